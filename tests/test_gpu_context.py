"""Contexts and allocators (the library's data is allocated through the
caller's allocator, Sec. 4): every device buffer of a hierarchy, of its
multi-RHS engine and of a coefficient update comes from the context; a
failing allocation is reported as PAMG_E_OOM with everything that call
allocated freed again, and it leaves an existing hierarchy as it was."""
import numpy as np
import pytest

import paper_2210_16660_amd as pamg
from workloads import SplitMix64, q1_rhs, q1_stretched

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


class Injector:
    """torch's caching allocator with a switch that fails the k-th call from now."""

    def __init__(self):
        self.calls = 0
        self.fail_at = None
        self.live = {}

    def fail_after(self, k):
        self.fail_at = self.calls + k

    def alloc(self, nbytes, stream):
        i = self.calls
        self.calls += 1
        if self.fail_at is not None and i == self.fail_at:
            self.fail_at = None
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes, torch.cuda.current_device(), stream)
        self.live[p] = nbytes
        return p

    def free(self, ptr, stream):
        assert ptr in self.live, "freed a pointer the allocator never handed out"
        del self.live[ptr]
        torch.cuda.caching_allocator_delete(ptr)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda:0")


def test_setup_oom_at_every_stage_frees_everything():
    A = q1_stretched(12, 1.05)
    inj = Injector()
    ctx = pamg.Context(allocator=(inj.alloc, inj.free))
    H = pamg.Hierarchy(A, context=ctx, build_f32=1)
    n_setup = inj.calls
    H.close()
    st = ctx.stats()
    assert st.allocs == st.frees == n_setup and st.live_bytes == 0 and not inj.live
    assert n_setup > 20
    for k in sorted({0, 1, 2, n_setup // 3, n_setup // 2, n_setup - 2, n_setup - 1}):
        inj.fail_after(k)
        with pytest.raises(pamg.PamgError) as e:
            pamg.Hierarchy(A, context=ctx, build_f32=1)
        assert e.value.code == pamg.E_OOM, k
        st = ctx.stats()
        assert st.allocs == st.frees and st.live_bytes == 0 and st.users == 0, k
        assert not inj.live, k
    assert ctx.stats().failed >= 7
    ctx.close()


@pytest.mark.parametrize("steps", [1, 2])
def test_device_setup_oom_frees_everything(steps):
    # the device construction: canonical temporaries, layout arrays, the
    # host-built levels' uploads; a failure anywhere leaves nothing behind
    A = q1_stretched(32, 1.05)
    kw = dict(build_f32=1, device_setup=1, device_min_rows=1000, agg_steps=steps)
    inj = Injector()
    ctx = pamg.Context(allocator=(inj.alloc, inj.free))
    H = pamg.Hierarchy(A, context=ctx, **kw)
    assert H.info().device_levels >= 1
    n_setup = inj.calls
    H.close()
    st = ctx.stats()
    assert st.allocs == st.frees == n_setup and st.live_bytes == 0 and not inj.live
    assert n_setup > 60
    for k in sorted({0, 1, 5, n_setup // 4, n_setup // 3, n_setup // 2, 2 * n_setup // 3, n_setup - 2,
                     n_setup - 1}):
        inj.fail_after(k)
        with pytest.raises(pamg.PamgError) as e:
            pamg.Hierarchy(A, context=ctx, **kw)
        assert e.value.code == pamg.E_OOM, k
        st = ctx.stats()
        assert st.allocs == st.frees and st.live_bytes == 0 and st.users == 0, k
        assert not inj.live, k
    ctx.close()


def test_oom_leaves_an_existing_hierarchy_unchanged():
    N = 12
    A = q1_stretched(N, 1.05)
    b = dev(q1_rhs(N, 1.05, 2))
    inj = Injector()
    ctx = pamg.Context(allocator=(inj.alloc, inj.free))
    H = pamg.Hierarchy(A, context=ctx, build_f32=1)
    base = ctx.stats()

    def solve_bits():
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        info = H.solve(b, x, tol=1e-8)
        return x.cpu().numpy().view(np.uint64).copy(), info.iterations

    def same(u, v):
        return u[1] == v[1] and np.array_equal(u[0], v[0])

    ref = solve_bits()
    B = torch.from_numpy(np.stack([SplitMix64(40 + j).uniform(A.n) for j in range(16)])).cuda()
    # the 16-column engine: fail its k-th buffer, then build it for real
    for k in (0, 3, 9, 20):
        inj.fail_after(k)
        X = torch.zeros_like(B)
        with pytest.raises(pamg.PamgError) as e:
            H.solve_batch(B, X, tol=1e-8)
        assert e.value.code == pamg.E_OOM
        st = ctx.stats()
        assert st.allocs - st.frees == base.allocs - base.frees and st.live_bytes == base.live_bytes
        assert same(solve_bits(), ref)
    X = torch.zeros_like(B)
    infos = H.solve_batch(B, X, tol=1e-8)
    assert all(i.status == pamg.OK for i in infos)
    engine = ctx.stats()
    assert engine.live_bytes > base.live_bytes
    # coefficient update: its plan's k-th buffer fails, the hierarchy keeps its values
    v2 = torch.from_numpy(q1_stretched(N, 1.06).val).cuda()
    for k in (0, 5, 11):
        inj.fail_after(k)
        with pytest.raises(pamg.PamgError) as e:
            H.update_values(v2)
        assert e.value.code == pamg.E_OOM
        st = ctx.stats()
        assert st.live_bytes == engine.live_bytes and st.allocs - st.frees == engine.allocs - engine.frees
        assert same(solve_bits(), ref)
    H.update_values(v2)
    assert not same(solve_bits(), ref)
    # a context in use cannot be destroyed
    with pytest.raises(pamg.PamgError) as e:
        ctx.close()
    assert e.value.code == pamg.E_BUSY
    H.close()
    st = ctx.stats()
    assert st.allocs == st.frees and st.live_bytes == 0 and st.users == 0 and not inj.live
    ctx.close()


def test_hip_context_and_torch_context_give_the_same_result():
    A = q1_stretched(10, 1.05)
    b = dev(q1_rhs(10, 1.05, 2))
    out = []
    for allocator in ("hip", "torch"):
        ctx = pamg.Context(allocator=allocator)
        H = pamg.Hierarchy(A, context=ctx)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        H.solve(b, x, tol=1e-8)
        out.append(x.cpu().numpy())
        assert ctx.stats().live_bytes == H.info().device_bytes
        H.close()
        ctx.close()
    assert np.array_equal(out[0].view(np.uint64), out[1].view(np.uint64))
