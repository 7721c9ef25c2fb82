"""Trilinear (Q1) hexahedral finite-element Laplacian on a boundary-layer
stretched mesh, and a discrete-divergence right-hand side (input generators).

Mesh: nodes (i, j, k), 0 <= i, j, k <= N, at x_i = i/N, y_j = j/N and
z_k = (r^k - 1)/(r^N - 1): element heights grow geometrically by r from the
bottom wall z = 0.  Element (ex, ey, ez) has sizes hx = hy = 1/N and
hz = z_{ez+1} - z_{ez}.

Element stiffness (exact for trilinear shape functions on a box):
    K_e[a, b] = (hy hz / hx) K[ax,bx] M[ay,by] M[az,bz]
              + (hx hz / hy) M[ax,bx] K[ay,by] M[az,bz]
              + (hx hy / hz) M[ax,bx] M[ay,by] K[az,bz]
with the unit-interval 1D matrices K = [[1,-1],[-1,1]] and
M = [[1/3,1/6],[1/6,1/3]], and local corners a = (ax, ay, az) in {0,1}^3.

Boundary conditions: Dirichlet on the top face z = 1 (the k = N layer is
eliminated), natural (Neumann) elsewhere, and node (0,0,0) pinned and
eliminated.  The remaining nodes are numbered lexicographically (x fastest,
then y, then z from the bottom).  The pattern keeps every in-grid neighbour
that shares an element (27-point stencil), including entries whose value
is exactly zero.

Right-hand side: b_a = sum over elements of int phi_a div(u_h), with u_h the
Q1 interpolant of a smooth random velocity field
u(x) = sum_{m<64} a_m sin(2 pi k_m . x + phi_m),  k_m in Z^3 \\ {0}, |k_m| <= 8,
a_m ~ U[-1,1]^3, phi_m ~ U[0, 2 pi).  Rows of eliminated nodes are dropped.
"""
from __future__ import annotations

import numpy as np

from .csr import CSR
from .rng import SplitMix64

_K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
_M1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
# int_0^1 phi_a dphi_b/dx dx for phi_0 = 1-x, phi_1 = x
_C1 = np.array([[-0.5, 0.5], [-0.5, 0.5]])

_CORNERS = [(ax, ay, az) for az in (0, 1) for ay in (0, 1) for ax in (0, 1)]
# the 27 neighbour offsets in ascending column order (z slowest, x fastest)
_OFFS27 = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def node_z(N: int, ratio: float) -> np.ndarray:
    k = np.arange(N + 1, dtype=np.float64)
    if ratio == 1.0:
        return k / N
    return (ratio ** k - 1.0) / (ratio ** N - 1.0)


def _elem_entry(a, b, hz: np.ndarray, h: float) -> np.ndarray:
    """K_e[a, b] for all element heights hz (hx = hy = h)."""
    ax, ay, az = a
    bx, by, bz = b
    t1 = (h * hz / h) * (_K1[ax, bx] * _M1[ay, by] * _M1[az, bz])
    t2 = (h * hz / h) * (_M1[ax, bx] * _K1[ay, by] * _M1[az, bz])
    t3 = (h * h / hz) * (_M1[ax, bx] * _M1[ay, by] * _K1[az, bz])
    return (t1 + t2) + t3


def _dof_numbering(N: int) -> np.ndarray:
    """dof index of node (i,j,k) (array [i,j,k]); -1 for eliminated nodes."""
    keep = np.ones((N + 1, N + 1, N + 1), dtype=bool)
    keep[:, :, N] = False         # Dirichlet top layer
    keep[0, 0, 0] = False         # pinned node
    flat_keep = keep.transpose(2, 1, 0).reshape(-1)   # x-fastest order
    num = np.full(flat_keep.shape, -1, dtype=np.int64)
    num[flat_keep] = np.arange(int(flat_keep.sum()))
    return num.reshape(N + 1, N + 1, N + 1).transpose(2, 1, 0)


def q1_stretched(N: int, ratio: float = 1.05, progress=None) -> CSR:
    """Assemble the Q1 stiffness matrix described in the module docstring.

    An entry depends on the x and y position of its row node only through
    whether that node is on the first, an interior or the last plane (which
    element corners exist), so the coefficients are summed once per such
    class and gathered; the per-element sums keep the corner order.
    ``progress(msg)`` is called after each stencil offset."""
    P = N + 1
    h = 1.0 / N
    z = node_z(N, ratio)
    hz = z[1:] - z[:-1]                       # (N,)
    rep = np.array([0, min(1, N), N])         # a node of each class: first, interior, last
    cls = np.ones(P, dtype=np.intp)
    cls[0], cls[N] = 0, 2
    kk = np.arange(P)
    # coef[d][cx, cy, k]: entry (u, u + d) for offsets d >= 0 in column order;
    # the lower half is mirrored from the upper half for bitwise symmetry.
    upper = [d for d in _OFFS27 if (d[2], d[1], d[0]) >= (0, 0, 0)]
    coef = {}
    for d in upper:
        acc = np.zeros((3, 3, P))
        for a in _CORNERS:
            b = (a[0] + d[0], a[1] + d[1], a[2] + d[2])
            if min(b) < 0 or max(b) > 1:
                continue
            # element e = u - a must exist: 0 <= u_c - a_c < N
            vx = (rep - a[0] >= 0) & (rep - a[0] < N)
            vy = (rep - a[1] >= 0) & (rep - a[1] < N)
            ez = np.clip(kk - a[2], 0, N - 1)
            vz = (kk - a[2] >= 0) & (kk - a[2] < N)
            ent_z = np.where(vz, _elem_entry(a, b, hz[ez], h), 0.0)       # (P,)
            m = (vx[:, None, None] & vy[None, :, None] & vz[None, None, :])
            acc += np.where(m, ent_z[None, None, :], 0.0)
        coef[d] = acc
    # kept nodes in dof order: lexicographic index lex = i + P j + P^2 k (x
    # fastest) with the top layer k = N and the pinned node lex = 0 removed,
    # so dof = lex - 1.  Rows are assembled in cache-sized chunks.
    n = P * P * N - 1
    chunk = 1 << 16
    rp_parts, col_parts, val_parts = [], [], []
    cols = np.empty((chunk, 27), dtype=np.int32)
    vals = np.empty((chunk, 27))
    next_report = 0.1
    for r0 in range(0, n, chunk):
        lex = np.arange(r0 + 1, min(n, r0 + chunk) + 1, dtype=np.int64)
        m = lex.size
        i = lex % P
        j = (lex // P) % P
        k = lex // (P * P)
        ci, cj = cls[i], cls[j]
        for s, d in enumerate(_OFFS27):
            dx, dy, dz = d
            i2, j2, k2 = i + dx, j + dy, k + dz
            keep2 = ((i2 >= 0) & (i2 <= N) & (j2 >= 0) & (j2 <= N) & (k2 >= 0) & (k2 < N)
                     & ~((i2 == 0) & (j2 == 0) & (k2 == 0)))
            cols[:m, s] = np.where(keep2, lex + (dx + P * dy + P * P * dz) - 1, -1)
            if d in coef:
                vals[:m, s] = coef[d][ci, cj, k]
            else:  # mirror: a(u, u+d) = a(u+d, u) = coef[-d] at node u+d
                vals[:m, s] = coef[(-dx, -dy, -dz)][cls[np.clip(i2, 0, N)], cls[np.clip(j2, 0, N)],
                                                    np.clip(k2, 0, N)]
        mask = cols[:m] >= 0
        rp_parts.append(mask.sum(axis=1))
        col_parts.append(cols[:m][mask])
        val_parts.append(vals[:m][mask])
        if progress is not None and (r0 + m) / n >= next_report:
            progress(f"Q1 {N}^3 assembly: {100 * (r0 + m) // n}% of rows")
            next_report += 0.1
    counts = np.concatenate(rp_parts)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("nnz does not fit int32 indices")
    return CSR(n, row_ptr.astype(np.int32), np.concatenate(col_parts), np.concatenate(val_parts))


def random_modes(seed: int, n_modes: int = 64, kmax: int = 8):
    """Wave vectors (rejection sampling of components in [-kmax, kmax] with
    0 < |k| <= kmax), amplitudes U[-1,1]^3 and phases U[0, 2 pi)."""
    rng = SplitMix64(seed)
    ks = []
    while len(ks) < n_modes:
        cand = rng.integers(3, -kmax, kmax)
        r2 = int((cand * cand).sum())
        if 0 < r2 <= kmax * kmax:
            ks.append(cand)
    k = np.array(ks, dtype=np.float64)
    amp = rng.uniform(3 * n_modes).reshape(n_modes, 3)
    phase = 2.0 * np.pi * rng.uniform01(n_modes)
    return k, amp, phase


def velocity_field(N: int, ratio: float, seed: int, progress=None) -> np.ndarray:
    """Nodal velocity u[c, i, j, k] (c = component) of the random smooth field."""
    k, amp, phase = random_modes(seed)
    x = np.arange(N + 1) / N
    zc = node_z(N, ratio)
    u = np.zeros((3, N + 1, N + 1, N + 1))
    for m in range(k.shape[0]):
        ex = np.exp(2j * np.pi * k[m, 0] * x)
        ey = np.exp(2j * np.pi * k[m, 1] * x)
        ez = np.exp(2j * np.pi * k[m, 2] * zc) * np.exp(1j * phase[m])
        s = np.imag(ex[:, None, None] * ey[None, :, None] * ez[None, None, :])
        for c in range(3):
            u[c] += amp[m, c] * s
        if progress is not None and (m + 1) % 16 == 0:
            progress(f"velocity field {N}^3: {m + 1}/{k.shape[0]} modes")
    return u


def divergence_rhs(N: int, ratio: float, u: np.ndarray) -> np.ndarray:
    """b = D u assembled over elements (rows of eliminated nodes dropped)."""
    h = 1.0 / N
    z = node_z(N, ratio)
    hz = z[1:] - z[:-1]
    P = N + 1
    b = np.zeros((P, P, P))
    for a in _CORNERS:
        acc = np.zeros((N, N, N))
        for bc in _CORNERS:
            ux = u[0][bc[0]:bc[0] + N, bc[1]:bc[1] + N, bc[2]:bc[2] + N]
            uy = u[1][bc[0]:bc[0] + N, bc[1]:bc[1] + N, bc[2]:bc[2] + N]
            uz = u[2][bc[0]:bc[0] + N, bc[1]:bc[1] + N, bc[2]:bc[2] + N]
            dx = _C1[a[0], bc[0]] * (h * _M1[a[1], bc[1]]) * (hz * _M1[a[2], bc[2]])
            dy = (h * _M1[a[0], bc[0]]) * _C1[a[1], bc[1]] * (hz * _M1[a[2], bc[2]])
            dz = (h * _M1[a[0], bc[0]]) * (h * _M1[a[1], bc[1]]) * _C1[a[2], bc[2]]
            acc += ux * dx[None, None, :] + uy * dy[None, None, :] + uz * dz
        b[a[0]:a[0] + N, a[1]:a[1] + N, a[2]:a[2] + N] += acc
    num = _dof_numbering(N)
    keep = num >= 0
    out = np.empty(int(keep.sum()))
    out[num[keep]] = b[keep]
    return out


def q1_rhs(N: int, ratio: float, seed: int, progress=None) -> np.ndarray:
    return divergence_rhs(N, ratio, velocity_field(N, ratio, seed, progress))


def q1_rhs_sequence(N: int, ratio: float, seed: int, count: int = 16, amp: float = 0.05):
    """Consecutive-time-step stand-in: u(0) from seed, then
    u(t) = u(t-1) + amp * (rms(u(0)) / rms(delta(t))) * delta(t), delta(t) from seed + t."""
    u0 = velocity_field(N, ratio, seed)
    rms0 = np.sqrt(np.mean(u0 * u0))
    out = [divergence_rhs(N, ratio, u0)]
    u = u0
    for t in range(1, count):
        d = velocity_field(N, ratio, seed + t)
        u = u + amp * (rms0 / np.sqrt(np.mean(d * d))) * d
        out.append(divergence_rhs(N, ratio, u))
    return np.stack(out, axis=1)   # (n, count), row-major
