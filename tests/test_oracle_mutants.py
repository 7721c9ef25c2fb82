"""The oracle's pins must reject plausible mistakes.

Each case plants one mistake in a copy of the oracle source (a dropped term,
a wrong sign or index, a transposed operand, a flipped tie-break), compiles
it on the CPU and runs the pin suite against it in a subprocess: every mutant
must make at least one pin fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "post_smooth_sign": ("z[i] += dinv[i] * (r[i] - t[i]);", "z[i] += dinv[i] * (t[i] - r[i]);"),
    "residual_sign": ("t[i] = r[i] - t[i];             /* residual */", "t[i] = r[i] + t[i];             /* residual */"),
    "hgs_residual_sign": ("t[i] = r[i] - t[i];         /* residual */", "t[i] = r[i] + t[i];         /* residual */"),
    "prolong_drops_p": ("z[i] += h->p[l][i] * e[h->agg[l][i]];", "z[i] += e[h->agg[l][i]];"),
    "restrict_drops_p": ("rc[h->agg[l][i]] += h->p[l][i] * t[i];", "rc[h->agg[l][i]] += t[i];"),
    "weight_wrong_index": ("double num = ((2.0 * a_lohi) * w_lo) * w_hi;",
                           "double num = ((2.0 * a_lohi) * w_lo) * w_lo;"),
    "eligibility_all": ("if (match_all || c > 1.0)", "if (match_all || c > 0.0)"),
    "galerkin_transposed_p": ("t[m].t = a->v[k] * (p[i] * p[j]);", "t[m].t = a->v[k] * (p[i] * p[i]);"),
    "tie_break_flipped": ("if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;",
                          "if (a->lo != b->lo) return a->lo < b->lo ? 1 : -1;"),
    "fcg_beta_sign": ("double beta = -dot(n, z, q) / delta_old;", "double beta = dot(n, z, q) / delta_old;"),
    "pcg_direction_sign": ("double beta = rho / rho_old; for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];",
                           "double beta = rho / rho_old; for (int i = 0; i < n; ++i) p[i] = z[i] - beta * p[i];"),
    "cholesky_drops_term": ("for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];",
                            "for (int k = 1; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];"),
    "l1_not_absolute": ("for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) d += fabs(a->v[k]);",
                        "for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) d += a->v[k];"),
    "pair_norm_wrong": ("double nu = sqrt(w[i] * w[i] + w[m] * w[m]);", "double nu = sqrt(w[i] * w[i] + w[i] * w[m]);"),
    "stop_rule_not_strict": ("(double)A->n < min_ratio * (double)(A->n - pairs)",
                             "(double)A->n <= min_ratio * (double)(A->n - pairs)"),
    "stop_rule_ignores_dense_limit": ("if (A->n <= max_dense && (double)A->n < min_ratio",
                                      "if ((double)A->n < min_ratio"),
    "compose_drops_p": ("                pc = pc * h->p[m][I];", "                pc = pc * h->p[a][I];"),
    "compose_wrong_chain": ("                I = h->agg[m][I];", "                I = h->agg[a][I];"),
    "update_stale_smoother": ("        st = l1_inverse(&g->A[j], g->dinv[j]);\n        if (st) break;",
                              "        memcpy(g->dinv[j], h->dinv[j], sizeof(double) * (size_t)n);"),
    "update_wrong_step_p": ("st = galerkin(&chain[m], h->pw_agg[m], h->pw_p[m], h->pw_n[m + 1], &chain[m + 1]);",
                            "st = galerkin(&chain[m], h->pw_agg[m], h->pw_p[0], h->pw_n[m + 1], &chain[m + 1]);"),
    "update_ignores_kept_map": ("        const int m = h->kept[j], n = chain[m].n;", "        const int m = j, n = chain[m].n;"),
    "update_old_coarse_factor": ("if (!st) st = dense_cholesky(&g->A[g->nlev - 1], &g->chol);",
                                 "if (!st) st = dense_cholesky(&h->A[h->nlev - 1], &g->chol);"),
    "hgs_fresh_wrong_side": ("if (qj >= b0 && qj < b1 && (backward ? qj > q : qj < q)) fresh",
                             "if (qj >= b0 && qj < b1 && (backward ? qj < q : qj > q)) fresh"),
    "hgs_ignores_blocks": ("if (qj >= b0 && qj < b1 && (backward ? qj > q : qj < q)) fresh",
                           "if ((backward ? qj > q : qj < q)) fresh"),
    "hgs_post_forward": ("oracle_hgs_smooth(h, l, 1, 0, r, z);", "oracle_hgs_smooth(h, l, 0, 0, r, z);"),
    "hgs_omega_dropped": ("x_new[i] = x_old[i] + d[i] / h->gs_omega;", "x_new[i] = x_old[i] + d[i];"),
    "hgs_omega_inside": ("d[i] = ((r[i] - old) - fresh) / aii;", "d[i] = ((r[i] - old) - fresh) / (h->gs_omega * aii);"),
    "nested_members_descending": ("for (int i = 0; i < nf; ++i) finer[first[h->agg[m][i]]++] = i;",
                                  "for (int i = nf - 1; i >= 0; --i) finer[first[h->agg[m][i]]++] = i;"),
    "sa_omega_l1_diagonal": ("        double r = s / aii;\n        if (r > mx) mx = r;", "        double r = s / s;\n        if (r > mx) mx = r;"),
    "sa_smoothing_sign": ("P->v[u] = P->v[u] - (omega * (a->v[k] / aii)) * p[j];",
                          "P->v[u] = P->v[u] + (omega * (a->v[k] / aii)) * p[j];"),
    "sa_wrong_column_weight": ("P->v[u] = P->v[u] - (omega * (a->v[k] / aii)) * p[j];",
                               "P->v[u] = P->v[u] - (omega * (a->v[k] / aii)) * p[i];"),
    "sa_restrict_uses_tentative": ("for (int u = P->rp[i]; u < P->rp[i + 1]; ++u) rc[P->ci[u]] += P->v[u] * t[i];",
                                   "rc[h->agg[l][i]] += h->p[l][i] * t[i];"),
    "sa_galerkin_drops_lower_mirror": ("if (J != I) { out->ci[mark[J]] = I; out->v[mark[J]] = U.v[u]; mark[J]++; }",
                                       "if (J != I) { out->ci[mark[J]] = I; out->v[mark[J]] = 0.0; mark[J]++; }"),
    "sa_composed_p_not_multiplied": ("                    cp[i] = cp[i] * p[I];", "                    cp[i] = p[I];"),
    "sa_composed_smooths_wrong_matrix": ("st = smoothed_prolongator(K, cagg, cp, &h->P[j], &h->omega_p[j]);",
                                         "st = smoothed_prolongator(&h->A[0], cagg, cp, &h->P[j], &h->omega_p[j]);"),
    "backsolve_transposed": ("for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * z[k];",
                             "for (int k = i + 1; k < n; ++k) s -= L[(size_t)i * n + k] * z[k];"),
    "round_f32_dinv_unrounded": ("g->dinv[l][i] = (double)(float)h->dinv[l][i];", "g->dinv[l][i] = h->dinv[l][i];"),
    "round_f32_rounds_w": ("g->w[l][i] = h->w[l][i];", "g->w[l][i] = (double)(float)h->w[l][i];"),
    "round_f32_p_unrounded": ("for (int i = 0; i < a->n; ++i) g->p[l][i] = (double)(float)h->p[l][i];",
                              "for (int i = 0; i < a->n; ++i) g->p[l][i] = h->p[l][i];"),
    "round_f32_chol_unrounded": ("g->chol[k] = (double)(float)h->chol[k];", "g->chol[k] = h->chol[k];"),
    "restart_from_recurrence_residual": (
        "restart:\n    csr_mv(A, x, q);\n    for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];",
        "    csr_mv(A, x, q);\n    for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];\nrestart:"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", str(mut), "-o", str(so), "-lm"],
                   check=True)
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
