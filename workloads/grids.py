"""Finite-difference Laplacians on the unit cube (input generators).

* ``lap7(n)``: the 7-point Laplacian on n^3 interior nodes with homogeneous
  Dirichlet boundary, h = 1/(n+1), scaled by 1/h^2 (6 on the diagonal,
  -1 to each of the six neighbours).  The scale is an exact integer.
* ``varcoef7(n, seed)``: the 7-point discretisation of -div(k grad p) with a
  log-normal coefficient per cell: k_c = exp(g_c), g_c ~ N(0, 1), one value
  for each of the (n+1)^3 cells; the coupling across a grid edge is the mean
  of the four cells touching that edge divided by h^2.  With k == 1 it is
  bitwise the ``lap7`` operator.

Dofs are numbered lexicographically, x fastest: idx = i + n*j + n*n*k.
Off-diagonal values are computed once per edge and mirrored, so every
matrix is bitwise symmetric.
"""
from __future__ import annotations

import numpy as np

from .csr import CSR, from_dense_rows
from .rng import SplitMix64

# stencil offsets in ascending column order for x-fastest numbering
_OFFS7 = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def _assemble7(n: int, cx: np.ndarray, cy: np.ndarray, cz: np.ndarray) -> CSR:
    """cx[i,j,k] is the coupling of grid edge (i-1 -> i) along x for interior
    node (i,j,k) in extended grid coords, arrays of shape (n+1, n, n) etc.
    Shapes: cx (n+1, n, n) indexed [i_edge, j, k] with edge i_edge joining
    interior x-positions i_edge-1 and i_edge (positions -1 and n are boundary).
    """
    N = n * n * n
    i = np.arange(n)
    I, J, K = np.meshgrid(i, i, i, indexing="ij")
    # per-node coefficients of the 6 edges
    west = cx[I, J, K]          # edge between i-1 and i
    east = cx[I + 1, J, K]      # edge between i and i+1
    south = cy[I, J, K]
    north = cy[I, J + 1, K]
    down = cz[I, J, K]
    up = cz[I, J, K + 1]
    diag = ((west + east) + (south + north)) + (down + up)
    idx = (I + n * J + n * n * K)
    cols = np.empty((n, n, n, 7), dtype=np.int64)
    vals = np.empty((n, n, n, 7), dtype=np.float64)
    mask = np.empty((n, n, n, 7), dtype=bool)
    coefs = [-down, -south, -west, diag, -east, -north, -up]
    for s, (dx, dy, dz) in enumerate(_OFFS7):
        cols[..., s] = idx + dx + n * dy + n * n * dz
        vals[..., s] = coefs[s]
        mask[..., s] = ((I + dx >= 0) & (I + dx < n) & (J + dy >= 0) & (J + dy < n)
                        & (K + dz >= 0) & (K + dz < n))
    # reorder to row-major over idx (x fastest): transpose (i,j,k) -> (k,j,i)
    cols = cols.transpose(2, 1, 0, 3).reshape(N, 7)
    vals = vals.transpose(2, 1, 0, 3).reshape(N, 7)
    mask = mask.transpose(2, 1, 0, 3).reshape(N, 7)
    return from_dense_rows(N, cols, vals, mask)


def lap7(n: int) -> CSR:
    """7-point Laplacian on n^3 interior nodes, homogeneous Dirichlet, 1/h^2 scaling."""
    inv_h2 = float((n + 1) * (n + 1))
    cx = np.full((n + 1, n, n), inv_h2)
    cy = np.full((n, n + 1, n), inv_h2)
    cz = np.full((n, n, n + 1), inv_h2)
    return _assemble7(n, cx, cy, cz)


def cell_coefficients(n: int, seed: int) -> np.ndarray:
    """k_c = exp(g_c), g_c ~ N(0,1) from SplitMix64(seed), shape (n+1,)*3 indexed [cx, cy, cz]
    (draw order: cx fastest)."""
    g = SplitMix64(seed).normal((n + 1) ** 3)
    return np.exp(g).reshape(n + 1, n + 1, n + 1).transpose(2, 1, 0).copy()


def varcoef7(n: int, seed: int | None = None, kappa: np.ndarray | None = None) -> CSR:
    """Variable-coefficient 7-point operator.  Grid positions 0..n+1 per axis,
    interior nodes 1..n; cell c spans positions [c, c+1], c = 0..n."""
    if kappa is None:
        kappa = cell_coefficients(n, seed)
    inv_h2 = float((n + 1) * (n + 1))
    k = kappa
    # x-edge between positions a and a+1 (a = 0..n) at interior (j, l) positions 1..n:
    # touching cells: cx = a, cy in {j-1, j}, cz in {l-1, l}
    a = np.arange(n + 1)
    j = np.arange(1, n + 1)
    A, Jg, Lg = np.meshgrid(a, j, j, indexing="ij")
    cx = ((k[A, Jg - 1, Lg - 1] + k[A, Jg, Lg - 1]) + (k[A, Jg - 1, Lg] + k[A, Jg, Lg])) * 0.25 * inv_h2
    Jg, A, Lg = np.meshgrid(j, a, j, indexing="ij")
    cy = ((k[Jg - 1, A, Lg - 1] + k[Jg, A, Lg - 1]) + (k[Jg - 1, A, Lg] + k[Jg, A, Lg])) * 0.25 * inv_h2
    Jg, Lg, A = np.meshgrid(j, j, a, indexing="ij")
    cz = ((k[Jg - 1, Lg - 1, A] + k[Jg, Lg - 1, A]) + (k[Jg - 1, Lg, A] + k[Jg, Lg, A])) * 0.25 * inv_h2
    return _assemble7(n, cx, cy, cz)


def uniform_rhs(n_dofs: int, seed: int) -> np.ndarray:
    """b_i ~ U[-1, 1] i.i.d. from SplitMix64(seed)."""
    return SplitMix64(seed).uniform(n_dofs)
