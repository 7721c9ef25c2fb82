"""Plain CSR container shared by the workload generators (input data only)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """0-based CSR, full symmetric storage, columns sorted in every row."""
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def check(self, symmetric: bool = True) -> None:
        """Structural checks plus (optionally) bitwise symmetry."""
        rp, c = self.row_ptr, self.col
        assert rp.dtype == np.int32 and c.dtype == np.int32 and self.val.dtype == np.float64
        assert rp[0] == 0 and len(rp) == self.n + 1
        assert np.all(np.diff(rp) > 0)
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(rp))
        key = rows * self.n + c
        assert np.all(np.diff(key) > 0), "columns must be strictly ascending"
        if symmetric:
            order = np.lexsort((rows, c.astype(np.int64)))
            assert np.array_equal(c[order].astype(np.int64), rows), "pattern not symmetric"
            # entries sorted by (col,row) are the transpose in CSR order
            assert np.array_equal(self.val[order].view(np.uint64), self.val.view(np.uint64)), \
                "values not bitwise symmetric"


def from_dense_rows(n: int, cols: np.ndarray, vals: np.ndarray, mask: np.ndarray) -> CSR:
    """Build CSR from an (n, k) table of candidate entries whose columns are
    already ascending along axis 1; ``mask`` selects the stored ones."""
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("nnz does not fit int32 indices")
    col = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    return CSR(n, row_ptr.astype(np.int32), col, val)
