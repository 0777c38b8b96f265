"""Compressed sparse row container shared by the generators."""
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """A square sparse matrix in CSR form.

    ``row_ptr`` is int32[n+1], ``col`` int32[nnz] (sorted and distinct within
    each row), ``val`` float64[nnz].  ``meta`` records how it was generated.
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    meta: dict

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def check(self) -> None:
        """Raise ValueError unless the arrays form a valid CSR matrix."""
        rp, c = self.row_ptr, self.col
        if rp.dtype != np.int32 or c.dtype != np.int32 or self.val.dtype != np.float64:
            raise ValueError("CSR dtypes must be int32/int32/float64")
        if rp.shape != (self.n + 1,) or rp[0] != 0 or np.any(np.diff(rp) < 0):
            raise ValueError("row_ptr must be monotone, start at 0, have n+1 entries")
        if c.shape != (self.nnz,) or self.val.shape != (self.nnz,):
            raise ValueError("col/val length must equal nnz")
        if self.nnz and (c.min() < 0 or c.max() >= self.n):
            raise ValueError("column index out of range")
        # strictly increasing columns inside every row
        d = np.diff(c.astype(np.int64))
        row_start = np.zeros(self.nnz, dtype=bool)
        row_start[rp[:-1][np.diff(rp) > 0]] = True
        if self.nnz > 1 and np.any((d <= 0) & ~row_start[1:]):
            raise ValueError("columns must be strictly increasing within a row")

    def norm1(self) -> float:
        """Largest absolute column sum (the matrix 1-norm)."""
        s = np.zeros(self.n)
        np.add.at(s, self.col, np.abs(self.val))
        return float(s.max()) if self.n else 0.0

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        a[rows, self.col] = self.val
        return a


def from_triplets(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray, meta: dict) -> CSR:
    """Assemble a CSR matrix from (row, col, val) triplets with distinct (row, col)."""
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    return CSR(n, row_ptr.astype(np.int32), cols.astype(np.int32),
               np.ascontiguousarray(vals, dtype=np.float64), meta)
