"""Minimal CSR container used by the oracle (test infrastructure only).

Sums that feed the setup phase are formed strictly left to right in IEEE
double precision (one rounding per addition, products rounded before they are
added), so that every value is fixed by the order in which the terms are
listed.  ``ordered_segment_sum`` is that rule written out.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    rowptr: np.ndarray   # int64 (nrows+1)
    col: np.ndarray      # int64 (nnz), sorted within each row
    val: np.ndarray      # float64 (nnz)
    ncols: int

    @property
    def nrows(self) -> int:
        return self.rowptr.size - 1

    @property
    def nnz(self) -> int:
        return self.col.size

    def rows(self) -> np.ndarray:
        """Row index of every stored entry."""
        return np.repeat(np.arange(self.nrows), np.diff(self.rowptr))

    def scipy(self) -> sp.csr_matrix:
        m = sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.nrows, self.ncols))
        m.has_sorted_indices = True
        return m

    def matvec(self, x: np.ndarray) -> np.ndarray:
        return self.scipy() @ x

    def dense(self) -> np.ndarray:
        d = np.zeros((self.nrows, self.ncols))
        d[self.rows(), self.col] = self.val
        return d

    def diag(self) -> np.ndarray:
        r = self.rows()
        m = r == self.col
        d = np.zeros(self.nrows)
        d[r[m]] = self.val[m]
        return d

    def astype32(self) -> "CSR":
        return CSR(self.rowptr, self.col, self.val.astype(np.float32), self.ncols)


def ordered_segment_sum(vals: np.ndarray, segptr: np.ndarray) -> np.ndarray:
    """out[s] = (((0 + v[p0]) + v[p0+1]) + ...) for p in segment s, in order."""
    nseg = segptr.size - 1
    lens = np.diff(segptr)
    out = np.zeros(nseg, dtype=vals.dtype)
    if nseg == 0 or vals.size == 0:
        return out
    order = np.argsort(-lens, kind="stable")      # longest segments first
    slens = lens[order]
    starts = segptr[:-1][order]
    neg = -slens                                   # ascending
    for p in range(int(slens[0])):
        k = int(np.searchsorted(neg, -p, side="left"))   # segments longer than p: a prefix
        idx = order[:k]
        out[idx] = out[idx] + vals[starts[:k] + p]
    return out


def from_sorted_triples(rows: np.ndarray, cols: np.ndarray, vals: np.ndarray,
                        nrows: int, ncols: int) -> CSR:
    """Build a CSR from triples already grouped by (row, col) in the order the
    terms must be summed; duplicate (row, col) keys are summed in that order."""
    key = rows.astype(np.int64) * ncols + cols.astype(np.int64)
    if key.size:
        new = np.empty(key.size, dtype=bool)
        new[0] = True
        new[1:] = key[1:] != key[:-1]
        starts = np.nonzero(new)[0]
    else:
        starts = np.zeros(0, dtype=np.int64)
    segptr = np.append(starts, key.size)
    v = ordered_segment_sum(vals, segptr)
    ukey = key[starts]
    urow = ukey // ncols
    ucol = ukey % ncols
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.add.at(rowptr, urow + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(rowptr, ucol, v, ncols)


def sum_by_key(rows, cols, vals, nrows, ncols) -> CSR:
    """Stable-sort triples by (row, col) (keeping the given order inside each
    key) and sum each key left to right."""
    key = rows.astype(np.int64) * ncols + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    return from_sorted_triples(rows[order], cols[order], vals[order], nrows, ncols)


def transpose(a: CSR) -> CSR:
    """Stable transpose: row J of the result lists the rows i of a that hold
    column J, in ascending i."""
    r = a.rows()
    order = np.argsort(a.col, kind="stable")
    rowptr = np.zeros(a.ncols + 1, dtype=np.int64)
    np.add.at(rowptr, a.col + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(rowptr, r[order], a.val[order], a.nrows)


def find(a: CSR, i: int, k: int):
    """Value of a[i, k] if stored, else None."""
    s, e = a.rowptr[i], a.rowptr[i + 1]
    p = np.searchsorted(a.col[s:e], k)
    if p < e - s and a.col[s + p] == k:
        return a.val[s + p]
    return None


def is_structurally_symmetric_and_equal(a: CSR) -> bool:
    t = transpose(a)
    return (np.array_equal(a.rowptr, t.rowptr) and np.array_equal(a.col, t.col)
            and np.array_equal(a.val.view(np.uint64), t.val.view(np.uint64)))
