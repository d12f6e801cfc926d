"""Block-sparse storage used by the oracle (test infrastructure only).

A ``BlockCSR`` keeps the *structural* pattern of a matrix: an entry exists for
every pair of nodes coupled through an element (or, on coarse levels, through
the Galerkin product of such patterns), even where its value is exactly zero.
The coarsening of Section 3.2 works on the connectivity graph of the matrix,
so the pattern, not the numerical value, defines the graph.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class BlockCSR:
    indptr: np.ndarray   # (nrows+1,) int64
    indices: np.ndarray  # (nnz,) int64, sorted within each row
    vals: np.ndarray     # (nnz, br, bc) float64
    ncols: int           # number of block columns

    @property
    def nrows(self) -> int:
        return self.indptr.shape[0] - 1

    @property
    def nnz(self) -> int:
        return self.indices.shape[0]

    @property
    def bshape(self) -> tuple[int, int]:
        return self.vals.shape[1], self.vals.shape[2]

    def scipy(self) -> sp.csr_matrix:
        br, bc = self.bshape
        m = sp.bsr_matrix((self.vals, self.indices, self.indptr),
                          shape=(self.nrows * br, self.ncols * bc))
        return m.tocsr()

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = M x with x of shape (ncols, bc) (or flat); returns (nrows, br)."""
        br, bc = self.bshape
        xs = np.asarray(x, dtype=np.float64).reshape(self.ncols, bc)
        y = np.zeros((self.nrows, br))
        rows = np.repeat(np.arange(self.nrows), np.diff(self.indptr))
        contrib = np.einsum("kij,kj->ki", self.vals, xs[self.indices])
        for c in range(br):
            y[:, c] = np.bincount(rows, weights=contrib[:, c], minlength=self.nrows)
        return y

    def dense(self) -> np.ndarray:
        return self.scipy().toarray()

    def pattern(self) -> sp.csr_matrix:
        """Node-level structural pattern as a 0/1 CSR matrix."""
        return sp.csr_matrix((np.ones(self.nnz), self.indices, self.indptr),
                             shape=(self.nrows, self.ncols))

    def row_of(self) -> np.ndarray:
        return np.repeat(np.arange(self.nrows), np.diff(self.indptr))

    def diag_blocks(self) -> np.ndarray:
        """Diagonal blocks (square matrices only), shape (n, br, bc)."""
        rows = self.row_of()
        on = np.nonzero(rows == self.indices)[0]
        assert on.shape[0] == self.nrows, "every row must hold its diagonal block"
        return self.vals[on]

    def transpose(self) -> "BlockCSR":
        br, bc = self.bshape
        rows = self.row_of()
        order = np.lexsort((rows, self.indices))
        t_rows = self.indices[order]
        indptr = np.zeros(self.ncols + 1, dtype=np.int64)
        np.add.at(indptr, t_rows + 1, 1)
        indptr = np.cumsum(indptr)
        return BlockCSR(indptr, rows[order].astype(np.int64),
                        np.ascontiguousarray(self.vals[order].transpose(0, 2, 1)), self.nrows)


def from_pairs(rows: np.ndarray, cols: np.ndarray, nrows: int, ncols: int,
               br: int, bc: int) -> tuple[BlockCSR, np.ndarray]:
    """Structural pattern from (row, col) pairs with duplicates.

    Returns an all-zero BlockCSR with the sorted unique pattern and, for every
    input pair, the position of its entry (for scatter-add of element values).
    """
    keys = rows.astype(np.int64) * ncols + cols.astype(np.int64)
    uk, inv = np.unique(keys, return_inverse=True)
    r = uk // ncols
    indptr = np.zeros(nrows + 1, dtype=np.int64)
    np.add.at(indptr, r + 1, 1)
    indptr = np.cumsum(indptr)
    M = BlockCSR(indptr, (uk % ncols).astype(np.int64), np.zeros((uk.shape[0], br, bc)), ncols)
    return M, inv.ravel()


def scatter_add(M: BlockCSR, pos: np.ndarray, vals: np.ndarray) -> None:
    """M.vals[pos[k]] += vals[k] for every k (duplicates summed in index order)."""
    br, bc = M.bshape
    v = vals.reshape(-1, br, bc)
    for i in range(br):
        for j in range(bc):
            M.vals[:, i, j] += np.bincount(pos, weights=v[:, i, j], minlength=M.nnz)


def csr_scalar(indptr, indices, data, nrows, ncols) -> sp.csr_matrix:
    return sp.csr_matrix((data, indices, indptr), shape=(nrows, ncols))
