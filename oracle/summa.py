"""Sparse SUMMA stage accumulation on one process, and the hypersparse
row-compressed format (TEST INFRASTRUCTURE ONLY: only the tests, the smoke
check and the benchmark's CPU-baseline leg import this module; the product
path never does).

DCSR is the row-wise counterpart of the DCSC format of Section 4.2: the
matrix keeps only its rows that hold at least one entry, each with its row
index, so its storage is O(nnz) whatever the row dimension (the column-wise
DCSC drops repeated column pointers the same way; C = A B by rows is the
transpose of the paper's column-wise formulation, so rows take the place of
columns).

summa_local is one process's share of Algorithm 2's stage loop (Section
4.1, Section 4.4): the process holds A's columns and B's rows of its
layer's inner range, split into `stages` stage blocks of equal width; each
stage block is cut further into blocks of b inner indices (the blocking
parameter b, which must divide the stage block).  Every block gives one
local product A(:,block) B(block,:), a rank-b update; the products are kept
and summed at the end by one multiway merge that adds equal entries in
stage order (Section 4.3).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from synth import CSR

from . import merge, spgemm, VAL_DTYPE


@dataclass
class DCSR:
    """Row-compressed sparse matrix: row_ids int64[nzr] strictly increasing,
    row_ptr int64[nzr+1], col int32[nnz], val[nnz]; every kept row holds at
    least one entry."""

    nrows: int
    ncols: int
    row_ids: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    val: Optional[np.ndarray]

    @property
    def nzr(self) -> int:
        return int(self.row_ids.size)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def compress(M: CSR) -> DCSR:
    """The DCSR of a CSR matrix: drop the row pointers of empty rows and
    record the indices of the rows kept (Section 4.2)."""
    lens = np.diff(M.row_ptr)
    keep = np.nonzero(lens > 0)[0].astype(np.int64)
    row_ptr = np.append(M.row_ptr[keep], M.row_ptr[-1]).astype(np.int64)
    val = None if M.val is None else M.val.copy()
    return DCSR(M.nrows, M.ncols, keep, row_ptr, M.col.astype(np.int32).copy(), val)


def expand(D: DCSR) -> CSR:
    """The CSR of a DCSR matrix: absent rows are empty."""
    lens = np.zeros(D.nrows, dtype=np.int64)
    lens[D.row_ids] = np.diff(D.row_ptr)
    row_ptr = np.zeros(D.nrows + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    val = None if D.val is None else D.val.copy()
    return CSR(D.nrows, D.ncols, row_ptr, D.col.copy(), val)


def stage_blocks(inner: int, stages: int, b: int):
    """Inner-index windows [lo, hi) of the local products, in stage order:
    `stages` stage blocks of inner/stages indices, each cut into blocks of b
    (Algorithm 2: the stage loop over r and the loop over the b-wide blocks
    of the local inner dimension)."""
    if stages < 1 or b < 1:
        raise ValueError("stages and b must be positive")
    if inner % stages:
        raise ValueError("the stage count must divide the inner dimension")
    per_stage = inner // stages
    if per_stage % b:
        raise ValueError("b must divide the inner width of a stage")
    return [(r * per_stage + q * b, r * per_stage + (q + 1) * b)
            for r in range(stages) for q in range(per_stage // b)]


def summa_local(A: DCSR, B: CSR, stages: int, b: int, sr: str = "f64"):
    """C = sum over the blocks, in stage order, of A(:,block) B(block,:).

    Returns (C as DCSR, the total number of entries of the kept block
    products: the intermediate the merge reads)."""
    if A.ncols != B.nrows:
        raise ValueError("inner dimensions differ")
    Ac = expand(A)
    prods = [spgemm(Ac, B, sr, lo, hi) for lo, hi in stage_blocks(A.ncols, stages, b)]
    stage_nnz = sum(P.nnz for P in prods)
    if prods:
        C = merge(prods, sr)
    else:
        C = CSR(A.nrows, B.ncols, np.zeros(A.nrows + 1, np.int64), np.zeros(0, np.int32),
                np.zeros(0, VAL_DTYPE[sr]))
    return compress(C), stage_nnz
