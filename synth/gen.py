"""Seeded generators for the synthetic workloads of the SpGEMM experiments.

Matrix classes follow the experimental setup of the paper (Section 5):
R-MAT with the G500, SSCA and Erdos-Renyi seed parameters, scale s giving a
2^s x 2^s matrix with an average of 16 (G500, ER) or 8 (SSCA) nonzeros per
row, and a random symmetric permutation P A P^T applied to spread load.
The restriction workload of Section 5.3 is stood in for by a 7-point 3D
Poisson operator and a piecewise-constant 2x2x2 aggregation R.

All randomness comes from numpy's Philox counter-based generator keyed by
the seed, so every input is reproducible on any machine.  Matrices are
returned as canonical CSR: int64 row pointers, int32 column indices sorted
strictly increasing within each row, one value array (float64, int64 or
uint8 for the three semirings).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# R-MAT seed parameters (a, b, c, d), Section 5.
G500 = (0.57, 0.19, 0.19, 0.05)
SSCA = (0.6, 0.4 / 3, 0.4 / 3, 0.4 / 3)
ER = (0.25, 0.25, 0.25, 0.25)


@dataclass
class CSR:
    """Host CSR matrix: row_ptr int64[nrows+1], col int32[nnz], val[nnz]."""

    nrows: int
    ncols: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: Optional[np.ndarray]
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row(self, i: int):
        s, e = int(self.row_ptr[i]), int(self.row_ptr[i + 1])
        v = None if self.val is None else self.val[s:e]
        return self.col[s:e], v

    def is_canonical(self) -> bool:
        rp = self.row_ptr
        if rp.shape != (self.nrows + 1,) or rp[0] != 0:
            return False
        if np.any(np.diff(rp) < 0):
            return False
        if self.col.shape[0] != rp[-1]:
            return False
        if self.nnz == 0:
            return True
        c = self.col.astype(np.int64)
        if c.min() < 0 or c.max() >= self.ncols:
            return False
        # strictly increasing inside rows: every step inside a row is > 0
        d = np.diff(c)
        row_of = np.repeat(np.arange(self.nrows), np.diff(rp))
        same_row = row_of[1:] == row_of[:-1]
        return bool(np.all(d[same_row] > 0))

    def to_dense(self, dtype=np.float64) -> np.ndarray:
        d = np.zeros((self.nrows, self.ncols), dtype=dtype)
        row_of = np.repeat(np.arange(self.nrows), np.diff(self.row_ptr))
        vals = np.ones(self.nnz, dtype=dtype) if self.val is None else self.val
        d[row_of, self.col.astype(np.int64)] = vals
        return d

    def pattern(self) -> np.ndarray:
        p = np.zeros((self.nrows, self.ncols), dtype=bool)
        row_of = np.repeat(np.arange(self.nrows), np.diff(self.row_ptr))
        p[row_of, self.col.astype(np.int64)] = True
        return p


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed)))


def canonical_from_coo(nrows, ncols, rows, cols, vals, dup="sum") -> CSR:
    """Sort (row, col) pairs, combine duplicates, build canonical CSR.

    dup="sum" adds the values of repeated coordinates in generation order
    (the R-MAT workloads sum duplicates); dup="first" keeps the first one.
    Combining duplicates is input preparation, not part of the product.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = rows * np.int64(ncols) + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size:
        starts = np.concatenate(([0], np.nonzero(np.diff(key))[0] + 1))
    else:
        starts = np.zeros(0, dtype=np.int64)
    ukey = key[starts]
    if vals is None:
        uval = None
    else:
        v = np.asarray(vals)[order]
        if dup == "sum" and v.size:
            uval = np.add.reduceat(v, starts)
        else:
            uval = v[starts]
    urow = ukey // ncols if ncols else ukey
    ucol = (ukey - urow * ncols).astype(np.int32)
    counts = np.bincount(urow, minlength=nrows) if nrows else np.zeros(0, np.int64)
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(nrows, ncols, row_ptr, ucol, uval)


def rmat(scale: int, edge_factor: int = 16, abcd=G500, seed: int = 0,
         permute: bool = True, dup: str = "sum") -> CSR:
    """R-MAT matrix of scale s (2^s x 2^s) with edge_factor * 2^s edges.

    Each edge picks one of the four quadrants with probabilities (a,b,c,d)
    at each of the s recursion levels, independently, with no noise.
    Values are U(0,1) per generated edge; duplicates are summed; self loops
    are kept; the matrix is not symmetrised.  With permute=True a seeded
    random symmetric permutation P A P^T is applied (Section 5).
    """
    n = 1 << scale
    ne = edge_factor * n
    rng = _rng(seed)
    a, b, c, _ = abcd
    t1, t2, t3 = a, a + b, a + b + c
    rows = np.zeros(ne, dtype=np.int64)
    cols = np.zeros(ne, dtype=np.int64)
    for level in range(scale):
        u = rng.random(ne)
        q = (u >= t1).astype(np.int64) + (u >= t2) + (u >= t3)
        bit = np.int64(1) << np.int64(scale - 1 - level)
        rows |= np.where(q >= 2, bit, 0)
        cols |= np.where((q & 1) == 1, bit, 0)
    vals = rng.random(ne)
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        rows = perm[rows]
        cols = perm[cols]
    m = canonical_from_coo(n, n, rows, cols, vals, dup=dup)
    m.meta = dict(kind="rmat", scale=scale, edge_factor=edge_factor,
                  abcd=tuple(abcd), seed=seed, permuted=permute)
    return m


def er_uniform_columns(n: int, per_col: int, seed: int) -> CSR:
    """n x n matrix with exactly per_col distinct uniform-random rows in each
    column (sampling without replacement) and U(0,1) values."""
    rng = _rng(seed)
    rows = np.empty(n * per_col, dtype=np.int64)
    for j in range(n):
        rows[j * per_col:(j + 1) * per_col] = rng.choice(n, per_col, replace=False)
    cols = np.repeat(np.arange(n, dtype=np.int64), per_col)
    vals = rng.random(n * per_col)
    m = canonical_from_coo(n, n, rows, cols, vals, dup="first")
    m.meta = dict(kind="er_uniform_columns", n=n, per_col=per_col, seed=seed)
    return m


def random_csr(m: int, n: int, density: float, seed: int, kind="f64",
               explicit_zero_frac: float = 0.0) -> CSR:
    """Small random matrix for tests: independent Bernoulli(density)
    pattern; values per semiring kind ("f64": U(-1,1) with some exact zeros,
    "i64": integers in [-3,3], "bool": 0/1)."""
    rng = _rng(seed)
    mask = rng.random((m, n)) < density
    rows, cols = np.nonzero(mask)
    nnz = rows.size
    if kind == "f64":
        vals = rng.uniform(-1.0, 1.0, nnz)
        z = rng.random(nnz) < explicit_zero_frac
        vals[z] = 0.0
    elif kind == "i64":
        vals = rng.integers(-3, 4, nnz).astype(np.int64)
    elif kind == "bool":
        vals = (rng.random(nnz) >= explicit_zero_frac).astype(np.uint8)
    else:
        raise ValueError(kind)
    return canonical_from_coo(m, n, rows, cols, vals, dup="first")


def with_values(a: CSR, kind: str, seed: Optional[int] = None) -> CSR:
    """Same structure, new values: "ones_i64", "true_bool", "ones_f64",
    or "uniform_f64" (U(0,1), needs a seed)."""
    nnz = a.nnz
    if kind == "ones_i64":
        v = np.ones(nnz, dtype=np.int64)
    elif kind == "true_bool":
        v = np.ones(nnz, dtype=np.uint8)
    elif kind == "ones_f64":
        v = np.ones(nnz, dtype=np.float64)
    elif kind == "uniform_f64":
        v = _rng(seed).random(nnz)
    else:
        raise ValueError(kind)
    return CSR(a.nrows, a.ncols, a.row_ptr, a.col, v, dict(a.meta))


def identity(n: int, kind: str = "f64") -> CSR:
    dt = {"f64": np.float64, "i64": np.int64, "bool": np.uint8}[kind]
    return CSR(n, n, np.arange(n + 1, dtype=np.int64),
               np.arange(n, dtype=np.int32), np.ones(n, dtype=dt))


def permutation_matrix(perm: np.ndarray, kind: str = "f64") -> CSR:
    """P with P(i, perm[i]) = 1, so (P X)(i,:) = X(perm[i], :)."""
    n = perm.size
    dt = {"f64": np.float64, "i64": np.int64, "bool": np.uint8}[kind]
    return CSR(n, n, np.arange(n + 1, dtype=np.int64),
               perm.astype(np.int32), np.ones(n, dtype=dt))


def permute_symmetric(a: CSR, perm: np.ndarray) -> CSR:
    """Return B with B(perm[i], perm[j]) = A(i, j) (square A)."""
    row_of = np.repeat(np.arange(a.nrows, dtype=np.int64), np.diff(a.row_ptr))
    p = perm.astype(np.int64)
    return canonical_from_coo(a.nrows, a.ncols, p[row_of], p[a.col.astype(np.int64)],
                              a.val, dup="first")


def poisson7(N: int) -> CSR:
    """Unscaled 7-point Laplacian on an N^3 grid with Dirichlet boundaries:
    6 on the diagonal and -1 for each in-grid face neighbour.  The grid
    point (x, y, z) has index x + N*(y + N*z)."""
    idx = np.arange(N ** 3, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    rows = [idx]
    cols = [idx]
    vals = [np.full(idx.size, 6.0)]
    for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
        xx, yy, zz = x + dx, y + dy, z + dz
        ok = (xx >= 0) & (xx < N) & (yy >= 0) & (yy < N) & (zz >= 0) & (zz < N)
        rows.append(idx[ok])
        cols.append((xx + N * (yy + N * zz))[ok])
        vals.append(np.full(int(ok.sum()), -1.0))
    m = canonical_from_coo(N ** 3, N ** 3, np.concatenate(rows), np.concatenate(cols),
                           np.concatenate(vals), dup="first")
    m.meta = dict(kind="poisson7", N=N)
    return m


def aggregation_2x2x2(N: int):
    """Piecewise-constant aggregation over 2x2x2 blocks of an N^3 grid.

    Returns (RT, R): R is N^3 x M^3 with R(i, agg(i)) = 1, M = ceil(N/2),
    agg(x,y,z) = (x//2) + M*((y//2) + M*(z//2)); RT is its transpose, built
    directly as CSR (rows = aggregates, fine points increasing)."""
    M = (N + 1) // 2
    idx = np.arange(N ** 3, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    agg = (x // 2) + M * ((y // 2) + M * (z // 2))
    R = canonical_from_coo(N ** 3, M ** 3, idx, agg, np.ones(idx.size), dup="first")
    RT = canonical_from_coo(M ** 3, N ** 3, agg, idx, np.ones(idx.size), dup="first")
    R.meta = dict(kind="aggregation_R", N=N, M=M)
    RT.meta = dict(kind="aggregation_RT", N=N, M=M)
    return RT, R


def galerkin_batch(count: int = 64, nmin: int = 16, nmax: int = 64, seed: int = 5):
    """Batch of AMG Galerkin instances: grid sizes N_i ~ UniformInt[nmin, nmax]
    and, per instance, (RT_i, A_i, R_i) with A_i = poisson7(N_i)."""
    rng = _rng(seed)
    sizes = rng.integers(nmin, nmax + 1, count)
    out = []
    for N in sizes.tolist():
        A = poisson7(N)
        RT, R = aggregation_2x2x2(N)
        out.append((RT, A, R))
    return sizes, out


def layer_bounds(K: int, c: int):
    """Contiguous inner-dimension layers K_l = [floor(l*K/c), floor((l+1)*K/c)),
    the split distribution of Section 4 along the third grid dimension."""
    return [((l * K) // c, ((l + 1) * K) // c) for l in range(c)]


def submatrix(M: CSR, r0: int, r1: int, c0: int, c1: int) -> CSR:
    """Rows [r0, r1) and columns [c0, c1) of M, renumbered from 0."""
    rp = M.row_ptr
    s, e = int(rp[r0]), int(rp[r1])
    rows = np.repeat(np.arange(r1 - r0, dtype=np.int64), np.diff(rp[r0:r1 + 1]))
    cols = M.col[s:e].astype(np.int64)
    keep = (cols >= c0) & (cols < c1)
    val = None if M.val is None else M.val[s:e][keep]
    out = canonical_from_coo(r1 - r0, c1 - c0, rows[keep], cols[keep] - c0, val, dup="first")
    return out


def process_share(M: CSR, grid: int, layers: int, i: int, j: int, k: int):
    """The blocks of A = B = M that process P(i, j, k) of a grid x grid x
    layers process grid multiplies in its Sparse SUMMA stages: A's rows of
    process row i and B's columns of process column j, both over the inner
    range of layer k (the layer's n/layers inner indices, which the grid
    stages cover in `grid` equal stage blocks).  Returns (A_loc, B_loc)."""
    n = M.nrows
    if n % grid or n % layers or (n // layers) % grid:
        raise ValueError("the grid must divide the dimension")
    mb, kb = n // grid, n // layers
    A = submatrix(M, i * mb, (i + 1) * mb, k * kb, (k + 1) * kb)
    B = submatrix(M, k * kb, (k + 1) * kb, j * mb, (j + 1) * mb)
    return A, B
