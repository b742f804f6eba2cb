"""CPU oracle for the SpGEMM hot path (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never loads it; the two share no code.  Inputs come from the separate
``synth`` generators.

The arithmetic lives in ``oracle.c`` (row-wise Gustavson with a dense
sparse accumulator, Algorithm 1 of the paper written by rows; the merge adds
c layers entry by entry in ascending layer order, Section 4.3).  This file
compiles it with gcc on first use and marshals numpy arrays.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from synth import CSR

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

SEMIRINGS = {"f64": 0, "i64": 1, "bool": 2}
VAL_DTYPE = {"f64": np.float64, "i64": np.int64, "bool": np.uint8}


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-std=c99", "-Wall", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I64 = ctypes.c_int64
            lib.oracle_row_flops.argtypes = [I64, P, P, P, I64, I64, P]
            lib.oracle_spgemm_count.argtypes = [ctypes.c_int, I64, P, P, P, P, I64, I64, I64,
                                                P, P, ctypes.c_int]
            lib.oracle_spgemm_fill.argtypes = [ctypes.c_int, I64, P, P, P, P, P, P, I64, I64,
                                               I64, P, P, P, P, ctypes.c_int]
            lib.oracle_spgemm_f64_check.argtypes = [I64, P, P, P, P, P, P, I64, I64, I64, P, P, P, P, P,
                                                    ctypes.c_int]
            lib.oracle_merge_count.argtypes = [I64, I64, ctypes.c_int, P, P, P, ctypes.c_int]
            lib.oracle_merge_fill.argtypes = [ctypes.c_int, I64, I64, ctypes.c_int, P, P, P, P,
                                              P, P, ctypes.c_int]
            for f in (lib.oracle_row_flops, lib.oracle_spgemm_count, lib.oracle_spgemm_fill,
                      lib.oracle_spgemm_f64_check, lib.oracle_merge_count, lib.oracle_merge_fill):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def _window(A: CSR, k_lo, k_hi):
    k_lo = 0 if k_lo is None else int(k_lo)
    k_hi = A.ncols if k_hi is None else int(k_hi)
    return k_lo, k_hi


def row_flops(A: CSR, B: CSR, k_lo=None, k_hi=None) -> np.ndarray:
    """flops_i: scalar multiplications of row i (inner window [k_lo,k_hi))."""
    lib = _load()
    assert A.ncols == B.nrows
    k_lo, k_hi = _window(A, k_lo, k_hi)
    arp, acol, brp = _c(A.row_ptr, np.int64), _c(A.col, np.int32), _c(B.row_ptr, np.int64)
    out = np.zeros(A.nrows, dtype=np.int64)
    lib.oracle_row_flops(A.nrows, _p(arp), _p(acol), _p(brp), k_lo, k_hi, _p(out))
    return out


def row_counts(A: CSR, B: CSR, k_lo=None, k_hi=None, rows=None, nthreads: int = 0) -> np.ndarray:
    """nnz(C(i,:)) of every row (or of the rows given), structure only."""
    lib = _load()
    if A.ncols != B.nrows:
        raise ValueError("inner dimensions differ")
    k_lo, k_hi = _window(A, k_lo, k_hi)
    arp, acol = _c(A.row_ptr, np.int64), _c(A.col, np.int32)
    brp, bcol = _c(B.row_ptr, np.int64), _c(B.col, np.int32)
    sel = None if rows is None else _c(rows, np.int64)
    nsel = A.nrows if sel is None else sel.size
    cnt = np.zeros(nsel, dtype=np.int64)
    if lib.oracle_spgemm_count(2, B.ncols, _p(arp), _p(acol), _p(brp), _p(bcol), k_lo, k_hi, nsel, _p(sel),
                               _p(cnt), nthreads):
        raise MemoryError("oracle scratch allocation failed")
    return cnt


def _vals(M: CSR, sr: str):
    if M.val is None:
        if sr == "bool":
            return None
        raise ValueError("value array required for semiring %s" % sr)
    return _c(M.val, VAL_DTYPE[sr])


def spgemm(A: CSR, B: CSR, sr: str = "f64", k_lo=None, k_hi=None, rows=None,
           nthreads: int = 0, values: bool = True) -> CSR:
    """C = A(:,K) * B(K,:) over the semiring, K = [k_lo, k_hi).

    rows: optional subset of row indices; the result then holds exactly those
    rows, in the order given.  values=False returns the structure only."""
    lib = _load()
    if A.ncols != B.nrows:
        raise ValueError("inner dimensions differ")
    k_lo, k_hi = _window(A, k_lo, k_hi)
    srid = SEMIRINGS[sr]
    arp, acol = _c(A.row_ptr, np.int64), _c(A.col, np.int32)
    brp, bcol = _c(B.row_ptr, np.int64), _c(B.col, np.int32)
    sel = None if rows is None else _c(rows, np.int64)
    nsel = A.nrows if sel is None else sel.size
    cnt = np.zeros(nsel, dtype=np.int64)
    rc = lib.oracle_spgemm_count(srid, B.ncols, _p(arp), _p(acol), _p(brp), _p(bcol), k_lo, k_hi,
                                 nsel, _p(sel), _p(cnt), nthreads)
    if rc:
        raise MemoryError("oracle scratch allocation failed")
    ptr = np.zeros(nsel + 1, dtype=np.int64)
    np.cumsum(cnt, out=ptr[1:])
    col = np.zeros(int(ptr[-1]), dtype=np.int32)
    av = bv = val = None
    if values:
        av, bv = _vals(A, sr), _vals(B, sr)
        val = np.zeros(int(ptr[-1]), dtype=VAL_DTYPE[sr])
    rc = lib.oracle_spgemm_fill(srid, B.ncols, _p(arp), _p(acol), _p(av), _p(brp), _p(bcol), _p(bv),
                                k_lo, k_hi, nsel, _p(sel), _p(ptr), _p(col), _p(val), nthreads)
    if rc:
        raise MemoryError("oracle scratch allocation failed")
    return CSR(nsel, B.ncols, ptr, col, val)


def merge(layers, sr: str = "f64", nthreads: int = 0) -> CSR:
    """Entry-wise sum over the semiring of c same-shape CSR layers; equal
    (i,j) combine in ascending layer order (Section 4.3)."""
    lib = _load()
    c = len(layers)
    if c == 0:
        raise ValueError("need at least one layer")
    m, n = layers[0].nrows, layers[0].ncols
    for L in layers:
        if (L.nrows, L.ncols) != (m, n):
            raise ValueError("layer shapes differ")
    rps = [_c(L.row_ptr, np.int64) for L in layers]
    cols = [_c(L.col, np.int32) for L in layers]
    vals = [_vals(L, sr) for L in layers]
    P = ctypes.c_void_p
    rp_arr = (P * c)(*[r.ctypes.data for r in rps])
    col_arr = (P * c)(*[x.ctypes.data for x in cols])
    val_arr = (P * c)(*[(v.ctypes.data if v is not None else None) for v in vals])
    cnt = np.zeros(m, dtype=np.int64)
    if lib.oracle_merge_count(m, n, c, rp_arr, col_arr, _p(cnt), nthreads):
        raise MemoryError("oracle scratch allocation failed")
    ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(cnt, out=ptr[1:])
    col = np.zeros(int(ptr[-1]), dtype=np.int32)
    val = np.zeros(int(ptr[-1]), dtype=VAL_DTYPE[sr])
    if lib.oracle_merge_fill(SEMIRINGS[sr], m, n, c, rp_arr, col_arr, val_arr, _p(ptr), _p(col),
                             _p(val), nthreads):
        raise MemoryError("oracle scratch allocation failed")
    return CSR(m, n, ptr, col, val)


def f64_check(A: CSR, B: CSR, ref: CSR, k_lo=None, k_hi=None, rows=None, nthreads=0):
    """Per-entry data for checking an FP64 product summed in another order.

    ``ref`` is the oracle's product of A and B over the same window and rows
    (its structure fixes the entry order).  Returns three arrays aligned with
    ``ref.col``:

    comp    the entry's terms A(i,k)*B(k,j), each rounded once, added in
            ascending k with Neumaier's compensated summation: within
            u*|S| + (N-1)^2 u^2 sum|terms| of their exact sum S
            (u = 2^-53, N terms);
    abs_sum the sum of the terms' magnitudes;
    nterms  N, the number of terms.

    Any order of N-1 additions of the same rounded terms lands within
    (N-1) u / (1 - (N-1) u) * sum|terms| of S (the recursive-summation
    bound), so a result and comp differ by at most that plus u*|comp| and
    second-order terms (``f64_bound``)."""
    lib = _load()
    if A.ncols != B.nrows:
        raise ValueError("inner dimensions differ")
    k_lo, k_hi = _window(A, k_lo, k_hi)
    arp, acol, av = _c(A.row_ptr, np.int64), _c(A.col, np.int32), _c(A.val, np.float64)
    brp, bcol, bv = _c(B.row_ptr, np.int64), _c(B.col, np.int32), _c(B.val, np.float64)
    sel = None if rows is None else _c(rows, np.int64)
    nsel = A.nrows if sel is None else sel.size
    ptr = _c(ref.row_ptr, np.int64)
    assert ptr.size == nsel + 1
    nz = int(ptr[-1])
    comp = np.zeros(nz, dtype=np.float64)
    absum = np.zeros(nz, dtype=np.float64)
    nterms = np.zeros(nz, dtype=np.int64)
    rc = lib.oracle_spgemm_f64_check(B.ncols, _p(arp), _p(acol), _p(av), _p(brp), _p(bcol), _p(bv), k_lo, k_hi,
                                     nsel, _p(sel), _p(ptr), _p(comp), _p(absum), _p(nterms), nthreads)
    if rc:
        raise MemoryError("oracle scratch allocation failed")
    return comp, absum, nterms


U = 2.0 ** -53


def f64_bound(comp, abs_sum, nterms):
    """Largest |g - comp| of a value g that sums the same N rounded terms in
    any order: gamma_{N-1} * sum|terms| (recursive summation in any order)
    plus u*|comp| and 2 gamma_{N-1}^2 * sum|terms| for comp's own error, with
    gamma_k = k u / (1 - k u); sum|terms| is taken as abs_sum * (1 + 2 gamma)
    to cover abs_sum's own rounding."""
    n1 = np.maximum(np.asarray(nterms, dtype=np.float64) - 1.0, 0.0)
    g = n1 * U / (1.0 - n1 * U)
    a = np.asarray(abs_sum, dtype=np.float64) * (1.0 + 2.0 * g)
    return g * a + U * np.abs(np.asarray(comp)) + 2.0 * g * g * a
