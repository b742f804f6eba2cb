"""Helpers shared by the tests: brute-force references and comparisons.

The brute-force products here are independent of the oracle: plain Python
loops over dense arrays that follow the definition of the product over a
semiring (Section 2 and Algorithm 1 of the paper), usable on tiny inputs.
"""

from __future__ import annotations

import os

import numpy as np

from synth import CSR

U = 2.0 ** -53
M64 = (1 << 64) - 1


def _to_signed(x: int) -> int:
    x &= M64
    return x - (1 << 64) if x >> 63 else x


def dense_of(M: CSR):
    """(stored mask, python value table) of a small CSR."""
    st = [[False] * M.ncols for _ in range(M.nrows)]
    va = [[None] * M.ncols for _ in range(M.nrows)]
    for i in range(M.nrows):
        for p in range(int(M.row_ptr[i]), int(M.row_ptr[i + 1])):
            j = int(M.col[p])
            st[i][j] = True
            va[i][j] = 1 if M.val is None else M.val[p].item()
    return st, va


def brute_product(A: CSR, B: CSR, sr: str, k_lo=0, k_hi=None):
    """Dict (i,j) -> value by the definition: triple loop, k ascending, the
    first term taken as is and later terms folded with the semiring add."""
    if k_hi is None:
        k_hi = A.ncols
    sa, va = dense_of(A)
    sb, vb = dense_of(B)
    out = {}
    for i in range(A.nrows):
        for j in range(B.ncols):
            acc = None
            for k in range(k_lo, k_hi):
                if not (sa[i][k] and sb[k][j]):
                    continue
                if sr == "f64":
                    t = float(va[i][k]) * float(vb[k][j])
                    acc = t if acc is None else acc + t
                elif sr == "i64":
                    t = _to_signed(int(va[i][k]) * int(vb[k][j]))
                    acc = t if acc is None else _to_signed(acc + t)
                else:
                    t = int(bool(va[i][k]) and bool(vb[k][j]))
                    acc = t if acc is None else (acc | t)
            if acc is not None:
                out[(i, j)] = acc
    return out


def brute_merge(layers, sr: str):
    out = {}
    for L in layers:
        st, va = dense_of(L)
        for i in range(L.nrows):
            for j in range(L.ncols):
                if not st[i][j]:
                    continue
                v = va[i][j]
                if (i, j) not in out:
                    out[(i, j)] = v if sr != "bool" else int(bool(v))
                elif sr == "f64":
                    out[(i, j)] = out[(i, j)] + float(v)
                elif sr == "i64":
                    out[(i, j)] = _to_signed(out[(i, j)] + int(v))
                else:
                    out[(i, j)] = out[(i, j)] | int(bool(v))
    return out


def csr_to_dict(C: CSR):
    d = {}
    for i in range(C.nrows):
        for p in range(int(C.row_ptr[i]), int(C.row_ptr[i + 1])):
            d[(i, int(C.col[p]))] = C.val[p].item() if C.val is not None else 1
    return d


def assert_same_structure(got: CSR, ref: CSR):
    assert got.nrows == ref.nrows and got.ncols == ref.ncols
    assert np.array_equal(np.asarray(got.row_ptr), np.asarray(ref.row_ptr)), "row pointers differ"
    assert np.array_equal(np.asarray(got.col), np.asarray(ref.col)), "column indices differ"


# FP64 entries that needed the second test, per calling test:
# (test id, entries over 1e-12 relative, entries compared); printed in the
# session summary by conftest.py
FP64_RECHECKS = []


def assert_values(got: CSR, ref: CSR, sr: str, check=None):
    """Integer and boolean values bit-exact.  FP64: every entry within 1e-12
    relative of the oracle's ascending-k value; an entry over that is
    re-checked against the compensated sum of the same terms (``check`` =
    oracle.f64_check(...) for the same entries, or a function returning it,
    called only when some entry needs it) and must lie within the
    bound of any summation order of those terms, oracle.f64_bound.  Returns
    the number of entries that needed the re-check; the count is recorded
    for the session summary and named in any failure message."""
    g = np.asarray(got.val)
    r = np.asarray(ref.val)
    if sr != "f64":
        assert g.dtype == r.dtype
        bad = np.nonzero(g != r)[0]
        assert bad.size == 0, "values differ at %s: got %s ref %s" % (
            bad[:5], g[bad[:5]], r[bad[:5]])
        return 0
    assert g.shape == r.shape
    err = np.abs(g - r)
    ok = err <= 1e-12 * np.abs(r)
    over = np.nonzero(~ok)[0]
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    FP64_RECHECKS.append((test, int(over.size), int(r.size)))
    if over.size == 0:
        return 0
    if callable(check):
        check = check()
    assert check is not None, (
        "%d FP64 entries over 1e-12 relative and no compensated check supplied: idx %s got %s ref %s" % (
            over.size, over[:5], g[over[:5]], r[over[:5]]))
    import oracle
    comp, absum, nterms = (np.asarray(x)[over] for x in check)
    bound = oracle.f64_bound(comp, absum, nterms)
    dev = np.abs(g[over] - comp)
    bad = over[dev > bound]
    assert bad.size == 0, (
        "%d of %d FP64 entries were over 1e-12 relative; %d of them are beyond the summation-order bound "
        "around the compensated sum, at %s (got %s, compensated %s)" % (
            over.size, r.size, bad.size, bad[:5], g[bad[:5]], np.asarray(check[0])[bad[:5]]))
    return int(over.size)


def column_form_flops(A: CSR, B: CSR, k_lo=0, k_hi=None) -> int:
    """flops = sum over k of nnz(A(:,k)) * nnz(B(k,:)) (column times row
    counts), an independent form of the per-row count."""
    if k_hi is None:
        k_hi = A.ncols
    colcnt = np.bincount(np.asarray(A.col, dtype=np.int64), minlength=A.ncols)
    rowlen = np.diff(np.asarray(B.row_ptr))
    k = np.arange(A.ncols)
    sel = (k >= k_lo) & (k < k_hi)
    return int(np.sum(colcnt[sel].astype(np.int64) * rowlen[sel]))
