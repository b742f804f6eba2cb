"""Pins of the oracle's FP64 check data (oracle.f64_check, oracle.f64_bound).

The GPU sums an entry's terms A(i,k)*B(k,j) in another order than the
oracle's ascending k (LDS atomics, merge trees), so an FP64 entry is accepted
when it is within 1e-12 relative of the oracle's value, or within the bound
of any summation order around a compensated sum of the same terms.  These
tests pin the three arrays behind that second test against exact rational
arithmetic (Python's Fraction) on tiny inputs, and the bound against sums
taken in shuffled orders:

* nterms is the number of k in the window with A(i,k) and B(k,j) stored;
* abs_sum is sum |A(i,k)*B(k,j)| up to the rounding of a sum of positives;
* comp is within u*|S| + 2 gamma^2 sum|terms| of the exact sum S of the
  rounded terms (Neumaier's compensated summation);
* a case whose plain ascending-k sum cancels to 0 while the exact sum is 1.
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth import CSR
from util import dense_of

U = 2.0 ** -53


def _terms(A: CSR, B: CSR, k_lo=0, k_hi=None):
    """(i, j) -> list of rounded products in ascending k, by the definition."""
    if k_hi is None:
        k_hi = A.ncols
    sa, va = dense_of(A)
    sb, vb = dense_of(B)
    out = {}
    for i in range(A.nrows):
        for j in range(B.ncols):
            t = [float(va[i][k]) * float(vb[k][j]) for k in range(k_lo, k_hi) if sa[i][k] and sb[k][j]]
            if t:
                out[(i, j)] = t
    return out


def _check_against_exact(A, B, k_lo=0, k_hi=None, rows=None):
    ref = oracle.spgemm(A, B, "f64", k_lo, k_hi, rows=rows)
    comp, absum, nterms = oracle.f64_check(A, B, ref, k_lo, k_hi, rows=rows)
    terms = _terms(A, B, k_lo, k_hi)
    sel = range(A.nrows) if rows is None else rows
    e = 0
    for r, i in enumerate(sel):
        for p in range(int(ref.row_ptr[r]), int(ref.row_ptr[r + 1])):
            t = terms[(int(i), int(ref.col[p]))]
            n = len(t)
            assert nterms[p] == n
            S = sum(Fraction(x) for x in t)
            Aex = sum(Fraction(abs(x)) for x in t)
            g = (n - 1) * U / (1 - (n - 1) * U)
            # a recursive sum of non-negative terms: relative error <= gamma_{n-1}
            assert abs(Fraction(absum[p]) - Aex) <= Fraction(g) * Aex
            # compensated sum: u|S| + 2 gamma^2 sum|t|
            assert abs(Fraction(comp[p]) - S) <= Fraction(U) * abs(S) + 2 * Fraction(g) ** 2 * Aex
            e += 1
    assert e == ref.nnz
    return ref, comp, absum, nterms


def test_check_data_against_exact_sums():
    """Random tiny products with mixed signs, explicit zeros and windows."""
    rng = np.random.default_rng(71)
    for trial in range(30):
        m, k, n = (int(x) for x in rng.integers(1, 9, 3))
        dens = float(rng.choice([0.3, 0.6, 1.0]))
        A = synth.random_csr(m, k, dens, int(rng.integers(1 << 30)), "f64")
        B = synth.random_csr(k, n, dens, int(rng.integers(1 << 30)), "f64")
        A = CSR(A.nrows, A.ncols, A.row_ptr, A.col, (A.val - 0.5) * 10.0 ** rng.integers(-3, 4, A.nnz))
        B = CSR(B.nrows, B.ncols, B.row_ptr, B.col, (B.val - 0.5) * 10.0 ** rng.integers(-3, 4, B.nnz))
        if A.nnz:
            A.val[rng.random(A.nnz) < 0.1] = 0.0  # explicit zeros stay terms
        lo = int(rng.integers(0, k + 1))
        hi = int(rng.integers(lo, k + 1))
        _check_against_exact(A, B, lo, hi)
        rows = rng.permutation(m)[: max(1, m // 2)].astype(np.int64)
        _check_against_exact(A, B, rows=rows)


def test_compensated_sum_survives_cancellation():
    """Terms 1e16, 1, -1e16 (ascending k): the plain sum rounds 1e16 + 1 to
    1e16 and ends at 0; the exact sum is 1, and so is the compensated one."""
    A = synth.canonical_from_coo(1, 3, [0, 0, 0], [0, 1, 2], np.array([1e16, 1.0, -1e16]), dup="first")
    B = synth.canonical_from_coo(3, 1, [0, 1, 2], [0, 0, 0], np.ones(3), dup="first")
    ref, comp, absum, nterms = _check_against_exact(A, B)
    assert ref.val[0] == 0.0
    assert comp[0] == 1.0
    assert nterms[0] == 3
    assert absum[0] == 2e16 + 1.0 or absum[0] == 2e16  # rounded sum of magnitudes


def test_bound_covers_every_summation_order():
    """Entries with many terms summed in shuffled orders (pairwise trees and
    left-to-right) stay within f64_bound of comp; a value moved by twice the
    bound does not."""
    rng = np.random.default_rng(72)
    A = synth.random_csr(6, 3000, 0.5, 73, "f64")
    B = synth.random_csr(3000, 4, 0.5, 74, "f64")
    A = CSR(A.nrows, A.ncols, A.row_ptr, A.col, A.val - 0.5)
    ref = oracle.spgemm(A, B, "f64")
    comp, absum, nterms = oracle.f64_check(A, B, ref)
    terms = _terms(A, B)
    bound = oracle.f64_bound(comp, absum, nterms)
    assert np.all(bound > 0)
    for r in range(A.nrows):
        for p in range(int(ref.row_ptr[r]), int(ref.row_ptr[r + 1])):
            t = np.array(terms[(r, int(ref.col[p]))])
            for _ in range(4):
                x = list(rng.permutation(t))
                s = 0.0
                for v in x:
                    s += v
                assert abs(s - comp[p]) <= bound[p]
                while len(x) > 1:  # a pairwise tree in a random order
                    x = [x[q] + x[q + 1] if q + 1 < len(x) else x[q] for q in range(0, len(x), 2)]
                assert abs(x[0] - comp[p]) <= bound[p]
            assert abs((comp[p] + 2 * bound[p]) - comp[p]) > bound[p]


@pytest.mark.parametrize("n,expect", [(1, 0.0), (2, U / (1 - U))])
def test_bound_closed_form(n, expect):
    """One term: no addition, so the bound is u|comp| alone; two terms: one
    rounding, gamma_1 = u/(1-u) of the magnitude sum (plus second-order terms)."""
    b = oracle.f64_bound(np.array([3.0]), np.array([5.0]), np.array([n]))
    g = expect
    a = 5.0 * (1 + 2 * g)
    assert b[0] == pytest.approx(g * a + U * 3.0 + 2 * g * g * a, rel=1e-15)
