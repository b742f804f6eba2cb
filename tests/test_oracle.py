"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: hand-worked
products, brute force by the definition on tiny inputs, an independent
library product, closed forms (flop identity, C1's exact flop count, the
AMG Galerkin stencil), and invariants (identity and permutation operands,
layer split = unsplit product).
"""

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from synth import CSR
from util import (assert_same_structure, assert_values, brute_merge, brute_product,
                  column_form_flops, csr_to_dict)

HERE = os.path.dirname(os.path.abspath(__file__))


def _from_dense_lists(D, sr):
    rows, cols, vals = [], [], []
    for i, r in enumerate(D):
        for j, v in enumerate(r):
            if v is not None:
                rows.append(i)
                cols.append(j)
                vals.append(v)
    dt = oracle.VAL_DTYPE[sr]
    return synth.canonical_from_coo(len(D), len(D[0]), rows, cols, np.array(vals, dtype=dt),
                                    dup="first")


def test_hand_worked_products():
    """Products worked out by hand (tests/golden/hand_products.json)."""
    cases = json.load(open(os.path.join(HERE, "golden", "hand_products.json")))["cases"]
    for case in cases:
        sr = case["semiring"]
        A = _from_dense_lists(case["A"], sr)
        B = _from_dense_lists(case["B"], sr)
        lo, hi = case["window"]
        C = oracle.spgemm(A, B, sr, lo, hi)
        got = [[i, int(C.col[p]), C.val[p].item()]
               for i in range(C.nrows) for p in range(C.row_ptr[i], C.row_ptr[i + 1])]
        assert got == case["C"], case["name"]


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_brute_force_tiny(sr):
    """Oracle == triple-loop definition, bit-exact (same summation order),
    over tiny shapes including empty dimensions, all densities, explicit
    zeros and cancelling values, full and partial inner windows."""
    rng = np.random.default_rng(11)
    seed = 0
    for m in (0, 1, 3, 7, 12):
        for kk in (0, 1, 5, 12):
            for n in (0, 2, 9, 12):
                for dens in (0.0, 0.1, 0.3, 1.0):
                    seed += 1
                    A = synth.random_csr(m, kk, dens, seed, sr, explicit_zero_frac=0.2)
                    B = synth.random_csr(kk, n, dens, seed + 7919, sr, explicit_zero_frac=0.2)
                    windows = [(0, kk)]
                    if kk > 1:
                        lo = int(rng.integers(0, kk))
                        hi = int(rng.integers(lo, kk + 1))
                        windows.append((lo, hi))
                    for lo, hi in windows:
                        C = oracle.spgemm(A, B, sr, lo, hi)
                        assert C.is_canonical()
                        ref = brute_product(A, B, sr, lo, hi)
                        got = csr_to_dict(C)
                        assert got.keys() == ref.keys()
                        for key, v in ref.items():
                            if sr == "f64":
                                assert np.float64(got[key]).tobytes() == np.float64(v).tobytes()
                            else:
                                assert got[key] == v


def test_flop_identity_and_c1_closed_form():
    """Row form sum_i flops_i == column form sum_k nnz(A(:,k)) nnz(B(k,:));
    for C1 (exactly 4 entries per column of A) flops(A,A) = 4 nnz(A) =
    65,536 and nnz(A) = 16,384."""
    A = synth.er_uniform_columns(4096, 4, seed=1)
    assert A.nnz == 16384
    f = oracle.row_flops(A, A)
    assert int(f.sum()) == 65536 == column_form_flops(A, A)
    R = synth.rmat(12, 16, synth.G500, seed=21)
    for lo, hi in [(0, R.ncols), (100, 2000), (0, 0), (4095, 4096)]:
        assert int(oracle.row_flops(R, R, lo, hi).sum()) == column_form_flops(R, R, lo, hi)


def test_bounds_max_b_row_and_flops():
    """max_{k in A(i,:)} nnz(B(k,:)) <= nnz(C(i,:)) <= min(flops_i, n) and
    nnz(C) <= flops (Section 4.4)."""
    A = synth.rmat(12, 16, synth.G500, seed=22)
    C = oracle.spgemm(A, A, "bool")
    cnt = np.diff(C.row_ptr)
    f = oracle.row_flops(A, A)
    blen = np.diff(A.row_ptr)
    maxb = np.zeros(A.nrows, dtype=np.int64)
    for i in range(A.nrows):
        cs, _ = A.row(i)
        if cs.size:
            maxb[i] = blen[cs].max()
    assert np.all(maxb <= cnt)
    assert np.all(cnt <= np.minimum(f, A.ncols))
    assert C.nnz <= f.sum()


def test_against_independent_library_product():
    """Structure and path counts equal scipy's product of the 0/1 patterns
    (no cancellation possible with positive counts); FP64 with U(0,1)
    values within the summation-order bound of scipy's product."""
    A = synth.rmat(12, 16, synth.G500, seed=23)
    B = synth.rmat(12, 16, synth.ER, seed=24)
    Sa = sp.csr_matrix((np.ones(A.nnz, np.int64), A.col, A.row_ptr), shape=(A.nrows, A.ncols))
    Sb = sp.csr_matrix((np.ones(B.nnz, np.int64), B.col, B.row_ptr), shape=(B.nrows, B.ncols))
    P = (Sa @ Sb).tocsr()
    P.sort_indices()
    A1 = synth.with_values(A, "ones_i64")
    B1 = synth.with_values(B, "ones_i64")
    C = oracle.spgemm(A1, B1, "i64")
    assert np.array_equal(C.row_ptr, P.indptr.astype(np.int64))
    assert np.array_equal(C.col, P.indices.astype(np.int32))
    assert np.array_equal(C.val, P.data.astype(np.int64))
    Fa = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.nrows, A.ncols))
    Fb = sp.csr_matrix((B.val, B.col, B.row_ptr), shape=(B.nrows, B.ncols))
    Q = (Fa @ Fb).tocsr()
    Q.sort_indices()
    Cf = oracle.spgemm(A, B, "f64")
    assert np.array_equal(Cf.col, Q.indices.astype(np.int32))
    ref = CSR(Q.shape[0], Q.shape[1], Q.indptr.astype(np.int64), Q.indices.astype(np.int32), Q.data)
    # scipy sums in its own order: within the order bound of the same terms
    assert_values(Cf, ref, "f64", oracle.f64_check(A, B, Cf))


def test_cross_semiring_and_path_counts():
    """Same stored set for all three semirings; with all-ones INT64 the sum
    of C is exactly flops (each entry counts length-2 paths); boolean values
    are all true."""
    A = synth.rmat(11, 16, synth.G500, seed=25)
    f = int(oracle.row_flops(A, A).sum())
    Cf = oracle.spgemm(A, A, "f64")
    Ci = oracle.spgemm(synth.with_values(A, "ones_i64"), synth.with_values(A, "ones_i64"), "i64")
    Cb = oracle.spgemm(synth.with_values(A, "true_bool"), synth.with_values(A, "true_bool"), "bool")
    assert_same_structure(Ci, Cf)
    assert_same_structure(Cb, Cf)
    assert int(Ci.val.sum()) == f
    assert np.all(Cb.val == 1)


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_identity_operands(sr):
    """A I = A and I A = A exactly (each entry has a single term)."""
    kind = {"f64": "uniform_f64", "i64": "ones_i64", "bool": "true_bool"}[sr]
    A = synth.rmat(10, 8, synth.G500, seed=26)
    A = synth.with_values(A, kind, seed=3)
    I = synth.identity(A.ncols, sr)
    for C in (oracle.spgemm(A, I, sr), oracle.spgemm(I, A, sr)):
        assert_same_structure(C, A)
        assert C.val.tobytes() == A.val.tobytes()


def test_column_permutation_operand():
    """A P^T, with P a permutation matrix, moves column j of A to perm^-1..:
    (A Q)(i, j) = A(i, k) where Q(k, j) = 1."""
    A = synth.rmat(10, 8, synth.G500, seed=27)
    perm = np.random.default_rng(5).permutation(A.ncols)
    Q = synth.permutation_matrix(perm)  # Q(i, perm[i]) = 1
    C = oracle.spgemm(A, Q, "f64")
    row_of = np.repeat(np.arange(A.nrows), np.diff(A.row_ptr))
    ref = synth.canonical_from_coo(A.nrows, A.ncols, row_of, perm[A.col], A.val, dup="first")
    assert_same_structure(C, ref)
    assert C.val.tobytes() == ref.val.tobytes()


def test_symmetric_permutation_invariance():
    """(P A P^T)(P B P^T) = P (A B) P^T (Section 5): structure and INT64
    exact, FP64 within the summation-order bound."""
    A = synth.rmat(11, 16, synth.G500, seed=28, permute=False)
    B = synth.rmat(11, 16, synth.G500, seed=29, permute=False)
    perm = np.random.default_rng(9).permutation(A.nrows)
    PA, PB = synth.permute_symmetric(A, perm), synth.permute_symmetric(B, perm)
    C = oracle.spgemm(A, B, "f64")
    PC = synth.permute_symmetric(C, perm)
    got = oracle.spgemm(PA, PB, "f64")
    assert_same_structure(got, PC)
    assert_values(got, PC, "f64", oracle.f64_check(PA, PB, got))
    Ai, Bi = synth.with_values(A, "ones_i64"), synth.with_values(B, "ones_i64")
    Ci = synth.permute_symmetric(oracle.spgemm(Ai, Bi, "i64"), perm)
    gi = oracle.spgemm(synth.permute_symmetric(Ai, perm), synth.permute_symmetric(Bi, perm), "i64")
    assert_same_structure(gi, Ci)
    assert np.array_equal(gi.val, Ci.val)


def test_single_entry_rows_are_scaled_b_rows():
    """A row of A with one stored entry a at column k gives C(i,:) = a B(k,:)
    exactly, in B's column order."""
    A = synth.rmat(12, 16, synth.G500, seed=30)
    C = oracle.spgemm(A, A, "f64")
    lens = np.diff(A.row_ptr)
    rows = np.nonzero(lens == 1)[0]
    assert rows.size > 50
    for i in rows[:400]:
        p = A.row_ptr[i]
        k, a = A.col[p], A.val[p]
        bc, bv = A.row(k)
        cc, cv = C.row(i)
        assert np.array_equal(cc, bc)
        assert (a * bv).tobytes() == cv.tobytes()


@pytest.mark.parametrize("c", [1, 2, 4, 16])
def test_layer_split_equals_unsplit(c):
    """Split 3D identity (Section 4.4, Algorithm 2): with contiguous inner
    layers K_l, the flops add up exactly, nnz(C) <= sum_l nnz(C_l) <= flops,
    and merging the layer products gives the unsplit product (structure and
    INT64 exact, FP64 within the order bound); c = 1 merge is the identity."""
    A = synth.rmat(12, 16, synth.ER, seed=31)
    B = synth.rmat(12, 16, synth.ER, seed=32)
    bounds = synth.layer_bounds(A.ncols, c)
    C = oracle.spgemm(A, B, "f64")
    f = int(oracle.row_flops(A, B).sum())
    layers = [oracle.spgemm(A, B, "f64", lo, hi) for lo, hi in bounds]
    assert sum(int(oracle.row_flops(A, B, lo, hi).sum()) for lo, hi in bounds) == f
    tot = sum(L.nnz for L in layers)
    assert C.nnz <= tot <= f
    M = oracle.merge(layers, "f64")
    assert_same_structure(M, C)
    assert_values(M, C, "f64", oracle.f64_check(A, B, C))
    Ai, Bi = synth.with_values(A, "ones_i64"), synth.with_values(B, "ones_i64")
    Ci = oracle.spgemm(Ai, Bi, "i64")
    Mi = oracle.merge([oracle.spgemm(Ai, Bi, "i64", lo, hi) for lo, hi in bounds], "i64")
    assert_same_structure(Mi, Ci)
    assert np.array_equal(Mi.val, Ci.val)
    if c == 1:
        assert M.val.tobytes() == C.val.tobytes()


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_merge_brute_force(sr):
    """Merge == entry-wise fold of dense layers in layer order (bit-exact)."""
    seed = 100
    for c in (1, 2, 3, 5):
        for m, n in ((0, 4), (4, 0), (6, 9), (12, 12)):
            for dens in (0.0, 0.2, 0.7):
                seed += 1
                layers = [synth.random_csr(m, n, dens, seed * 31 + l, sr, explicit_zero_frac=0.2)
                          for l in range(c)]
                M = oracle.merge(layers, sr)
                assert M.is_canonical()
                ref = brute_merge(layers, sr)
                got = csr_to_dict(M)
                assert got.keys() == ref.keys()
                for key, v in ref.items():
                    if sr == "f64":
                        assert np.float64(got[key]).tobytes() == np.float64(v).tobytes()
                    else:
                        assert got[key] == v


@pytest.mark.parametrize("N", [2, 3, 5, 8])
def test_galerkin_closed_forms(N):
    """2x2x2 aggregation of the 7-point operator: nnz(A) = 7N^3 - 6N^2,
    nnz(R) = N^3, flops(R^T, A) = nnz(A), flops(T, R) = nnz(T); the coarse
    operator is the 7-point stencil on M^3 (nnz = 7M^3 - 6M^2), with
    C(I,I) = 6|I| - 2e(I) (24 for full blocks), C(I,J) = -(fine edges
    between I and J) (-4 for full faces), row sums of C equal the sums of
    the fine row sums, and T(I,j) = 6 - (neighbours of j inside I) for j in
    I, -1 for j outside I next to I."""
    A = synth.poisson7(N)
    RT, R = synth.aggregation_2x2x2(N)
    M = (N + 1) // 2
    assert A.nnz == 7 * N ** 3 - 6 * N ** 2
    assert R.nnz == N ** 3 and RT.nnz == N ** 3
    assert int(oracle.row_flops(RT, A).sum()) == A.nnz
    T = oracle.spgemm(RT, A, "f64")
    assert int(oracle.row_flops(T, R).sum()) == T.nnz
    C = oracle.spgemm(T, R, "f64")
    assert C.nnz == 7 * M ** 3 - 6 * M ** 2
    # aggregate membership
    idx = np.arange(N ** 3)
    x, y, z = idx % N, (idx // N) % N, idx // (N * N)
    agg = (x // 2) + M * ((y // 2) + M * (z // 2))
    Ad = A.to_dense()
    members = [np.nonzero(agg == I)[0] for I in range(M ** 3)]
    Cd = C.to_dense()
    for I in range(M ** 3):
        mI = members[I]
        inside = (Ad[np.ix_(mI, mI)] == -1).sum() // 2
        assert Cd[I, I] == 6 * len(mI) - 2 * inside
        if len(mI) == 8:
            assert Cd[I, I] == 24
        for J in range(M ** 3):
            if J != I:
                e = (Ad[np.ix_(mI, members[J])] == -1).sum()
                assert Cd[I, J] == -e
    assert np.array_equal(Cd.sum(axis=1), np.array([Ad[m].sum() for m in members]))
    Td = T.to_dense()
    for I in range(M ** 3):
        mI = members[I]
        for j in range(N ** 3):
            nbr_in = int((Ad[mI, j] == -1).sum())
            if agg[j] == I:
                assert Td[I, j] == 6 - nbr_in
            elif nbr_in:
                assert Td[I, j] == -nbr_in
    assert np.all(np.abs(Cd - np.round(Cd)) == 0)
