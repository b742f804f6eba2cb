"""Pins of the oracle's stage accumulation and hypersparse format
(Section 4.1 Sparse SUMMA stages with blocking b; Section 4.2 DCSC, here by
rows; Section 4.3 multiway merge in stage order).

* DCSR round trips: compress then expand gives the CSR back; a DCSR keeps
  exactly the non-empty rows, with strictly increasing row indices, and its
  pointer array has nzr + 1 entries whatever the row dimension;
* the stage blocks tile the inner dimension in stage order and reject a
  blocking that does not divide a stage;
* brute force on tiny matrices: every entry equals, bit for bit, the sum
  over the blocks in stage order of the block's terms added in ascending k,
  written out here entry by entry in plain Python;
* the distributive law: the stage sum equals the unsplit product exactly
  for INT64 and boolean values, and with one block it is the unsplit FP64
  product bit for bit.
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import summa
from synth import CSR


def _rand(m, n, density, seed, kind):
    return synth.random_csr(m, n, density, seed, kind=kind, explicit_zero_frac=0.1 if kind == "f64" else 0.0)


def _with_empty_rows(M: CSR, seed) -> CSR:
    """Zero out about half of the rows (hypersparse-like row set)."""
    rng = np.random.default_rng(seed)
    drop = rng.random(M.nrows) < 0.5
    rows = np.repeat(np.arange(M.nrows), np.diff(M.row_ptr))
    keep = ~drop[rows]
    return synth.canonical_from_coo(M.nrows, M.ncols, rows[keep], M.col[keep].astype(np.int64),
                                    None if M.val is None else M.val[keep], dup="first")


@pytest.mark.parametrize("m,n,density", [(0, 5, 0.3), (7, 0, 0.3), (9, 6, 0.0), (40, 30, 0.05), (200, 50, 0.02)])
def test_dcsr_round_trip(m, n, density):
    M = _with_empty_rows(_rand(m, n, density, 3, "f64"), 4) if m and n else _rand(m, n, density, 3, "f64")
    D = summa.compress(M)
    lens = np.diff(M.row_ptr)
    nonempty = [i for i in range(m) if lens[i] > 0]
    assert D.row_ids.tolist() == nonempty
    assert D.row_ptr.size == D.nzr + 1 and D.row_ptr[0] == 0
    assert np.all(np.diff(D.row_ptr) > 0)
    assert D.col.tolist() == M.col.tolist()
    for r, i in enumerate(D.row_ids):
        assert D.row_ptr[r] == M.row_ptr[i] and D.row_ptr[r + 1] == M.row_ptr[i + 1]
    E = summa.expand(D)
    assert E.row_ptr.tolist() == M.row_ptr.tolist()
    assert E.col.tolist() == M.col.tolist()
    assert E.val.tobytes() == M.val.tobytes()


def test_dcsr_storage_does_not_grow_with_rows():
    """Three entries in a matrix of 2^40 rows: the DCSR holds 3 row indices
    and 4 pointers (the CSR would need 2^40 + 1)."""
    D = summa.DCSR(1 << 40, 8, np.array([5, 1 << 20, (1 << 40) - 1], np.int64), np.array([0, 1, 2, 3], np.int64),
                   np.array([0, 3, 7], np.int32), np.array([1.0, 2.0, 3.0]))
    assert D.nzr == 3 and D.nnz == 3 and D.row_ptr.size == 4


def test_stage_blocks_tile_in_stage_order():
    w = summa.stage_blocks(24, 3, 4)
    assert w == [(0, 4), (4, 8), (8, 12), (12, 16), (16, 20), (20, 24)]
    assert summa.stage_blocks(24, 3, 8) == [(0, 8), (8, 16), (16, 24)]
    assert summa.stage_blocks(24, 1, 24) == [(0, 24)]
    assert summa.stage_blocks(0, 4, 2) == []
    for bad in ((24, 5, 1), (24, 3, 3), (24, 0, 1), (24, 3, 0)):
        with pytest.raises(ValueError):
            summa.stage_blocks(*bad)


def _brute(A: CSR, B: CSR, stages, b, sr):
    """Entry by entry: within a block, terms A(i,k) B(k,j) in ascending k
    (the first term starts the sum); blocks combined in stage order (the
    first block holding the entry starts it)."""
    blocks = summa.stage_blocks(A.ncols, stages, b)
    Ad = {}
    for i in range(A.nrows):
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            Ad[(i, int(A.col[p]))] = A.val[p] if A.val is not None else 1
    Bd = {}
    for k in range(B.nrows):
        for p in range(B.row_ptr[k], B.row_ptr[k + 1]):
            Bd.setdefault(k, []).append((int(B.col[p]), B.val[p] if B.val is not None else 1))
    out = {}
    for i in range(A.nrows):
        for lo, hi in blocks:
            part = {}
            for k in range(lo, hi):
                if (i, k) not in Ad:
                    continue
                a = Ad[(i, k)]
                for j, bv in Bd.get(k, []):
                    if sr == "f64":
                        t = float(a) * float(bv)
                        part[j] = t if j not in part else part[j] + t
                    elif sr == "i64":
                        t = int(a) * int(bv)
                        part[j] = t if j not in part else part[j] + t
                    else:
                        t = bool(a) and bool(bv)
                        part[j] = t if j not in part else (part[j] or t)
            for j, v in part.items():
                if (i, j) not in out:
                    out[(i, j)] = v
                elif sr == "bool":
                    out[(i, j)] = out[(i, j)] or v
                else:
                    out[(i, j)] = out[(i, j)] + v
    return out


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
@pytest.mark.parametrize("stages,b,density", [(1, 24, 0.15), (2, 3, 0.15), (3, 4, 0.15), (4, 1, 0.15), (6, 2, 0.15),
                                              (4, 2, 0.7), (8, 1, 0.7)])
def test_summa_local_brute_force(sr, stages, b, density):
    """The dense cases give entries many blocks' partial sums, so adding the
    blocks in any other order changes some FP64 results."""
    A = _with_empty_rows(_rand(30, 24, density, 11, sr), 12)
    B = _rand(24, 17, density, 13, sr)
    C, stage_nnz = summa.summa_local(summa.compress(A), B, stages, b, sr)
    ref = _brute(A, B, stages, b, sr)
    got = {}
    for r, i in enumerate(C.row_ids):
        for p in range(C.row_ptr[r], C.row_ptr[r + 1]):
            got[(int(i), int(C.col[p]))] = C.val[p]
    assert sorted(got) == sorted(ref)
    for key, v in ref.items():
        if sr == "f64":
            assert np.float64(got[key]).tobytes() == np.float64(v).tobytes(), key
        elif sr == "i64":
            assert int(got[key]) == v, key
        else:
            assert bool(got[key]) == v, key
    # the kept block products hold one entry per (block, i, j) with a term
    blocks = summa.stage_blocks(A.ncols, stages, b)
    want = sum(int(oracle.row_counts(A, B, lo, hi).sum()) for lo, hi in blocks)
    assert stage_nnz == want
    assert np.all(np.diff(C.row_ptr) > 0) and np.all(np.diff(C.row_ids) > 0)


@pytest.mark.parametrize("stages,b", [(4, 8), (8, 2), (2, 32)])
def test_summa_local_is_the_product(stages, b):
    """Sum of rank-b updates = the product (distributive law): exact for
    INT64 and boolean values; FP64 within the reordering bound."""
    A0 = synth.rmat(6, 8, synth.G500, seed=21)
    B0 = synth.rmat(6, 8, synth.ER, seed=22)
    for sr in ("i64", "bool"):
        kind = "ones_i64" if sr == "i64" else "true_bool"
        A, B = synth.with_values(A0, kind), synth.with_values(B0, kind)
        C, _ = summa.summa_local(summa.compress(A), B, stages, b, sr)
        U = oracle.spgemm(A, B, sr)
        E = summa.expand(C)
        assert E.row_ptr.tolist() == U.row_ptr.tolist()
        assert E.col.tolist() == U.col.tolist()
        assert E.val.tolist() == U.val.tolist()
    C, _ = summa.summa_local(summa.compress(A0), B0, stages, b, "f64")
    E = summa.expand(C)
    U = oracle.spgemm(A0, B0, "f64")
    assert E.col.tolist() == U.col.tolist()
    comp, absum, nterms = oracle.f64_check(A0, B0, U)
    assert np.all(np.abs(E.val - comp) <= oracle.f64_bound(comp, absum, nterms))
    # one block: the unsplit product itself, bit for bit
    C1, _ = summa.summa_local(summa.compress(A0), B0, 1, A0.ncols, "f64")
    assert summa.expand(C1).val.tobytes() == U.val.tobytes()


def test_summa_local_no_inner_indices():
    A = summa.compress(CSR(5, 0, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0)))
    B = CSR(0, 4, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    C, stage_nnz = summa.summa_local(A, B, 2, 3, "f64")
    assert C.nzr == 0 and C.nnz == 0 and stage_nnz == 0 and C.nrows == 5 and C.ncols == 4
