"""GPU parity of the heap bin (HeapSpGEMM, Section 4.2): rows whose window
holds few A entries are merged from their B rows by one wave (k-way merge,
column range split over the lanes).  Rows are forced into the bin and
compared with the oracle element by element; since equal columns add in
ascending k, FP64 values equal the oracle's ascending-k sums bit for bit.
The same products with the bin switched off (hash tables instead) agree
exactly in structure and in INT64/boolean values."""

import numpy as np
import pytest
import torch

import oracle
import paper_1510_00844_amd as spg
import synth
from gpu_util import check_full_vs_oracle, to_dev, to_host
from util import assert_same_structure

pytestmark = pytest.mark.gpu
HEAP = spg.BIN_HEAP
ROW_MAX = 384  # most products a heap-bin row takes (the entries one wave merges)


def heap_rows(seed, m=3000, k_max=32, n=20000, K=6000):
    """A (m x K) with 2..k_max entries per row against B (K x n) whose rows
    hold 0..60 entries, so rows have 65..ROW_MAX products; plus rows built
    to stress the merge: every list equal (each column k times), lists of
    one entry, lists clustered in a narrow column range, empty B rows, and
    rows at exactly k_max lists."""
    rng = np.random.default_rng(seed)
    blen = rng.integers(0, 61, K)
    blen[:50] = 0  # empty B rows
    rows_b, cols_b = [], []
    for r in range(K):
        if r < 100:  # B rows 100..: random; 50..99: a narrow cluster
            c = np.sort(rng.choice(200, min(blen[r], 200), replace=False)) + 9000 if r >= 50 else np.zeros(0, int)
        elif r < 120:  # identical rows: the same 30 columns
            c = np.arange(30) * 17 + 5
        else:
            c = np.sort(rng.choice(n, blen[r], replace=False))
        rows_b += [r] * len(c)
        cols_b += c.tolist()
    B = synth.canonical_from_coo(K, n, np.array(rows_b), np.array(cols_b), rng.random(len(rows_b)) - 0.5,
                                 dup="first")
    bl = np.diff(B.row_ptr)
    rows_a, cols_a = [], []
    for i in range(m):
        kind = i % 5
        if kind == 0:  # identical lists
            ks = rng.choice(np.arange(100, 120), int(rng.integers(3, min(k_max, 20) + 1)), replace=False)
        elif kind == 1:  # clustered columns and empty rows mixed in
            ks = np.concatenate([rng.choice(np.arange(50, 100), int(rng.integers(2, 12)), replace=False),
                                 rng.choice(50, 3, replace=False)])
        else:  # random lists
            kk = int(rng.integers(2, k_max + 1))
            ks = rng.choice(np.arange(120, K), kk, replace=False)
        ks = np.sort(ks)[:k_max]
        # keep the row at 65..ROW_MAX products
        while bl[ks].sum() > ROW_MAX and len(ks) > 2:
            ks = ks[:-1]
        rows_a += [i] * len(ks)
        cols_a += ks.tolist()
    A = synth.canonical_from_coo(m, K, np.array(rows_a), np.array(cols_a), rng.random(len(rows_a)) + 0.25,
                                 dup="first")
    return A, B


def with_kind(M, sr):
    kind = {"f64": None, "i64": "ones_i64", "bool": "true_bool"}[sr]
    return M if kind is None else synth.with_values(M, kind)


@pytest.mark.parametrize("kmax", [8, 16, 32])
@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_heap_bin_forced(sr, kmax):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A, B = heap_rows(80 + kmax, k_max=kmax)
    A, B = with_kind(A, sr), with_kind(B, sr)
    f = oracle.row_flops(A, B)
    annz = np.diff(A.row_ptr)
    want = int(np.sum((annz > 1) & (f > 64) & (f <= ROW_MAX) & (annz <= kmax)))
    assert want > 1000
    p = spg.Plan(heap_max_lists=kmax)
    try:
        print("case heap kmax=%d sr=%s" % (kmax, sr), flush=True)
        C = spg.spgemm(p, sr, to_dev(A, sr), to_dev(B, sr))
        st = p.stats()
        assert st["sym_rows"][HEAP] == want and st["num_rows"][HEAP] == want, (st["sym_rows"][HEAP], want)
        check_full_vs_oracle(C, A, B, sr)
        if sr == "f64":
            # ascending-k sums: bit for bit the oracle's on every row of the bin
            got = to_host(C)
            ref = oracle.spgemm(A, B, "f64")
            heap = (annz > 1) & (f > 64) & (f <= ROW_MAX) & (annz <= kmax)
            sel = np.repeat(heap, np.diff(ref.row_ptr))
            assert got.val[sel].tobytes() == ref.val[sel].tobytes()
        # the same product through the hash tables
        q = spg.Plan(heap_max_lists=-1)
        try:
            H = spg.spgemm(q, sr, to_dev(A, sr), to_dev(B, sr))
            assert q.stats()["num_rows"][HEAP] == 0
            assert torch.equal(H.row_ptr, C.row_ptr) and torch.equal(H.col, C.col)
            if sr != "f64":
                assert torch.equal(H.val, C.val)
        finally:
            q.close()
    finally:
        p.close()


def test_heap_bin_structure_only_and_windows():
    """Structure-only numeric pass (no value arrays) and inner windows."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A, B = heap_rows(91)
    p = spg.Plan(heap_max_lists=32)
    try:
        dA, dB = to_dev(A), to_dev(B)
        for lo, hi in [(0, A.ncols), (1000, 4000), (3000, 3001)]:
            C = spg.spgemm(p, "f64", dA, dB, lo, hi)
            check_full_vs_oracle(C, A, B, "f64", lo, hi)
        S = spg.spgemm(p, "f64", dA, dB, values=False)
        ref = oracle.spgemm(A, B, "bool", values=False)
        got = to_host(S)
        assert_same_structure(got, ref)
    finally:
        p.close()


def test_heap_bin_er_rows():
    """ER rows (about 16 A entries of about 16 products each, the layer
    shape of the scale-18 workload at a smaller scale): nearly every row
    takes the heap bin."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A = synth.rmat(14, 16, synth.ER, seed=93)
    B = synth.rmat(14, 16, synth.ER, seed=94)
    p = spg.Plan(heap_max_lists=32)
    try:
        C = spg.spgemm(p, "f64", to_dev(A), to_dev(B))
        st = p.stats()
        assert st["num_rows"][HEAP] > 0.9 * A.nrows
        check_full_vs_oracle(C, A, B, "f64")
    finally:
        p.close()
