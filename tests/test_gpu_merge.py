"""GPU parity of the layered product and the k-way layer merge (Section 4.4
split of the inner dimension into c contiguous layers; Section 4.3 merge)."""

import numpy as np
import pytest
import torch

import oracle
import paper_1510_00844_amd as spg
import synth
from gpu_util import check_full_vs_oracle, to_dev, to_host
from synth import CSR
from util import assert_same_structure, assert_values

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def plan():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = spg.Plan()
    yield p
    p.close()


def layered(plan, sr, A, B, c):
    dA, dB = to_dev(A, sr), to_dev(B, sr)
    layers = [spg.spgemm(plan, sr, dA, dB, lo, hi) for lo, hi in synth.layer_bounds(A.ncols, c)]
    return layers, spg.spgemm_merge_layers(plan, sr, layers), spg.spgemm(plan, sr, dA, dB)


@pytest.mark.parametrize("c", [1, 2, 4, 16])
@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_layers_merge_small(plan, c, sr):
    A = synth.rmat(12, 16, synth.ER, seed=31)
    B = synth.rmat(12, 16, synth.G500, seed=32)
    if sr != "f64":
        kind = "ones_i64" if sr == "i64" else "true_bool"
        A, B = synth.with_values(A, kind), synth.with_values(B, kind)
    layers, M, U = layered(plan, sr, A, B, c)
    # every layer equals the oracle's windowed product
    for (lo, hi), L in zip(synth.layer_bounds(A.ncols, c), layers):
        check_full_vs_oracle(L, A, B, sr, lo, hi)
    # merge of the device layers equals the oracle merge of the same layers
    hl = [to_host(L) for L in layers]
    ref_m = oracle.merge(hl, sr)
    got_m = to_host(M)
    assert_same_structure(got_m, ref_m)
    assert_values(got_m, ref_m, sr)
    # every merge path adds equal columns in ascending layer order, as the
    # oracle's merge does: bit for bit
    assert got_m.val.tobytes() == ref_m.val.tobytes()
    # and the merged result equals the oracle's unsplit product
    check_full_vs_oracle(M, A, B, sr)
    assert torch.equal(M.row_ptr, U.row_ptr) and torch.equal(M.col, U.col)


@pytest.mark.parametrize("c", [4, 16])
def test_c3_er_s18_layers(plan, c):
    """C3: ER scale 18, edge factor 16, A and B independent, c layers.
    Every layer against the oracle's windowed product, the merged result
    against the oracle's merge of the same layers and against the oracle's
    unsplit product, all element by element."""
    A = synth.rmat(18, 16, synth.ER, seed=3)
    B = synth.rmat(18, 16, synth.ER, seed=4)
    print("case C3 c=%d" % c, flush=True)
    layers, M, U = layered(plan, "f64", A, B, c)
    del U
    f = int(oracle.row_flops(A, B).sum())
    tot = sum(L.nnz for L in layers)
    assert M.nnz <= tot <= f
    hl = []
    for (lo, hi), L in zip(synth.layer_bounds(A.ncols, c), layers):
        check_full_vs_oracle(L, A, B, "f64", lo, hi)
        hl.append(to_host(L))
    ref_m = oracle.merge(hl, "f64")
    got_m = to_host(M)
    assert_same_structure(got_m, ref_m)
    assert got_m.val.tobytes() == ref_m.val.tobytes()
    over = check_full_vs_oracle(M, A, B, "f64")
    print("C3 c=%d merged: %d entries, %d over 1e-12 relative" % (c, M.nnz, over), flush=True)


def _layer(m, n, rows_lens, seed, sr="f64"):
    rng = np.random.default_rng(seed)
    rr, cc = [], []
    for i, L in enumerate(rows_lens):
        cs = rng.choice(n, min(L, n), replace=False)
        rr += [i] * len(cs)
        cc += cs.tolist()
    vals = {"f64": rng.random(len(rr)), "i64": rng.integers(-5, 6, len(rr)),
            "bool": (rng.random(len(rr)) < 0.7).astype(np.uint8)}[sr]
    return synth.canonical_from_coo(m, n, rr, cc, vals, dup="first")


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_merge_edge_cases(plan, sr):
    """Empty layers, c = 1, rows in every merge bin (the wave k-way merge up
    to 384 entries, rank placement up to 4096, the chunked dense path above),
    bit for bit against the oracle's merge (ascending layer order)."""
    n = 20000
    lens = [0, 1, 5, 30, 64, 65, 127, 128, 129, 170, 171, 300, 383, 384, 385, 511, 512, 513, 1500, 3000, 5000,
            9000, 19000]
    layers_h = [_layer(len(lens), n, lens, 10 + l, sr) for l in range(3)]
    layers_h.append(_layer(len(lens), n, [0] * len(lens), 99, sr))  # an empty layer
    for sel in ([0], [3], [0, 1], [0, 1, 2, 3], [0, 3, 1]):
        hl = [layers_h[x] for x in sel]
        M = spg.spgemm_merge_layers(plan, sr, [to_dev(L, sr) for L in hl])
        ref = oracle.merge(hl, sr)
        got = to_host(M)
        assert_same_structure(got, ref)
        assert_values(got, ref, sr)
        assert got.val.tobytes() == ref.val.tobytes()


@pytest.mark.parametrize("c", [5, 8, 9, 16, 17, 32, 33, 64])
def test_merge_many_layers(plan, c):
    """Layer counts around the wave merge's list limits (4, 8, 16, 32) and
    above them (33..64 take the wave sort and rank paths): rows of 0..600
    entries over c layers, many columns shared between layers."""
    rng = np.random.default_rng(200 + c)
    m, n = 400, 3000
    hl = []
    for l in range(c):
        lens = rng.integers(0, max(2, 600 // c + 2), m)
        hl.append(_layer(m, n, lens.tolist(), 300 + 7 * c + l))
    M = spg.spgemm_merge_layers(plan, "f64", [to_dev(L) for L in hl])
    ref = oracle.merge(hl, "f64")
    got = to_host(M)
    assert_same_structure(got, ref)
    assert got.val.tobytes() == ref.val.tobytes()


def _layers_from_rows(n, row_cols, c, seed, sr="f64"):
    """c layers whose row i together hold the columns row_cols[i] (each
    column goes to 1..3 random layers, so many columns are shared)."""
    rng = np.random.default_rng(seed)
    per = [([], []) for _ in range(c)]
    for i, cols in enumerate(row_cols):
        for j in cols:
            for l in rng.choice(c, int(rng.integers(1, min(3, c) + 1)), replace=False):
                per[l][0].append(i)
                per[l][1].append(int(j))
    out = []
    for l, (rr, cc) in enumerate(per):
        vals = {"f64": rng.random(len(rr)), "i64": rng.integers(-5, 6, len(rr)),
                "bool": (rng.random(len(rr)) < 0.7).astype(np.uint8)}[sr]
        out.append(synth.canonical_from_coo(len(row_cols), n, rr, cc, vals, dup="first"))
    return out


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
@pytest.mark.parametrize("c", [2, 4, 16])
def test_merge_sort_bin_shapes(plan, sr, c):
    """Rows of the bucket-sort merge bin (65..512 entries over the layers)
    with uniform columns (buckets of at most 8 or 16, sorted in registers),
    with a band of columns next to a few far ones (larger buckets: the whole
    row is sorted by the wave), and rows whose columns span 2^23 or more
    (left to the other merge paths), all bit for bit against the oracle's
    merge."""
    rng = np.random.default_rng(500 + c)
    n = (1 << 24) + 5
    rows = []
    for target in (30, 60, 100, 170, 250):
        rows.append(np.unique(rng.choice(1 << 20, target, replace=False)))          # uniform
        for band in (20, 28, 45, 160):                                             # clustered
            start = int(rng.integers(0, (1 << 20) - band))
            far = rng.choice(1 << 20, max(1, target // 10), replace=False)
            rows.append(np.unique(np.concatenate([start + np.arange(band), far])))
        rows.append(np.unique(np.concatenate([[0, n - 1], rng.choice(n, target, replace=False)])))  # wide
    hl = _layers_from_rows(n, rows, c, 600 + c, sr)
    M = spg.spgemm_merge_layers(plan, sr, [to_dev(L, sr) for L in hl])
    ref = oracle.merge(hl, sr, nthreads=2)
    got = to_host(M)
    assert_same_structure(got, ref)
    assert_values(got, ref, sr)
    assert got.val.tobytes() == ref.val.tobytes()
