"""GPU parity of the HIP SpGEMM path (through the C ABI) against the oracle.

Structure and INT64/boolean values are compared exactly; FP64 values to
1e-12 relative per entry, or, for an entry over that, within the bound of
any summation order around the compensated sum of its terms (tests/util.py).
Every configuration here is compared with the oracle element by element over
all rows; the scale-19 workload is in test_gpu_c5.py.
"""

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


def run(plan, sr, A, B, k_lo=None, k_hi=None):
    return spg.spgemm(plan, sr, to_dev(A, sr), to_dev(B, sr), k_lo, k_hi)


def with_kind(M, sr, seed=0):
    kind = {"f64": "uniform_f64", "i64": "ones_i64", "bool": "true_bool"}[sr]
    return synth.with_values(M, kind, seed=seed)


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_c1_er_uniform_full(plan, sr):
    print("case C1 ER-uniform n=4096 sr=%s" % sr, flush=True)
    A = synth.er_uniform_columns(4096, 4, seed=1)
    A = A if sr == "f64" else with_kind(A, sr)
    C = run(plan, sr, A, A)
    check_full_vs_oracle(C, A, A, sr)
    st = plan.stats()
    assert st["flops"] == 65536


def _binned_matrices(seed=7):
    """A (m x K) whose rows cover every accumulator bin against an R-MAT B
    with hub rows: empty rows, one-entry rows, a few products, each hash
    size, and rows whose products exceed the hash limit."""
    # B: the first 8192 rows of an R-MAT scale-17 matrix (131072 columns, so
    # rows up to 4096 products stay in the hash bins and hub rows appear)
    R = synth.rmat(17, 16, synth.G500, seed=seed)
    K = 8192
    B = synth.CSR(K, R.ncols, R.row_ptr[:K + 1].copy(), R.col[:R.row_ptr[K]].copy(),
                  R.val[:R.row_ptr[K]].copy())
    rng = np.random.default_rng(seed)
    blen = np.diff(B.row_ptr)
    order = np.argsort(-blen)
    rows, cols = [], []
    r = 0
    # (the hash tables hold at most 3/4 of their slots: rows of 1900 and
    # 3000 products take the 4096-slot table, below the 4096 where the
    # bitmap starts)
    targets = [0, 1, 1, 2, 3, 5, 8, 12, 20, 40, 60, 100, 200, 400, 800, 1500, 1900, 3000, 6000, 12000, 30000, 60000]
    for rep in range(6):
        for tf in targets:
            if tf == 0:
                r += 1
                continue
            if tf == 1:
                k = int(rng.integers(0, K))
                rows.append(r); cols.append(k)
                r += 1
                continue
            picked, f = set(), 0
            pool = order if tf > 2000 else rng.permutation(K)
            for k in pool:
                k = int(k)
                if k in picked or blen[k] == 0:
                    continue
                if f + blen[k] > tf and f > 0:
                    continue
                picked.add(k)
                f += int(blen[k])
                if f >= tf * 0.9:
                    break
            for k in picked:
                rows.append(r); cols.append(k)
            r += 1
    # rows whose products collide heavily: B rows K..K+59 share the same 12
    # columns, so 8 of them give 96 products but only 12 outputs
    extra = 60
    shared = rng.choice(B.ncols, 12, replace=False)
    brow = np.repeat(np.arange(K, K + extra), 12)
    bcol = np.tile(shared, extra)
    B_rows = np.repeat(np.arange(K), np.diff(B.row_ptr))
    B = synth.canonical_from_coo(K + extra, B.ncols, np.concatenate([B_rows, brow]),
                                 np.concatenate([B.col.astype(np.int64), bcol]),
                                 np.concatenate([B.val, rng.random(brow.size)]), dup="first")
    for rep in range(20):
        ks = rng.choice(extra, 8, replace=False) + K
        rows += [r] * 8
        cols += ks.tolist()
        r += 1
    A = synth.canonical_from_coo(r, K + extra, rows, cols, rng.random(len(rows)), dup="first")
    return A, B


@pytest.mark.parametrize("heap", [False, True])
@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_every_bin_full(sr, heap):
    """Rows in every bin; with the heap bin off every hash table size is
    used, with it on the rows of few A entries move to the heap bin."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A, B = _binned_matrices()
    print("case bins m=%d sr=%s heap=%s" % (A.nrows, sr, heap), flush=True)
    A, B = (A, B) if sr == "f64" else (with_kind(A, sr), with_kind(B, sr))
    plan = spg.Plan(heap_max_lists=32 if heap else -1)
    try:
        C = run(plan, sr, A, B)
        st = plan.stats()
    finally:
        plan.close()
    used_sym = [b for b in range(spg.NBINS) if st["sym_rows"][b]]
    used_num = [b for b in range(spg.NBINS) if st["num_rows"][b]]
    expect = (0, 1, 2, 12) + ((spg.BIN_HEAP,) if heap else (3, 4, 5, 6, 7, 8))
    for b in expect:
        assert b in used_sym or b in used_num, "bin %s not exercised" % spg.BIN_NAMES[b]
    assert 12 in used_sym
    assert any(b in used_num for b in (13, 14, 15)), "no rank-space rows"
    for b in ((6, 7, 8) if not heap else (spg.BIN_HEAP,)):
        assert b in used_num, "numeric bin %s not exercised" % spg.BIN_NAMES[b]
    check_full_vs_oracle(C, A, B, sr)


def test_small_rows_exact_order(plan):
    """Rows with <= 64 products fold equal columns in ascending k, the
    oracle's order, so FP64 matches bit for bit there."""
    A = synth.random_csr(300, 200, 0.02, seed=41, kind="f64")
    B = synth.random_csr(200, 150, 0.03, seed=42, kind="f64")
    f = oracle.row_flops(A, B)
    assert f.max() <= 64
    C = to_host(run(plan, "f64", A, B))
    ref = oracle.spgemm(A, B, "f64")
    assert_same_structure(C, ref)
    assert C.val.tobytes() == ref.val.tobytes()


def test_small_rows_with_many_empty_b_rows(plan):
    """Rows of at most 64 products whose A windows hold more than 64 entries
    (most point at empty B rows): the small-row kernels take two rows per
    wave and fall back to the one-row search for such pairs; rows of every
    kind are mixed so that both paths share waves.  FP64 bit-exact."""
    rng = np.random.default_rng(47)
    k, n, m = 400, 120, 97
    # B: rows 0..39 hold 1-2 entries, the rest are empty
    brows, bcols = [], []
    for r in range(40):
        for c in rng.choice(n, size=int(rng.integers(1, 3)), replace=False):
            brows.append(r)
            bcols.append(int(c))
    B = synth.canonical_from_coo(k, n, np.array(brows), np.array(bcols), rng.random(len(brows)) + 0.5, dup="first")
    arows, acols = [], []
    for i in range(m):
        if i % 3 == 0:  # > 64 entries, mostly empty B rows
            cols = rng.choice(np.arange(40, k), size=80, replace=False).tolist() + rng.choice(40, size=3, replace=False).tolist()
        else:
            cols = rng.choice(k, size=int(rng.integers(1, 12)), replace=False).tolist()
        arows += [i] * len(cols)
        acols += cols
    A = synth.canonical_from_coo(m, k, np.array(arows), np.array(acols), rng.random(len(arows)) + 0.5, dup="first")
    f = oracle.row_flops(A, B)
    assert f.max() <= 64 and np.diff(A.row_ptr).max() > 64
    C = to_host(run(plan, "f64", A, B))
    ref = oracle.spgemm(A, B, "f64")
    assert_same_structure(C, ref)
    assert C.val.tobytes() == ref.val.tobytes()


@pytest.mark.parametrize("window", [(0, 0), (0, 1), (100, 1000), (4000, 8192), (8191, 8192), (0, 8192)])
def test_inner_windows(plan, window):
    A = synth.rmat(13, 16, synth.G500, seed=43)
    B = synth.rmat(13, 16, synth.ER, seed=44)
    lo, hi = window
    print("case window %s" % (window,), flush=True)
    C = run(plan, "f64", A, B, lo, hi)
    check_full_vs_oracle(C, A, B, "f64", lo, hi)


def test_degenerate_shapes(plan):
    cases = [
        (synth.random_csr(0, 5, 0.5, 1), synth.random_csr(5, 4, 0.5, 2)),
        (synth.random_csr(4, 0, 0.5, 1), synth.random_csr(0, 4, 0.5, 2)),
        (synth.random_csr(4, 5, 0.5, 1), synth.random_csr(5, 0, 0.5, 2)),
        (synth.random_csr(7, 6, 0.0, 1), synth.random_csr(6, 3, 0.5, 2)),
        (synth.random_csr(7, 6, 1.0, 1), synth.random_csr(6, 3, 1.0, 2)),
    ]
    for A, B in cases:
        print("case degenerate %dx%d * %dx%d" % (A.nrows, A.ncols, B.nrows, B.ncols), flush=True)
        C = run(plan, "f64", A, B)
        ref = oracle.spgemm(A, B, "f64")
        got = to_host(C)
        assert_same_structure(got, ref)
        assert_values(got, ref, "f64")


def test_all_products_in_one_column(plan):
    """Every product lands in column 0: one output per row with up to
    thousands of terms (hash and dense paths under maximal collision)."""
    K = 5000
    B = synth.canonical_from_coo(K, 3, np.arange(K), np.zeros(K, np.int64), np.ones(K), dup="first")
    rng = np.random.default_rng(3)
    rows, cols = [], []
    for r, nz in enumerate([1, 2, 30, 64, 65, 500, 2000, 4999, 5000]):
        ks = rng.choice(K, nz, replace=False)
        rows += [r] * nz
        cols += ks.tolist()
    A = synth.canonical_from_coo(9, K, rows, cols, rng.integers(1, 5, len(rows)).astype(np.float64))
    for sr in ("f64", "i64", "bool"):
        AA = A if sr == "f64" else synth.CSR(A.nrows, A.ncols, A.row_ptr, A.col,
                                             A.val.astype(np.int64) if sr == "i64" else np.ones(A.nnz, np.uint8))
        BB = B if sr == "f64" else with_kind(B, sr)
        check_full_vs_oracle(run(plan, sr, AA, BB), AA, BB, sr)


@pytest.mark.parametrize("ncols,want,opts", [
    (9000, 15, dict(rank_max_nnz=16384)), (9000, 11, {}), (6000, 14, dict(rank_block=1024)),
    (9000, 15, dict(rank_block=1024, rank_max_nnz=16384)), (20000, 11, {}), (20000, 11, dict(chunk_group=1)),
    (262144, 14, {}), (1 << 20, 12, {}),
    # one column chunk covers every column: rank chunks without a split table
    (9000, 11, dict(dense_chunk_cols=16384)), (6000, 11, dict(rank_max_nnz=4096, dense_chunk_cols=8192))])
def test_dense_operands(ncols, want, opts):
    """Large output rows.  Dense operands with 9000 columns fit the
    rank-space accumulator of 16384 outputs when it is enabled (rank16384),
    else take rank chunks of the saved bitmap (dense_par); with 1024-thread
    rank workgroups 6000 outputs take rank8192; with 20000 outputs per row
    rank chunks, also one chunk per item; with 262144 columns and 20 entries
    per B row, rank8192; with 2^20 columns one LDS bitmap no longer covers a
    row, so the bitmap pass counts in column blocks and the numeric pass
    sweeps column chunks in one workgroup (dense)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    plan = spg.Plan(**opts)
    A = synth.random_csr(40, 300, 1.0, 5, "f64")
    if ncols < 100000:
        B = synth.random_csr(300, ncols, 1.0, 6, "f64")
    else:
        rng = np.random.default_rng(6)
        rr = np.repeat(np.arange(300), 20)
        cc = np.concatenate([rng.choice(ncols, 20, replace=False) for _ in range(300)])
        B = synth.canonical_from_coo(300, ncols, rr, cc, rng.random(rr.size), dup="first")
    C = run(plan, "f64", A, B)
    st = plan.stats()
    plan.close()
    assert st["num_rows"][want] == 40, st["num_rows"]
    check_full_vs_oracle(C, A, B, "f64")


def test_rmat_s16_c2(plan):
    """C2: R-MAT G500 scale 16, edge factor 16, FP64 U(0,1), INT64 all-ones
    and boolean: all 65,536 rows compared with the oracle, element by
    element (columns exact, INT64/boolean values exact, FP64 within 1e-12
    relative or the summation-order bound around the compensated sum).
    Also: total flops, INT64 all-ones sums to flops, boolean values all true."""
    A = synth.rmat(16, 16, synth.G500, seed=2)
    print("case C2 f64 nnz(A)=%d" % A.nnz, flush=True)
    C = run(plan, "f64", A, A)
    st = plan.stats()
    f = oracle.row_flops(A, A)
    assert st["flops"] == int(f.sum())
    over = check_full_vs_oracle(C, A, A, "f64")
    print("C2 f64: %d of %d entries over 1e-12 relative, all within the compensated bound" % (over, C.nnz),
          flush=True)
    A1 = with_kind(A, "i64")
    print("case C2 i64", flush=True)
    Ci = run(plan, "i64", A1, A1)
    assert torch.equal(Ci.row_ptr, C.row_ptr) and torch.equal(Ci.col, C.col)
    assert int(Ci.val.sum().item()) == int(f.sum())
    del C
    check_full_vs_oracle(Ci, A1, A1, "i64")
    del Ci
    Ab = with_kind(A, "bool")
    print("case C2 bool", flush=True)
    Cb = run(plan, "bool", Ab, Ab)
    assert bool((Cb.val == 1).all().item())
    check_full_vs_oracle(Cb, Ab, Ab, "bool")


def test_determinism_integer(plan):
    A = synth.with_values(synth.rmat(14, 16, synth.G500, seed=12), "ones_i64")
    C1 = run(plan, "i64", A, A)
    C2 = run(plan, "i64", A, A)
    assert torch.equal(C1.row_ptr, C2.row_ptr) and torch.equal(C1.col, C2.col) and torch.equal(C1.val, C2.val)


def test_errors(plan):
    A = to_dev(synth.random_csr(5, 6, 0.5, 1))
    B = to_dev(synth.random_csr(7, 3, 0.5, 2))
    with pytest.raises(spg.SpgError) as e:
        spg.spgemm_symbolic(plan, "f64", A, B)
    assert e.value.name == "SPG_ERR_SHAPE"
    B2 = to_dev(synth.random_csr(6, 3, 0.5, 2))
    with pytest.raises(spg.SpgError) as e:
        spg.spgemm_symbolic(plan, "f64", A, B2, 3, 2)
    assert e.value.name == "SPG_ERR_ARG"
    with pytest.raises(spg.SpgError) as e:
        spg.spgemm_symbolic(plan, "f64", A, B2, 0, 7)
    assert e.value.name == "SPG_ERR_ARG"
    rp, nnz = spg.spgemm_symbolic(plan, "f64", A, B2)
    other = to_dev(synth.random_csr(5, 6, 0.5, 9))
    with pytest.raises(spg.SpgError) as e:
        spg.spgemm_numeric(plan, "f64", other, B2, rp, nnz)
    assert e.value.name == "SPG_ERR_STATE"
    vplan = spg.Plan(validate=True)
    bad = spg.DeviceCSR.from_arrays(2, 4, [0, 2, 3], [3, 1, 0], np.ones(3))
    with pytest.raises(spg.SpgError) as e:
        spg.spgemm_symbolic(vplan, "f64", bad, to_dev(synth.random_csr(4, 2, 0.5, 3)))
    assert e.value.name == "SPG_ERR_NOT_CANONICAL"
    vplan.close()
    # a B whose row-length sums could exceed int32 inside the product
    # kernels (2^31 entries over more than 2^21 columns) is refused before
    # any launch; the descriptor's arrays are small stand-ins, never read
    rows = 1 << 22
    huge = spg.DeviceCSR(rows, 1 << 22, torch.zeros(2, dtype=torch.int64, device=plan.device),
                         torch.zeros(1, dtype=torch.int32, device=plan.device),
                         torch.zeros(1, dtype=torch.float64, device=plan.device))
    a = spg.DeviceCSR(4, rows, torch.zeros(5, dtype=torch.int64, device=plan.device),
                      torch.zeros(1, dtype=torch.int32, device=plan.device),
                      torch.zeros(1, dtype=torch.float64, device=plan.device))
    import ctypes
    hb, ha = huge._c("f64"), a._c("f64")
    hb.nnz = 1 << 31
    hb.nrows = rows
    rp = torch.zeros(5, dtype=torch.int64, device=plan.device)
    nnz = ctypes.c_int64()
    st = spg.lib().spgemm_symbolic(plan.handle, 0, ctypes.byref(ha), ctypes.byref(hb), 0, rows,
                                   ctypes.c_void_p(rp.data_ptr()), ctypes.byref(nnz))
    assert st == 4  # SPG_ERR_INDEX_RANGE


@pytest.mark.parametrize("opts", [
    dict(hash_max_nnz=1024), dict(hash_max_nnz=512, chunk_min_nnz=256), dict(chunk_unroll=8),
    dict(serial_heavy=2), dict(serial_heavy=16, streams=2), dict(streams=1, rank_block=512),
    dict(rank_max_nnz=16384, rank_block=512), dict(rank_max_nnz=1, chunk_group=1),
    dict(gather_map=2, unroll=8, sym_gather_map=2, sym_unroll=8), dict(small_max_flops=1, hash_max_flops=128),
    dict(gather_pipeline=2), dict(gather_pipeline=2, rank_max_nnz=1, dense_chunk_cols=2048)])
def test_option_variants(opts):
    """Every tuning option gives the oracle's product (R-MAT G500 scale 13,
    FP64, plus an INT64 run for the exact values)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A = synth.rmat(13, 16, synth.G500, seed=50)
    p = spg.Plan(**opts)
    try:
        check_full_vs_oracle(run(p, "f64", A, A), A, A, "f64")
        Ai = synth.with_values(A, "ones_i64")
        check_full_vs_oracle(run(p, "i64", Ai, Ai), Ai, Ai, "i64")
    finally:
        p.close()


def test_profile_select_times_one_kernel():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A = synth.rmat(13, 16, synth.G500, seed=51)
    p = spg.Plan(profile=True)
    try:
        run(p, "f64", A, A)
        names = set(p.profile_read())
        assert "rowinfo" in names and len(names) > 3
        p.profile_reset()
        p.profile_select("rowinfo")
        run(p, "f64", A, A)
        assert set(p.profile_read()) == {"rowinfo"}
        p.profile_select(None)
    finally:
        p.close()


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_ssca_class(plan, sr):
    """The third synthetic class of the paper's experiments: R-MAT with the
    SSCA parameters (.6, .4/3, .4/3, .4/3), edge factor 8, scale 15."""
    A = synth.rmat(15, 8, synth.SSCA, seed=60)
    if sr != "f64":
        A = with_kind(A, sr)
    check_full_vs_oracle(run(plan, sr, A, A), A, A, sr)


# table size -> threads of the numeric hash kernel for that size
_HASH_NT = {7: 64, 8: 64, 9: 64, 10: 128, 11: 256, 12: 256, 13: 512}


def _order_path(cols):
    """How the numeric hash kernel orders a row with these distinct sorted
    output columns: by bitmap rank (narrow span), by per-thread column
    buckets sorted in registers (at most 8, 16, or -- with 16 table slots per
    thread -- 32 per bucket, columns that fit beside a slot index in 32
    bits), by buckets sorted in place (at most 32), or by the full sort.  The
    bucket of a column is (column - min) * threads / span in FP32, as in the
    kernel."""
    cnt = cols.size
    lg = max(7, int(np.ceil(np.log2((4 * cnt + 2) // 3))))
    T, NT = 1 << lg, _HASH_NT[lg]
    kmin, kmax = int(cols[0]), int(cols[-1])
    nw = ((kmax - kmin) >> 5) + 1
    if nw <= T and nw <= 8 * cnt + 64:
        return "bitmap"
    scale = np.float32(NT) / np.float32(kmax - kmin + 1)
    b = np.minimum(((cols - kmin).astype(np.float32) * scale).astype(np.int64), NT - 1)
    bmax = int(np.bincount(b).max())
    if bmax > 32:
        return "full_sort"
    net_max = 32 if T // NT >= 16 else 16
    if bmax <= net_max and kmax - kmin < (1 << (32 - lg)):
        return "net8" if bmax <= 8 else ("net16" if bmax <= 16 else "net32")
    return "in_place"


def _hash_order_rows(n, specs, seed):
    """A (len(specs) rows) times B (one entry per row, at a chosen column):
    row r of A holds f_r consecutive B rows, so C(r,:) has exactly the
    chosen columns.  A tenth of each row's products repeat a column of the
    row, so equal columns are summed.  Patterns: "uniform" over [0, n),
    "narrow" inside a window of 4 f columns, "clusterW": W consecutive
    columns plus uniform ones."""
    rng = np.random.default_rng(seed)
    arow, bcol, rows_cols = [], [], []
    for r, (f, pat) in enumerate(specs):
        nd = f - f // 10
        if pat == "uniform":
            cols = rng.choice(n, nd, replace=False)
        elif pat == "narrow":
            cols = int(rng.integers(0, n - 4 * f)) + rng.choice(4 * f, nd, replace=False)
        else:
            w = int(pat[len("cluster"):])
            start = int(rng.integers(0, n - w))
            cols = np.unique(np.concatenate([start + np.arange(w), rng.choice(n, nd - w, replace=False)]))
        cols = np.unique(cols)
        allc = np.concatenate([cols, rng.choice(cols, f - cols.size)])
        rng.shuffle(allc)
        arow += [r] * allc.size
        bcol += allc.tolist()
        rows_cols.append(cols)
    k = len(bcol)
    A = CSR(len(specs), k, np.concatenate([[0], np.cumsum([f for f, _ in specs])]).astype(np.int64),
            np.arange(k, dtype=np.int32), rng.random(k) + 0.5)
    B = CSR(k, n, np.arange(k + 1, dtype=np.int64), np.asarray(bcol, dtype=np.int32), rng.random(k) + 0.5)
    return A, B, rows_cols


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_hash_row_orders(plan, sr):
    """Rows of the hash bins reaching every way the numeric hash kernel
    puts a row in column order (bitmap rank, register sorting networks of 8,
    16 and 32, in-place bucket sort, full sort; columns too far apart to pack
    beside a slot index), all against the oracle."""
    specs = []
    for f in (100, 150, 300, 700, 1400, 2500):
        specs += [(f, "uniform"), (f, "narrow"), (f, "cluster20"), (f, "cluster28"), (f, "cluster40"),
                  (f, "cluster70")]
    seen = set()
    for n, seed, sp in ((1 << 18, 71, specs), (1 << 21, 72, [(f, "uniform") for f in (1400, 2000, 2500, 2900)]
                                                                         + [(100, "cluster20"), (300, "cluster28")])):
        A, B, rows_cols = _hash_order_rows(n, sp, seed)
        paths = [_order_path(c) for c in rows_cols]
        seen |= set(paths)
        print("case hash orders n=%d sr=%s paths=%s" % (n, sr, sorted(set(paths))), flush=True)
        A, B = (A, B) if sr == "f64" else (with_kind(A, sr, seed), with_kind(B, sr, seed))
        C = run(plan, sr, A, B)
        st = plan.stats()
        assert sum(st["num_rows"][3:11]) == A.nrows, "rows outside the hash bins"
        check_full_vs_oracle(C, A, B, sr)
    assert seen >= {"bitmap", "net8", "net16", "net32", "in_place", "full_sort"}, seen


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_wave_enumeration_rows(plan, sr):
    """Rows of the one-wave hash kernels whose products span several batches
    of 64 A entries (150 and 200 A entries over short or empty B rows) and
    rows with few outputs but thousands of products (50 B rows sharing the
    same 300 columns: 15,000 products, 300 outputs, so the numeric pass
    takes the 512-slot one-wave kernel), also through inner windows, all
    against the oracle."""
    rng = np.random.default_rng(81)
    n = 50000
    brows, bcols = [], []
    k = 0
    shared = rng.choice(n, 300, replace=False)
    dup_rows = list(range(k, k + 50))
    for r in dup_rows:
        brows += [r] * 300
        bcols += shared.tolist()
    k += 50
    short_rows = list(range(k, k + 600))
    for r in short_rows:
        c = int(rng.integers(0, 4))  # 0..3 entries, some rows empty
        brows += [r] * c
        bcols += rng.choice(n, c, replace=False).tolist()
    k += 600
    B = synth.canonical_from_coo(k, n, np.array(brows), np.array(bcols), rng.random(len(brows)) + 0.5, dup="first")
    arows, acols = [], []
    specs = [dup_rows, dup_rows[:20], rng.choice(short_rows, 150, replace=False).tolist(),
             rng.choice(short_rows, 200, replace=False).tolist(), short_rows[:70],
             rng.choice(short_rows, 100, replace=False).tolist() + dup_rows[:3]]
    for i, ks in enumerate(specs):
        arows += [i] * len(ks)
        acols += [int(x) for x in ks]
    A = synth.canonical_from_coo(len(specs), k, np.array(arows), np.array(acols), rng.random(len(arows)) + 0.5,
                                 dup="first")
    A, B = (A, B) if sr == "f64" else (with_kind(A, sr), with_kind(B, sr))
    for lo, hi in ((0, k), (10, 400), (40, 650)):
        print("case wave rows sr=%s window=(%d,%d)" % (sr, lo, hi), flush=True)
        C = run(plan, sr, A, B, lo, hi)
        check_full_vs_oracle(C, A, B, sr, lo, hi)
    run(plan, sr, A, B)
    st = plan.stats()
    assert st["num_rows"][5] > 0, "no row in the 512-slot numeric bin"
