"""GPU checks of the batched Galerkin products C_b = (R_b^T A_b) R_b.

Every instance of a batched call must equal the oracle's two products and
the library's own unbatched two-phase run (the values of the 7-point
operator times 0/1 aggregations are small integers, so FP64 is exact too),
the coarse operators must have the closed-form structure of the 7-point
stencil on the coarse grid, and graph replays must reproduce the first
(eager) call and follow value updates of the inputs."""

import numpy as np
import pytest
import torch

import oracle
import paper_1510_00844_amd as spg
import synth
from gpu_util import to_dev, to_host
from util import assert_same_structure, assert_values

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def plan():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = spg.Plan()
    yield p
    p.close()


def _typed(M, sr):
    if sr == "f64" or M.val is None:
        return M
    if sr == "i64":
        return synth.CSR(M.nrows, M.ncols, M.row_ptr, M.col, np.asarray(M.val).astype(np.int64), M.meta)
    return synth.with_values(M, "true_bool")


def _oracle_galerkin(RT, A, R, sr):
    return oracle.spgemm(oracle.spgemm(RT, A, sr), R, sr)


def _empty_instance(n):
    """M = 0 aggregates: RT is 0 x n, R is n x 0."""
    RT = synth.CSR(0, n, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    R = synth.CSR(n, 0, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    return RT, synth.poisson7(round(n ** (1 / 3))), R


def _zero_operator(N):
    RT, R = synth.aggregation_2x2x2(N)
    n = N ** 3
    A = synth.CSR(n, n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    return RT, A, R


def _small_batch():
    _, inst = synth.galerkin_batch(count=9, nmin=1, nmax=13, seed=11)
    inst = list(inst)
    inst.insert(3, _empty_instance(27))
    inst.append(_zero_operator(4))
    return inst


def _run(plan, inst, sr, use_graph=True):
    dev = [(to_dev(_typed(RT, sr), sr), to_dev(_typed(A, sr), sr), to_dev(_typed(R, sr), sr)) for RT, A, R in inst]
    res = spg.spgemm_galerkin_batched(plan, sr, [d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev],
                                      use_graph=use_graph)
    return dev, res


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_batched_equals_oracle_and_unbatched(plan, sr):
    inst = _small_batch()
    dev, res = _run(plan, inst, sr)
    got = res.fetch(plan)
    assert len(got) == len(inst)
    for b, ((RT, A, R), (dRT, dA, dR), C) in enumerate(zip(inst, dev, got)):
        ref = _oracle_galerkin(_typed(RT, sr), _typed(A, sr), _typed(R, sr), sr)
        h = to_host(C)
        assert (h.nrows, h.ncols) == (RT.nrows, R.ncols), b
        assert_same_structure(h, ref)
        if sr == "f64":
            assert np.array_equal(h.val, ref.val), b  # small integers: exact
        else:
            assert_values(h, ref, sr)
        T = spg.spgemm(plan, sr, dRT, dA)
        U = spg.spgemm(plan, sr, T, dR)
        assert torch.equal(U.row_ptr, C.row_ptr) and torch.equal(U.col, C.col), b
        assert torch.equal(U.val, C.val), b


def test_c4_closed_forms_and_oracle(plan):
    """The full batch: 64 grids with N uniform in [16, 64]."""
    sizes, inst = synth.galerkin_batch()
    dev, res = _run(plan, inst, "f64")
    got = res.fetch(plan)
    for b, (N, (RT, A, R), C) in enumerate(zip(sizes.tolist(), inst, got)):
        M = (N + 1) // 2
        assert C.nrows == C.ncols == M ** 3
        assert C.nnz == 7 * M ** 3 - 6 * M ** 2, (b, N)
        h = to_host(C)
        ref = _oracle_galerkin(RT, A, R, "f64")
        assert_same_structure(h, ref)
        assert np.array_equal(h.val, ref.val), b
        # row sums of C are the sums of A's rows over each aggregate
        rs = np.add.reduceat(h.val, h.row_ptr[:-1]) if h.nnz else np.zeros(0)
        a_rs = np.add.reduceat(A.val, A.row_ptr[:-1])
        want = np.zeros(M ** 3)
        np.add.at(want, R.col, a_rs)
        assert np.array_equal(rs, want), b


def test_graph_replay_and_value_update(plan):
    inst = _small_batch()[:6]
    dev, res = _run(plan, inst, "f64", use_graph=True)
    first = [to_host(C) for C in res.fetch(plan)]
    for rep in range(3):
        # eager work and a synchronization between replays
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        res2 = spg.spgemm_galerkin_batched(plan, "f64", [d[0] for d in dev], [d[1] for d in dev],
                                           [d[2] for d in dev], use_graph=True)
        assert res2.nnz == res.nnz
        for b, C in enumerate(res2.fetch(plan)):
            h = to_host(C)
            assert_same_structure(h, first[b])
            assert np.array_equal(h.val, first[b].val), (rep, b)
    # new values in the same buffers: the replay follows them
    rng = np.random.default_rng(3)
    newA = []
    for (RT, A, R), (_, dA, _) in zip(inst, dev):
        v = rng.integers(-3, 4, A.nnz).astype(np.float64)
        dA.val.copy_(torch.as_tensor(v, device="cuda"))
        newA.append(synth.CSR(A.nrows, A.ncols, A.row_ptr, A.col, v))
    res3 = spg.spgemm_galerkin_batched(plan, "f64", [d[0] for d in dev], [d[1] for d in dev],
                                       [d[2] for d in dev], use_graph=True)
    for b, ((RT, _, R), A2, C) in enumerate(zip(inst, newA, res3.fetch(plan))):
        ref = _oracle_galerkin(RT, A2, R, "f64")
        h = to_host(C)
        # numerical cancellation may leave explicit zeros; structure is symbolic
        assert np.array_equal(h.row_ptr, first[b].row_ptr) and np.array_equal(h.col, first[b].col)
        dense_ref = np.zeros((ref.nrows, ref.ncols))
        for i in range(ref.nrows):
            dense_ref[i, ref.col[ref.row_ptr[i]:ref.row_ptr[i + 1]]] = ref.val[ref.row_ptr[i]:ref.row_ptr[i + 1]]
        dense_got = np.zeros_like(dense_ref)
        for i in range(h.nrows):
            dense_got[i, h.col[h.row_ptr[i]:h.row_ptr[i + 1]]] = h.val[h.row_ptr[i]:h.row_ptr[i + 1]]
        assert np.array_equal(dense_got, dense_ref), b


def _heavy_instance(n, agg, density, seed):
    """Aggregation of `agg` fine points per coarse point over a random
    operator dense enough that the rows of R^T A take the bitmap and rank
    paths (the heavy bins the captured graph orders by work)."""
    rng = np.random.default_rng(seed)
    a = rng.random((n, n)) < density
    r, c = np.nonzero(a)
    A = synth.canonical_from_coo(n, n, r, c, rng.integers(-2, 3, r.size).astype(np.float64), dup="first")
    m = (n + agg - 1) // agg
    rows = np.arange(n)
    R = synth.canonical_from_coo(n, m, rows, rows // agg, np.ones(n), dup="first")
    RT = synth.canonical_from_coo(m, n, rows // agg, rows, np.ones(n), dup="first")
    return RT, A, R


def test_graph_replay_with_heavy_rows(plan):
    """Instances whose products have heavy rows: the captured graph holds
    the heavy bins' work ordering and the bitmap and rank kernels; replays
    match the eager call and the oracle bit for bit (integer values)."""
    inst = [_heavy_instance(512, 64, 0.2, 1), _heavy_instance(300, 50, 0.3, 2), _heavy_instance(640, 80, 0.15, 3)]
    dev, res = _run(plan, inst, "f64", use_graph=True)
    first = [to_host(C) for C in res.fetch(plan)]
    for b, ((RT, A, R), h) in enumerate(zip(inst, first)):
        ref = _oracle_galerkin(RT, A, R, "f64")
        assert_same_structure(h, ref)
        assert np.array_equal(h.val, ref.val), b
    for rep in range(3):
        torch.cuda.synchronize()
        res2 = spg.spgemm_galerkin_batched(plan, "f64", [d[0] for d in dev], [d[1] for d in dev],
                                           [d[2] for d in dev], use_graph=True)
        for b, C in enumerate(res2.fetch(plan)):
            h = to_host(C)
            assert_same_structure(h, first[b])
            assert np.array_equal(h.val, first[b].val), (rep, b)


def test_eager_and_graph_agree(plan):
    inst = _small_batch()[:5]
    p2 = spg.Plan()
    try:
        _, r1 = _run(plan, inst, "i64", use_graph=False)
        a = [to_host(C) for C in r1.fetch(plan)]
        dev, r2 = _run(p2, inst, "i64", use_graph=True)
        r2 = spg.spgemm_galerkin_batched(p2, "i64", [d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev])
        b_ = [to_host(C) for C in r2.fetch(p2)]
        for x, y in zip(a, b_):
            assert_same_structure(x, y)
            assert np.array_equal(x.val, y.val)
    finally:
        p2.close()


def test_batched_errors(plan):
    p = spg.Plan()
    try:
        with pytest.raises(spg.SpgError):
            spg.GalerkinBatch([], "f64").fetch(p)  # nothing computed on this plan
    finally:
        p.close()
    RT, A, R = synth.galerkin_batch(count=1, nmin=4, nmax=4)[1][0]
    dRT, dA, dR = to_dev(RT), to_dev(A), to_dev(R)
    with pytest.raises(spg.SpgError):
        spg.spgemm_galerkin_batched(plan, "f64", [dR], [dA], [dR])  # R in place of RT: shapes
    with pytest.raises(ValueError):
        spg.spgemm_galerkin_batched(plan, "f64", [dRT, dRT], [dA], [dR])


def test_autotune_cache(tmp_path):
    """The tuner returns valid options, the tuned plan gives the same
    result, and a second call reads the cache instead of timing."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    inst = _small_batch()
    cache = str(tmp_path / "tune.jsonl")
    p = spg.Plan()
    try:
        dev = [(to_dev(RT), to_dev(A), to_dev(R)) for RT, A, R in inst]
        args = ([d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev])
        ref = [to_host(C) for C in spg.spgemm_galerkin_batched(p, "f64", *args).fetch(p)]
        opts, hit = spg.spg_autotune_galerkin(p, "f64", *args, cache_path=cache, budget_ms=3000)
        assert not hit
        assert opts["streams"] in (1, 2, 4) and opts["gather_map"] in (1, 2) and opts["unroll"] in (4, 8)
        assert 0 < opts["small_max_flops"] <= 64 and 0 < opts["hash_max_nnz"] <= 4096
        got = [to_host(C) for C in spg.spgemm_galerkin_batched(p, "f64", *args).fetch(p)]
        for x, y in zip(got, ref):
            assert_same_structure(x, y)
            assert np.array_equal(x.val, y.val)
        opts2, hit2 = spg.spg_autotune_galerkin(p, "f64", *args, cache_path=cache, budget_ms=3000)
        assert hit2 and opts2 == opts
        lines = open(cache).read().strip().splitlines()
        assert len(lines) == 1 and '"key": "galerkin:' in lines[0]
    finally:
        p.close()
