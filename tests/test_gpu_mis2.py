"""GPU parity of the distance-2 maximal independent set, the aggregation and
the restriction operator (Section 5.3, Algorithm 3) with the oracle: the
same set, aggregates, round count and R bit for bit, since both sides draw
the per-round keys from the same counter-based generator definition."""

import numpy as np
import pytest
import torch

import oracle
import paper_1510_00844_amd as spg
import synth
from gpu_util import to_dev, to_host
from oracle import mis2 as M
from util import assert_same_structure

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def plan():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = spg.Plan()
    yield p
    p.close()


def sym_graph(n, p, seed, diag=True, isolated=0):
    rng = np.random.default_rng(seed)
    a = rng.random((n, n)) < p
    a = a | a.T
    np.fill_diagonal(a, diag)
    if isolated:
        a[:isolated, :] = False
        a[:, :isolated] = False
    r, c = np.nonzero(a)
    return synth.canonical_from_coo(n, n, r, c, np.ones(r.size), dup="first")


def check(plan, A, seed):
    in_mis, agg, na, rounds = spg.spg_mis2_aggregate(plan, to_dev(A), seed)
    ref_mis, ref_rounds = M.mis2(A, seed)
    ref_agg, ref_na = M.aggregate(A, ref_mis, seed)
    assert np.array_equal(in_mis.cpu().numpy().astype(bool), ref_mis)
    assert rounds == ref_rounds and na == ref_na
    assert np.array_equal(agg.cpu().numpy(), ref_agg)
    return agg, na


@pytest.mark.parametrize("N", [2, 5, 8, 13, 48])
def test_poisson_grids(plan, N):
    check(plan, synth.poisson7(N), seed=100 + N)


@pytest.mark.parametrize("n,p,seed,diag,iso", [(50, 0.1, 1, True, 0), (300, 0.01, 2, False, 0),
                                               (200, 0.02, 3, True, 7), (64, 1.0, 4, False, 0)])
def test_random_graphs(plan, n, p, seed, diag, iso):
    check(plan, sym_graph(n, p, seed, diag, iso), seed=seed * 17)


def test_edgeless_and_empty(plan):
    E = synth.CSR(10, 10, np.zeros(11, np.int64), np.zeros(0, np.int32), np.zeros(0))
    agg, na = check(plan, E, 3)
    assert na == 10 and agg.cpu().numpy().tolist() == list(range(10))
    Z = synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    in_mis, agg, na, rounds = spg.spg_mis2_aggregate(plan, to_dev(Z), 1)
    assert na == 0 and in_mis.numel() == 0


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_restriction_matches_oracle(plan, sr):
    A = synth.poisson7(9)
    agg, na = check(plan, A, 21)
    R, RT = spg.spg_restriction(plan, sr, agg, na)
    ref_R, ref_RT = M.restriction(A.nrows, na, agg.cpu().numpy())
    for got, ref in ((to_host(R), ref_R), (to_host(RT), ref_RT)):
        assert_same_structure(got, ref)
        assert (got.val == 1).all()


def test_large_aggregate_rows_sorted(plan):
    """A star graph: one aggregate of 3000 vertices (the LDS row sort)."""
    n = 3000
    r = np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n)])
    c = np.concatenate([np.arange(1, n), np.zeros(n - 1, np.int64)])
    A = synth.canonical_from_coo(n, n, r, c, np.ones(r.size), dup="first")
    agg, na = check(plan, A, 5)
    assert na == 1
    R, RT = spg.spg_restriction(plan, "f64", agg, na)
    assert np.array_equal(RT.col.cpu().numpy(), np.arange(n))


def test_galerkin_with_algebraic_restriction(plan):
    """Batched (R^T A) R with MIS-2 restrictions of three grids equals the
    oracle's products exactly (integer values)."""
    RTs, As, Rs, host = [], [], [], []
    for N, seed in ((6, 1), (9, 2), (12, 3)):
        A = synth.poisson7(N)
        agg, na = check(plan, A, seed)
        R, RT = spg.spg_restriction(plan, "f64", agg, na)
        dA = to_dev(A)
        RTs.append(RT); As.append(dA); Rs.append(R)
        host.append((to_host(RT), A, to_host(R)))
    res = spg.spgemm_galerkin_batched(plan, "f64", RTs, As, Rs)
    for (hRT, hA, hR), C in zip(host, res.fetch(plan)):
        ref = oracle.spgemm(oracle.spgemm(hRT, hA, "f64"), hR, "f64")
        got = to_host(C)
        assert_same_structure(got, ref)
        assert np.array_equal(got.val, ref.val)


def test_errors(plan):
    A = synth.random_csr(5, 7, 0.5, 1, "f64")
    with pytest.raises(spg.SpgError):
        spg.spg_mis2_aggregate(plan, to_dev(A), 1)
