"""GPU checks of the row-size predictor and the single-pass product.

The HIP forward pass and gradient are compared with the FP64 reference
(oracle/mlp.py), the Adam step with torch's CPU Adam, and the single-pass
product with the oracle and with the two-phase path: the structure must be
identical whatever the predictions, including when every predicted row
overflows its capacity."""

import numpy as np
import pytest
import torch

import oracle
import paper_1510_00844_amd as spg
import synth
from oracle import mlp
from gpu_util import check_full_vs_oracle, to_dev, to_host
from util import assert_same_structure, assert_values

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def plan():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = spg.Plan()
    yield p
    p.close()


def _xt(seed, n):
    rng = np.random.default_rng(seed)
    X = mlp.features(rng.integers(2, 300, n), rng.integers(65, 50000, n), rng.integers(1, 2000, n))
    t = np.log1p(rng.integers(1, 20000, n).astype(np.float64))
    return X, t


def test_forward_matches_reference(plan):
    X, _ = _xt(1, 3000)
    p = mlp.init_params(3)
    y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
    spg.spg_mlp_forward(plan, torch.tensor(p, dtype=torch.float32, device="cuda"),
                        torch.tensor(X, dtype=torch.float32, device="cuda"), y)
    ref, _ = mlp.forward(p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    assert np.allclose(y.cpu().numpy(), ref, rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("n", [1, 255, 256, 1000, 5000])
def test_gradient_matches_reference(plan, n):
    X, t = _xt(2 + n, n)
    p = mlp.init_params(4)
    p32 = p.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    t32 = t.astype(np.float32).astype(np.float64)
    grad = torch.zeros(spg.MLP_NPARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    spg.spg_mlp_grad(plan, torch.tensor(p32, dtype=torch.float32, device="cuda"),
                     torch.tensor(X32, dtype=torch.float32, device="cuda"),
                     torch.tensor(t32, dtype=torch.float32, device="cuda"), 4.0, grad, loss)
    g_ref = mlp.backward(p32, X32, t32, 4.0)
    g = grad.cpu().numpy().astype(np.float64)
    scale = np.abs(g_ref).max()
    assert np.max(np.abs(g - g_ref)) <= 1e-4 * scale + 1e-7, np.max(np.abs(g - g_ref)) / scale
    assert abs(loss.item() - mlp.loss(p32, X32, t32, 4.0)) <= 1e-4 * mlp.loss(p32, X32, t32, 4.0)


def test_adam_matches_torch(plan):
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=spg.MLP_NPARAMS).astype(np.float32)
    grads = [rng.normal(size=spg.MLP_NPARAMS).astype(np.float32) for _ in range(3)]
    ref = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([ref], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    dp = torch.tensor(p0, device="cuda")
    m = torch.zeros_like(dp)
    v = torch.zeros_like(dp)
    for k, g in enumerate(grads):
        opt.zero_grad()
        ref.grad = torch.tensor(g)
        opt.step()
        dg = torch.tensor(g, device="cuda")
        spg.spg_mlp_adam(plan, dp, dg, m, v, k + 1, 1e-2)
        assert float(dg.abs().max()) == 0.0  # cleared after the step
    assert np.allclose(dp.cpu().numpy(), ref.detach().numpy(), rtol=1e-5, atol=1e-6)


def test_training_lowers_the_loss(plan):
    from paper_1510_00844_amd import learned
    x, t = learned.training_rows(plan, [("g500", 12, 100), ("er", 12, 101), ("g500", 13, 102)])
    assert x.shape[0] == t.shape[0] > 500
    params, hist = learned.train(plan, x, t, epochs=15, batch=2048)
    assert hist[-1] < 0.25 * hist[0], hist


def _learned_vs_plain(plan, A, sr, params, margin=0.15):
    dA = to_dev(A, sr)
    C, st = spg.spgemm_learned(plan, sr, dA, dA, params, margin)
    P = spg.spgemm(plan, sr, dA, dA)
    assert torch.equal(C.row_ptr, P.row_ptr) and torch.equal(C.col, P.col)
    if sr != "f64":
        assert torch.equal(C.val, P.val)
    return C, st


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_single_pass_equals_two_phase_and_oracle(plan, sr):
    A = synth.rmat(13, 16, synth.G500, seed=40)
    if sr != "f64":
        A = synth.with_values(A, "ones_i64" if sr == "i64" else "true_bool")
    params = torch.tensor(mlp.init_params(2), dtype=torch.float32, device="cuda")
    C, st = _learned_vs_plain(plan, A, sr, params)
    check_full_vs_oracle(C, A, A, sr)


def test_fused_single_pass_equals_oracle():
    """The fused bitmap-and-rank single pass (off by default), for rows
    predicted above the hash tables."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A = synth.rmat(13, 16, synth.G500, seed=44)
    params = torch.tensor(mlp.init_params(2), dtype=torch.float32, device="cuda")
    p = spg.Plan(fused_max_nnz=16384)
    try:
        C, st = _learned_vs_plain(p, A, "f64", params)
        fused = sum(st["bin_rows"][b] for b in range(13, 16))
        assert fused > 0, st
        check_full_vs_oracle(C, A, A, "f64")
    finally:
        p.close()


def test_forced_overflow_falls_back(plan):
    """A network that predicts 0 for every row sizes each slot at its lower
    bound max_k nnz(B(k,:)): nearly every predicted row overflows and is
    recomputed exactly; the result is unchanged."""
    A = synth.rmat(13, 16, synth.G500, seed=41)
    p = np.zeros(spg.MLP_NPARAMS, dtype=np.float32)
    p[-1] = -30.0  # y = -30 everywhere
    C, st = _learned_vs_plain(plan, A, "f64", torch.tensor(p, device="cuda"), margin=0.0)
    assert st["rows_overflow"] > 0.5 * st["rows_predicted"], st
    check_full_vs_oracle(C, A, A, "f64")


def test_upper_bound_sizing_never_overflows(plan):
    A = synth.rmat(13, 16, synth.ER, seed=42)
    C, st = _learned_vs_plain(plan, A, "f64", None)
    assert st["rows_overflow"] == 0
    check_full_vs_oracle(C, A, A, "f64")


def test_window_single_pass(plan):
    A = synth.rmat(12, 16, synth.G500, seed=43)
    B = synth.rmat(12, 16, synth.ER, seed=44)
    dA, dB = to_dev(A), to_dev(B)
    params = torch.tensor(mlp.init_params(7), dtype=torch.float32, device="cuda")
    for lo, hi in [(0, 1000), (1000, 4096), (0, 0)]:
        nnz, st = spg.spgemm_learned_run(plan, "f64", dA, dB, params, 0.15, lo, hi)
        C = spg.spgemm_learned_fetch(plan, "f64", dA, dB, nnz)
        check_full_vs_oracle(C, A, B, "f64", lo, hi)


def test_trained_predictor_gain():
    """The shipped trained weights against sizing without a predictor
    (capacity = min(flops, n)), on an R-MAT G500 scale-16 product (not in
    the training set), with the fused single pass on (rows up to 8192
    predicted outputs), where the capacities depend on the prediction: the
    same result; with the predictor more of C is produced in the single
    pass, fewer rows need the exact method, and the padded slots are used
    far more fully."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_00844_amd import learned
    import os
    if not os.path.exists(learned.WEIGHTS):
        pytest.skip("no trained weights")
    plan = spg.Plan(fused_max_nnz=8192)
    try:
        _predictor_gain(plan, learned.load())
    finally:
        plan.close()


def _predictor_gain(plan, params):
    A = synth.rmat(16, 16, synth.G500, seed=2)
    dA = to_dev(A)
    nnz_l, st_l = spg.spgemm_learned_run(plan, "f64", dA, dA, params, 0.15)
    C = spg.spgemm_learned_fetch(plan, "f64", dA, dA, nnz_l)
    nnz_u, st_u = spg.spgemm_learned_run(plan, "f64", dA, dA, None, 0.15)
    assert nnz_l == nnz_u
    print("learned", st_l, "upper bound", st_u)
    eff_l = st_l["nnz_single"] / max(st_l["slots"], 1)
    eff_u = st_u["nnz_single"] / max(st_u["slots"], 1)
    assert eff_l > 1.05 * eff_u, (eff_l, eff_u)
    assert st_l["nnz_single"] > st_u["nnz_single"]
    assert st_l["rows_exact"] + st_l["rows_overflow"] < st_u["rows_exact"] + st_u["rows_overflow"]
    assert st_l["rows_overflow"] < 0.1 * max(st_l["rows_predicted"], 1), st_l
    check_full_vs_oracle(C, A, A, "f64")
