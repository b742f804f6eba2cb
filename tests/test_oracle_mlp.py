"""Pins of the FP64 predictor reference: central finite differences, an
independent autograd implementation (torch, float64, CPU), and closed
forms."""

import numpy as np
import pytest
import torch

from oracle import mlp


def _data(seed, n=200):
    rng = np.random.default_rng(seed)
    X = mlp.features(rng.integers(1, 300, n), rng.integers(2, 50000, n), rng.integers(1, 2000, n))
    t = np.log1p(rng.integers(1, 20000, n).astype(np.float64))
    return X, t


@pytest.mark.parametrize("alpha", [1.0, 4.0])
def test_gradient_matches_finite_differences(alpha):
    X, t = _data(1)
    p = mlp.init_params(3)
    g = mlp.backward(p, X, t, alpha)
    rng = np.random.default_rng(7)
    idx = rng.choice(mlp.NPARAMS, 60, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAMS)
        e[k] = h
        fd = (mlp.loss(p + e, X, t, alpha) - mlp.loss(p - e, X, t, alpha)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_forward_and_gradient_match_torch_autograd():
    X, t = _data(2)
    p = mlp.init_params(5)
    alpha = 4.0
    W1, b1, W2, b2, w3, b3 = [torch.tensor(np.array(a), dtype=torch.float64, requires_grad=True)
                              for a in mlp.unpack(p)]
    Xt = torch.tensor(X)
    tt = torch.tensor(t)
    y = torch.relu(torch.relu(Xt @ W1.T + b1) @ W2.T + b2) @ w3 + b3
    d = y - tt
    a = torch.where(d < 0, torch.full_like(d, alpha), torch.ones_like(d))
    L = (a * d * d).mean()
    L.backward()
    y_ref, _ = mlp.forward(p, X)
    assert np.allclose(y.detach().numpy(), y_ref, rtol=1e-13, atol=1e-13)
    assert abs(L.item() - mlp.loss(p, X, t, alpha)) <= 1e-13 * abs(L.item())
    g_ref = mlp.pack(W1.grad.numpy(), b1.grad.numpy(), W2.grad.numpy(), b2.grad.numpy(),
                     w3.grad.numpy(), b3.grad.item())
    assert np.allclose(mlp.backward(p, X, t, alpha), g_ref, rtol=1e-12, atol=1e-14)


def test_closed_forms():
    X, t = _data(3, 50)
    # zero weights: y = b3 everywhere, only b3 has a gradient, equal to the
    # mean of 2 a (b3 - t)
    p = np.zeros(mlp.NPARAMS)
    p[-1] = 2.5
    y, _ = mlp.forward(p, X)
    assert np.all(y == 2.5)
    g = mlp.backward(p, X, t, 4.0)
    d = 2.5 - t
    a = np.where(d < 0, 4.0, 1.0)
    assert np.allclose(g[-1], np.mean(2 * a * d))
    assert np.all(g[:-1] == 0.0)
    # a unit whose pre-activation is negative for every row passes no gradient
    p = mlp.init_params(9)
    W1, b1, W2, b2, w3, b3 = [np.array(v, dtype=np.float64) for v in mlp.unpack(p)]
    W1[0] = 0.0
    b1[0] = -1.0
    p = mlp.pack(W1, b1, W2, b2, w3, b3)
    g = mlp.backward(p, X, t, 1.0)
    gW1 = g[:3 * mlp.H].reshape(mlp.H, 3)
    assert np.all(gW1[0] == 0.0) and g[3 * mlp.H] == 0.0


def test_capacity_bounds():
    y = np.log1p(np.array([0.0, 10.0, 1000.0, 1e9]))
    maxb = np.array([5, 50, 20, 7])
    flops = np.array([6, 40, 5000, 800])
    cap = mlp.capacity(y, maxb, flops, n=6000, margin=0.25)
    # 8 -> upper bound 6; 20 -> lower bound 50 -> upper bound 40; 1250+8; upper bound flops
    assert list(cap) == [6, 40, 1258, 800]
    cap = mlp.capacity(y, maxb, flops, n=700, margin=0.25)
    assert list(cap) == [6, 40, 700, 700]  # upper bound n
