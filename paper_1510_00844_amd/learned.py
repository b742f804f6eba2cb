"""Training driver of the row-size predictor.

The network is trained on the GPU by the library's own kernels
(spg_mlp_grad, spg_mlp_adam) on rows whose exact sizes come from the
library's symbolic pass over R-MAT G500 and Erdos-Renyi matrices of scales
14 to 17 (the generators of Section 5).  This module only sequences those
calls and moves the resulting weights to and from a JSON file.

Usage (on a GPU): python -m paper_1510_00844_amd.learned --out sizer_weights.json
"""

from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import (DeviceCSR, MLP_NPARAMS, Plan, spg_mlp_adam, spg_mlp_grad, spg_row_training_data,
               spgemm_symbolic)

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "sizer_weights.json")

# (class, scale, seed): the training matrices, seeds 100-115
TRAIN_SET = [(cls, s, 100 + 2 * i + j) for i, (cls, s) in
             enumerate([(c, s) for c in ("g500", "er") for s in (14, 15, 16, 17)]) for j in range(2)]


def he_init(seed: int = 0) -> np.ndarray:
    """Random initial weights (W1, b1, W2, b2, w3, b3), He scaling."""
    rng = np.random.default_rng(seed)
    H = 32
    W1 = rng.normal(0.0, np.sqrt(2.0 / 3), (H, 3))
    W2 = rng.normal(0.0, np.sqrt(2.0 / H), (H, H))
    w3 = rng.normal(0.0, np.sqrt(1.0 / H), H)
    p = np.concatenate([W1.ravel(), np.full(H, 0.01), W2.ravel(), np.full(H, 0.01), w3, [0.0]])
    assert p.size == MLP_NPARAMS
    return p.astype(np.float32)


def training_rows(plan: Plan, matrices, device="cuda", min_flops: int = 0):
    """Features and targets of the predicted rows of C = A*A for each
    (class, scale, seed), from the symbolic pass."""
    import synth
    xs, ts = [], []
    for cls, scale, seed in matrices:
        abcd = synth.G500 if cls == "g500" else synth.ER
        A = synth.rmat(scale, 16, abcd, seed=seed)
        dA = DeviceCSR.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col, A.val, device)
        rp, _ = spgemm_symbolic(plan, "f64", dA, dA)
        x, t = spg_row_training_data(plan, rp, A.nrows, min_flops)
        xs.append(x.clone())
        ts.append(t.clone())
    return torch.cat(xs), torch.cat(ts)


# Rows with fewer products have tight bounds already (their capacity is
# clamped to flops); training on the rows where sizing matters fits those.
MIN_FLOPS = 1024


def train(plan: Plan, x: torch.Tensor, t: torch.Tensor, epochs=100, batch=8192, lr=3e-3, alpha=4.0, seed=0,
          log=None):
    """Adam on the asymmetric squared loss; returns (params, per-epoch loss)."""
    dev = x.device
    params = torch.as_tensor(he_init(seed), device=dev)
    grad = torch.zeros(MLP_NPARAMS, dtype=torch.float32, device=dev)
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    n = t.shape[0]
    nb = (n + batch - 1) // batch
    step = 0
    history = []
    for ep in range(epochs):
        loss.zero_()
        shift = (ep * 7919) % max(nb, 1)
        for bi in range(nb):
            b0 = ((bi + shift) % nb) * batch
            b1 = min(b0 + batch, n)
            spg_mlp_grad(plan, params, x[b0:b1], t[b0:b1], alpha, grad, loss)
            step += 1
            spg_mlp_adam(plan, params, grad, m, v, step, lr)
        el = float(loss.item()) / nb
        history.append(el)
        if log:
            log("epoch %d loss %.5f" % (ep, el))
    return params, history


def save(params: torch.Tensor, path: str, meta: dict):
    with open(path, "w") as f:
        json.dump({"nparams": MLP_NPARAMS, "params": [float(v) for v in params.cpu().numpy()], "meta": meta}, f)


def load(path: str = WEIGHTS, device="cuda") -> torch.Tensor:
    with open(path) as f:
        d = json.load(f)
    assert d["nparams"] == MLP_NPARAMS
    return torch.tensor(d["params"], dtype=torch.float32, device=device)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--epochs", type=int, default=100)
    args = ap.parse_args()
    plan = Plan()
    t0 = time.time()
    x, t = training_rows(plan, TRAIN_SET, min_flops=MIN_FLOPS)
    t1 = time.time()
    params, hist = train(plan, x, t, epochs=args.epochs, log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    t2 = time.time()
    save(params, args.out, {"train_set": TRAIN_SET, "rows": int(t.shape[0]), "epochs": args.epochs,
                            "min_flops": MIN_FLOPS,
                            "loss_history": hist, "data_seconds": t1 - t0, "train_seconds": t2 - t1,
                            "loss": "mean a (y - t)^2, a = 4 if y < t else 1; t = log1p nnz(C(i,:))"})
    print(json.dumps({"rows": int(t.shape[0]), "final_loss": hist[-1], "train_seconds": t2 - t1}))


if __name__ == "__main__":
    main()
