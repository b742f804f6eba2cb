"""The merge entry point that allocates nothing (spgemm_merge_layers_noalloc,
its scratch in a fixed device array) against spgemm_merge_layers on the same
device layers: two calls in a row, the second with a smaller input, so the
second runs over what the first left in the array.  Row pointers, columns and
values must be equal bit for bit (both add equal columns in ascending layer
order, in the same kernels)."""

import numpy as np
import pytest
import torch

import paper_1510_00844_amd as spg
import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _layers(plan, sr, scale, kind, c, seed):
    A = synth.rmat(scale, 16, kind, seed=seed)
    B = synth.rmat(scale, 16, synth.G500, seed=seed + 1)
    if sr != "f64":
        v = "ones_i64" if sr == "i64" else "true_bool"
        A, B = synth.with_values(A, v), synth.with_values(B, v)
    dA, dB = to_dev(A, sr), to_dev(B, sr)
    return [spg.spgemm(plan, sr, dA, dB, lo, hi) for lo, hi in synth.layer_bounds(A.ncols, c)]


# (scale, kind, layers) of the first and the second, smaller, call; c <= 8
# takes the k-way wave merge for short rows, c = 16 the rank kernels
CALLS = {
    "kway_then_rank": ((14, synth.G500, 4), (12, synth.ER, 16)),
    "rank_then_kway": ((14, synth.G500, 16), (11, synth.G500, 3)),
}


@pytest.mark.parametrize("calls", sorted(CALLS))
@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
def test_merge_noalloc_matches_merge(sr, calls):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    plan = spg.Plan()
    try:
        prev_m = None
        for k, (scale, kind, c) in enumerate(CALLS[calls]):
            print("case noalloc sr=%s %s call %d: scale %d, %d layers" % (sr, calls, k, scale, c), flush=True)
            layers = _layers(plan, sr, scale, kind, c, seed=40 + k)
            m = layers[0].nrows
            assert prev_m is None or m < prev_m
            prev_m = m
            ref = spg.spgemm_merge_layers(plan, sr, layers)
            got = spg.spgemm_merge_layers_noalloc(sr, layers)
            torch.cuda.synchronize()
            assert got.nnz == ref.nnz and ref.nnz > 0
            assert torch.equal(got.row_ptr, ref.row_ptr)
            assert torch.equal(got.col, ref.col)
            assert got.val.dtype == ref.val.dtype
            assert got.val.cpu().numpy().tobytes() == ref.val.cpu().numpy().tobytes()
    finally:
        plan.close()


def test_merge_noalloc_empty_rows_and_one_layer():
    """Rows with no entry in any layer, and a single layer (a copy)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m, n = 300, 50
    rp = np.zeros(m + 1, np.int64)
    rp[101:] = 3  # row 100 holds three entries, every other row none
    L = spg.DeviceCSR.from_arrays(m, n, rp, np.array([1, 7, 40], np.int32), np.array([0.5, -2.0, 3.25]))
    for layers in ([L], [L, L, L]):
        got = spg.spgemm_merge_layers_noalloc("f64", layers)
        torch.cuda.synchronize()
        assert got.nnz == 3
        assert torch.equal(got.row_ptr.cpu(), torch.from_numpy(rp))
        assert got.col.cpu().tolist() == [1, 7, 40]
        assert got.val.cpu().tolist() == [0.5 * len(layers), -2.0 * len(layers), 3.25 * len(layers)]


def test_merge_noalloc_rejects_too_many_rows():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m = (1 << 20) + 1
    L = spg.DeviceCSR.from_arrays(m, 4, np.zeros(m + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    with pytest.raises(spg.SpgError) as e:
        spg.spgemm_merge_layers_noalloc("f64", [L, L])
    assert e.value.name == "SPG_ERR_CAPACITY"
