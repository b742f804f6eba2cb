"""GPU parity at the largest single-GPU workload: R-MAT G500 scale 19, edge
factor 16, FP64 (3.5 billion output entries).

* every row pointer equals the oracle's row counts;
* every row whose symbolic pass keeps an n-bit bitmap (they hold most of
  the output and include every rank-chunk row) is compared with the oracle element by element, in row blocks
  of bounded size, split over four tests so each stays short;
* every dense chunk width runs the heaviest rows against the oracle.
"""

import numpy as np
import pytest
import torch

import oracle
import paper_1510_00844_amd as spg
import synth
from gpu_util import check_blocks_vs_oracle, check_rows_vs_oracle, to_dev

pytestmark = pytest.mark.gpu

PARTS = 4


@pytest.fixture(scope="module")
def c5():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A = synth.rmat(19, 16, synth.G500, seed=6)
    print("case C5 nnz(A)=%d" % A.nnz, flush=True)
    plan = spg.Plan()
    dA = to_dev(A, "f64")
    C = spg.spgemm(plan, "f64", dA, dA)
    st = plan.stats()
    f = oracle.row_flops(A, A)
    # rows that take the bitmap in the symbolic pass (more than one A entry,
    # more than 64 products, and 32 flops >= n or more products than the
    # symbolic hash tables take, 4096); their numeric bins are rank and rank
    # chunks
    annz = np.diff(A.row_ptr)
    heavy = np.nonzero((annz > 1) & (f > 64) & ((32 * f >= A.ncols) | (f > 4096)))[0]
    yield A, C, st, f, heavy
    del C
    plan.close()
    torch.cuda.empty_cache()


def test_c5_row_pointers(c5):
    A, C, st, f, heavy = c5
    assert st["flops"] == int(f.sum())
    ref = oracle.row_counts(A, A)
    got = np.diff(C.row_ptr.cpu().numpy())
    assert np.array_equal(got, ref)
    # the rank and rank-chunk rows are among the bitmap rows (the others, of
    # at most chunk_min_nnz outputs, take the hash tables); all of them are
    # compared below
    nb = sum(st["num_rows"][b] for b in (11, 13, 14, 15))
    assert 0 < nb <= heavy.size, "bitmap rows %d, rank and rank-chunk rows %d" % (heavy.size, nb)


@pytest.mark.parametrize("part", range(PARTS))
def test_c5_heavy_rows(c5, part):
    A, C, st, f, heavy = c5
    rows = heavy[part::PARTS]
    print("case C5 heavy rows part %d: %d rows" % (part, rows.size), flush=True)
    nrows, ent, over = check_blocks_vs_oracle(C, A, A, "f64", rows)
    print("C5 part %d: %d rows, %d entries, %d over 1e-12 relative" % (part, nrows, ent, over), flush=True)


@pytest.mark.parametrize("cols", [2048, 4096, 8192, 16384])
def test_rmat_s19_c5_chunk_widths(cols):
    """C5 shape with every dense chunk width: with 4096 columns a row has
    128 chunks and the (row, chunk) work items exceed what one grid can hold,
    so the kernel must stride over them."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A = synth.rmat(19, 16, synth.G500, seed=6)
    p = spg.Plan(dense_chunk_cols=cols)
    C = spg.spgemm(p, "f64", to_dev(A, "f64"), to_dev(A, "f64"))
    st = p.stats()
    assert st["num_rows"][11] > 0  # rank chunks of saved bitmaps
    f = oracle.row_flops(A, A)
    rows = np.argsort(-f)[:60]
    check_rows_vs_oracle(C, A, A, "f64", rows)
    del C
    p.close()
    torch.cuda.empty_cache()
