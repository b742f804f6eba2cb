"""GPU parity of the hypersparse row-compressed format and of one process's
Sparse SUMMA stages with blocking b (Section 4.1 stage loop of Algorithm 2,
Section 4.2 DCSC by rows, Section 4.3 merge), against oracle/summa.py.

* compress / expand equal the oracle's DCSR and CSR arrays exactly;
* the stage result: row indices, row pointers and columns equal the
  oracle's; INT64 and boolean values exact; FP64 values within 1e-12 of the
  oracle's stage-order sum or, beyond, within the reordering bound of the
  compensated sum of the unsplit product's terms; the count of block-product
  entries equals the oracle's;
* shapes: several stage counts and blockings including b = 1 and a single
  block, rows whose products all vanish (dropped from the result), empty A,
  no inner indices, and a process share of an R-MAT scale-20 grid.
"""

import numpy as np
import pytest
import torch

import oracle
import paper_1510_00844_amd as spg
import synth
from gpu_util import to_dev
from oracle import summa
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


def _dcsr_dev(D: summa.DCSR, sr) -> spg.DeviceDCSR:
    val = None if D.val is None else np.asarray(D.val, dtype={"f64": np.float64, "i64": np.int64,
                                                              "bool": np.uint8}[sr])
    return spg.DeviceDCSR.from_arrays(D.nrows, D.ncols, D.row_ids, D.row_ptr, D.col, val)


def _host(C: spg.DeviceDCSR) -> summa.DCSR:
    return summa.DCSR(C.nrows, C.ncols, C.row_ids.cpu().numpy().astype(np.int64), C.row_ptr.cpu().numpy(),
                      C.col.cpu().numpy(), None if C.val is None else C.val.cpu().numpy())


def _values(sr, M: CSR) -> CSR:
    if sr == "f64":
        return M
    return synth.with_values(M, "ones_i64" if sr == "i64" else "true_bool")


def _sparse_rows(M: CSR, keep_frac, seed) -> CSR:
    rng = np.random.default_rng(seed)
    drop = rng.random(M.nrows) >= keep_frac
    rows = np.repeat(np.arange(M.nrows), np.diff(M.row_ptr))
    k = ~drop[rows]
    return synth.canonical_from_coo(M.nrows, M.ncols, rows[k], M.col[k].astype(np.int64),
                                    None if M.val is None else M.val[k], dup="first")


def check_summa(plan, sr, A: CSR, B: CSR, stages, b):
    Ad = summa.compress(A)
    print("case summa sr=%s m=%d K=%d n=%d nnzA=%d stages=%d b=%d" % (sr, A.nrows, A.ncols, B.ncols, A.nnz, stages, b),
          flush=True)
    C, snnz = spg.spgemm_summa_local(plan, sr, _dcsr_dev(Ad, sr), to_dev(B, sr), stages, b)
    ref, ref_snnz = summa.summa_local(Ad, B, stages, b, sr)
    got = _host(C)
    assert snnz == ref_snnz
    assert got.nrows == ref.nrows and got.ncols == ref.ncols
    assert np.array_equal(got.row_ids, ref.row_ids)
    g, r = summa.expand(got), summa.expand(ref)
    assert_same_structure(g, r)
    if sr == "f64":
        U = oracle.spgemm(A, B, "f64")
        assert_same_structure(g, U)
        assert_values(g, r, sr, lambda: oracle.f64_check(A, B, U))
    else:
        assert_values(g, r, sr)
    return got, snnz


@pytest.mark.parametrize("m,n,density,keep", [(0, 7, 0.1, 1.0), (5, 9, 0.0, 1.0), (1000, 300, 0.01, 0.3),
                                              (70000, 50, 0.02, 0.05)])
def test_dcsr_compress_expand(plan, m, n, density, keep):
    M = synth.random_csr(m, n, density, 5, kind="f64")
    if m:
        M = _sparse_rows(M, keep, 6)
    dM = to_dev(M, "f64")
    D = spg.dcsr_compress(plan, dM)
    ref = summa.compress(M)
    assert D.nzr == ref.nzr
    assert np.array_equal(D.row_ids.cpu().numpy().astype(np.int64), ref.row_ids)
    assert np.array_equal(D.row_ptr.cpu().numpy(), ref.row_ptr)
    E = spg.dcsr_expand(plan, D)
    assert np.array_equal(E.row_ptr.cpu().numpy(), M.row_ptr)


@pytest.mark.parametrize("sr", ["f64", "i64", "bool"])
@pytest.mark.parametrize("stages,b", [(1, 2048), (4, 512), (4, 64), (16, 8), (2, 1)])
def test_summa_stages(plan, sr, stages, b):
    """An R-MAT process share: 2048 inner indices, rows that keep about a
    third of their entries (hypersparse rows), every blocking from one block
    down to b = 1."""
    M = synth.rmat(13, 16, synth.G500, seed=51)
    A, B = synth.process_share(M, 4, 4, 1, 2, 3)
    A = _sparse_rows(A, 0.35, 52)
    check_summa(plan, sr, _values(sr, A), _values(sr, B), stages, b)


def test_summa_bool_without_values(plan):
    """Boolean operands without value arrays (every stored entry true)."""
    M = synth.rmat(12, 16, synth.G500, seed=95)
    A, B = synth.process_share(M, 4, 2, 0, 3, 1)
    A = synth.CSR(A.nrows, A.ncols, A.row_ptr, A.col, None)
    B = synth.CSR(B.nrows, B.ncols, B.row_ptr, B.col, None)
    Ad = summa.compress(A)
    C, snnz = spg.spgemm_summa_local(plan, "bool", spg.DeviceDCSR.from_arrays(Ad.nrows, Ad.ncols, Ad.row_ids,
                                                                            Ad.row_ptr, Ad.col, None),
                                     spg.DeviceCSR.from_arrays(B.nrows, B.ncols, B.row_ptr, B.col, None), 4, 64)
    ref, ref_snnz = summa.summa_local(Ad, B, 4, 64, "bool")
    got = _host(C)
    assert snnz == ref_snnz
    assert np.array_equal(got.row_ids, ref.row_ids)
    assert_same_structure(summa.expand(got), summa.expand(ref))
    assert np.all(got.val == 1) and np.array_equal(got.val, ref.val)


def test_summa_rows_without_products(plan):
    """Rows of A whose B rows are all empty give no result row: the DCSR
    result drops them."""
    A = synth.random_csr(3000, 640, 0.01, 61, kind="f64")
    B = synth.random_csr(640, 900, 0.02, 62, kind="f64")
    rows = np.repeat(np.arange(B.nrows), np.diff(B.row_ptr))
    k = rows % 3 != 0  # every third B row empty
    B = synth.canonical_from_coo(B.nrows, B.ncols, rows[k], B.col[k].astype(np.int64), B.val[k], dup="first")
    got, _ = check_summa(plan, "f64", A, B, 5, 32)
    assert got.nzr < summa.compress(A).nzr


@pytest.mark.parametrize("stages,b", [(1, 16), (4, 2)])
def test_summa_edge_cases(plan, stages, b):
    # A without entries
    A = CSR(100, 16, np.zeros(101, np.int64), np.zeros(0, np.int32), np.zeros(0))
    B = synth.random_csr(16, 40, 0.3, 71, kind="f64")
    check_summa(plan, "f64", A, B, stages, b)
    # one row, one entry per block
    A = synth.canonical_from_coo(9, 16, np.full(8, 4), np.arange(0, 16, 2), np.linspace(1, 2, 8), dup="first")
    check_summa(plan, "f64", A, B, stages, b)


def test_summa_fill_after_other_calls(plan):
    """Calls on the plan between the count and the fill call (a compression,
    an ordinary product) leave the stage state alone."""
    M = synth.rmat(11, 16, synth.G500, seed=91)
    A, B = synth.process_share(M, 2, 2, 1, 0, 1)
    Ad = summa.compress(A)
    import ctypes
    dA, dB = _dcsr_dev(Ad, "f64"), to_dev(B, "f64")
    a, bb = dA._c("f64"), dB._c("f64")
    L = spg.lib()
    nzr, nnz, snnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert L.spgemm_summa_local(plan.handle, 0, ctypes.byref(a), ctypes.byref(bb), 2, 64, None, None, None, None,
                                ctypes.byref(nzr), ctypes.byref(nnz), ctypes.byref(snnz)) == 0
    # other work on the same plan
    spg.dcsr_compress(plan, to_dev(synth.random_csr(5000, 300, 0.01, 92, kind="f64"), "f64"))
    X = to_dev(synth.random_csr(300, 300, 0.05, 93, kind="f64"), "f64")
    spg.spgemm(plan, "f64", X, X)
    ids = torch.empty(nzr.value, dtype=torch.int32, device=plan.device)
    rp = torch.empty(nzr.value + 1, dtype=torch.int64, device=plan.device)
    col = torch.empty(nnz.value, dtype=torch.int32, device=plan.device)
    val = torch.empty(nnz.value, dtype=torch.float64, device=plan.device)
    assert L.spgemm_summa_local(plan.handle, 0, ctypes.byref(a), ctypes.byref(bb), 2, 64,
                                ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(rp.data_ptr()),
                                ctypes.c_void_p(col.data_ptr()), ctypes.c_void_p(val.data_ptr()), None, None,
                                None) == 0
    ref, _ = summa.summa_local(Ad, B, 2, 64, "f64")
    got = summa.DCSR(A.nrows, B.ncols, ids.cpu().numpy().astype(np.int64), rp.cpu().numpy(), col.cpu().numpy(),
                     val.cpu().numpy())
    assert np.array_equal(got.row_ids, ref.row_ids)
    g, r = summa.expand(got), summa.expand(ref)
    assert_same_structure(g, r)
    U = oracle.spgemm(A, B, "f64")
    assert_values(g, r, "f64", lambda: oracle.f64_check(A, B, U))


def test_summa_no_inner_indices(plan):
    A = summa.DCSR(50, 0, np.zeros(0, np.int64), np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    B = CSR(0, 30, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    C, snnz = spg.spgemm_summa_local(plan, "f64", _dcsr_dev(A, "f64"), to_dev(B, "f64"), 3, 5)
    assert C.nzr == 0 and C.nnz == 0 and snnz == 0
    assert C.row_ptr.cpu().tolist() == [0]


def test_summa_argument_errors(plan):
    M = synth.random_csr(40, 24, 0.2, 81, kind="f64")
    D = _dcsr_dev(summa.compress(M), "f64")
    B = to_dev(synth.random_csr(24, 10, 0.2, 82, kind="f64"), "f64")
    for stages, b in ((5, 1), (3, 3), (0, 1), (2, 0)):
        with pytest.raises(spg.SpgError) as e:
            spg.spgemm_summa_local(plan, "f64", D, B, stages, b)
        assert e.value.name == "SPG_ERR_ARG"
    # a fill call that does not follow its count call
    L = spg.lib()
    import ctypes
    a, bb = D._c("f64"), B._c("f64")
    rp = torch.zeros(2, dtype=torch.int64, device=plan.device)
    nzr, nnz = ctypes.c_int64(), ctypes.c_int64()
    assert L.spgemm_summa_local(plan.handle, 0, ctypes.byref(a), ctypes.byref(bb), 2, 4, None, None, None, None,
                                ctypes.byref(nzr), ctypes.byref(nnz), None) == 0
    st = L.spgemm_summa_local(plan.handle, 0, ctypes.byref(a), ctypes.byref(bb), 2, 6, None,
                              ctypes.c_void_p(rp.data_ptr()), None, None, None, None, None)
    assert st == 8  # SPG_ERR_STATE
    # the validate option rejects row indices out of order
    p = spg.Plan(validate=True)
    try:
        bad = spg.DeviceDCSR(D.nrows, D.ncols, D.row_ids.flip(0).contiguous(), D.row_ptr, D.col, D.val)
        with pytest.raises(spg.SpgError) as e:
            spg.spgemm_summa_local(p, "f64", bad, B, 2, 4)
        assert e.value.name == "SPG_ERR_NOT_CANONICAL"
    finally:
        p.close()


@pytest.fixture(scope="module")
def share20():
    """The process P(0, 1, 1) of a 16 x 16 x 4 grid squaring R-MAT G500
    scale 20: 65,536 rows, 262,144 inner indices in 16 stages."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    M = synth.rmat(20, 16, synth.G500, seed=3)
    return synth.process_share(M, 16, 4, 0, 1, 1)


@pytest.mark.parametrize("b", [16384, 1024])
def test_summa_rmat_s20_share(plan, share20, b):
    A, B = share20
    got, snnz = check_summa(plan, "f64", A, B, 16, b)
    assert got.nzr > 0 and snnz >= got.nnz


@pytest.mark.parametrize("sr", ["f64", "i64"])
@pytest.mark.parametrize("c", [4, 16])
def test_summa_layers_in_one_call(plan, sr, c):
    """The layered product of the C3 shape (ER A and B, the inner dimension
    in c contiguous layers) as one stage call with one block per layer:
    equal to the oracle's sum of the c layer products in layer order."""
    A = synth.rmat(15, 16, synth.ER, seed=91)
    B = synth.rmat(15, 16, synth.ER, seed=92)
    check_summa(plan, sr, _values(sr, A), _values(sr, B), c, A.ncols // c)
