"""Python binding of the MI355X SpGEMM library (libspgemm.so).

Argument marshalling only: every step of the product and the merge runs in
the HIP kernels behind the C ABI of include/spgemm.h.  torch tensors own the
device buffers and supply the stream; no torch operation takes part in the
computation.  If the library is not built this module raises on first use;
there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspgemm.so")

SEMIRINGS = {"f64": 0, "i64": 1, "bool": 2}
TORCH_DTYPE = {"f64": torch.float64, "i64": torch.int64, "bool": torch.uint8}

NBINS = 17
BIN_NAMES = (["empty", "tiny", "small"] + ["hash%d" % (128 << b) for b in range(8)] + ["dense_par", "dense"]
             + ["rank%d" % (4096 << b) for b in range(3)] + ["heap"])
BIN_HEAP = 16


class SpgError(RuntimeError):
    def __init__(self, status: int, name: str, msg: str):
        super().__init__("%s: %s" % (name, msg))
        self.status = status
        self.name = name


class _Csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Dcsr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nzr", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("row_ids", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("validate", ctypes.c_int32), ("small_max_flops", ctypes.c_int32),
                ("hash_max_flops", ctypes.c_int32), ("hash_max_nnz", ctypes.c_int32),
                ("dense_chunk_cols", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("gather_map", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("sym_gather_map", ctypes.c_int32), ("sym_unroll", ctypes.c_int32),
                ("chunk_min_nnz", ctypes.c_int32), ("chunk_group", ctypes.c_int32),
                ("rank_max_nnz", ctypes.c_int32), ("rank_block", ctypes.c_int32),
                ("serial_heavy", ctypes.c_int32), ("chunk_unroll", ctypes.c_int32),
                ("gather_pipeline", ctypes.c_int32), ("fused_max_nnz", ctypes.c_int32),
                ("heap_max_lists", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("flops", ctypes.c_int64), ("nnz_c", ctypes.c_int64),
                ("sym_rows", ctypes.c_int64 * NBINS), ("sym_flops", ctypes.c_int64 * NBINS),
                ("sym_annz", ctypes.c_int64 * NBINS),
                ("num_rows", ctypes.c_int64 * NBINS), ("num_flops", ctypes.c_int64 * NBINS),
                ("num_annz", ctypes.c_int64 * NBINS), ("num_cnnz", ctypes.c_int64 * NBINS),
                ("dense_chunk_cols", ctypes.c_int32), ("dense_chunks", ctypes.c_int32)]


MLP_NPARAMS = 1217


class LearnedStats(ctypes.Structure):
    _fields_ = [("rows_predicted", ctypes.c_int64), ("rows_exact", ctypes.c_int64),
                ("rows_overflow", ctypes.c_int64), ("slots", ctypes.c_int64), ("nnz_c", ctypes.c_int64),
                ("nnz_single", ctypes.c_int64), ("bin_rows", ctypes.c_int64 * NBINS)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


_lib = None


def lib():
    """Load libspgemm.so (built in-tree by build.py); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libspgemm.so is not built (run __graft_entry__.build() or "
                               "python paper_1510_00844_amd/build.py); no fallback exists")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        CP = ctypes.POINTER(_Csr)
        sig = {
            "spg_default_opts": ([ctypes.POINTER(Opts)], None),
            "spg_plan_create": ([ctypes.POINTER(P), P, ctypes.POINTER(Opts)], ctypes.c_int),
            "spg_plan_destroy": ([P], ctypes.c_int),
            "spg_plan_set_stream": ([P, P], ctypes.c_int),
            "spgemm_symbolic": ([P, ctypes.c_int, CP, CP, I64, I64, P, ctypes.POINTER(I64)], ctypes.c_int),
            "spgemm_numeric": ([P, ctypes.c_int, CP, CP, I64, I64, P, P, P], ctypes.c_int),
            "spgemm_merge_layers": ([P, ctypes.c_int, I32, CP, P, P, P, ctypes.POINTER(I64)], ctypes.c_int),
            "spgemm_merge_layers_noalloc": ([P, ctypes.c_int, I32, CP, P, P, P, ctypes.POINTER(I64)], ctypes.c_int),
            "spg_dcsr_compress": ([P, CP, P, P, ctypes.POINTER(I64)], ctypes.c_int),
            "spg_dcsr_expand": ([P, ctypes.POINTER(_Dcsr), P], ctypes.c_int),
            "spgemm_summa_local": ([P, ctypes.c_int, ctypes.POINTER(_Dcsr), CP, I64, I64, P, P, P, P,
                                    ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)], ctypes.c_int),
            "spg_plan_stats": ([P, ctypes.POINTER(Stats)], ctypes.c_int),
            "spg_profile_read": ([P, ctypes.POINTER(KernelTime), I32, ctypes.POINTER(I32)], ctypes.c_int),
            "spg_profile_reset": ([P], ctypes.c_int),
            "spg_profile_select": ([P, ctypes.c_char_p], ctypes.c_int),
            "spg_mlp_forward": ([P, P, P, I64, P], ctypes.c_int),
            "spg_mlp_grad": ([P, P, P, P, I64, ctypes.c_float, P, P], ctypes.c_int),
            "spg_mlp_adam": ([P, P, P, P, P, I64, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float],
                             ctypes.c_int),
            "spg_row_training_data": ([P, P, I64, P, P, ctypes.POINTER(I64)], ctypes.c_int),
            "spgemm_learned_run": ([P, ctypes.c_int, CP, CP, I64, I64, P, ctypes.c_float, ctypes.POINTER(I64),
                                    ctypes.POINTER(LearnedStats)], ctypes.c_int),
            "spgemm_learned_fetch": ([P, CP, CP, P, P, P], ctypes.c_int),
            "spgemm_galerkin_batched": ([P, ctypes.c_int, I32, CP, CP, CP, CP, I32], ctypes.c_int),
            "spgemm_galerkin_copy": ([P, P, P, P], ctypes.c_int),
            "spg_autotune_galerkin": ([P, ctypes.c_int, I32, CP, CP, CP, ctypes.c_char_p, I32, ctypes.POINTER(Opts),
                                       ctypes.POINTER(I32)], ctypes.c_int),
            "spg_mis2_aggregate": ([P, CP, ctypes.c_uint64, P, P, ctypes.POINTER(I64), ctypes.POINTER(I32)],
                                   ctypes.c_int),
            "spg_restriction": ([P, ctypes.c_int, I64, I64, P, P, P, P, P, P, P], ctypes.c_int),
            "spg_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "spg_last_error": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        L = lib()
        raise SpgError(status, L.spg_status_string(status).decode(), L.spg_last_error().decode())


@dataclass
class DeviceCSR:
    """CSR matrix in device memory: int64 row_ptr, int32 col, typed val."""

    nrows: int
    ncols: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: Optional[torch.Tensor]

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @staticmethod
    def from_arrays(nrows, ncols, row_ptr, col, val, device="cuda") -> "DeviceCSR":
        rp = torch.as_tensor(row_ptr, dtype=torch.int64).to(device).contiguous()
        c = torch.as_tensor(col, dtype=torch.int32).to(device).contiguous()
        v = None if val is None else torch.as_tensor(val).to(device).contiguous()
        return DeviceCSR(int(nrows), int(ncols), rp, c, v)

    def to_numpy(self):
        return (self.row_ptr.cpu().numpy(), self.col.cpu().numpy(),
                None if self.val is None else self.val.cpu().numpy())

    def _c(self, sr: Optional[str] = None) -> _Csr:
        if self.val is not None and sr is not None:
            want = TORCH_DTYPE[sr]
            if self.val.dtype != want:
                raise TypeError("values are %s, semiring %s needs %s" % (self.val.dtype, sr, want))
        return _Csr(self.nrows, self.ncols, self.nnz, self.row_ptr.data_ptr(),
                    self.col.data_ptr() if self.nnz else None,
                    None if self.val is None or self.nnz == 0 else self.val.data_ptr())


@dataclass
class DeviceDCSR:
    """Row-compressed (hypersparse) device matrix: only the nzr rows holding
    entries, with their indices (row_ids int32, strictly increasing)."""
    nrows: int
    ncols: int
    row_ids: torch.Tensor
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: Optional[torch.Tensor]

    @property
    def nzr(self) -> int:
        return int(self.row_ids.numel())

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @staticmethod
    def from_arrays(nrows, ncols, row_ids, row_ptr, col, val, device="cuda") -> "DeviceDCSR":
        ids = torch.as_tensor(row_ids, dtype=torch.int32).to(device).contiguous()
        rp = torch.as_tensor(row_ptr, dtype=torch.int64).to(device).contiguous()
        c = torch.as_tensor(col, dtype=torch.int32).to(device).contiguous()
        v = None if val is None else torch.as_tensor(val).to(device).contiguous()
        return DeviceDCSR(int(nrows), int(ncols), ids, rp, c, v)

    def _c(self, sr: Optional[str] = None) -> _Dcsr:
        if self.val is not None and sr is not None:
            want = TORCH_DTYPE[sr]
            if self.val.dtype != want:
                raise TypeError("values are %s, semiring %s needs %s" % (self.val.dtype, sr, want))
        return _Dcsr(self.nrows, self.ncols, self.nzr, self.nnz, self.row_ids.data_ptr() if self.nzr else None,
                     self.row_ptr.data_ptr(), self.col.data_ptr() if self.nnz else None,
                     None if self.val is None or self.nnz == 0 else self.val.data_ptr())


class Plan:
    """Owns an spg_plan bound to a device and a stream (default: torch's
    current stream on that device)."""

    def __init__(self, device=None, stream: Optional[torch.cuda.Stream] = None, validate=False,
                 profile=False, small_max_flops=0, hash_max_flops=0, hash_max_nnz=0,
                 dense_chunk_cols=0, streams=0, gather_map=0, unroll=0, sym_gather_map=0, sym_unroll=0,
                 chunk_min_nnz=0, chunk_group=0, rank_max_nnz=0, rank_block=0, serial_heavy=-1,
                 chunk_unroll=0, gather_pipeline=0, fused_max_nnz=0, heap_max_lists=0):
        L = lib()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            o = Opts()
            L.spg_default_opts(ctypes.byref(o))
            o.validate = int(validate)
            o.profile = int(profile)
            for name, v in (("small_max_flops", small_max_flops), ("hash_max_flops", hash_max_flops),
                            ("hash_max_nnz", hash_max_nnz), ("dense_chunk_cols", dense_chunk_cols),
                            ("streams", streams), ("gather_map", gather_map), ("unroll", unroll),
                            ("sym_gather_map", sym_gather_map), ("sym_unroll", sym_unroll),
                            ("chunk_min_nnz", chunk_min_nnz), ("chunk_group", chunk_group),
                            ("rank_max_nnz", rank_max_nnz), ("rank_block", rank_block),
                            ("chunk_unroll", chunk_unroll), ("gather_pipeline", gather_pipeline),
                            ("fused_max_nnz", fused_max_nnz), ("heap_max_lists", heap_max_lists)):
                if v:
                    setattr(o, name, int(v))
            if serial_heavy >= 0:
                o.serial_heavy = int(serial_heavy)
            h = ctypes.c_void_p()
            _check(L.spg_plan_create(ctypes.byref(h), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(o)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().spg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        s = Stats()
        _check(lib().spg_plan_stats(self.handle, ctypes.byref(s)))
        d = {k: getattr(s, k) for k in ("m", "n", "k", "flops", "nnz_c", "dense_chunk_cols", "dense_chunks")}
        for k in ("sym_rows", "sym_flops", "sym_annz", "num_rows", "num_flops", "num_annz", "num_cnnz"):
            d[k] = list(getattr(s, k))
        return d

    def profile_read(self) -> dict:
        arr = (KernelTime * 64)()
        n = ctypes.c_int32()
        _check(lib().spg_profile_read(self.handle, arr, 64, ctypes.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(n.value, 64))}

    def profile_reset(self):
        _check(lib().spg_profile_reset(self.handle))

    def profile_select(self, name: Optional[str] = None):
        """Time only launches of this name (None: all)."""
        _check(lib().spg_profile_select(self.handle, None if name is None else name.encode()))


def _window(A: DeviceCSR, k_lo, k_hi):
    return (0 if k_lo is None else int(k_lo)), (A.ncols if k_hi is None else int(k_hi))


def spgemm_symbolic(plan: Plan, sr: str, A: DeviceCSR, B: DeviceCSR, k_lo=None, k_hi=None,
                    c_row_ptr: Optional[torch.Tensor] = None, want_nnz: bool = True):
    """Row pointers of C = A(:,K) B(K,:) (device tensor, m+1) and nnz(C)."""
    k_lo, k_hi = _window(A, k_lo, k_hi)
    if c_row_ptr is None:
        c_row_ptr = torch.empty(A.nrows + 1, dtype=torch.int64, device=plan.device)
    nnz = ctypes.c_int64(-1)
    a, b = A._c(), B._c()
    _check(lib().spgemm_symbolic(plan.handle, SEMIRINGS[sr], ctypes.byref(a), ctypes.byref(b), k_lo, k_hi,
                                 ctypes.c_void_p(c_row_ptr.data_ptr()),
                                 ctypes.byref(nnz) if want_nnz else None))
    return c_row_ptr, (nnz.value if want_nnz else None)


def spgemm_numeric(plan: Plan, sr: str, A: DeviceCSR, B: DeviceCSR, c_row_ptr: torch.Tensor, nnz: int,
                   k_lo=None, k_hi=None, values: bool = True, c_col=None, c_val=None):
    """Column indices and values of C for the row pointers of the matching
    symbolic call."""
    k_lo, k_hi = _window(A, k_lo, k_hi)
    if c_col is None:
        c_col = torch.empty(max(nnz, 0), dtype=torch.int32, device=plan.device)
    if values and c_val is None:
        c_val = torch.empty(max(nnz, 0), dtype=TORCH_DTYPE[sr], device=plan.device)
    a, b = A._c(sr), B._c(sr)
    _check(lib().spgemm_numeric(plan.handle, SEMIRINGS[sr], ctypes.byref(a), ctypes.byref(b), k_lo, k_hi,
                                ctypes.c_void_p(c_row_ptr.data_ptr()),
                                ctypes.c_void_p(c_col.data_ptr()) if nnz > 0 else None,
                                ctypes.c_void_p(c_val.data_ptr()) if (values and nnz > 0) else None))
    return c_col, (c_val if values else None)


def spgemm(plan: Plan, sr: str, A: DeviceCSR, B: DeviceCSR, k_lo=None, k_hi=None, values=True) -> DeviceCSR:
    """Two-phase product C = A(:,K) B(K,:) as a DeviceCSR."""
    rp, nnz = spgemm_symbolic(plan, sr, A, B, k_lo, k_hi)
    col, val = spgemm_numeric(plan, sr, A, B, rp, nnz, k_lo, k_hi, values=values)
    return DeviceCSR(A.nrows, B.ncols, rp, col, val)


def spgemm_merge_layers(plan: Plan, sr: str, layers: Sequence[DeviceCSR], values=True) -> DeviceCSR:
    """LocalMerge: entry-wise semiring sum of the layers (count + fill pass)."""
    c = len(layers)
    arr = (_Csr * c)(*[L._c(sr if values else None) for L in layers])
    m, n = layers[0].nrows, layers[0].ncols
    rp = torch.empty(m + 1, dtype=torch.int64, device=plan.device)
    nnz = ctypes.c_int64(-1)
    _check(lib().spgemm_merge_layers(plan.handle, SEMIRINGS[sr], c, arr, ctypes.c_void_p(rp.data_ptr()),
                                     None, None, ctypes.byref(nnz)))
    col = torch.empty(max(nnz.value, 0), dtype=torch.int32, device=plan.device)
    val = torch.empty(max(nnz.value, 0), dtype=TORCH_DTYPE[sr], device=plan.device) if values else None
    if nnz.value > 0:
        _check(lib().spgemm_merge_layers(plan.handle, SEMIRINGS[sr], c, arr, ctypes.c_void_p(rp.data_ptr()),
                                         ctypes.c_void_p(col.data_ptr()),
                                         ctypes.c_void_p(val.data_ptr()) if values else None, None))
    return DeviceCSR(m, n, rp, col, val)


def spgemm_merge_layers_noalloc(sr: str, layers: Sequence[DeviceCSR], stream: Optional[torch.cuda.Stream] = None,
                                values=True) -> DeviceCSR:
    """The merge through the entry point that allocates nothing (its scratch
    is a fixed device array, at most 2^20 rows); the output tensors are
    allocated here, by the caller side."""
    c = len(layers)
    arr = (_Csr * c)(*[L._c(sr if values else None) for L in layers])
    m, n = layers[0].nrows, layers[0].ncols
    dev = layers[0].row_ptr.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    rp = torch.empty(m + 1, dtype=torch.int64, device=dev)
    nnz = ctypes.c_int64(-1)
    _check(lib().spgemm_merge_layers_noalloc(ctypes.c_void_p(st.cuda_stream), SEMIRINGS[sr], c, arr,
                                             ctypes.c_void_p(rp.data_ptr()), None, None, ctypes.byref(nnz)))
    col = torch.empty(max(nnz.value, 0), dtype=torch.int32, device=dev)
    val = torch.empty(max(nnz.value, 0), dtype=TORCH_DTYPE[sr], device=dev) if values else None
    if nnz.value > 0:
        _check(lib().spgemm_merge_layers_noalloc(ctypes.c_void_p(st.cuda_stream), SEMIRINGS[sr], c, arr,
                                                 ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                                                 ctypes.c_void_p(val.data_ptr()) if values else None, None))
    return DeviceCSR(m, n, rp, col, val)


def dcsr_compress(plan: Plan, A: DeviceCSR) -> DeviceDCSR:
    """CSR -> DCSR; the result shares A's column and value tensors."""
    a = A._c()
    nzr = ctypes.c_int64(-1)
    _check(lib().spg_dcsr_compress(plan.handle, ctypes.byref(a), None, None, ctypes.byref(nzr)))
    ids = torch.empty(nzr.value, dtype=torch.int32, device=plan.device)
    rp = torch.empty(nzr.value + 1, dtype=torch.int64, device=plan.device)
    _check(lib().spg_dcsr_compress(plan.handle, ctypes.byref(a), ctypes.c_void_p(ids.data_ptr() or None),
                                   ctypes.c_void_p(rp.data_ptr()), None))
    return DeviceDCSR(A.nrows, A.ncols, ids, rp, A.col, A.val)


def dcsr_expand(plan: Plan, D: DeviceDCSR) -> DeviceCSR:
    """DCSR -> CSR; the result shares D's column and value tensors."""
    d = D._c()
    rp = torch.empty(D.nrows + 1, dtype=torch.int64, device=plan.device)
    _check(lib().spg_dcsr_expand(plan.handle, ctypes.byref(d), ctypes.c_void_p(rp.data_ptr())))
    return DeviceCSR(D.nrows, D.ncols, rp, D.col, D.val)


def spgemm_summa_local(plan: Plan, sr: str, A: DeviceDCSR, B: DeviceCSR, stages: int, b: int, values=True):
    """One process's Sparse SUMMA stages with blocking b (count + fill
    call).  Returns (C as DeviceDCSR, entries of all kept block products)."""
    a, bb = A._c(sr if values else None), B._c(sr if values else None)
    nzr, nnz, snnz = ctypes.c_int64(-1), ctypes.c_int64(-1), ctypes.c_int64(-1)
    L = lib()
    _check(L.spgemm_summa_local(plan.handle, SEMIRINGS[sr], ctypes.byref(a), ctypes.byref(bb), int(stages), int(b),
                                None, None, None, None, ctypes.byref(nzr), ctypes.byref(nnz), ctypes.byref(snnz)))
    ids = torch.empty(nzr.value, dtype=torch.int32, device=plan.device)
    rp = torch.empty(nzr.value + 1, dtype=torch.int64, device=plan.device)
    col = torch.empty(nnz.value, dtype=torch.int32, device=plan.device)
    val = torch.empty(nnz.value, dtype=TORCH_DTYPE[sr], device=plan.device) if values else None
    _check(L.spgemm_summa_local(plan.handle, SEMIRINGS[sr], ctypes.byref(a), ctypes.byref(bb), int(stages), int(b),
                                ctypes.c_void_p(ids.data_ptr() or None), ctypes.c_void_p(rp.data_ptr()),
                                ctypes.c_void_p(col.data_ptr() or None),
                                ctypes.c_void_p(val.data_ptr() or None) if values else None, None, None, None))
    return DeviceDCSR(A.nrows, B.ncols, ids, rp, col, val), snnz.value


def _vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def spg_mlp_forward(plan: Plan, params: torch.Tensor, x: torch.Tensor, y: torch.Tensor):
    _check(lib().spg_mlp_forward(plan.handle, _vp(params), _vp(x), x.shape[0], _vp(y)))


def spg_mlp_grad(plan: Plan, params, x, t, alpha: float, grad, loss=None):
    _check(lib().spg_mlp_grad(plan.handle, _vp(params), _vp(x), _vp(t), t.shape[0], float(alpha), _vp(grad),
                              _vp(loss)))


def spg_mlp_adam(plan: Plan, params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().spg_mlp_adam(plan.handle, _vp(params), _vp(grad), _vp(m), _vp(v), int(step), float(lr),
                              float(beta1), float(beta2), float(eps)))


def spg_row_training_data(plan: Plan, c_row_ptr: torch.Tensor, m: int, min_flops: int = 0):
    """Features (n, 3) and targets (n,) of the predicted rows (with at least
    min_flops products) of the last symbolic call."""
    x = torch.empty(max(m, 1) * 3, dtype=torch.float32, device=plan.device)
    t = torch.empty(max(m, 1), dtype=torch.float32, device=plan.device)
    n = ctypes.c_int64()
    _check(lib().spg_row_training_data(plan.handle, _vp(c_row_ptr), int(min_flops), _vp(x), _vp(t),
                                       ctypes.byref(n)))
    return x[: 3 * n.value].view(n.value, 3), t[: n.value]


def spgemm_learned_run(plan: Plan, sr: str, A: DeviceCSR, B: DeviceCSR, params: Optional[torch.Tensor],
                       margin: float = 0.15, k_lo=None, k_hi=None):
    """Single-pass product with predicted row sizes; returns (nnz, stats)."""
    k_lo, k_hi = _window(A, k_lo, k_hi)
    a, b = A._c(sr), B._c(sr)
    nnz = ctypes.c_int64()
    st = LearnedStats()
    _check(lib().spgemm_learned_run(plan.handle, SEMIRINGS[sr], ctypes.byref(a), ctypes.byref(b), k_lo, k_hi,
                                    _vp(params), float(margin), ctypes.byref(nnz), ctypes.byref(st)))
    stats = {k: getattr(st, k) for k in ("rows_predicted", "rows_exact", "rows_overflow", "slots", "nnz_c",
                                         "nnz_single")}
    stats["bin_rows"] = list(st.bin_rows)
    return nnz.value, stats


def spgemm_learned_fetch(plan: Plan, sr: str, A: DeviceCSR, B: DeviceCSR, nnz: int, values=True) -> DeviceCSR:
    a, b = A._c(sr), B._c(sr)
    rp = torch.empty(A.nrows + 1, dtype=torch.int64, device=plan.device)
    col = torch.empty(max(nnz, 0), dtype=torch.int32, device=plan.device)
    val = torch.empty(max(nnz, 0), dtype=TORCH_DTYPE[sr], device=plan.device) if values else None
    _check(lib().spgemm_learned_fetch(plan.handle, ctypes.byref(a), ctypes.byref(b), _vp(rp),
                                      _vp(col) if nnz > 0 else None, _vp(val) if (values and nnz > 0) else None))
    return DeviceCSR(A.nrows, B.ncols, rp, col, val)


def spgemm_learned(plan: Plan, sr: str, A: DeviceCSR, B: DeviceCSR, params, margin=0.15, k_lo=None, k_hi=None):
    nnz, st = spgemm_learned_run(plan, sr, A, B, params, margin, k_lo, k_hi)
    return spgemm_learned_fetch(plan, sr, A, B, nnz), st


class GalerkinBatch:
    """Result descriptors of one spgemm_galerkin_batched call (device memory
    owned by the plan)."""

    def __init__(self, out, sr):
        self.out = out
        self.sr = sr

    @property
    def nnz(self):
        return [int(o.nnz) for o in self.out]

    def fetch(self, plan: "Plan", values=True) -> list:
        """Copy the instances into torch tensors (one DeviceCSR each)."""
        nb = len(self.out)
        rows = [int(o.nrows) for o in self.out]
        nnz = self.nnz
        tot = sum(nnz)
        rp = torch.empty(sum(rows) + nb, dtype=torch.int64, device=plan.device)
        col = torch.empty(max(tot, 1), dtype=torch.int32, device=plan.device)
        val = torch.empty(max(tot, 1), dtype=TORCH_DTYPE[self.sr], device=plan.device) if values else None
        _check(lib().spgemm_galerkin_copy(plan.handle, _vp(rp), _vp(col), _vp(val)))
        res, r0, z0 = [], 0, 0
        for b in range(nb):
            res.append(DeviceCSR(rows[b], int(self.out[b].ncols), rp[r0:r0 + rows[b] + 1], col[z0:z0 + nnz[b]],
                                 None if val is None else val[z0:z0 + nnz[b]]))
            r0 += rows[b] + 1
            z0 += nnz[b]
        return res


def spgemm_galerkin_batched(plan: Plan, sr: str, RT: Sequence[DeviceCSR], A: Sequence[DeviceCSR],
                            R: Sequence[DeviceCSR], use_graph=True) -> GalerkinBatch:
    """C_b = (RT_b A_b) R_b for all b in one block-diagonal product; with
    use_graph, repeated calls on the same matrices replay one HIP graph."""
    nb = len(A)
    if not (len(RT) == len(R) == nb):
        raise ValueError("RT, A and R need the same number of instances")
    keep = (RT, A, R)  # noqa: F841  (descriptors reference these tensors)
    rt = (_Csr * nb)(*[m._c(sr) for m in RT])
    a = (_Csr * nb)(*[m._c(sr) for m in A])
    r = (_Csr * nb)(*[m._c(sr) for m in R])
    out = (_Csr * nb)()
    _check(lib().spgemm_galerkin_batched(plan.handle, SEMIRINGS[sr], nb, rt, a, r, out, int(bool(use_graph))))
    return GalerkinBatch(out, sr)


TUNED_FIELDS = ("small_max_flops", "streams", "gather_map", "unroll", "sym_gather_map", "hash_max_nnz")


def spg_autotune_galerkin(plan: Plan, sr: str, RT: Sequence[DeviceCSR], A: Sequence[DeviceCSR],
                          R: Sequence[DeviceCSR], cache_path: Optional[str] = None, budget_ms: int = 5000):
    """Tune the plan's options for these batched Galerkin instances (or take
    them from the JSON-lines cache); returns (chosen options, from_cache)."""
    nb = len(A)
    rt = (_Csr * nb)(*[m._c(sr) for m in RT])
    a = (_Csr * nb)(*[m._c(sr) for m in A])
    r = (_Csr * nb)(*[m._c(sr) for m in R])
    best = Opts()
    hit = ctypes.c_int32()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().spg_autotune_galerkin(plan.handle, SEMIRINGS[sr], nb, rt, a, r, path, int(budget_ms),
                                       ctypes.byref(best), ctypes.byref(hit)))
    return {k: int(getattr(best, k)) for k in TUNED_FIELDS}, bool(hit.value)


def spg_mis2_aggregate(plan: Plan, A: DeviceCSR, seed: int):
    """Distance-2 maximal independent set and aggregates of A's graph;
    returns (in_mis uint8 tensor, agg int32 tensor, n_agg, rounds)."""
    n = A.nrows
    in_mis = torch.empty(max(n, 1), dtype=torch.uint8, device=plan.device)
    agg = torch.empty(max(n, 1), dtype=torch.int32, device=plan.device)
    na = ctypes.c_int64()
    rounds = ctypes.c_int32()
    a = A._c(None)
    _check(lib().spg_mis2_aggregate(plan.handle, ctypes.byref(a), ctypes.c_uint64(seed & ((1 << 64) - 1)),
                                    _vp(in_mis), _vp(agg), ctypes.byref(na), ctypes.byref(rounds)))
    return in_mis[:n], agg[:n], na.value, rounds.value


def spg_restriction(plan: Plan, sr: str, agg: torch.Tensor, n_agg: int):
    """(R, R^T) as DeviceCSR from the aggregate of every vertex."""
    n = agg.numel()
    dt = TORCH_DTYPE[sr]
    r_rp = torch.empty(n + 1, dtype=torch.int64, device=plan.device)
    r_col = torch.empty(max(n, 1), dtype=torch.int32, device=plan.device)
    r_val = torch.empty(max(n, 1), dtype=dt, device=plan.device)
    rt_rp = torch.empty(n_agg + 1, dtype=torch.int64, device=plan.device)
    rt_col = torch.empty(max(n, 1), dtype=torch.int32, device=plan.device)
    rt_val = torch.empty(max(n, 1), dtype=dt, device=plan.device)
    _check(lib().spg_restriction(plan.handle, SEMIRINGS[sr], n, n_agg, _vp(agg), _vp(r_rp), _vp(r_col), _vp(r_val),
                                 _vp(rt_rp), _vp(rt_col), _vp(rt_val)))
    R = DeviceCSR(n, n_agg, r_rp, r_col[:n], r_val[:n])
    RT = DeviceCSR(n_agg, n, rt_rp, rt_col[:n], rt_val[:n])
    return R, RT
