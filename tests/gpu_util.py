"""Helpers for the GPU parity tests: move inputs to the device, fetch rows of
a device result, and compare them with the oracle row by row."""

from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_1510_00844_amd as spg
from synth import CSR
from util import assert_same_structure, assert_values

VAL_DTYPE = {"f64": np.float64, "i64": np.int64, "bool": np.uint8}


def to_dev(M: CSR, sr: str = "f64") -> spg.DeviceCSR:
    val = None if M.val is None else np.asarray(M.val, dtype=VAL_DTYPE[sr])
    return spg.DeviceCSR.from_arrays(M.nrows, M.ncols, M.row_ptr, M.col, val)


def to_host(C: spg.DeviceCSR) -> CSR:
    rp, col, val = C.to_numpy()
    return CSR(C.nrows, C.ncols, rp, col, val)


def rows_of(C: spg.DeviceCSR, rows: np.ndarray) -> CSR:
    """Rows of a device CSR, in the given order, as a host CSR."""
    rp = C.row_ptr.cpu().numpy()
    rows = np.asarray(rows, dtype=np.int64)
    starts, ends = rp[rows], rp[rows + 1]
    lens = ends - starts
    ptr = np.zeros(rows.size + 1, dtype=np.int64)
    np.cumsum(lens, out=ptr[1:])
    if ptr[-1]:
        idx = np.repeat(starts - ptr[:-1], lens) + np.arange(ptr[-1])
        it = torch.as_tensor(idx, device=C.col.device)
        col = C.col[it].cpu().numpy()
        val = None if C.val is None else C.val[it].cpu().numpy()
    else:
        col = np.zeros(0, np.int32)
        val = None if C.val is None else np.zeros(0, VAL_DTYPE_T[C.val.dtype])
    return CSR(rows.size, C.ncols, ptr, col, val)


VAL_DTYPE_T = {torch.float64: np.float64, torch.int64: np.int64, torch.uint8: np.uint8}


def check_rows_vs_oracle(C: spg.DeviceCSR, A: CSR, B: CSR, sr: str, rows, k_lo=None, k_hi=None):
    """Sampled rows of the device result equal the oracle's rows (structure
    and integer/boolean values exact, FP64 within the per-entry bound)."""
    rows = np.asarray(rows, dtype=np.int64)
    got = rows_of(C, rows)
    ref = oracle.spgemm(A, B, sr, k_lo, k_hi, rows=rows)
    assert_same_structure(got, ref)
    if sr == "f64":
        return assert_values(got, ref, sr, lambda: oracle.f64_check(A, B, ref, k_lo, k_hi, rows=rows))
    return assert_values(got, ref, sr)


def check_full_vs_oracle(C: spg.DeviceCSR, A: CSR, B: CSR, sr: str, k_lo=None, k_hi=None):
    got = to_host(C)
    ref = oracle.spgemm(A, B, sr, k_lo, k_hi)
    assert_same_structure(got, ref)
    if sr == "f64":
        return assert_values(got, ref, sr, lambda: oracle.f64_check(A, B, ref, k_lo, k_hi))
    return assert_values(got, ref, sr)


def sample_rows(A: CSR, B: CSR, count: int, seed: int, k_lo=None, k_hi=None):
    """The heaviest rows by flops, the lightest non-empty ones, and a uniform
    random set: covers every accumulator bin."""
    f = oracle.row_flops(A, B, k_lo, k_hi)
    order = np.argsort(-f, kind="stable")
    heavy = order[: count // 4]
    nz = order[f[order] > 0]
    light = nz[-(count // 8):] if nz.size else nz
    rng = np.random.default_rng(seed)
    rnd = rng.choice(A.nrows, size=min(A.nrows, count // 2), replace=False)
    return np.unique(np.concatenate([heavy, light, rnd]))


def check_blocks_vs_oracle(C: spg.DeviceCSR, A: CSR, B: CSR, sr: str, rows, block_entries=60_000_000,
                           k_lo=None, k_hi=None):
    """Every given row of the device result against the oracle, in row
    blocks of about block_entries outputs (bounded host memory).  Returns
    (rows compared, entries compared, FP64 entries that needed the re-check)."""
    rows = np.asarray(rows, dtype=np.int64)
    rp = C.row_ptr.cpu().numpy()
    lens = rp[rows + 1] - rp[rows]
    ent = over = 0
    s = 0
    while s < rows.size:
        e = s + 1
        tot = int(lens[s])
        while e < rows.size and tot + lens[e] <= block_entries:
            tot += int(lens[e])
            e += 1
        over += check_rows_vs_oracle(C, A, B, sr, rows[s:e], k_lo, k_hi) or 0
        ent += tot
        s = e
    return rows.size, ent, over
