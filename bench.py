"""Benchmark of the SpGEMM hot path on one MI355X.

Headline step: one two-phase product C = A*A (symbolic + numeric, FP64
plus-times) of an R-MAT G500 matrix of scale 16, edge factor 16
(duplicates summed, random symmetric permutation), inputs resident in HBM.
value = 2 * flops / step time (flops = scalar multiplications).

The JSON line also carries the roofline of the dominant kernel (algorithmic
bytes per launch over its average launch time, HIP events on the plan's
stream), the oracle timed on the host cores, and secondary modes.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpGEMM GFLOP/s (2·mults/s) + HBM GB/s, R-MAT A·A; learned/batched vs plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-launch events")
    ap.add_argument("--dense-cols", type=int, default=0, help="columns per dense accumulator chunk")
    ap.add_argument("--streams", type=int, default=0, help="streams for independent bins (1..4)")
    ap.add_argument("--gather-map", type=int, default=0, help="1 coalesced, 2 per-lane ranges")
    ap.add_argument("--unroll", type=int, default=0, help="gathers in flight per lane (4 or 8)")
    ap.add_argument("--sym-gather-map", type=int, default=0)
    ap.add_argument("--sym-unroll", type=int, default=0)
    ap.add_argument("--no-c5", action="store_true", help="skip the scale-19 learned-sizing comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB (3 times), the reference for "
                         "scaling the HBM byte counters")
    ap.add_argument("--no-isolated", action="store_true",
                    help="skip the second pass that times every kernel alone (roofline_isolated)")
    ap.add_argument("--tune-cache", default=None, help="JSON-lines cache of the batched autotuner")
    ap.add_argument("--tune-budget-ms", type=int, default=3000)
    ap.add_argument("--pmc-summary", nargs="+", default=None, metavar="CSV",
                    help="only print a markdown table of per-kernel averages of rocprofv3 --pmc csv files")
    ap.add_argument("--trace-summary", default=None, metavar="CSV",
                    help="only print a markdown table of a rocprofv3 kernel_stats.csv")
    ap.add_argument("--traffic-summary", nargs=5, default=None,
                    metavar=("WORKLOAD", "FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="only write profiles/pmc_traffic_<WORKLOAD>.json from FETCH_SIZE / WRITE_SIZE passes "
                         "and print its table")
    ap.add_argument("--traffic-commands", default="", help="the counter commands, recorded in the json")
    ap.add_argument("--mode", default="c2", choices=["c2", "c3", "c4", "c5", "summa"],
                    help="c2: the headline product (default); c3, c4, c5, summa: only that secondary "
                         "workload, with its per-kernel times (for profiling)")
    return ap.parse_args()


def _kernel_short(name: str) -> str:
    name = name.split("(")[0].strip()
    return name[5:] if name.startswith("void ") else name


def pmc_summary(paths, top=30):
    """Per-kernel averages over the dispatches of rocprofv3 --pmc csv files:
    duration, and each counter per dispatch; SQ_INSTS_* also per wave."""
    import csv
    from collections import defaultdict
    recs = defaultdict(lambda: {"disp": {}, "c": defaultdict(list)})
    counters = []
    for p in paths:
        with open(p) as f:
            for r in csv.DictReader(f):
                k = _kernel_short(r["Kernel_Name"])
                d = recs[k]
                did = (p, r["Dispatch_Id"])
                d["disp"][did] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                d["c"][r["Counter_Name"]].append(float(r["Counter_Value"]))
                if r["Counter_Name"] not in counters:
                    counters.append(r["Counter_Name"])
    rows = []
    for k, d in recs.items():
        n = len(d["disp"])
        dur = sum(d["disp"].values()) / n / 1e3
        avg = {c: sum(v) / len(v) for c, v in d["c"].items()}
        rows.append((dur * n, k, n, dur, avg))
    rows.sort(key=lambda x: -x[0])
    cols = list(counters)
    per_wave = [c for c in cols if c.startswith("SQ_INSTS_")] if "SQ_WAVES" in cols else []
    head = ["kernel", "dispatches", "avg us"] + cols + [c + "/wave" for c in per_wave]
    print("| " + " | ".join(head) + " |")
    print("|" + "---|" + "---:|" * (len(head) - 1))
    for _, k, n, dur, avg in rows[:top]:
        vals = ["`%s`" % k, str(n), "%.1f" % dur]
        for c in cols:
            v = avg.get(c)
            vals.append("" if v is None else ("%.3g" % v if abs(v) < 1000 else "%.0f" % v))
        for c in per_wave:
            w = avg.get("SQ_WAVES") or 0
            vals.append("%.1f" % (avg.get(c, 0.0) / w) if w else "")
        print("| " + " | ".join(vals) + " |")


def traffic_summary(workload, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, commands):
    """Per-kernel HBM bytes per launch from one FETCH_SIZE and one WRITE_SIZE
    pass (KiB per dispatch), each scaled by what the same counter reads for
    the 256 MiB device copy of --copy-calibration; writes
    profiles/pmc_traffic_<workload>.json (stamped with the SHA-256 of the
    kernel sources) and prints the markdown table."""
    import csv
    from collections import defaultdict

    def per_kernel(path):
        acc = defaultdict(list)
        with open(path) as f:
            for r in csv.DictReader(f):
                acc[_kernel_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        return acc

    def copy_kib(path):
        v = per_kernel(path).get("__amd_rocclr_copyBuffer")
        if not v:
            raise SystemExit("no device copy in %s" % path)
        return sum(v) / len(v)

    copy_kib_total = (256 << 20) / 1024.0
    ff = copy_kib_total / copy_kib(copy_fetch_csv)
    wf = copy_kib_total / copy_kib(copy_write_csv)
    fe, wr = per_kernel(fetch_csv), per_kernel(write_csv)
    kernels = {}
    for k in fe:
        if k not in wr:
            continue
        kernels[k] = {"launches": len(fe[k]),
                      "fetch_bytes_per_launch": int(sum(fe[k]) / len(fe[k]) * 1024 * ff),
                      "write_bytes_per_launch": int(sum(wr[k]) / len(wr[k]) * 1024 * wf)}
    d = {"workload": workload, "source_sha256": kernel_source_sha256(), "fetch_factor": round(ff, 4),
         "write_factor": round(wf, 4), "commands": commands, "kernels": kernels}
    with open(os.path.join(ROOT, "profiles", "pmc_traffic_%s.json" % workload), "w") as f:
        json.dump(d, f, indent=1)
    print("| kernel | launches | fetch MB/launch | write MB/launch |")
    print("|---|---:|---:|---:|")
    for k, v in sorted(kernels.items(), key=lambda kv: -(kv[1]["fetch_bytes_per_launch"] +
                                                          kv[1]["write_bytes_per_launch"]))[:20]:
        print("| `%s` | %d | %.1f | %.1f |" % (k, v["launches"], v["fetch_bytes_per_launch"] / 1e6,
                                              v["write_bytes_per_launch"] / 1e6))
    print()
    print("Copy calibration: FETCH_SIZE factor %.4f, WRITE_SIZE factor %.4f; kernel sources SHA-256 `%s`"
          % (ff, wf, d["source_sha256"]))


def trace_summary(path, top=25):
    """Markdown table of a rocprofv3 --kernel-trace --stats kernel_stats.csv."""
    import csv
    with open(path) as f:
        rows = list(csv.DictReader(f))
    print("| kernel | calls | total us | average us | % |")
    print("|---|---:|---:|---:|---:|")
    for r in rows[:top]:
        print("| `%s` | %s | %.1f | %.1f | %.2f |" % (_kernel_short(r["Name"]), r["Calls"],
                                                    float(r["TotalDurationNs"]) / 1e3,
                                                    float(r["AverageNs"]) / 1e3, float(r["Percentage"])))


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """GB/s (bytes read + written) of a plain device-to-device copy of
    nbytes, timed with HIP events: the bandwidth a streaming kernel reaches
    on this GPU, beside the nominal 8 TB/s."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return round(2.0 * nbytes / (ms * 1e-3) / 1e9, 1)


def copy_calibration():
    import torch
    nbytes = 256 << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}))


def value_width(sr):
    return 1 if sr == "bool" else 8


def kernel_bytes(name: str, st: dict, sr: str) -> float:
    """Algorithmic bytes one launch of `name` moves (per-row byte model).

    numeric rows R:  16|R| + annz(4+w) + 16 annz + flops(4+w) + cnnz(4+w)
    symbolic rows R: 16|R| + 4 annz + 16 annz + 4 flops
    (row extents of A and C, A entries, B row extents, B entries gathered,
    C entries written; w = value bytes)."""
    import paper_1510_00844_amd as spg
    w = value_width(sr)
    bins = {"tiny": [1], "small": [2], "dense": [12], "bitmap": [12], "dense_par": [11]}
    kind, _, tail = name.partition("_")
    b = None
    if tail == "rankc":
        idx = [11]
    elif tail.startswith("hash"):
        T = int(tail[4:])
        b = 3 + (T.bit_length() - 1 - 7)
        idx = [b]
    elif tail.startswith("rank"):
        cap = int(tail[4:])
        idx = [13 + (cap.bit_length() - 1 - 12)]
    else:
        idx = bins.get(tail)
        if idx is None:
            return float("nan")
    if kind == "num":
        R = sum(st["num_rows"][x] for x in idx)
        an = sum(st["num_annz"][x] for x in idx)
        f = sum(st["num_flops"][x] for x in idx)
        cn = sum(st["num_cnnz"][x] for x in idx)
        return 16.0 * R + an * (4 + w) + 16.0 * an + f * (4 + w) + cn * (4 + w)
    if kind == "sym":
        R = sum(st["sym_rows"][x] for x in idx)
        an = sum(st["sym_annz"][x] for x in idx)
        f = sum(st["sym_flops"][x] for x in idx)
        return 16.0 * R + 4.0 * an + 16.0 * an + 4.0 * f
    return float("nan")


def kernel_source_sha256() -> str:
    """SHA-256 over the HIP sources (names and contents, sorted by name)."""
    import hashlib
    d = os.path.join(ROOT, "paper_1510_00844_amd", "csrc")
    h = hashlib.sha256()
    for n in sorted(os.listdir(d)):
        if n.endswith((".hpp", ".hip")):
            h.update(n.encode())
            with open(os.path.join(d, n), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str = "c2"):
    """HBM bytes per launch of `kernel` (a launch name such as num_rankc)
    from the committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated, written by --traffic-summary), or None when the sources
    changed since the counters were taken or the name is ambiguous."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256") != kernel_source_sha256():
        return None
    prefix = "spg::k_%s<" % kernel
    hits = [v for k, v in d["kernels"].items() if k.startswith(prefix)]
    if len(hits) != 1:
        return None
    k = hits[0]
    return {"fetch_bytes": k["fetch_bytes_per_launch"], "write_bytes": k["write_bytes_per_launch"],
            "total_bytes": k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"],
            "source": "profiles/pmc_traffic_%s.md" % workload}


def model_bytes(m, annz, flops, cnnz, sr):
    """One Gustavson numeric pass: 8(m+1) + nnzA(4+w) + 16 nnzA + flops(4+w)
    + 8(m+1) + nnzC(4+w)."""
    w = value_width(sr)
    return 8.0 * (m + 1) * 2 + annz * (4 + w) + 16.0 * annz + flops * (4 + w) + cnnz * (4 + w)


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps, r


def _time_median(fn, reps):
    """Median of per-call times (each call synchronized), after one warmup
    call: for calls that wait on the GPU themselves, so one slow call (an
    allocation, a clock change) does not move the figure."""
    import torch
    r = fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    ts.sort()
    return ts[len(ts) // 2], r


def learned_modes(A2, dA2, args):
    """Single-pass product with the trained predictor against the two-phase
    product and against single-pass sizing without a predictor (capacity =
    min(flops, n)): C2 and the R-MAT G500 scale-19 product."""
    import paper_1510_00844_amd as spg
    import synth
    from paper_1510_00844_amd import learned
    res = {}
    if not os.path.exists(learned.WEIGHTS):
        return res
    params = learned.load()
    cases = [("c2", A2, dA2)]
    if not args.no_c5:
        A5 = synth.rmat(19, 16, synth.G500, seed=6)
        cases.append(("c5", A5, spg.DeviceCSR.from_arrays(A5.nrows, A5.ncols, A5.row_ptr, A5.col, A5.val)))
    for name, A, dA in cases:
        plan = spg.Plan()

        def plain():
            rp, nnz = spg.spgemm_symbolic(plan, "f64", dA, dA)
            spg.spgemm_numeric(plan, "f64", dA, dA, rp, nnz)
            return nnz

        def single(p):
            def f():
                nnz, st = spg.spgemm_learned_run(plan, "f64", dA, dA, p, 0.15)
                spg.spgemm_learned_fetch(plan, "f64", dA, dA, nnz)
                return nnz, st
            return f

        reps = 3
        t_plain, nnz = _time(plain, reps)
        flops = plan.stats()["flops"]
        t_l, (nnz_l, st_l) = _time(single(params), reps)
        t_u, (nnz_u, st_u) = _time(single(None), reps)
        assert nnz_l == nnz == nnz_u
        g = lambda t: round(2.0 * flops / (t * 1e-3) / 1e9, 3)
        res[name + "_plain"] = {"ms": round(t_plain, 4), "gflops": g(t_plain), "flops": flops, "nnz_c": nnz}
        res[name + "_learned"] = {"ms": round(t_l, 4), "gflops": g(t_l), "speedup_vs_plain": round(t_plain / t_l, 3),
                                  "single_pass_share_of_c": round(st_l["nnz_single"] / max(nnz, 1), 4),
                                  "flops_per_output": round(flops / max(nnz, 1), 3),
                                  "stats": {k: v for k, v in st_l.items() if k != "bin_rows"}}
        res[name + "_upper_bound_sizing"] = {"ms": round(t_u, 4), "gflops": g(t_u),
                                             "stats": {k: v for k, v in st_u.items() if k != "bin_rows"}}
        plan.close()
        del dA
        import torch
        torch.cuda.empty_cache()
    return res


def batched_modes(args, reps=20):
    """64 AMG Galerkin products (R^T A) R, A = 7-point Poisson on N^3 grids
    with N uniform in [16, 64], R = 2x2x2 aggregation: one batched call
    replayed as a HIP graph, the same batched call without the graph, and
    the 128 products one by one with the plain two-phase entry points."""
    import torch

    import paper_1510_00844_amd as spg
    import synth
    sizes, inst = synth.galerkin_batch()
    dev = []
    for RT, A, R in inst:
        dev.append(tuple(spg.DeviceCSR.from_arrays(M.nrows, M.ncols, M.row_ptr, M.col, M.val) for M in (RT, A, R)))
    rts, As, Rs = [d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev]
    flops = sum(A.nnz for _, A, _ in inst)  # flops(R^T, A) = nnz(A): one entry per column of R^T
    plan = spg.Plan()
    res = spg.spgemm_galerkin_batched(plan, "f64", rts, As, Rs, use_graph=True)
    flops += sum(int(n) for n in _t_nnz(plan, rts, As))  # flops(T, R) = nnz(T): one entry per row of R
    t_graph, _ = _time(lambda: spg.spgemm_galerkin_batched(plan, "f64", rts, As, Rs, use_graph=True), reps)
    plan_e = spg.Plan()
    spg.spgemm_galerkin_batched(plan_e, "f64", rts, As, Rs, use_graph=False)
    t_eager, _ = _time(lambda: spg.spgemm_galerkin_batched(plan_e, "f64", rts, As, Rs, use_graph=False), reps)
    plan_s = spg.Plan()

    def seq():
        for rt, a, r in dev:
            T = spg.spgemm(plan_s, "f64", rt, a)
            spg.spgemm(plan_s, "f64", T, r)

    t_seq, _ = _time(seq, 3)
    nnz_c = sum(res.nnz)
    # the same products with algebraic restrictions: MIS-2 aggregation of
    # every grid (Algorithm 3), then the batched products on those R
    plan_m = spg.Plan()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rts_m, rs_m, rounds, naggs = [], [], [], []
    for b, (rt, a, r) in enumerate(dev):
        _, agg, na, rnd = spg.spg_mis2_aggregate(plan_m, a, seed=1000 + b)
        R_m, RT_m = spg.spg_restriction(plan_m, "f64", agg, na)
        rts_m.append(RT_m)
        rs_m.append(R_m)
        rounds.append(rnd)
        naggs.append(na)
    torch.cuda.synchronize()
    t_mis = (time.perf_counter() - t0) * 1e3
    res_m = spg.spgemm_galerkin_batched(plan_m, "f64", rts_m, As, rs_m, use_graph=True)
    flops_m = sum(A.nnz for _, A, _ in inst)
    flops_m += sum(int(n) for n in _t_nnz(plan_m, rts_m, As))
    t_graph_m, _ = _time(lambda: spg.spgemm_galerkin_batched(plan_m, "f64", rts_m, As, rs_m, use_graph=True), reps)
    mis_out = {"aggregation_ms": round(t_mis, 3), "rounds_max": max(rounds), "aggregates": sum(naggs),
               "flops": flops_m, "nnz_c": sum(res_m.nnz),
               "graph_replay": {"ms": round(t_graph_m, 4), "gflops": round(2.0 * flops_m / t_graph_m / 1e6, 3)}}
    plan_m.close()
    # autotuned options (bin thresholds, gather mappings, streams) for this batch
    plan_t = spg.Plan()
    t0 = time.perf_counter()
    tuned, hit = spg.spg_autotune_galerkin(plan_t, "f64", rts, As, Rs, cache_path=args.tune_cache,
                                           budget_ms=args.tune_budget_ms)
    tune_s = time.perf_counter() - t0
    spg.spgemm_galerkin_batched(plan_t, "f64", rts, As, Rs, use_graph=True)
    t_tuned, _ = _time(lambda: spg.spgemm_galerkin_batched(plan_t, "f64", rts, As, Rs, use_graph=True), reps)
    g = lambda t: round(2.0 * flops / (t * 1e-3) / 1e9, 3)
    out = {"workload": "64 x (R^T A) R, A 7-point Poisson N^3 (N uniform 16..64, seed 5), R 2x2x2 aggregation, FP64",
           "grid_sizes": [int(x) for x in sizes], "flops": flops, "nnz_c": nnz_c,
           "graph_replay": {"ms": round(t_graph, 4), "gflops": g(t_graph)},
           "graph_replay_autotuned": {"ms": round(t_tuned, 4), "gflops": g(t_tuned), "opts": tuned,
                                      "from_cache": hit, "tune_seconds": round(tune_s, 3)},
           "batched_no_graph": {"ms": round(t_eager, 4), "gflops": g(t_eager)},
           "sequential_128_products": {"ms": round(t_seq, 4), "gflops": g(t_seq)},
           "mis2_restriction": mis_out,
           "speedup_graph_vs_sequential": round(t_seq / t_graph, 3)}
    for p in (plan, plan_e, plan_s, plan_t):
        p.close()
    torch.cuda.empty_cache()
    return out


def _t_nnz(plan, rts, As):
    """nnz(R_b^T A_b) per instance, from the two-phase symbolic pass."""
    import paper_1510_00844_amd as spg
    out = []
    for rt, a in zip(rts, As):
        _, nnz = spg.spgemm_symbolic(plan, "f64", rt, a)
        out.append(nnz)
    return out


def layered_modes(args, profile=False):
    """Split-3D layer shape: ER scale 18, edge factor 16; the inner dimension
    in c contiguous layers, C_l = A(:,K_l) B(K_l,:), then the merge."""
    import torch

    import paper_1510_00844_amd as spg
    import synth
    A = synth.rmat(18, 16, synth.ER, seed=3)
    B = synth.rmat(18, 16, synth.ER, seed=4)
    dA = spg.DeviceCSR.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col, A.val)
    dB = spg.DeviceCSR.from_arrays(B.nrows, B.ncols, B.row_ptr, B.col, B.val)
    plan = spg.Plan(profile=profile)
    t_full, C = _time_median(lambda: spg.spgemm(plan, "f64", dA, dB), 5)
    flops = plan.stats()["flops"]
    if profile:
        unsplit_kernels = kernel_table(plan, 6)
        plan.profile_reset()
    out = {"workload": "ER (.25,.25,.25,.25) scale 18 edge factor 16, A*B FP64", "flops": flops,
           "nnz_c": C.nnz, "unsplit": {"ms": round(t_full, 4), "gflops": round(2.0 * flops / t_full / 1e6, 3)}}
    for c in (4, 16):
        bounds = synth.layer_bounds(A.ncols, c)
        layers = []

        def products():
            layers.clear()
            for lo, hi in bounds:
                layers.append(spg.spgemm(plan, "f64", dA, dB, lo, hi))
            return layers

        t_prod, _ = _time_median(products, 5)
        if profile:
            prod_kernels = kernel_table(plan, 6)
            plan.profile_reset()
        t_merge, M = _time_median(lambda: spg.spgemm_merge_layers(plan, "f64", layers), 5)
        assert M.nnz == C.nnz
        # merge model: every layer read once, C written once (CSR bytes)
        w_merge = sum(8.0 * (L.nrows + 1) + 12.0 * L.nnz for L in layers) + 8.0 * (M.nrows + 1) + 12.0 * M.nnz
        out["c%d" % c] = {"layers_ms": round(t_prod, 4), "merge_ms": round(t_merge, 4),
                          "gflops_layers": round(2.0 * flops / t_prod / 1e6, 3),
                          "layer_nnz": sum(L.nnz for L in layers),
                          "merge_model_bytes": int(w_merge),
                          "merge_model_gbs": round(w_merge / t_merge / 1e6, 2),
                          "merge_model_frac": round(w_merge / t_merge / 1e6 / HBM_PEAK_GBS, 4)}
        if profile:
            out["c%d" % c]["layer_kernels"] = prod_kernels
            out["c%d" % c]["merge_kernels"] = kernel_table(plan, 6)
            plan.profile_reset()
        del layers, M
        # the same c layer products and their merge in one call: A's rows
        # cut at the layer bounds (piece rows), one product, the merge as a
        # selection product (the SUMMA stage call with one block per stage)
        D = spg.dcsr_compress(plan, dA)
        t_one, (Cs, snnz) = _time_median(lambda: spg.spgemm_summa_local(plan, "f64", D, dB, c, A.ncols // c), 5)
        assert Cs.nnz == C.nnz and snnz == out["c%d" % c]["layer_nnz"]
        out["c%d" % c]["one_call_ms"] = round(t_one, 4)
        out["c%d" % c]["one_call_speedup"] = round((t_prod + t_merge) / t_one, 3)
        if profile:
            plan.profile_reset()
        del D, Cs
    if profile:
        out["unsplit_kernels"] = unsplit_kernels
    plan.close()
    torch.cuda.empty_cache()
    return out


def heap_modes(reps=5):
    """The heap bin (k-way merge of a row's few B rows, HeapSpGEMM) against
    the hash tables for the same rows: each workload's two-phase product with
    the bin taking rows of up to 32 and up to 8 A entries, and with the bin
    off (the default), and the rows the bin takes."""
    import torch

    import paper_1510_00844_amd as spg
    import synth
    cases = [("c2", synth.rmat(16, 16, synth.G500, seed=2), None),
             ("ssca_s16", synth.rmat(16, 8, synth.SSCA, seed=2), None),
             ("c3_unsplit", synth.rmat(18, 16, synth.ER, seed=3), synth.rmat(18, 16, synth.ER, seed=4))]
    out = {}
    for name, A, B in cases:
        B = A if B is None else B
        dA = spg.DeviceCSR.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col, A.val)
        dB = dA if B is A else spg.DeviceCSR.from_arrays(B.nrows, B.ncols, B.row_ptr, B.col, B.val)
        r = {}
        for label, opt in (("heap", 32), ("heap8", 8), ("hash", -1)):
            plan = spg.Plan(heap_max_lists=opt)
            t, C = _time(lambda: spg.spgemm(plan, "f64", dA, dB), reps)
            st = plan.stats()
            r[label] = {"ms": round(t, 4), "gflops": round(2.0 * st["flops"] / t / 1e6, 3),
                        "heap_rows": st["num_rows"][spg.BIN_HEAP]}
            plan.close()
            del C
        r["speedup_heap_vs_hash"] = round(r["hash"]["ms"] / r["heap"]["ms"], 3)
        out[name] = r
        del dA, dB
        torch.cuda.empty_cache()
    return out


def summa_modes(reps=5):
    """One process's Sparse SUMMA stages (Algorithm 2 stage loop, blocking b)
    on hypersparse blocks: the share of process P(0,1,1) of a 16 x 16 x 4
    grid squaring R-MAT G500 scale 20 (65,536 rows, 262,144 inner indices in
    16 stages, 65,536 columns), A as DCSR.  Times the count + fill calls for
    several b, the direct product of the DCSR rows (one block) and the same
    product on the uncompressed CSR rows.

    Byte model of the staged call (w = value bytes, G = row pieces):
    W = nnzA (4 + w + 16) + 4 flops (symbolic gathers) + flops (4 + w)
        + 2 nnzP (4 + w) + nnzC (4 + w) + 16 (G + nzr)
    (A read with its B row extents, B gathered twice, the block products
    written and read back by the merge, C written, piece and row extents)."""
    import numpy as np
    import torch

    import paper_1510_00844_amd as spg
    import synth
    M = synth.rmat(20, 16, synth.G500, seed=3)
    A, B = synth.process_share(M, 16, 4, 0, 1, 1)
    del M
    dA = spg.DeviceCSR.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col, A.val)
    dB = spg.DeviceCSR.from_arrays(B.nrows, B.ncols, B.row_ptr, B.col, B.val)
    plan = spg.Plan()
    D = spg.dcsr_compress(plan, dA)
    t_csr, C = _time(lambda: spg.spgemm(plan, "f64", dA, dB), reps)
    flops = plan.stats()["flops"]
    nnz_c = C.nnz
    del C
    w = 8
    nz = np.diff(A.row_ptr) > 0
    out = {"workload": "Sparse SUMMA share of P(0,1,1), 16x16x4 grid, R-MAT G500 scale 20 squared: "
                       "A_loc 65536 x 262144 (DCSR), B_loc 262144 x 65536, 16 stages, FP64",
           "nnz_a": A.nnz, "nzr_a": int(nz.sum()), "nnz_b": B.nnz, "flops": flops, "nnz_c": nnz_c,
           "csr_product_ms": round(t_csr, 4)}
    t_dir, (Cd, _) = _time(lambda: spg.spgemm_summa_local(plan, "f64", D, dB, 1, A.ncols), reps)
    out["dcsr_product_ms"] = round(t_dir, 4)
    assert Cd.nnz == nnz_c
    del Cd
    for b in (16384, 4096, 1024):
        t, (Cs, snnz) = _time(lambda: spg.spgemm_summa_local(plan, "f64", D, dB, 16, b), reps)
        assert Cs.nnz == nnz_c
        cols = A.col.astype(np.int64) // b
        rows = np.repeat(np.arange(A.nrows), np.diff(A.row_ptr))
        pieces = int(np.count_nonzero(np.diff(rows * (A.ncols // b + 1) + cols, prepend=-1)))
        W = A.nnz * (4 + w + 16) + 4.0 * flops + flops * (4 + w) + 2.0 * snnz * (4 + w) + nnz_c * (4 + w) \
            + 16.0 * (pieces + int(nz.sum()))
        out["b%d" % b] = {"blocks": A.ncols // b, "pieces": pieces, "stage_nnz": snnz,
                          "stage_nnz_over_nnz_c": round(snnz / max(nnz_c, 1), 3), "ms": round(t, 4),
                          "gflops": round(2.0 * flops / t / 1e6, 3), "model_bytes": int(W),
                          "hbm_model_gbs": round(W / t / 1e6, 2), "hbm_model_frac": round(W / t / 1e6 / HBM_PEAK_GBS, 4)}
        del Cs
    plan.close()
    torch.cuda.empty_cache()
    return out


def kernel_table(plan, steps):
    out = {}
    for name, (launches, total) in plan.profile_read().items():
        out[name] = {"launches_per_step": launches / steps, "ms_per_step": round(total / steps, 4)}
    return dict(sorted(out.items(), key=lambda kv: -kv[1]["ms_per_step"]))


def secondary_mode(args):
    """One secondary workload alone: c3 (layers + merge), c4 (batched
    Galerkin), c5 (R-MAT scale 19 product)."""
    import torch

    import paper_1510_00844_amd as spg
    import synth
    torch.cuda.set_device(0)
    out = {"mode": args.mode}
    if args.mode == "c4":
        out.update(batched_modes(args, reps=args.steps))
    elif args.mode == "c3":
        out.update(layered_modes(args, profile=True))
        if not args.no_extras:
            out["heap_vs_hash"] = heap_modes()
    elif args.mode == "summa":
        out.update(summa_modes(reps=args.steps))
    else:
        A = synth.rmat(19, 16, synth.G500, seed=6)
        dA = spg.DeviceCSR.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col, A.val)
        plan = spg.Plan(profile=True, dense_chunk_cols=args.dense_cols, streams=args.streams)
        for _ in range(args.warmup):
            spg.spgemm(plan, "f64", dA, dA, values=True)
        torch.cuda.synchronize()
        plan.profile_reset()
        t, C = _time(lambda: spg.spgemm(plan, "f64", dA, dA), args.steps)
        flops = plan.stats()["flops"]
        st = plan.stats()
        out.update({"workload": "R-MAT G500 scale 19 edge factor 16, A*A FP64 two-phase", "ms": round(t, 4),
                    "gflops": round(2.0 * flops / t / 1e6, 3), "flops": flops, "nnz_c": C.nnz,
                    "num_rows": st["num_rows"], "sym_rows": st["sym_rows"],
                    "kernels": kernel_table(plan, args.steps + 1)})
        plan.close()
    print(json.dumps(out))


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary, args.traffic_commands)
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported "
              "(run with --gpus 1)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.mode != "c2":
        secondary_mode(args)
        return
    import numpy as np
    import torch

    import paper_1510_00844_amd as spg
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    A = synth.rmat(args.scale, 16, synth.G500, seed=2)
    sr = "f64"
    dA = spg.DeviceCSR.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col, A.val)
    plan = spg.Plan(profile=not args.no_profile, dense_chunk_cols=args.dense_cols, streams=args.streams,
                    gather_map=args.gather_map, unroll=args.unroll, sym_gather_map=args.sym_gather_map,
                    sym_unroll=args.sym_unroll)

    def step():
        rp, nnz = spg.spgemm_symbolic(plan, sr, dA, dA)
        col, val = spg.spgemm_numeric(plan, sr, dA, dA, rp, nnz)
        return nnz

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dom = None
    if not args.no_profile:
        # the dominant kernel: the one that moves the most algorithmic bytes
        # per step (over the warmup steps, every launch timed); the timed
        # steps then carry events around its launches only
        prof0 = plan.profile_read()
        st0 = plan.stats()
        cands = {}
        for k, (launches, _) in prof0.items():
            b = kernel_bytes(k, st0, sr)
            if b == b:  # kernels with a byte model (product kernels)
                cands[k] = b * launches
        dom = max(cands, key=cands.get) if cands else None
        plan.profile_select(dom)
        plan.profile_reset()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nnz = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    st = plan.stats()
    flops = st["flops"]
    gflops = 2.0 * flops / (ms * 1e-3) / 1e9
    W = model_bytes(A.nrows, A.nnz, flops, nnz, sr)
    prof = {} if args.no_profile else plan.profile_read()
    kernels = {}
    if not args.no_profile:
        for name, (launches, total) in prof0.items():
            kernels[name] = {"launches_per_step": launches / max(args.warmup, 1),
                             "ms_per_step": round(total / max(args.warmup, 1), 4)}
    roofline = None
    if dom is not None and dom in prof:
        launches, total = prof[dom]
        avg_ms = total / launches
        byts = kernel_bytes(dom, st, sr)
        ach = byts / (avg_ms * 1e-3) / 1e9
        tr = measured_traffic(dom)
        roofline = {"bound": "hbm", "kernel": dom, "dominant_by": "algorithmic bytes per step",
                    "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": None if tr is None else tr["total_bytes"],
                    "bytes_per_launch": byts, "avg_launch_ms": round(avg_ms, 5)}
        if tr is not None:
            roofline["traffic_detail"] = tr
    # context: every kernel alone (one stream), so each launch has the GPU to itself
    roofline_isolated = None
    if not args.no_profile and not args.no_isolated:
        piso = spg.Plan(profile=True, streams=1)
        for _ in range(2):
            rp_i, n_i = spg.spgemm_symbolic(piso, sr, dA, dA)
            spg.spgemm_numeric(piso, sr, dA, dA, rp_i, n_i)
        torch.cuda.synchronize()
        piso.profile_reset()
        t0 = time.perf_counter()
        for _ in range(3):
            rp_i, n_i = spg.spgemm_symbolic(piso, sr, dA, dA)
            spg.spgemm_numeric(piso, sr, dA, dA, rp_i, n_i)
        torch.cuda.synchronize()
        iso_ms = (time.perf_counter() - t0) * 1e3 / 3
        pi = piso.profile_read()
        sti = piso.stats()
        cand = {k: v for k, v in pi.items() if kernel_bytes(k, sti, sr) == kernel_bytes(k, sti, sr)}
        kd = max(cand, key=lambda k: kernel_bytes(k, sti, sr) * cand[k][0])
        launches, total = cand[kd]
        byts_i = kernel_bytes(kd, sti, sr)
        avg_i = total / launches
        roofline_isolated = {"kernel": kd, "achieved": round(byts_i / (avg_i * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(byts_i / (avg_i * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "bytes_per_launch": byts_i, "avg_launch_ms": round(avg_i, 5),
                             "step_ms_one_stream": round(iso_ms, 4),
                             "kernels_ms_per_step": {k: round(v[1] / 3, 4) for k, v in
                                                     sorted(pi.items(), key=lambda kv: -kv[1][1])[:8]}}
        piso.close()
    out = {
        "metric": METRIC,
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "R-MAT G500 (.57,.19,.19,.05) scale %d edge factor 16, duplicates summed, "
                               "symmetric permutation; C = A*A two-phase, plus-times FP64" % args.scale,
                   "m": A.nrows, "nnz_a": A.nnz, "flops": flops, "nnz_c": nnz, "seed": 2},
        "compulsory_bytes": int(A.nnz * 12 * 2 + (A.nrows + 1) * 16 + nnz * 12 + (A.nrows + 1) * 8),
        # what the two-phase step issues beyond the one-pass model W: the
        # symbolic pass's B row extents, B column gathers and row counts
        "issued_bytes": int(W + 16.0 * A.nnz + 4.0 * flops + 8.0 * (A.nrows + 1)),
        "model_bytes": int(W),
        "copy_kernel_gbs": copy_bandwidth(),
        "hbm_model_gbs": round(W / (ms * 1e-3) / 1e9, 2),
        "hbm_model_frac": round(W / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "roofline_isolated": roofline_isolated,
        "kernels_warmup": kernels,
        "bins": {spg.BIN_NAMES[b]: st["num_rows"][b] for b in range(spg.NBINS) if st["num_rows"][b]},
    }
    if not args.no_extras:
        extras = {}
        for xsr, kind in (("i64", "ones_i64"), ("bool", "true_bool")):
            Ax = synth.with_values(A, kind)
            dx = spg.DeviceCSR.from_arrays(Ax.nrows, Ax.ncols, Ax.row_ptr, Ax.col, Ax.val)
            p2 = spg.Plan()
            for _ in range(2):
                rp, n2 = spg.spgemm_symbolic(p2, xsr, dx, dx)
                spg.spgemm_numeric(p2, xsr, dx, dx, rp, n2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 5
            for _ in range(reps):
                rp, n2 = spg.spgemm_symbolic(p2, xsr, dx, dx)
                spg.spgemm_numeric(p2, xsr, dx, dx, rp, n2)
            torch.cuda.synchronize()
            xms = (time.perf_counter() - t0) * 1e3 / reps
            extras["c2_" + xsr] = {"ms_per_step": round(xms, 4),
                                   "gflops": round(2.0 * flops / (xms * 1e-3) / 1e9, 3),
                                   "hbm_model_gbs": round(model_bytes(A.nrows, A.nnz, flops, n2, xsr) / (xms * 1e-3) / 1e9, 2)}
            p2.close()
        # C1: ER-uniform n = 4096, 4 entries per column (latency-bound: 65,536 products)
        A1 = synth.er_uniform_columns(4096, 4, seed=1)
        d1 = spg.DeviceCSR.from_arrays(A1.nrows, A1.ncols, A1.row_ptr, A1.col, A1.val)
        p1 = spg.Plan()
        t1, C1 = _time(lambda: spg.spgemm(p1, "f64", d1, d1), 20)
        f1 = p1.stats()["flops"]
        extras["c1"] = {"workload": "ER-uniform n=4096, 4 distinct rows per column, FP64, C = A*A",
                        "ms": round(t1, 4), "flops": f1, "nnz_c": C1.nnz,
                        "gflops": round(2.0 * f1 / (t1 * 1e-3) / 1e9, 3)}
        p1.close()
        # the SSCA class (.6, .4/3, .4/3, .4/3), edge factor 8, scale 16
        As = synth.rmat(16, 8, synth.SSCA, seed=2)
        ds = spg.DeviceCSR.from_arrays(As.nrows, As.ncols, As.row_ptr, As.col, As.val)
        ps = spg.Plan()
        ts_, Cs = _time(lambda: spg.spgemm(ps, "f64", ds, ds), 10)
        fs_ = ps.stats()["flops"]
        extras["ssca_s16"] = {"workload": "R-MAT SSCA (.6,.4/3,.4/3,.4/3) scale 16 edge factor 8, A*A FP64",
                              "ms": round(ts_, 4), "flops": fs_, "nnz_c": Cs.nnz,
                              "gflops": round(2.0 * fs_ / (ts_ * 1e-3) / 1e9, 3)}
        ps.close()
        del Cs
        extras["heap_vs_hash"] = heap_modes()
        extras.update(learned_modes(A, dA, args))
        extras["c4_batched"] = batched_modes(args)
        extras["c3_layers"] = layered_modes(args)
        extras["summa_s20_share"] = summa_modes()
        out["modes"] = extras
    if not args.no_cpu_baseline:
        import oracle
        threads = os.cpu_count() or 1
        try:
            threads = len(os.sched_getaffinity(0))
        except Exception:
            pass
        # the whole product, repeated until about 12 s of wall time have passed
        runs, tc = 0, 0.0
        while runs < 60 and (runs == 0 or tc < 12.0):
            t0 = time.perf_counter()
            ref = oracle.spgemm(A, A, sr, nthreads=threads)
            tc += time.perf_counter() - t0
            runs += 1
        assert ref.nnz == nnz
        tc /= runs
        # one thread, on every 8th row (an eighth of the rows, spread over the matrix)
        rows = np.arange(0, A.nrows, 8)
        f_rows = int(oracle.row_flops(A, A)[rows].sum())
        t0 = time.perf_counter()
        oracle.spgemm(A, A, sr, rows=rows, nthreads=1)
        t1c = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(2.0 * flops / tc / 1e9, 4), "unit": "GFLOP/s", "cores": threads,
                               "kind": "oracle", "seconds": round(tc, 3),
                               "sample": "the whole C = A*A of this workload (count pass + fill pass), "
                                         "row-parallel OpenMP over %d threads, mean of %d runs" % (threads, runs),
                               "single_thread": {"value": round(2.0 * f_rows / t1c / 1e9, 4), "unit": "GFLOP/s",
                                                 "seconds": round(t1c, 3),
                                                 "sample": "every 8th row of the same product, one thread"}}
    plan.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
