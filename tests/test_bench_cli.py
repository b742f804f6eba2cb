"""bench.py command line on the CPU: more than one GPU is refused with a
message before anything is measured, and the profile summarizers turn
rocprofv3 csv output into the committed tables."""

import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_pmc_summary_averages_per_kernel(tmp_path):
    path = tmp_path / "pmc.csv"
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    rows = [
        (1, "void spg::k_a<1>(int)", "SQ_WAVES", 10, 0, 2000),
        (1, "void spg::k_a<1>(int)", "SQ_INSTS_LDS", 100, 0, 2000),
        (2, "void spg::k_a<1>(int)", "SQ_WAVES", 30, 5000, 9000),
        (2, "void spg::k_a<1>(int)", "SQ_INSTS_LDS", 300, 5000, 9000),
        (3, "k_b(long)", "SQ_WAVES", 4, 0, 1000),
        (3, "k_b(long)", "SQ_INSTS_LDS", 8, 0, 1000),
    ]
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(fields)
        w.writerows(rows)
    r = _run("--pmc-summary", str(path))
    assert r.returncode == 0, r.stderr
    lines = [l for l in r.stdout.splitlines() if l.startswith("| `")]
    # k_a: two dispatches of 2 and 4 us, 20 waves and 200 LDS instructions on average, 10 per wave
    assert lines[0].startswith("| `spg::k_a<1>` | 2 | 3.0 |")
    assert "| 20 |" in lines[0] and lines[0].rstrip().endswith("| 10.0 |")
    assert lines[1].startswith("| `k_b` | 1 | 1.0 |")


def test_trace_summary_table(tmp_path):
    path = tmp_path / "stats.csv"
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["void spg::k_x<0>(spg::Csr)", 4, 8000, 2000, 80.0, 1000, 3000, 1.0])
    r = _run("--trace-summary", str(path))
    assert r.returncode == 0, r.stderr
    assert "| `spg::k_x<0>` | 4 | 8.0 | 2.0 | 80.00 |" in r.stdout
