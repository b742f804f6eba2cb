"""Planted mistakes in a copy of the oracle must fail the oracle's pins.

Each mutant edits one line of a private copy of oracle.c (a window bound off
by one, a dropped term, a wrong operand index, unsorted output, the wrong
boolean operation, a miscounted flop, a dropped compensation, a signed
magnitude sum, a miscounted term, a wrong error term); the pin suites run
against that copy have to fail.  The real oracle is never modified.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("if (k < k_lo || k >= k_hi) continue;", "if (k < k_lo || k > k_hi) continue;"),
    ("else spa_f[j] = spa_f[j] + t;", "else spa_f[j] = t;"),
    ("((const double*)b_val)[q];", "((const double*)b_val)[p];"),
    ("if (out_col) qsort", "if (0) qsort"),
    ("uint64_t t = av & bv;", "uint64_t t = av | bv;"),
    ("f += b_rp[k + 1] - b_rp[k];", "f += b_rp[k + 1] - b_rp[k] + (k == 0);"),
    ("else spa_u[j] = spa_u[j] + t;", "else spa_u[j] = spa_u[j] - t;"),
    # the FP64 check data (compensated sum, magnitude sum, term count)
    ("comp_out[t] = sum[j] + comp[j];", "comp_out[t] = sum[j];"),
    ("absum[j] += at;", "absum[j] += t;"),
    ("nterms[j] += 1;", "nterms[j] += 1 + (nterms[j] > 2);"),
    ("if (as >= at) comp[j] += (s - r) + t;", "if (as >= at) comp[j] += (s - r) - t;"),
]


@pytest.mark.slow
@pytest.mark.parametrize("idx", range(len(MUTANTS)))
def test_mutant_is_caught(tmp_path, idx):
    old, new = MUTANTS[idx]
    for d in ("oracle", "synth", "tests"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d,
                        ignore=shutil.ignore_patterns("*.so", "__pycache__", "*.tmp*"))
    src = tmp_path / "oracle" / "oracle.c"
    text = src.read_text()
    assert old in text, "mutation target not found"
    src.write_text(text.replace(old, new, 1))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle.py", "tests/test_oracle_f64.py"], cwd=tmp_path, capture_output=True,
                       text=True,
                       timeout=600)
    assert r.returncode != 0, "mutant %d survived the pins:\n%s" % (idx, r.stdout[-2000:])
