"""Planted mistakes in a copy of the oracle must fail the oracle's pins.

Each mutant edits one line of a private copy of the oracle (in oracle.c: a
window bound off by one, a dropped term, a wrong operand index, unsorted
output, the wrong boolean operation, a miscounted flop, a dropped
compensation, a signed magnitude sum, a miscounted term, a wrong error term;
in summa.py: a block bound off by one, single-entry rows dropped, stages
merged in reverse order, row lengths assigned to the wrong rows); the pin
suites run against that copy have to fail.  The real oracle is never modified.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("oracle.c", "if (k < k_lo || k >= k_hi) continue;", "if (k < k_lo || k > k_hi) continue;"),
    ("oracle.c", "else spa_f[j] = spa_f[j] + t;", "else spa_f[j] = t;"),
    ("oracle.c", "((const double*)b_val)[q];", "((const double*)b_val)[p];"),
    ("oracle.c", "if (out_col) qsort", "if (0) qsort"),
    ("oracle.c", "uint64_t t = av & bv;", "uint64_t t = av | bv;"),
    ("oracle.c", "f += b_rp[k + 1] - b_rp[k];", "f += b_rp[k + 1] - b_rp[k] + (k == 0);"),
    ("oracle.c", "else spa_u[j] = spa_u[j] + t;", "else spa_u[j] = spa_u[j] - t;"),
    # the FP64 check data (compensated sum, magnitude sum, term count)
    ("oracle.c", "comp_out[t] = sum[j] + comp[j];", "comp_out[t] = sum[j];"),
    ("oracle.c", "absum[j] += at;", "absum[j] += t;"),
    ("oracle.c", "nterms[j] += 1;", "nterms[j] += 1 + (nterms[j] > 2);"),
    ("oracle.c", "if (as >= at) comp[j] += (s - r) + t;", "if (as >= at) comp[j] += (s - r) - t;"),
    # the stage accumulation and the row-compressed format
    ("summa.py", "r * per_stage + (q + 1) * b)", "r * per_stage + (q + 1) * b - 1)"),
    ("summa.py", "keep = np.nonzero(lens > 0)[0]", "keep = np.nonzero(lens > 1)[0]"),
    ("summa.py", "for lo, hi in stage_blocks(A.ncols, stages, b)]", "for lo, hi in stage_blocks(A.ncols, stages, b)[::-1]]"),
    ("summa.py", "lens[D.row_ids] = np.diff(D.row_ptr)", "lens[D.row_ids] = np.diff(D.row_ptr)[::-1]"),
]


@pytest.mark.slow
@pytest.mark.parametrize("idx", range(len(MUTANTS)))
def test_mutant_is_caught(tmp_path, idx):
    fname, old, new = MUTANTS[idx]
    for d in ("oracle", "synth", "tests"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d,
                        ignore=shutil.ignore_patterns("*.so", "__pycache__", "*.tmp*"))
    src = tmp_path / "oracle" / fname
    text = src.read_text()
    assert old in text, "mutation target not found"
    src.write_text(text.replace(old, new, 1))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle.py", "tests/test_oracle_f64.py", "tests/test_oracle_summa.py"], cwd=tmp_path, capture_output=True,
                       text=True,
                       timeout=600)
    assert r.returncode != 0, "mutant %d survived the pins:\n%s" % (idx, r.stdout[-2000:])
