import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def gpu_available():
    import torch
    return torch.cuda.is_available()


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """FP64 entries over 1e-12 relative that each test re-checked against the
    compensated sum of their terms (always printed, also under -q)."""
    try:
        from util import FP64_RECHECKS
    except ImportError:
        return
    if not FP64_RECHECKS:
        return
    per = {}
    for test, over, total in FP64_RECHECKS:
        o, t = per.get(test, (0, 0))
        per[test] = (o + over, t + total)
    tr = terminalreporter
    tr.write_sep("-", "FP64 entries over 1e-12 relative (re-checked against the compensated sum)")
    for test, (o, t) in per.items():
        tr.write_line("%s: %d of %d entries" % (test, o, t))
