"""The C ABI library loads and exports every function include/*.h declares
(no compute call: this runs without a GPU), and the binding marshals the
structures with the header's layout."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                             text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("spgemm_symbolic", "spgemm_numeric", "spgemm_merge_layers", "spg_plan_create",
                 "spg_plan_destroy", "spg_status_string", "spg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1510_00844_amd as spg
    if not os.path.exists(spg.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(spg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_entry_points():
    import paper_1510_00844_amd as spg
    if not os.path.exists(spg.LIB_PATH):
        pytest.skip("library not built")
    L = spg.lib()
    assert L.spg_status_string(0) == b"SPG_OK"
    assert L.spg_status_string(2) == b"SPG_ERR_SHAPE"
    o = spg.Opts()
    L.spg_default_opts(ctypes.byref(o))
    assert o.small_max_flops == 64 and o.hash_max_nnz == 4096 and o.streams == 4
    assert o.gather_pipeline == 0 and o.fused_max_nnz == 0 and o.heap_max_lists == -1
    assert ctypes.sizeof(spg.Opts) == 20 * 4
    assert ctypes.sizeof(spg._Csr) == 6 * 8
