"""The C-ABI library loads and exports every function include/csbq.h declares
(no compute call: this runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "csbq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(csbq_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("csbq_create", "csbq_set_geometry", "csbq_eval", "csbq_smooth_sum", "csbq_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2310_00889_amd as pk
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("libcsbq.so not built")
    lib = C.CDLL(pk.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options_without_device():
    import paper_2310_00889_amd as pk
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("libcsbq.so not built")
    lib = pk.load_library()
    opt = pk._Options()
    lib.csbq_default_options(C.byref(opt))
    assert opt.quad_tol == 1e-12 and opt.precision == 0 and opt.device == 0
