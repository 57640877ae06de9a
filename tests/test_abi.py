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
    assert opt.kernel == pk.CSBQ_KERNEL_STOKES and opt.srule == pk.CSBQ_SRULE_AUTO
    assert opt.far_rule == pk.CSBQ_FAR_AUTO


def test_options_struct_matches_header():
    """The binding's options struct has the header's fields in the header's
    order (a missing or reordered field would shift every later one)."""
    import paper_2310_00889_amd as pk
    src = open(os.path.join(ROOT, "include", "csbq.h")).read()
    body = re.search(r"typedef struct \{([^}]*)\} csbq_options;", src, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"(\w+)\s*;", body)
    assert names == [f[0] for f in pk._Options._fields_]


def test_unknown_srule_refused_before_the_library():
    import paper_2310_00889_amd as pk
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("libcsbq.so not built")
    with pytest.raises(pk.CsbqError):
        pk.Evaluator(srule="dyadic-only")


def test_unknown_far_rule_refused_before_the_library():
    import paper_2310_00889_amd as pk
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("libcsbq.so not built")
    with pytest.raises(pk.CsbqError):
        pk.Evaluator(far_rule="nearest")
