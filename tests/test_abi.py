"""The C ABI (CPU only): libmeb.so loads and exports every function that
include/meb.h declares.  No compute call is made (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2605_31425_amd", "libmeb.so")
HDR = os.path.join(ROOT, "include", "meb.h")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(meb_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["meb_solve", "meb_al_eval", "meb_screen", "meb_check_feasible"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmeb.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmeb.so not built")
def test_binding_export_list_matches_header():
    import sys
    sys.path.insert(0, ROOT)
    src = open(os.path.join(ROOT, "paper_2605_31425_amd", "meb.py")).read()
    listed = re.search(r"EXPORTS = \[(.*?)\]", src, flags=re.S).group(1)
    listed = sorted(re.findall(r'"(meb_\w+)"', listed))
    assert listed == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmeb.so not built")
def test_options_defaults_without_gpu():
    # meb_default_options and meb_workspace_size are pure host code
    import sys
    sys.path.insert(0, ROOT)
    from paper_2605_31425_amd import meb
    o = meb.options()
    assert o.rho == 0.9 and o.tol_kkt == 1e-9 and o.tol_kkt_low == 1e-2 and o.mode == meb.MEB_MODE_MIXED
    assert o.hess == meb.MEB_HESS_AUTO and o.newton == 0 and o.cg_max_iter == 20 and o.first_order_outer == 0
    n = ctypes.c_size_t()
    assert meb.lib.meb_workspace_size(1000, 10, 0, ctypes.byref(o), ctypes.byref(n)) == 0
    assert n.value > 1000 * 10 * 8
    assert meb.lib.meb_workspace_size(0, 10, 0, ctypes.byref(o), ctypes.byref(n)) < 0
    assert meb.lib.meb_last_error().decode() != ""


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmeb.so not built")
def test_library_was_built_from_these_sources():
    import sys
    sys.path.insert(0, ROOT)
    from paper_2605_31425_amd import build
    lib = ctypes.CDLL(LIB)
    lib.meb_source_hash.restype = ctypes.c_char_p
    assert lib.meb_source_hash().decode() == build.source_hash(), "libmeb.so is stale: rebuild it"
