"""The C ABI library loads and exports every function that include/tns.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "tns.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tns_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("tns_build_tasklist", "tns_apply_heff", "tns_apply_heff_backward", "tns_davidson"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2305_05581_amd.tns import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("libtns.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
