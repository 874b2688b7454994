"""CPU checks of the C-ABI library: it loads and exports every entry point
that include/qtb.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "qtb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qtb_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_four_core_calls():
    names = declared_functions()
    for n in ("qtb_init", "qtb_build_filter", "qtb_step", "qtb_observables"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1905_02521_amd import qtb
    if not os.path.exists(qtb.LIB_PATH):
        pytest.skip("libqtb.so not built")
    lib = ctypes.CDLL(qtb.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(qtb.EXPORTS) == set(declared_functions())


def test_version_string():
    from paper_1905_02521_amd import qtb
    if not os.path.exists(qtb.LIB_PATH):
        pytest.skip("libqtb.so not built")
    assert b"gfx950" in qtb.lib().qtb_version()
