"""CPU checks of the C ABI: the built library loads and exports every entry point
declared in include/genpcg.h (no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "genpcg.h")
LIB = os.path.join(ROOT, "paper_1901_05188_amd", "libgenpcg.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gn_[a-z_]+)\s*\(", src)))


def test_header_declares_the_three_calls():
    names = declared_functions()
    for f in ("gn_assemble", "gn_setup_geneo", "gn_solve"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_every_declared_symbol():
    from paper_1901_05188_amd import binding
    assert sorted(binding.EXPORTS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_last_error_is_empty_string_initially():
    lib = ctypes.CDLL(LIB)
    lib.gn_last_error.restype = ctypes.c_char_p
    assert lib.gn_last_error() == b""


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_arguments_rejected_without_device_work():
    lib = ctypes.CDLL(LIB)
    lib.gn_problem_info.restype = ctypes.c_int32
    lib.gn_last_error.restype = ctypes.c_char_p
    assert lib.gn_problem_info(None, None, None, None) == -1
    assert b"null" in lib.gn_last_error()
