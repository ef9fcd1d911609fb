"""CPU checks of the C ABI: the built library loads and exports every entry point
declared in include/genpcg.h (no compute call is made without a GPU)."""
import ctypes
import numpy as np
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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_footprint_estimate_on_the_host():
    """gn_footprint needs no device: it sizes an operator and its preconditioner
    from the grid and decomposition.  Checked against the sizes it must at
    least cover (A, element matrices, local factor bands, coarse factor), and
    for its response to the options."""
    from paper_1901_05188_amd import binding as gb
    from workloads import generate as gen
    w = gen.config_c1()
    est64 = gb.footprint(w, local_prec=64)
    est32 = gb.footprint(w, local_prec=32)
    one = gb.footprint(w, coarse=False)
    op_only = gb.footprint(w, with_precond=False)
    nn = (w.ne[0] + 1) * (w.ne[1] + 1) * (w.ne[2] + 1)
    assert op_only >= nn * 27 * 9 * 8 + w.n_elem * 24 * 24 * 8
    assert op_only < one < est64 and est32 < est64
    # the coarse part: N_H = 4 x 10, its dense factor inverse of ceil(40/32)^2 tiles
    assert est64 - one >= 2 * 2 * 32 * 32 * 8
    bad = gen.config_c1()
    bad.cuts = [np.array([0, 9, 8, 16]), bad.cuts[1], bad.cuts[2]]
    bad.nparts = (3, bad.nparts[1], bad.nparts[2])
    with pytest.raises(gb.GenPCGError) as e:
        gb.footprint(bad)
    assert e.value.code == -1
    # c5, the largest single-GPU configuration: FP64 local factors fit one MI355X
    c5 = gen.config_c5()
    b5 = gb.footprint(c5, local_prec=64)
    assert 30e9 < b5 < 200e9, b5
