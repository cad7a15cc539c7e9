"""The C-ABI library loads and exports every symbol the header declares.

Host-only entry points (argument validation that fails before any device
call, the Chebyshev order rule) are exercised without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "procmv.h")).read()
    return sorted(set(re.findall(r"\b(procmv_[a-z_]+)\s*\(", text)))


def test_header_matches_binding_list():
    from paper_2606_31598_amd import procmv
    assert sorted(procmv.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_2606_31598_amd import procmv
    L = procmv.load()
    for name in _declared():
        assert hasattr(L, name), name


def test_cheb_order_matches_oracle():
    from paper_2606_31598_amd import procmv
    from oracle import chebyshev as ch
    for x in [0.125, 1.0, 7.3, 141.37, 4000.0, 82792.0]:
        for tol in [1e-7, 1e-10]:
            assert procmv.cheb_order(x, tol) == ch.cheb_order(x, tol)


def test_invalid_arguments_rejected_on_host():
    from paper_2606_31598_amd import procmv
    L = procmv.load()
    h = ctypes.c_void_p()
    assert L.procmv_create_operator(7, 1, 16, None, ctypes.byref(h)) == 1
    assert L.procmv_create_operator(0, 1, 0, None, ctypes.byref(h)) == 1
    assert L.procmv_create_operator(0, 1, 1 << 31, None, ctypes.byref(h)) == 1
    assert b"outside" in L.procmv_last_error()
    assert L.procmv_create_operator(0, 1, 100, None, None) == 1
    # a Philox-GUE operator is host state only until it is planned
    assert L.procmv_create_operator(0, 1, 100, None, ctypes.byref(h)) == 0
    assert L.procmv_plan(h, 100, 0, 0.0, 0, None) == 1         # not a multiple of 64
    assert L.procmv_plan(h, 64, 9, 0.0, 0, None) == 1          # unknown strategy
    assert L.procmv_plan(h, 64, 1, 1.5, 0, None) == 1          # fraction outside [0, 1]
    x = ctypes.c_void_p(16)
    assert L.procmv_apply(h, x, 100, x, 100, 1, None) == 4     # not planned
    info = procmv.PlanInfo()
    assert L.procmv_plan_info(h, ctypes.byref(info)) == 4
    assert L.procmv_get_entries(h, 90, 0, 20, 1, x, None) == 1  # window outside
    L.procmv_destroy(h)
    L.procmv_destroy(None)
