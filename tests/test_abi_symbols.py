"""The C ABI library loads and exports every entry point include/clak.h
declares, and the binding knows each one (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1207_2169_amd import clak

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "clak.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(clak_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["clak_plan_create", "clak_plan_workspace_size", "clak_plan_set_workspace",
                     "clak_plan_set_stream", "clak_set_kinship", "clak_set_eigen", "clak_set_covariates",
                     "clak_set_traits", "clak_run_block", "clak_plan_destroy", "clak_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(clak.LIB_PATH):
        pytest.fail("libclak.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(clak.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in clak.SIGNATURES, f"binding lacks {name}"


def test_host_only_calls_without_a_gpu():
    """Calls that touch no device memory work on a host without a GPU."""
    lib = clak.lib()
    assert b"gfx950" in lib.clak_version()
    assert lib.clak_plan_create(None, 10, 3, 1, 10, 0, 0) == clak.CLAK_E_ARG
    assert b"null" in lib.clak_last_error()
    assert lib.clak_plan_destroy(None) == clak.CLAK_E_ARG
    assert lib.clak_plan_set_tuning(None, 0, 2, 64, 8) == clak.CLAK_E_ARG
    assert lib.clak_plan_get_tuning(None, None, None, None, None) == clak.CLAK_E_ARG
    assert lib.clak_autotune(None, 1, None, 0, 1, None, None, 0, 1, None, None) == clak.CLAK_E_ARG
    assert lib.clak_estimate_vc(None, None, 1, clak.CLAK_VC_REML, None, None, None) == clak.CLAK_E_ARG
    assert b"null" in lib.clak_last_error()
    h = ctypes.c_void_p()
    assert lib.clak_plan_create(ctypes.byref(h), 10, 3, 2, 10, 0, clak.CLAK_CHOL) == clak.CLAK_E_ARG
    assert b"t = 1" in lib.clak_last_error()
    # sizes outside what a precision supports are refused before any device work
    assert lib.clak_plan_create(ctypes.byref(h), 40000, 3, 1, 10, clak.CLAK_PREC_MIXED, 0) == clak.CLAK_E_UNSUPPORTED
    assert lib.clak_plan_create(ctypes.byref(h), 100, 9, 1, 10, clak.CLAK_PREC_MIXED, 0) == clak.CLAK_E_UNSUPPORTED
    assert lib.clak_plan_create(ctypes.byref(h), 100, 17, 1, 10, clak.CLAK_PREC_FP64, 0) == clak.CLAK_E_ARG
    assert lib.clak_plan_create(ctypes.byref(h), 3, 3, 1, 10, clak.CLAK_PREC_FP64, 0) == clak.CLAK_E_ARG
    assert lib.clak_plan_create(ctypes.byref(h), 100, 3, 1, 10, 0, 1 << 5) == clak.CLAK_E_ARG
