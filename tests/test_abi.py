"""The C-ABI library loads and exports every entry point include/grasp.h
declares, and the Python binding covers exactly those (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grasp.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grasp_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2306_08132_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2306_08132_amd import build
        build.build()
    return _lib


def test_every_declared_symbol_is_exported(lib):
    dll = C.CDLL(lib.LIB_PATH)
    names = declared()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(dll, n)]
    assert not missing, missing


def test_binding_covers_header(lib):
    bound = sorted(n for n, _, _ in lib.SIGNATURES)
    assert bound == declared()


def test_null_arguments_are_rejected_without_a_device(lib):
    L = lib.Library.get()
    assert L.grasp_create_hand(None, None, None) == lib.GRASP_EINVAL
    assert b"NULL" in L.grasp_last_error()
    assert L.grasp_step_fwd(None, 0, 0, None, 0, None, None, None, None, 0, None) == lib.GRASP_EINVAL
    assert L.grasp_init(0, None, 1 << 20, None) == lib.GRASP_EINVAL
    p = lib.StepParamsC()
    L.grasp_default_params(C.byref(p))
    assert (p.dt, p.K, p.ckpt_every, p.alpha_leak) == (C.c_float(1e-3).value, 1, 1, C.c_float(0.1).value)
