"""The C-ABI library loads and exports what include/bim.h declares (CPU only; no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1709_08803_amd", "libbim.so")


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(bim_[a-z0-9_]+|precond_[a-z0-9_]+|jfnk_[a-z0-9_]+|lg_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libbim.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("bim_residual", "bim_jv", "bim_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_invalid_arguments_are_rejected_without_gpu(lib):
    lib.bim_residual.restype = ctypes.c_int
    lib.bim_residual.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int, ctypes.c_void_p]
    lib.bim_last_error.restype = ctypes.c_char_p
    assert lib.bim_residual(None, None, None, 0, None) == -1
    assert b"NULL" in lib.bim_last_error()
