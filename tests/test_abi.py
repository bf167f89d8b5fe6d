"""The C-ABI library loads and exports every entry point that include/dycore.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dycore.h")
LIB = os.path.join(ROOT, "paper_2103_10114_amd", "libdycore.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+(dycore_[a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["dycore_create", "dycore_destroy", "dycore_step", "dycore_step_adjoint", "dycore_stage",
              "dycore_stage_adjoint", "dycore_diagnostics", "dycore_batch_create", "dycore_batch_step"]:
        assert n in names


def test_library_exports_every_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libdycore.so not built")
    L = ctypes.CDLL(LIB)          # fails on any undefined symbol
    for n in declared_functions():
        assert hasattr(L, n), n


def test_strerror_and_invalid_config_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("libdycore.so not built")
    L = ctypes.CDLL(LIB)
    L.dycore_strerror.restype = ctypes.c_char_p
    assert L.dycore_strerror(0) == b"ok"
    assert L.dycore_strerror(-1) == b"invalid argument"
    # a NULL config is rejected before any device call
    h = ctypes.c_void_p()
    assert L.dycore_create(None, ctypes.byref(h)) == -1
