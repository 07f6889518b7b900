"""The C-ABI library builds for gfx950, loads, and exports every symbol the header declares."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbffd.h")
LIB = os.path.join(ROOT, "paper_1912_13282_amd", "librbffd.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rbf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_1912_13282_amd import build
        build.build()
    return LIB


def test_header_declares_the_boundary():
    names = declared()
    for n in ["rbf_select_stencils", "rbf_compute_weights", "rbf_assemble_csr", "rbf_ctx_create"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s+(rbf_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_library_loads_with_ctypes(lib_path):
    import ctypes
    L = ctypes.CDLL(lib_path)
    for n in declared():
        assert hasattr(L, n)
    L.rbf_status_string.restype = ctypes.c_char_p
    assert L.rbf_status_string(-4) == b"workspace too small"


def test_host_argument_errors_without_gpu(lib_path):
    """Argument checks run on the host before any device call."""
    import ctypes
    L = ctypes.CDLL(lib_path)
    b = ctypes.c_size_t()
    assert L.rbf_select_stencils_workspace(ctypes.c_int64(1000), 4, 10, ctypes.byref(b)) == -3   # EDIM
    assert L.rbf_select_stencils_workspace(ctypes.c_int64(1000), 3, 10, None) == -1              # EINVAL
    assert L.rbf_select_stencils_workspace(ctypes.c_int64(1000), 3, 10, ctypes.byref(b)) == 0
    assert b.value > 1000 * (4 + 8 * 3)
    assert L.rbf_compute_weights(None, None, ctypes.c_int64(0), 2, None, None, ctypes.c_int64(0), 1, 2, 1,
                                 None, None, None) == -1
