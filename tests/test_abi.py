"""The C ABI: libaafwi.so loads and exports every entry point that
include/aafwi.h declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aafwi.h")
LIB = os.path.join(ROOT, "paper_2008_11778_amd", "libaafwi.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aafwi_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import shutil
        if not shutil.which("hipcc") and not os.path.exists("/opt/rocm/bin/hipcc"):
            pytest.skip("libaafwi.so not built and no hipcc available")
        import importlib.util
        spec = importlib.util.spec_from_file_location("aafwi_build", os.path.join(ROOT, "paper_2008_11778_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ("aafwi_create", "aafwi_forward_model", "aafwi_adjoint_gradient", "aafwi_born",
                 "aafwi_born_adjoint", "aafwi_aa_step", "aafwi_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_library_is_built_for_gfx950():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    out = subprocess.run(["strings", LIB], capture_output=True, text=True).stdout
    assert "gfx950" in out


def test_last_error_is_callable_without_gpu(lib):
    lib.aafwi_last_error.restype = ctypes.c_char_p
    assert lib.aafwi_last_error() is not None


def test_null_arguments_are_rejected_without_gpu(lib):
    lib.aafwi_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.aafwi_create(None, None, ctypes.byref(out)) == -1
    lib.aafwi_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.aafwi_last_error()
