"""CPU-side checks of the C-ABI library: it is built for gfx950, loads, and
exports every entry point include/fos_mc.h declares.  No compute call is
made (there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fos_mc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fos_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2409_00165_amd import fos
    if not os.path.exists(fos.LIB_PATH):
        from paper_2409_00165_amd import build
        build.build()
    return fos.LIB_PATH


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("fos_create", "fos_destroy", "fos_last_error", "fos_mc_prepare", "fos_mc_execute",
                 "fos_mc_run", "fos_philox_words"):
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (fos_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    L = ctypes.CDLL(libpath)
    for n in _declared():
        assert hasattr(L, n)


def test_library_carries_gfx950_code(libpath):
    blob = open(libpath, "rb").read()
    assert b"gfx950" in blob


def test_version_and_status_strings(libpath):
    from paper_2409_00165_amd import fos
    assert fos.fos_abi_version() == 5
    assert fos.fos_status_string(0) == "FOS_OK"
    assert fos.fos_status_string(1) == "FOS_E_INVALID_ARG"
    assert fos.fos_status_string(6) == "FOS_E_NOT_PREPARED"


def test_null_arguments_are_rejected_without_a_device(libpath):
    L = ctypes.CDLL(libpath)
    L.fos_create.argtypes = [ctypes.c_int, ctypes.c_void_p]
    assert L.fos_create(0, None) == 1
    L.fos_destroy.argtypes = [ctypes.c_void_p]
    L.fos_destroy(None)                       # NULL-safe
    L.fos_mc_prepare.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert L.fos_mc_prepare(None, None, None) == 1
    L.fos_mc_execute.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p]
    assert L.fos_mc_execute(None, 0, None, None, None) == 1
    L.fos_last_error.restype = ctypes.c_char_p
    L.fos_last_error.argtypes = [ctypes.c_void_p]
    assert L.fos_last_error(None) == b"null context"
