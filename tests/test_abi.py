"""CPU checks of the C ABI: the shared library loads and exports every entry point the header
declares, and the Python binding covers them (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gks.h")
LIB = os.path.join(ROOT, "paper_2306_04467_amd", "libgks.so")


def header_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gks_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    syms = header_symbols()
    for name in ("gks_mesh_create", "gks_state_init", "gks_stage", "gks_step"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_header_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in header_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_lists_every_header_symbol():
    from paper_2306_04467_amd import gks

    assert sorted(gks.SYMBOLS) == header_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_last_error_is_callable_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.gks_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.gks_last_error(), bytes)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_handles_are_rejected_on_the_host():
    """Argument checks run before any device call: null handles give GKS_EINVAL and a message."""
    lib = ctypes.CDLL(LIB)
    lib.gks_last_error.restype = ctypes.c_char_p
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64()
    assert lib.gks_mesh_info(vp(), ctypes.byref(i64), None, None, None) == 1
    assert b"null" in lib.gks_last_error()
    assert lib.gks_state_read(vp(), None, None, None) == 1
    assert lib.gks_stage(vp(), 0, None) == 1
    assert lib.gks_mesh_scenario(vp(), 0, None, None) == 1
    assert lib.gks_trainer_info(vp(), None, None) == 1
