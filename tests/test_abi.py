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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_mesh_checks_run_on_the_host():
    """gks_mesh_create checks its sizes and builds the host mesh before it touches a device: a size
    above the 32-bit index limit, an unknown boundary kind, clockwise, degenerate and non-manifold
    triangles are all rejected here, without a GPU (the size check reads no array)."""
    import numpy as np

    lib = ctypes.CDLL(LIB)
    lib.gks_last_error.restype = ctypes.c_char_p
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    lib.gks_mesh_create.argtypes = [dp, ctypes.c_int64, ip, ctypes.c_int64, dp, ctypes.c_int32, dp,
                                    ctypes.POINTER(ctypes.c_void_p)]
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.5]], dtype=np.float64)
    tri = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]], dtype=np.int32)
    out = ctypes.c_void_p()

    def create(xy_, tri_, n_tri=None, bc=0):
        return lib.gks_mesh_create(xy_.ctypes.data_as(dp), xy_.shape[0], tri_.ctypes.data_as(ip),
                                   tri_.shape[0] if n_tri is None else n_tri, None, bc, None, ctypes.byref(out))

    assert create(xy, tri, n_tri=(1 << 29) + 1) == 1 and b"32-bit" in lib.gks_last_error()
    assert create(xy, tri, bc=7) == 1 and b"boundary" in lib.gks_last_error()
    assert create(xy, np.ascontiguousarray(tri[:, ::-1])) == 4          # clockwise: GKS_EMESH
    flat = xy.copy()
    flat[4] = [0.5, 0.0]
    assert create(flat, tri) == 4                                        # zero-area triangle
    over = np.concatenate([tri, [[0, 1, 2]]]).astype(np.int32)
    assert create(xy, over) == 4 and b"same direction" in lib.gks_last_error()  # overlapping triangles
    xy3 = np.concatenate([xy, [[0.5, -0.5], [0.5, 0.2]]])
    three = np.concatenate([tri, [[1, 0, 5], [0, 1, 6]]]).astype(np.int32)
    assert create(xy3, three) == 4 and b"more than two" in lib.gks_last_error()  # edge 0-1 in three
    assert not out.value
