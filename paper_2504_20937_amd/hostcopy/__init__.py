"""Binding of the host-copy comparison renderer (libmm_hostcopy.so): the
frame drawn on host cores from positions copied out of device memory, as a
simulation without device interop would draw it. Only the benchmark and the
tests use it; the device path never does."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MM_HOSTCOPY_LIB names another build of hostcopy.c to load instead (the
# sanitizer test loads one built with AddressSanitizer and UBSan).
LIB_PATH = os.environ.get("MM_HOSTCOPY_LIB") or os.path.join(os.path.dirname(_HERE), "libmm_hostcopy.so")
_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2504_20937_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.hc_render.argtypes = [C.c_void_p, C.c_uint64, C.c_int, C.c_void_p, C.c_uint32,
                                C.c_uint32, C.c_uint32, C.c_uint64, C.c_void_p, C.c_int]
        L.hc_render.restype = C.c_int
        L.hc_max_threads.argtypes = []
        L.hc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def max_threads() -> int:
    return lib().hc_max_threads()


def render(pos: np.ndarray, seed: int, view_proj, width: int, height: int, footprint: int = 1,
           threads: int = 0, out: np.ndarray | None = None) -> np.ndarray:
    """pos: host (N, 2) or (N, 3) float32. Returns the (height, width) uint32 frame."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    m = np.ascontiguousarray(np.asarray(view_proj, dtype=np.float32).reshape(16))
    if out is None:
        out = np.empty((height, width), dtype=np.uint32)
    st = lib().hc_render(pos.ctypes.data, pos.shape[0], pos.shape[1], m.ctypes.data, width, height,
                         footprint, seed, out.ctypes.data, threads)
    if st != 0:
        raise RuntimeError(f"hc_render failed ({st})")
    return out
