"""CPU oracle of the displace+render frame (test infrastructure).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library never
loads it and shares no code with it.

The oracle is plain C (``mm_oracle.c``), built with gcc and FP contraction
off; this module builds it on demand and wraps it for numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mm_oracle.c")
# MM_ORACLE_LIB names another build of mm_oracle.c to load instead (the
# sanitizer test loads one built with AddressSanitizer and UBSan); it is used
# as built, never rebuilt here.
LIB = os.environ.get("MM_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
          "-fexcess-precision=standard", "-fPIC", "-shared", "-Wall", "-Wextra"]
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (also called by the package build)."""
    if os.environ.get("MM_ORACLE_LIB"):
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "mm_oracle.h"))):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        u32p, u64p, f32p = (C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                            C.POINTER(C.c_float))
        L.oracle_philox4x32_10_many.argtypes = [u32p, u32p, u32p, C.c_uint64]
        L.oracle_offset.argtypes = [C.c_uint32, C.c_float]
        L.oracle_offset.restype = C.c_float
        L.oracle_offset_many.argtypes = [u32p, C.c_uint64, C.c_float, f32p]
        L.oracle_wrap.argtypes = [C.c_float]
        L.oracle_wrap.restype = C.c_float
        L.oracle_displace.argtypes = [f32p, C.c_uint64, C.c_uint32, C.c_uint64,
                                      C.c_uint32, C.c_float, C.c_int]
        L.oracle_project.argtypes = [f32p, C.c_uint32, f32p, C.c_uint32, C.c_uint32,
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32), u32p]
        L.oracle_project.restype = C.c_int
        L.oracle_project_many.argtypes = [f32p, C.c_uint64, C.c_uint32, f32p, C.c_uint32,
                                          C.c_uint32, C.POINTER(C.c_int64)]
        L.oracle_splat.argtypes = [f32p, C.c_uint64, C.c_uint32, f32p, C.c_uint32,
                                   C.c_uint32, C.c_uint32, u64p, u64p]
        L.oracle_colour.argtypes = [C.c_uint32, C.c_uint64]
        L.oracle_colour.restype = C.c_uint32
        L.oracle_resolve.argtypes = [u64p, u32p, C.c_uint64, C.c_uint64]
        L.oracle_step_render.argtypes = [f32p, C.c_uint64, C.c_uint32, C.c_uint64,
                                         C.c_uint32, C.c_float, C.c_int, f32p,
                                         C.c_uint32, C.c_uint32, C.c_uint32, u64p, u32p]
        L.oracle_screen.argtypes = [f32p, C.c_uint32, f32p, C.c_uint32, C.c_uint32,
                                    f32p, f32p, f32p]
        L.oracle_screen.restype = C.c_int
        L.oracle_splat_edges.argtypes = [f32p, C.c_uint64, C.c_uint32, u32p, C.c_uint64,
                                         C.c_uint32, f32p, C.c_uint32, C.c_uint32, u64p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(ctype))


def _mat(m) -> np.ndarray:
    m = np.ascontiguousarray(np.asarray(m, dtype=np.float32).reshape(16))
    return m


def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """ctr (n, 4) uint32, key (n, 2) uint32 -> (n, 4) uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    assert ctr.shape[0] == key.shape[0]
    out = np.empty_like(ctr)
    lib().oracle_philox4x32_10_many(_ptr(ctr, C.c_uint32), _ptr(key, C.c_uint32),
                                    _ptr(out, C.c_uint32), ctr.shape[0])
    return out


def offset(r: int, a: float) -> float:
    return lib().oracle_offset(r, a)


def offset_many(r: np.ndarray, a: float) -> np.ndarray:
    r = np.ascontiguousarray(r, dtype=np.uint32)
    out = np.empty(r.shape, dtype=np.float32)
    lib().oracle_offset_many(_ptr(r, C.c_uint32), r.size, a, _ptr(out, C.c_float))
    return out


def wrap(x: float) -> float:
    return lib().oracle_wrap(x)


def displace(pos: np.ndarray, seed: int, step: int, a: float, wrap: bool) -> None:
    """In place on a C-contiguous float32 (n, dim) array."""
    assert pos.dtype == np.float32 and pos.ndim == 2
    lib().oracle_displace(_ptr(pos, C.c_float), pos.shape[0], pos.shape[1], seed,
                          step, a, int(wrap))


def project(p, m, width: int, height: int):
    """Returns (px, py, depth_bits) or None when the point is culled."""
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float32).reshape(-1))
    m = _mat(m)
    px, py, bits = C.c_int32(), C.c_int32(), C.c_uint32()
    ok = lib().oracle_project(_ptr(p, C.c_float), p.shape[0], _ptr(m, C.c_float),
                              width, height, C.byref(px), C.byref(py), C.byref(bits))
    return (px.value, py.value, bits.value) if ok else None


def project_many(pos: np.ndarray, m, width: int, height: int) -> np.ndarray:
    """Pixel index py * width + px of every point of an (n, dim) float32
    array, -1 for points off screen (the projection of ``project``)."""
    assert pos.dtype == np.float32 and pos.ndim == 2 and pos.flags.c_contiguous
    m = _mat(m)
    out = np.empty(pos.shape[0], dtype=np.int64)
    lib().oracle_project_many(_ptr(pos, C.c_float), pos.shape[0], pos.shape[1],
                              _ptr(m, C.c_float), width, height, _ptr(out, C.c_int64))
    return out


def new_depth(width: int, height: int) -> np.ndarray:
    return np.full(width * height, EMPTY, dtype=np.uint64)


def splat(pos: np.ndarray, m, width: int, height: int, footprint: int,
          depth: np.ndarray, order: np.ndarray | None = None) -> None:
    assert pos.dtype == np.float32 and depth.dtype == np.uint64
    m = _mat(m)
    optr = None
    if order is not None:
        order = np.ascontiguousarray(order, dtype=np.uint64)
        assert order.shape[0] == pos.shape[0]
        optr = _ptr(order, C.c_uint64)
    lib().oracle_splat(_ptr(pos, C.c_float), pos.shape[0], pos.shape[1], _ptr(m, C.c_float),
                       width, height, footprint, _ptr(depth, C.c_uint64), optr)


def colour(index: int, seed: int) -> int:
    return lib().oracle_colour(index, seed)


def resolve(depth: np.ndarray, seed: int) -> np.ndarray:
    out = np.empty(depth.shape[0], dtype=np.uint32)
    lib().oracle_resolve(_ptr(depth, C.c_uint64), _ptr(out, C.c_uint32), depth.shape[0], seed)
    return out


def step_render(pos: np.ndarray, seed: int, step: int, a: float, wrap: bool, m,
                width: int, height: int, footprint: int,
                depth: np.ndarray | None = None) -> np.ndarray:
    """Displace pos in place with step, then render; returns the RGBA8 frame
    as (height, width) uint32."""
    if depth is None:
        depth = new_depth(width, height)
    m = _mat(m)
    out = np.empty(width * height, dtype=np.uint32)
    lib().oracle_step_render(_ptr(pos, C.c_float), pos.shape[0], pos.shape[1], seed, step,
                             a, int(wrap), _ptr(m, C.c_float), width, height, footprint,
                             _ptr(depth, C.c_uint64), _ptr(out, C.c_uint32))
    return out.reshape(height, width)


def render(pos: np.ndarray, seed: int, m, width: int, height: int,
           footprint: int) -> np.ndarray:
    """Splat + resolve without displacement."""
    depth = new_depth(width, height)
    splat(pos, m, width, height, footprint, depth)
    return resolve(depth, seed).reshape(height, width)


def palette_colours(keys: np.ndarray, palette: np.ndarray,
                    indices: np.ndarray | None = None) -> np.ndarray:
    """Colours of resolved keys under a palette (section "Views": a colour
    property read per element, or through an index description into a
    table). A pixel with no point is 0. Otherwise i is the winning point's
    index (low word of its key); j = indices[i], or i without indices; the
    colour is palette[j], or 0 when j is past the palette's end.
    palette: uint32 RGBA8 entries; indices: unsigned integers per point."""
    keys = np.asarray(keys, dtype=np.uint64)
    palette = np.asarray(palette, dtype=np.uint32)
    out = np.zeros(keys.shape, dtype=np.uint32)
    drawn = keys != EMPTY
    i = (keys[drawn] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    j = np.asarray(indices)[i].astype(np.int64) if indices is not None else i
    inside = j < palette.shape[0]
    c = np.zeros(i.shape, dtype=np.uint32)
    c[inside] = palette[j[inside]]
    out[drawn] = c
    return out


def render_palette(pos: np.ndarray, m, width: int, height: int, footprint: int,
                   palette: np.ndarray, indices: np.ndarray | None = None) -> np.ndarray:
    """Splat without displacement, then the palette colours of the keys."""
    depth = new_depth(width, height)
    splat(pos, m, width, height, footprint, depth)
    return palette_colours(depth, palette, indices).reshape(height, width)


def render_grid(cols: int, rows: int, width: int, height: int, palette: np.ndarray,
                cells: np.ndarray) -> np.ndarray:
    """Structured-grid frame (the voxel view of a 2D lattice, section "Potts
    model": cell states drawn through a colormap). Pixel (px, py), row 0 at
    the top, shows the cell whose area holds the pixel centre: column
    floor((px + 1/2) cols / width), row floor((height - 1 - py + 1/2) rows /
    height) counted from the bottom; colour palette[value], or 0 when the
    value is past the palette. cells: cols * rows values, row-major from the
    bottom row. Returns (height, width) uint32."""
    palette = np.asarray(palette, dtype=np.uint32)
    cells = np.asarray(cells).reshape(-1).astype(np.int64)
    px = np.arange(width, dtype=np.int64)
    py = np.arange(height, dtype=np.int64)
    cx = (2 * px + 1) * cols // (2 * width)
    cy = (2 * (height - 1 - py) + 1) * rows // (2 * height)
    v = cells[cy[:, None] * cols + cx[None, :]]
    inside = v < palette.shape[0]
    return np.where(inside, palette[np.where(inside, v, 0)], 0).astype(np.uint32)


def screen(p, m, width: int, height: int):
    """(sx, sy, w) of a vertex before the pixel floor, or None when near-culled."""
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float32).reshape(-1))
    m = _mat(m)
    sx, sy, w = C.c_float(), C.c_float(), C.c_float()
    ok = lib().oracle_screen(_ptr(p, C.c_float), p.shape[0], _ptr(m, C.c_float), width, height,
                             C.byref(sx), C.byref(sy), C.byref(w))
    return (sx.value, sy.value, w.value) if ok else None


def render_edges(pos: np.ndarray, idx: np.ndarray, prim: int, seed: int, m, width: int,
                 height: int, depth: np.ndarray | None = None) -> np.ndarray:
    """Edges view frame: segments between indexed vertices (pairs, prim 2, or
    triangle sides, prim 3) sampled as oracle_splat_edge defines, resolved
    with the hash colour of the winning edge index."""
    assert pos.dtype == np.float32 and pos.ndim == 2
    idx = np.ascontiguousarray(idx, dtype=np.uint32).reshape(-1)
    assert idx.shape[0] % prim == 0
    if depth is None:
        depth = new_depth(width, height)
    lib().oracle_splat_edges(_ptr(pos, C.c_float), pos.shape[0], pos.shape[1],
                             _ptr(idx, C.c_uint32), idx.shape[0] // prim, prim, _ptr(_mat(m), C.c_float),
                             width, height, _ptr(depth, C.c_uint64))
    return resolve(depth, seed).reshape(height, width)
