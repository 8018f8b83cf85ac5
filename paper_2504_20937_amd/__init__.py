"""Python binding of libmm (the MI355X displace+render library).

A thin ctypes layer over the C ABI declared in ``include/mm.h``: the same
function names, arguments marshalled, errors raised as ``MMError``. Every
step of the frame runs in the library's HIP kernels; this module computes
nothing. Device memory and streams may come from PyTorch (pass
``tensor.data_ptr()`` and ``torch.cuda.current_stream().cuda_stream``), but
this module does not import torch.

The shared library must have been built (``python -m
paper_2504_20937_amd.build`` or ``__graft_entry__.build()``); importing the
binding without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MM_LIB names another build of the same library (e.g. one with host-side
# sanitizers, for tests)
LIB_PATH = os.environ.get("MM_LIB") or os.path.join(_HERE, "libmm.so")

MM_OK = 0
MM_ERR_INVALID_ARG = -1
MM_ERR_OUT_OF_MEMORY = -2
MM_ERR_HIP = -3
MM_ERR_BUDGET = -4
MM_ERR_IN_USE = -5
MM_ERR_UNSUPPORTED = -6
MM_ERR_NOT_READY = -7

MM_FLOAT2 = 2
MM_FLOAT3 = 3
MM_SPLAT_AUTO = 0
MM_SPLAT_DIRECT = 1
MM_SPLAT_BINNED = 2
MM_PIECES_STATIC = 0xFFFFFFFF
MM_CULL_AUTO, MM_CULL_ON, MM_CULL_OFF = 0, 1, 2
MM_DOMAIN_2D = 2
MM_DOMAIN_3D = 3


class MMError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {status_name(status)} ({status}): {detail}")
        self.status = status


class mm_instance_desc(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p)]


class mm_view_desc(C.Structure):
    _fields_ = [
        ("position", C.c_void_p),
        ("element_count", C.c_uint64),
        ("format", C.c_int),
        ("domain", C.c_int),
        ("width", C.c_uint32),
        ("height", C.c_uint32),
        ("footprint", C.c_uint32),
        ("seed", C.c_uint64),
        ("amplitude", C.c_float),
        ("wrap", C.c_int32),
        ("view_proj", C.c_float * 16),
    ]


class mm_tuning(C.Structure):
    _fields_ = [("splat", C.c_uint32), ("tile", C.c_uint32), ("points_per_thread", C.c_uint32),
                ("splits", C.c_uint32), ("bin_threads", C.c_uint32),
                ("piece_records", C.c_uint32), ("occlusion_cull", C.c_uint32)]


class mm_colour_desc(C.Structure):
    _fields_ = [
        ("palette", C.c_void_p),
        ("palette_size", C.c_uint32),
        ("indices", C.c_void_p),
        ("index_size", C.c_uint32),
    ]


class mm_grid_desc(C.Structure):
    _fields_ = [
        ("cols", C.c_uint32), ("rows", C.c_uint32),
        ("width", C.c_uint32), ("height", C.c_uint32),
        ("palette", C.c_void_p), ("palette_size", C.c_uint32),
        ("indices", C.c_void_p), ("index_size", C.c_uint32),
    ]


class mm_edges_desc(C.Structure):
    _fields_ = [
        ("position", C.c_void_p),
        ("element_count", C.c_uint64),
        ("format", C.c_int),
        ("domain", C.c_int),
        ("indices", C.c_void_p),
        ("primitive_count", C.c_uint64),
        ("vertices_per_primitive", C.c_uint32),
        ("width", C.c_uint32),
        ("height", C.c_uint32),
        ("seed", C.c_uint64),
        ("view_proj", C.c_float * 16),
    ]


class mm_cloud_desc(C.Structure):
    _fields_ = [
        ("position", C.c_void_p),
        ("element_count", C.c_uint64),
        ("format", C.c_int),
        ("seed", C.c_uint64),
        ("amplitude", C.c_float),
        ("wrap", C.c_int32),
    ]


class mm_batch_view_desc(C.Structure):
    _fields_ = [
        ("cloud", C.c_uint32),
        ("width", C.c_uint32),
        ("height", C.c_uint32),
        ("view_proj", C.c_float * 16),
    ]


class mm_batch_desc(C.Structure):
    _fields_ = [
        ("domain", C.c_int),
        ("footprint", C.c_uint32),
        ("n_clouds", C.c_uint32),
        ("clouds", C.POINTER(mm_cloud_desc)),
        ("n_views", C.c_uint32),
        ("views", C.POINTER(mm_batch_view_desc)),
    ]


class mm_batch_tuning(C.Structure):
    _fields_ = [("tile", C.c_uint32), ("points_per_thread", C.c_uint32), ("splits", C.c_uint32),
                ("grid_blocks", C.c_uint32), ("bin_threads", C.c_uint32)]


class mm_server_desc(C.Structure):
    _fields_ = [
        ("fb_budget_bytes", C.c_uint64),
        ("streams", C.c_uint32),
        ("max_batch", C.c_uint32),
        ("domain", C.c_int),
        ("footprint", C.c_uint32),
        ("tuning", mm_batch_tuning),
    ]


class mm_static_frame_desc(C.Structure):
    _fields_ = [
        ("dev_positions", C.c_void_p),
        ("element_count", C.c_uint64),
        ("domain", C.c_int32),
        ("width", C.c_uint32),
        ("height", C.c_uint32),
        ("footprint", C.c_uint32),
        ("seed", C.c_uint64),
        ("amplitude", C.c_float),
        ("wrap", C.c_int32),
        ("step", C.c_uint32),
        ("view_proj", C.c_float * 16),
        ("dev_rgba", C.c_void_p),
        ("stream", C.c_void_p),
    ]


class mm_server_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "completed", "launches",
                                           "admitted_sessions", "admissions", "evictions",
                                           "fb_bytes_in_use", "queued", "dropped",
                                           "max_in_flight", "max_batch")]


_lib = None
_status = C.c_int32
_vp = C.c_void_p


def _declare(L):
    sig = {
        "mm_version": ([], C.c_int32),
        "mm_last_error": ([], C.c_char_p),
        "mm_status_string": ([C.c_int32], C.c_char_p),
        "mm_create_instance": ([C.POINTER(mm_instance_desc), C.POINTER(_vp)], _status),
        "mm_destroy_instance": ([_vp], _status),
        "mm_synchronize": ([_vp], _status),
        "mm_alloc_linear": ([_vp, C.c_size_t, C.POINTER(_vp), C.POINTER(_vp)], _status),
        "mm_alloc_wrap": ([_vp, _vp, C.c_size_t, C.POINTER(_vp)], _status),
        "mm_free": ([_vp], _status),
        "mm_create_view": ([_vp, C.POINTER(mm_view_desc), C.POINTER(_vp)], _status),
        "mm_destroy_view": ([_vp], _status),
        "mm_set_camera": ([_vp, C.POINTER(C.c_float)], _status),
        "mm_step": ([_vp, C.c_uint32], _status),
        "mm_render": ([_vp], _status),
        "mm_step_render": ([_vp, C.c_uint32], _status),
        "mm_step_render_frames": ([_vp, C.c_uint32, C.c_uint32, C.POINTER(C.c_float)], _status),
        "mm_set_frame_overlap": ([_vp, C.c_uint32], _status),
        "mm_set_colour": ([_vp, C.POINTER(mm_colour_desc)], _status),
        "mm_create_grid": ([_vp, C.POINTER(mm_grid_desc), C.POINTER(_vp)], _status),
        "mm_create_edges": ([_vp, C.POINTER(mm_edges_desc), C.POINTER(_vp)], _status),
        "mm_destroy_edges": ([_vp], _status),
        "mm_edges_set_camera": ([_vp, C.POINTER(C.c_float)], _status),
        "mm_edges_render": ([_vp], _status),
        "mm_edges_frame_device_ptr": ([_vp, C.POINTER(_vp)], _status),
        "mm_edges_read_frame": ([_vp, _vp, C.c_size_t], _status),
        "mm_destroy_grid": ([_vp], _status),
        "mm_grid_render": ([_vp], _status),
        "mm_grid_frame_device_ptr": ([_vp, C.POINTER(_vp)], _status),
        "mm_grid_read_frame": ([_vp, _vp, C.c_size_t], _status),
        "mm_flush_frame": ([_vp], _status),
        "mm_frame_device_ptr": ([_vp, C.POINTER(_vp)], _status),
        "mm_read_frame": ([_vp, _vp, C.c_size_t], _status),
        "mm_set_tuning": ([_vp, C.POINTER(mm_tuning)], _status),
        "mm_get_tuning": ([_vp, C.POINTER(mm_tuning)], _status),
        "mm_profile_begin": ([_vp, C.c_uint32], _status),
        "mm_profile_every": ([_vp, C.c_uint32], _status),
        "mm_step_render_static": ([C.POINTER(mm_static_frame_desc)], _status),
        "mm_debug_fail_allocations": ([C.c_int64], _status),
        "mm_mark_begin": ([_vp, C.c_uint32], _status),
        "mm_mark_end": ([_vp], _status),
        "mm_mark_read": ([_vp, C.POINTER(C.c_float), C.POINTER(C.c_uint32)], _status),
        "mm_prepare_views": ([_vp, _vp], _status),
        "mm_update_views": ([_vp, _vp], _status),
        "mm_profile_end": ([_vp, C.POINTER(C.c_float), C.POINTER(C.c_float),
                            C.POINTER(C.c_float), C.POINTER(C.c_uint32)], _status),
        "mm_autotune": ([_vp, C.c_uint32, C.POINTER(mm_tuning)], _status),
        "mm_batch_autotune": ([_vp, C.c_uint32, C.POINTER(mm_batch_tuning)], _status),
        "mm_create_server": ([_vp, C.POINTER(mm_server_desc), C.POINTER(_vp)], _status),
        "mm_destroy_server": ([_vp], _status),
        "mm_server_add_cloud": ([_vp, C.POINTER(mm_cloud_desc), C.POINTER(C.c_uint32)], _status),
        "mm_server_submit": ([_vp, C.c_uint32, C.c_uint32, C.POINTER(C.c_float), C.c_uint32,
                              C.c_uint32, _vp, C.POINTER(C.c_uint64)], _status),
        "mm_server_poll": ([_vp, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double)], _status),
        "mm_server_wait": ([_vp, C.c_uint64, C.POINTER(C.c_double)], _status),
        "mm_server_read_frame": ([_vp, C.c_uint32, _vp, C.c_size_t], _status),
        "mm_server_close_session": ([_vp, C.c_uint32], _status),
        "mm_server_stats_get": ([_vp, C.POINTER(mm_server_stats)], _status),
        "mm_create_batch": ([_vp, C.POINTER(mm_batch_desc), C.POINTER(_vp)], _status),
        "mm_destroy_batch": ([_vp], _status),
        "mm_batch_set_camera": ([_vp, C.c_uint32, C.POINTER(C.c_float)], _status),
        "mm_batch_set_cameras": ([_vp, C.c_uint32, C.c_uint32, C.POINTER(C.c_float)], _status),
        "mm_batch_step_render": ([_vp, C.c_uint32], _status),
        "mm_batch_render": ([_vp], _status),
        "mm_batch_frame_device_ptr": ([_vp, C.c_uint32, C.POINTER(_vp)], _status),
        "mm_batch_read_frame": ([_vp, C.c_uint32, _vp, C.c_size_t], _status),
        "mm_batch_set_tuning": ([_vp, C.POINTER(mm_batch_tuning)], _status),
        "mm_batch_get_tuning": ([_vp, C.POINTER(mm_batch_tuning)], _status),
        "mm_batch_profile_begin": ([_vp, C.c_uint32], _status),
        "mm_batch_profile_end": ([_vp, C.POINTER(C.c_float), C.POINTER(C.c_uint32)], _status),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res


def lib() -> C.CDLL:
    """The loaded libmm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2504_20937_amd.build`")
        L = C.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def status_name(status: int) -> str:
    return lib().mm_status_string(status).decode()


def mm_last_error() -> str:
    return lib().mm_last_error().decode()


def mm_status_string(status: int) -> str:
    return status_name(status)


def mm_version() -> int:
    return lib().mm_version()


def _check(status: int, where: str) -> None:
    if status != MM_OK:
        raise MMError(status, where, mm_last_error())


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


# ------------------------------------------------------------------ instance
def mm_create_instance(device: int = 0, stream: int | None = None) -> int:
    desc = mm_instance_desc(device, stream or None)
    out = _vp()
    _check(lib().mm_create_instance(C.byref(desc), C.byref(out)), "mm_create_instance")
    return out.value


def mm_destroy_instance(inst: int) -> None:
    _check(lib().mm_destroy_instance(inst), "mm_destroy_instance")


def mm_synchronize(inst: int) -> None:
    _check(lib().mm_synchronize(inst), "mm_synchronize")


# --------------------------------------------------------------- allocations
def mm_prepare_views(inst: int, stream: int | None = None) -> None:
    """Start of a compute section: `stream` waits for the instance's work so far."""
    _check(lib().mm_prepare_views(inst, stream), "mm_prepare_views")


def mm_update_views(inst: int, stream: int | None = None) -> None:
    """End of a compute section: the instance's later work waits for `stream`."""
    _check(lib().mm_update_views(inst, stream), "mm_update_views")


def mm_alloc_linear(inst: int, nbytes: int) -> tuple[int, int]:
    """Returns (device pointer, alloc handle)."""
    ptr, out = _vp(), _vp()
    _check(lib().mm_alloc_linear(inst, nbytes, C.byref(ptr), C.byref(out)), "mm_alloc_linear")
    return ptr.value, out.value


def mm_alloc_wrap(inst: int, dev_ptr: int, nbytes: int) -> int:
    out = _vp()
    _check(lib().mm_alloc_wrap(inst, dev_ptr, nbytes, C.byref(out)), "mm_alloc_wrap")
    return out.value


def mm_free(alloc: int) -> None:
    _check(lib().mm_free(alloc), "mm_free")


# --------------------------------------------------------------------- views
def make_view_desc(position: int, element_count: int, dim: int, width: int, height: int,
                   footprint: int = 1, seed: int = 0, amplitude: float = 0.0,
                   wrap: bool = False, view_proj=None) -> mm_view_desc:
    d = mm_view_desc()
    d.position = position
    d.element_count = element_count
    d.format = MM_FLOAT2 if dim == 2 else MM_FLOAT3
    d.domain = MM_DOMAIN_2D if dim == 2 else MM_DOMAIN_3D
    d.width, d.height, d.footprint = width, height, footprint
    d.seed = seed
    d.amplitude = amplitude
    d.wrap = int(bool(wrap))
    m = np.eye(4, dtype=np.float32) if view_proj is None else view_proj
    m = np.ascontiguousarray(np.asarray(m, dtype=np.float32).reshape(16))
    for k in range(16):
        d.view_proj[k] = float(m[k])
    return d


def mm_create_view(inst: int, desc: mm_view_desc) -> int:
    out = _vp()
    _check(lib().mm_create_view(inst, C.byref(desc), C.byref(out)), "mm_create_view")
    return out.value


def mm_destroy_view(view: int) -> None:
    _check(lib().mm_destroy_view(view), "mm_destroy_view")


def mm_set_tuning(view: int, splat: int = MM_SPLAT_AUTO, tile: int = 0,
                  points_per_thread: int = 0, splits: int = 0, bin_threads: int = 0,
                  piece_records: int = 0, occlusion_cull: int = 0) -> None:
    t = mm_tuning(splat, tile, points_per_thread, splits, bin_threads, piece_records,
                  occlusion_cull)
    _check(lib().mm_set_tuning(view, C.byref(t)), "mm_set_tuning")


def _tuning_tuple(t: mm_tuning) -> tuple:
    return (t.splat, t.tile, t.points_per_thread, t.splits, t.bin_threads, t.piece_records,
            t.occlusion_cull)


def mm_get_tuning(view: int) -> tuple[int, int, int, int, int, int, int]:
    """(splat, tile, points_per_thread, splits, bin_threads, piece_records,
    occlusion_cull) in use."""
    t = mm_tuning()
    _check(lib().mm_get_tuning(view, C.byref(t)), "mm_get_tuning")
    return _tuning_tuple(t)


def mm_autotune(view: int, frames: int = 10) -> tuple[int, int, int, int, int, int, int]:
    """Times the supported shapes, keeps the fastest; returns it as mm_get_tuning does."""
    t = mm_tuning()
    _check(lib().mm_autotune(view, frames, C.byref(t)), "mm_autotune")
    return _tuning_tuple(t)


def mm_set_camera(view: int, view_proj) -> None:
    m = np.ascontiguousarray(np.asarray(view_proj, dtype=np.float32).reshape(16))
    _check(lib().mm_set_camera(view, _fptr(m)), "mm_set_camera")


def mm_step(view: int, step: int) -> None:
    _check(lib().mm_step(view, step), "mm_step")


def mm_render(view: int) -> None:
    _check(lib().mm_render(view), "mm_render")


def mm_step_render_frames(view: int, first_step: int, count: int, cameras=None) -> None:
    """`count` frames (steps first_step ..) in one graph launch; cameras: None
    or `count` 4x4 row-major matrices."""
    if cameras is None:
        _check(lib().mm_step_render_frames(view, first_step, count, None), "mm_step_render_frames")
        return
    m = np.ascontiguousarray(np.asarray(cameras, dtype=np.float32).reshape(-1))
    if m.size != 16 * count:
        raise ValueError(f"{count} frames need {16 * count} camera floats, got {m.size}")
    _check(lib().mm_step_render_frames(view, first_step, count, _fptr(m)), "mm_step_render_frames")


def mm_step_render(view: int, step: int) -> None:
    _check(lib().mm_step_render(view, step), "mm_step_render")


def mm_set_colour(view: int, palette=None, palette_size: int = 0, indices=None,
                  index_size: int = 0) -> None:
    """Colour source of the view: palette (an mm_alloc of RGBA8 entries) read
    through indices (an mm_alloc of index_size-byte integers) or by point
    index; palette None restores the default hash colour."""
    if palette is None:
        _check(lib().mm_set_colour(view, None), "mm_set_colour")
        return
    d = mm_colour_desc(palette, palette_size, indices, index_size)
    _check(lib().mm_set_colour(view, C.byref(d)), "mm_set_colour")


def mm_create_grid(inst: int, cols: int, rows: int, width: int, height: int, palette,
                   palette_size: int, indices, index_size: int) -> int:
    """Structured-grid view: a cols x rows lattice of cell values (indices, an
    mm_alloc) drawn through palette (an mm_alloc of RGBA8 entries)."""
    d = mm_grid_desc(cols, rows, width, height, palette, palette_size, indices, index_size)
    out = _vp()
    _check(lib().mm_create_grid(inst, C.byref(d), C.byref(out)), "mm_create_grid")
    return out.value


def mm_destroy_grid(grid: int) -> None:
    _check(lib().mm_destroy_grid(grid), "mm_destroy_grid")


def mm_grid_render(grid: int) -> None:
    _check(lib().mm_grid_render(grid), "mm_grid_render")


def mm_grid_frame_device_ptr(grid: int) -> int:
    out = _vp()
    _check(lib().mm_grid_frame_device_ptr(grid, C.byref(out)), "mm_grid_frame_device_ptr")
    return out.value


def mm_grid_read_frame(grid: int, width: int, height: int) -> np.ndarray:
    out = np.empty((height, width), dtype=np.uint32)
    _check(lib().mm_grid_read_frame(grid, out.ctypes.data, out.nbytes), "mm_grid_read_frame")
    return out


def mm_create_edges(inst: int, position, n: int, dim: int, indices, nprim: int, prim: int,
                    width: int, height: int, seed: int, view_proj=None) -> int:
    """Edges view over n vertices (position, an mm_alloc) joined by nprim
    vertex pairs (prim 2) or triangles (prim 3) of uint32 indices (an mm_alloc)."""
    m = np.eye(4, dtype=np.float32).reshape(16) if view_proj is None else \
        np.ascontiguousarray(np.asarray(view_proj, dtype=np.float32).reshape(16))
    d = mm_edges_desc(position, n, dim, dim, indices, nprim, prim, width, height, seed,
                      (C.c_float * 16)(*m.tolist()))
    out = _vp()
    _check(lib().mm_create_edges(inst, C.byref(d), C.byref(out)), "mm_create_edges")
    return out.value


def mm_destroy_edges(view: int) -> None:
    _check(lib().mm_destroy_edges(view), "mm_destroy_edges")


def mm_edges_set_camera(view: int, view_proj) -> None:
    m = np.ascontiguousarray(np.asarray(view_proj, dtype=np.float32).reshape(16))
    _check(lib().mm_edges_set_camera(view, m.ctypes.data_as(C.POINTER(C.c_float))),
           "mm_edges_set_camera")


def mm_edges_render(view: int) -> None:
    _check(lib().mm_edges_render(view), "mm_edges_render")


def mm_edges_frame_device_ptr(view: int) -> int:
    out = _vp()
    _check(lib().mm_edges_frame_device_ptr(view, C.byref(out)), "mm_edges_frame_device_ptr")
    return out.value


def mm_edges_read_frame(view: int, width: int, height: int) -> np.ndarray:
    out = np.empty((height, width), dtype=np.uint32)
    _check(lib().mm_edges_read_frame(view, out.ctypes.data, out.nbytes), "mm_edges_read_frame")
    return out


def mm_set_frame_overlap(view: int, on: bool) -> None:
    """Frame overlap: frame f is binned while frame f - 1 is drawn; the frame
    buffer then lags mm_step_render by one frame until mm_flush_frame."""
    _check(lib().mm_set_frame_overlap(view, int(on)), "mm_set_frame_overlap")


def mm_flush_frame(view: int) -> None:
    _check(lib().mm_flush_frame(view), "mm_flush_frame")


def mm_frame_device_ptr(view: int) -> int:
    out = _vp()
    _check(lib().mm_frame_device_ptr(view, C.byref(out)), "mm_frame_device_ptr")
    return out.value


def mm_read_frame(view: int, width: int, height: int) -> np.ndarray:
    """The view's RGBA8 frame as a (height, width) uint32 array (synchronises)."""
    out = np.empty((height, width), dtype=np.uint32)
    _check(lib().mm_read_frame(view, out.ctypes.data, out.nbytes), "mm_read_frame")
    return out


def mm_profile_every(view: int, every: int) -> None:
    _check(lib().mm_profile_every(view, every), "mm_profile_every")


def mm_profile_begin(view: int, capacity: int) -> None:
    _check(lib().mm_profile_begin(view, capacity), "mm_profile_begin")


def mm_profile_end(view: int, capacity: int):
    """Returns (splat_ms, resolve_ms, frame_ms) float32 arrays of the recorded frames."""
    s = np.zeros(capacity, dtype=np.float32)
    r = np.zeros(capacity, dtype=np.float32)
    f = np.zeros(capacity, dtype=np.float32)
    n = C.c_uint32()
    _check(lib().mm_profile_end(view, _fptr(s), _fptr(r), _fptr(f), C.byref(n)),
           "mm_profile_end")
    k = n.value
    return s[:k], r[:k], f[:k]


def mm_mark_begin(view: int, capacity: int) -> None:
    _check(lib().mm_mark_begin(view, capacity), "mm_mark_begin")


def mm_mark_end(view: int) -> None:
    _check(lib().mm_mark_end(view), "mm_mark_end")


def mm_mark_read(view: int, capacity: int) -> np.ndarray:
    """Intervals (ms) between consecutive frame marks: one per marked frame
    (a loop of K frames takes capacity K + 1)."""
    out = np.zeros(max(1, capacity - 1), dtype=np.float32)
    n = C.c_uint32()
    _check(lib().mm_mark_read(view, _fptr(out), C.byref(n)), "mm_mark_read")
    return out[:n.value]


def mm_debug_fail_allocations(after: int) -> None:
    """Lets `after` library allocations succeed and fails the next one (tests)."""
    _check(lib().mm_debug_fail_allocations(after), "mm_debug_fail_allocations")


def mm_step_render_static(dev_positions: int, element_count: int, dim: int, width: int,
                          height: int, dev_rgba: int, step: int, footprint: int = 1,
                          seed: int = 0, amplitude: float = 0.0, wrap: bool = False,
                          view_proj=None, stream: int = 0) -> None:
    """One direct-splat frame with no allocation (keys in the library's static array)."""
    d = mm_static_frame_desc()
    d.dev_positions = dev_positions
    d.element_count = element_count
    d.domain = MM_DOMAIN_2D if dim == 2 else MM_DOMAIN_3D
    d.width, d.height, d.footprint = width, height, footprint
    d.seed, d.amplitude, d.wrap, d.step = seed, amplitude, int(bool(wrap)), step
    m = np.eye(4, dtype=np.float32) if view_proj is None else view_proj
    m = np.ascontiguousarray(np.asarray(m, dtype=np.float32).reshape(16))
    for k in range(16):
        d.view_proj[k] = float(m[k])
    d.dev_rgba = dev_rgba
    d.stream = stream or None
    _check(lib().mm_step_render_static(C.byref(d)), "mm_step_render_static")


# ------------------------------------------------------------------- batches
def make_cloud_desc(position: int, element_count: int, dim: int, seed: int = 0,
                    amplitude: float = 0.0, wrap: bool = False) -> mm_cloud_desc:
    c = mm_cloud_desc()
    c.position = position
    c.element_count = element_count
    c.format = MM_FLOAT2 if dim == 2 else MM_FLOAT3
    c.seed = seed
    c.amplitude = amplitude
    c.wrap = int(bool(wrap))
    return c


def make_batch_view_desc(cloud: int, width: int, height: int,
                         view_proj=None) -> mm_batch_view_desc:
    v = mm_batch_view_desc()
    v.cloud, v.width, v.height = cloud, width, height
    m = np.eye(4, dtype=np.float32) if view_proj is None else view_proj
    m = np.ascontiguousarray(np.asarray(m, dtype=np.float32).reshape(16))
    for k in range(16):
        v.view_proj[k] = float(m[k])
    return v


def mm_create_batch(inst: int, dim: int, footprint: int, clouds, views) -> int:
    """clouds: sequence of mm_cloud_desc; views: sequence of mm_batch_view_desc."""
    ca = (mm_cloud_desc * max(1, len(clouds)))(*clouds)
    va = (mm_batch_view_desc * max(1, len(views)))(*views)
    d = mm_batch_desc()
    d.domain = MM_DOMAIN_2D if dim == 2 else MM_DOMAIN_3D
    d.footprint = footprint
    d.n_clouds, d.clouds = len(clouds), ca
    d.n_views, d.views = len(views), va
    out = _vp()
    _check(lib().mm_create_batch(inst, C.byref(d), C.byref(out)), "mm_create_batch")
    return out.value


def mm_destroy_batch(batch: int) -> None:
    _check(lib().mm_destroy_batch(batch), "mm_destroy_batch")


def mm_batch_set_camera(batch: int, view: int, view_proj) -> None:
    m = np.ascontiguousarray(np.asarray(view_proj, dtype=np.float32).reshape(16))
    _check(lib().mm_batch_set_camera(batch, view, _fptr(m)), "mm_batch_set_camera")


def mm_batch_set_cameras(batch: int, first: int, view_proj) -> None:
    """view_proj: (count, 4, 4) or (count, 16) float32, for views first.. first+count-1."""
    m = np.ascontiguousarray(np.asarray(view_proj, dtype=np.float32).reshape(-1, 16))
    _check(lib().mm_batch_set_cameras(batch, first, m.shape[0], _fptr(m)), "mm_batch_set_cameras")


def mm_batch_step_render(batch: int, step: int) -> None:
    _check(lib().mm_batch_step_render(batch, step), "mm_batch_step_render")


def mm_batch_render(batch: int) -> None:
    _check(lib().mm_batch_render(batch), "mm_batch_render")


def mm_batch_frame_device_ptr(batch: int, view: int) -> int:
    out = _vp()
    _check(lib().mm_batch_frame_device_ptr(batch, view, C.byref(out)),
           "mm_batch_frame_device_ptr")
    return out.value


def mm_batch_read_frame(batch: int, view: int, width: int, height: int) -> np.ndarray:
    out = np.empty((height, width), dtype=np.uint32)
    _check(lib().mm_batch_read_frame(batch, view, out.ctypes.data, out.nbytes),
           "mm_batch_read_frame")
    return out


def mm_batch_set_tuning(batch: int, tile: int = 0, points_per_thread: int = 0, splits: int = 0,
                        grid_blocks: int = 0, bin_threads: int = 0) -> None:
    t = mm_batch_tuning(tile, points_per_thread, splits, grid_blocks, bin_threads)
    _check(lib().mm_batch_set_tuning(batch, C.byref(t)), "mm_batch_set_tuning")


def mm_batch_get_tuning(batch: int) -> tuple[int, int, int, int, int]:
    """(tile, points_per_thread, splits, grid_blocks, bin_threads) in use."""
    t = mm_batch_tuning()
    _check(lib().mm_batch_get_tuning(batch, C.byref(t)), "mm_batch_get_tuning")
    return t.tile, t.points_per_thread, t.splits, t.grid_blocks, t.bin_threads


def mm_batch_autotune(batch: int, frames: int = 5) -> tuple[int, int, int, int, int]:
    t = mm_batch_tuning()
    _check(lib().mm_batch_autotune(batch, frames, C.byref(t)), "mm_batch_autotune")
    return t.tile, t.points_per_thread, t.splits, t.grid_blocks, t.bin_threads


def mm_batch_profile_begin(batch: int, capacity: int) -> None:
    _check(lib().mm_batch_profile_begin(batch, capacity), "mm_batch_profile_begin")


def mm_batch_profile_end(batch: int, capacity: int) -> np.ndarray:
    """Frame times (ms) of the recorded frames."""
    f = np.zeros(capacity, dtype=np.float32)
    n = C.c_uint32()
    _check(lib().mm_batch_profile_end(batch, _fptr(f), C.byref(n)), "mm_batch_profile_end")
    return f[:n.value]


# -------------------------------------------------------------------- server
def mm_create_server(inst: int, fb_budget_bytes: int, streams: int = 2, max_batch: int = 256,
                     dim: int = 3, footprint: int = 1, tile: int = 0, points_per_thread: int = 0,
                     splits: int = 0, grid_blocks: int = 0, bin_threads: int = 0) -> int:
    d = mm_server_desc()
    d.fb_budget_bytes = fb_budget_bytes
    d.streams, d.max_batch = streams, max_batch
    d.domain = MM_DOMAIN_2D if dim == 2 else MM_DOMAIN_3D
    d.footprint = footprint
    d.tuning = mm_batch_tuning(tile, points_per_thread, splits, grid_blocks, bin_threads)
    out = _vp()
    _check(lib().mm_create_server(inst, C.byref(d), C.byref(out)), "mm_create_server")
    return out.value


def mm_destroy_server(server: int) -> None:
    _check(lib().mm_destroy_server(server), "mm_destroy_server")


def mm_server_add_cloud(server: int, cloud: mm_cloud_desc) -> int:
    out = C.c_uint32()
    _check(lib().mm_server_add_cloud(server, C.byref(cloud), C.byref(out)), "mm_server_add_cloud")
    return out.value


def mm_server_submit(server: int, session: int, cloud: int, view_proj, width: int, height: int,
                     dev_out: int | None = None) -> int:
    m = np.ascontiguousarray(np.asarray(view_proj, dtype=np.float32).reshape(16))
    out = C.c_uint64()
    _check(lib().mm_server_submit(server, session, cloud, _fptr(m), width, height, dev_out or None,
                                  C.byref(out)), "mm_server_submit")
    return out.value


def mm_server_poll(server: int, request_id: int) -> tuple[bool, float | None]:
    done = C.c_int32()
    lat = C.c_double()
    _check(lib().mm_server_poll(server, request_id, C.byref(done), C.byref(lat)), "mm_server_poll")
    return bool(done.value), (lat.value if done.value else None)


def mm_server_wait(server: int, request_id: int) -> float:
    """Blocks until the request is complete; returns its latency in seconds."""
    lat = C.c_double()
    _check(lib().mm_server_wait(server, request_id, C.byref(lat)), "mm_server_wait")
    return lat.value


def mm_server_read_frame(server: int, session: int, width: int, height: int) -> np.ndarray:
    out = np.empty((height, width), dtype=np.uint32)
    _check(lib().mm_server_read_frame(server, session, out.ctypes.data, out.nbytes),
           "mm_server_read_frame")
    return out


def mm_server_close_session(server: int, session: int) -> None:
    _check(lib().mm_server_close_session(server, session), "mm_server_close_session")


def mm_server_stats_get(server: int) -> dict:
    st = mm_server_stats()
    _check(lib().mm_server_stats_get(server, C.byref(st)), "mm_server_stats_get")
    return {n: getattr(st, n) for n, _ in mm_server_stats._fields_}
