"""Helpers shared by the GPU tests (through the C ABI only)."""
from __future__ import annotations

import ctypes as C
import sys

import numpy as np


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


class Rig:
    """An instance on torch's current stream, with views over torch tensors."""

    def __init__(self):
        import torch

        import paper_2504_20937_amd as mm

        self.torch, self.mm = torch, mm
        self.inst = mm.mm_create_instance(0, torch.cuda.current_stream().cuda_stream)
        self.keep = []

    def cloud(self, pts: np.ndarray):
        dev = self.torch.from_numpy(np.ascontiguousarray(pts)).cuda()
        alloc = self.mm.mm_alloc_wrap(self.inst, dev.data_ptr(), dev.numel() * 4)
        self.keep.append(dev)
        return dev, alloc

    def view(self, alloc, n, dim, w, h, foot=1, seed=0, amp=0.0, wrap=False, cam=None):
        d = self.mm.make_view_desc(alloc, n, dim, w, h, foot, seed, amp, wrap, cam)
        return self.mm.mm_create_view(self.inst, d)

    def positions(self, dev) -> np.ndarray:
        self.mm.mm_synchronize(self.inst)
        return dev.cpu().numpy()

    def close(self):
        self.mm.mm_destroy_instance(self.inst)
        self.keep.clear()


def same_bits(a: np.ndarray, b: np.ndarray) -> bool:
    return a.shape == b.shape and np.array_equal(a.view(np.uint32), b.view(np.uint32))


def first_diff(got: np.ndarray, want: np.ndarray) -> str:
    g, w = got.reshape(-1), want.reshape(-1)
    bad = np.flatnonzero(g.view(np.uint32) != w.view(np.uint32))
    if bad.size == 0:
        return "identical"
    k = bad[0]
    return f"{bad.size} differ; first at flat {k}: got {g[k]!r} want {w[k]!r}"


_hip = None


def hip():
    """libamdhip64 for the few raw copies the alloc_linear test needs."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    return _hip


HIP_H2D, HIP_D2H = 1, 2
