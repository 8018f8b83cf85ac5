"""The frame that allocates nothing (mm_step_render_static), through the C
ABI: its frames and positions equal those of mm_step_render with the direct
splat on the same inputs, bit for bit, over two calls in a row, the second
with a smaller cloud and screen; a screen beyond its static key array is
refused; and device memory in use does not change across calls."""
import ctypes as C

import numpy as np
import pytest

import synth
from gpu_util import Rig, first_diff, same_bits, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture
def rig(torch_gpu):
    r = Rig()
    yield r
    r.close()


def _free_bytes():
    hip = C.CDLL("libamdhip64.so")
    free, total = C.c_size_t(), C.c_size_t()
    assert hip.hipMemGetInfo(C.byref(free), C.byref(total)) == 0
    return free.value


def _reference(rig, pts, dim, w, h, foot, seed, amp, wrap, step, cam):
    """The existing entry point: a view with the direct splat, one frame."""
    mm = rig.mm
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, pts.shape[0], dim, w, h, foot, seed, amp, wrap, cam)
    mm.mm_set_tuning(view, mm.MM_SPLAT_DIRECT)
    mm.mm_step_render(view, step)
    frame = mm.mm_read_frame(view, w, h)
    pos = rig.positions(dev).copy()
    mm.mm_destroy_view(view)
    mm.mm_free(alloc)
    return frame, pos


CASES = [  # dim, n, w, h, footprint, seed, amplitude, wrap, step
    (3, 200003, 640, 480, 1, 7, 0.002, False, 5),
    (3, 50001, 320, 200, 3, 8, 0.001, False, 6),   # smaller cloud and screen
    (2, 30000, 256, 256, 1, 9, 0.005, True, 0),
]


def test_static_frames_equal_the_direct_view_frames(rig):
    torch, mm = rig.torch, rig.mm
    stream = torch.cuda.current_stream()
    free_after_first = None
    for k, (dim, n, w, h, foot, seed, amp, wrap, step) in enumerate(CASES):
        say(f"case: static frame {k}: {dim}D, {n} points, {w}x{h}, footprint {foot}, step {step}")
        pts = synth.uniform_square(n, seed) if dim == 2 else synth.uniform_cube(n, seed)
        cam = synth.IDENTITY if dim == 2 else synth.orbit_camera(step, w, h)
        want_frame, want_pos = _reference(rig, pts, dim, w, h, foot, seed, amp, wrap, step, cam)
        dev = torch.from_numpy(pts.copy()).cuda()
        out = torch.full((h, w), -1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        free_before = _free_bytes()
        mm.mm_step_render_static(dev.data_ptr(), n, dim, w, h, out.data_ptr(), step, foot, seed,
                                 amp, wrap, cam, stream.cuda_stream)
        torch.cuda.synchronize()
        if k > 0:  # the library's code object (and the key array) is loaded by now
            assert _free_bytes() == free_before, "device memory changed across the call"
        free_after_first = free_after_first or _free_bytes()
        got = out.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want_frame), f"frame {k}: {first_diff(got, want_frame)}"
        assert same_bits(dev.cpu().numpy(), want_pos), f"positions {k}"
    assert free_after_first is not None


def test_static_frame_refuses_a_screen_beyond_its_keys(rig):
    torch, mm = rig.torch, rig.mm
    pts = synth.uniform_cube(1000, 1)
    dev = torch.from_numpy(pts).cuda()
    out = torch.zeros((2050, 2048), dtype=torch.int32, device="cuda")
    with pytest.raises(mm.MMError) as e:
        mm.mm_step_render_static(dev.data_ptr(), 1000, 3, 2048, 2050, out.data_ptr(), 0, 1, 0, 0.0,
                                 False, synth.orbit_camera(0, 2048, 2050))
    assert e.value.status == mm.MM_ERR_BUDGET
    # the largest screen it takes, 2048 x 2048, renders
    out2 = torch.zeros((2048, 2048), dtype=torch.int32, device="cuda")
    mm.mm_step_render_static(dev.data_ptr(), 1000, 3, 2048, 2048, out2.data_ptr(), 0, 1, 0, 0.0,
                             False, synth.orbit_camera(0, 2048, 2048))
    torch.cuda.synchronize()
    assert int((out2 != 0).sum()) > 0
