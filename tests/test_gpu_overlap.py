"""GPU parity of frame overlap: with mm_set_frame_overlap on, the frame of
mm_step_render(f) is drawn during the call for step f + 1 (or by
mm_flush_frame), and every frame is still bit-identical to the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import Rig, first_diff, same_bits, say

pytestmark = pytest.mark.gpu

ST = 0xFFFFFFFF


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


def _overlap_run(rig, pts, w, h, foot, seed, amp, frames, cam_fn, tuning=None):
    """Steps 0 .. frames - 1 with overlap on; after the call for step s the
    frame buffer must hold frame s - 1, and after the flush frame s."""
    mm = rig.mm
    n = pts.shape[0]
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, n, 3, w, h, foot, seed, amp, False, cam_fn(0))
    if tuning is not None:
        mm.mm_set_tuning(view, *tuning)
    mm.mm_set_frame_overlap(view, True)
    say(f"  tuning {mm.mm_get_tuning(view)}")
    assert mm.mm_get_tuning(view)[6] == mm.MM_CULL_OFF  # no occlusion cull with overlap
    ref = pts.copy()
    prev = np.zeros((h, w), dtype=np.uint32)  # the frame buffer starts cleared
    for s in range(frames):
        cam = cam_fn(s)
        mm.mm_set_camera(view, cam)
        mm.mm_step_render(view, s)
        got = mm.mm_read_frame(view, w, h)
        assert np.array_equal(got, prev), f"after step {s}: {first_diff(got, prev)}"
        prev = oracle.step_render(ref, seed, s, amp, False, cam, w, h, foot)
    mm.mm_flush_frame(view)
    got = mm.mm_read_frame(view, w, h)
    assert np.array_equal(got, prev), f"after the flush: {first_diff(got, prev)}"
    assert same_bits(rig.positions(dev), ref)
    return view, alloc, dev, ref


@pytest.mark.parametrize("tuning", [None, (2, 32, 8, 2, 1024, ST), (2, 64, 16, 0, 256, 4096),
                                    (2, 16, 4, 1, 512, ST)],
                         ids=["auto", "t32-z2", "t64-balanced", "t16"])
def test_overlap_lags_one_frame_and_matches(rig, tuning):
    say("case: overlap, 3D uniform, 200003 points, 640x360, 8 frames, moving camera")
    pts = synth.uniform_cube(200003, seed=5)
    view, alloc, _, _ = _overlap_run(rig, pts, 640, 360, 1, 5, 0.002, 8,
                                     lambda s: synth.orbit_camera(9 * s, 640, 360), tuning)
    rig.mm.mm_destroy_view(view)
    rig.mm.mm_free(alloc)


def test_overlap_footprint3_mixture_tiles_leave_the_screen(rig):
    say("case: overlap, 3D mixture, 3x3 footprint, 2^18 points, 480x270, zooming camera")
    pts = synth.gaussian_mixture(1 << 18, seed=2)
    # the camera turns far enough that clusters leave and enter tiles
    view, alloc, _, _ = _overlap_run(rig, pts, 480, 270, 3, 2, 0.001, 6,
                                     lambda s: synth.orbit_camera(25 * s, 480, 270))
    rig.mm.mm_destroy_view(view)
    rig.mm.mm_free(alloc)


def test_overlap_render_toggle_and_errors(rig):
    say("case: overlap: mm_render draws at once, turning it off flushes, direct refused")
    mm = rig.mm
    w, h, seed, amp = 320, 240, 7, 0.001
    pts = synth.uniform_cube(50000, seed=7)
    cam = synth.orbit_camera(4, w, h)
    view, alloc, dev, ref = _overlap_run(rig, pts, w, h, 1, seed, amp, 3, lambda s: cam)
    # mm_render with overlap: drawn before it returns to the stream
    mm.mm_render(view)
    assert np.array_equal(mm.mm_read_frame(view, w, h), oracle.render(ref, seed, cam, w, h, 1))
    # a pending frame is drawn when overlap is turned off
    mm.mm_step_render(view, 3)
    want = oracle.step_render(ref, seed, 3, amp, False, cam, w, h, 1)
    mm.mm_set_frame_overlap(view, False)
    assert np.array_equal(mm.mm_read_frame(view, w, h), want)
    # serial again: no lag
    mm.mm_step_render(view, 4)
    want = oracle.step_render(ref, seed, 4, amp, False, cam, w, h, 1)
    assert np.array_equal(mm.mm_read_frame(view, w, h), want)
    assert same_bits(rig.positions(dev), ref)
    # direct splat and overlap exclude each other; so do overlap and a cull asked for
    mm.mm_set_frame_overlap(view, True)
    with pytest.raises(mm.MMError) as e:
        mm.mm_set_tuning(view, 2, 32, 8, 1, 1024, 0xFFFFFFFF, mm.MM_CULL_ON)
    assert e.value.status == mm.MM_ERR_UNSUPPORTED
    with pytest.raises(mm.MMError) as e:
        mm.mm_set_tuning(view, 1, 0, 0, 0, 0, 0)
    assert e.value.status == mm.MM_ERR_UNSUPPORTED
    mm.mm_set_frame_overlap(view, False)
    mm.mm_set_tuning(view, 1, 0, 0, 0, 0, 0)
    with pytest.raises(mm.MMError) as e:
        mm.mm_set_frame_overlap(view, True)
    assert e.value.status == mm.MM_ERR_UNSUPPORTED
    with pytest.raises(mm.MMError):
        mm.mm_set_frame_overlap(view, 2)
    mm.mm_destroy_view(view)
    mm.mm_free(alloc)


def test_overlap_profile_events(rig):
    say("case: overlap with profiling: the bin kernel is timed on the instance stream")
    mm = rig.mm
    pts = synth.uniform_cube(1 << 20, seed=1)
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, 1 << 20, 3, 1920, 1080, 1, 1, 0.001, False, synth.orbit_camera(0, 1920, 1080))
    mm.mm_set_frame_overlap(view, True)
    mm.mm_profile_begin(view, 8)
    for s in range(8):
        mm.mm_step_render(view, s)
    mm.mm_flush_frame(view)
    sp, rs, fr = mm.mm_profile_end(view, 8)
    assert len(sp) == 8 and all(x > 0 for x in sp)
    mm.mm_destroy_view(view)
    mm.mm_free(alloc)


def test_compute_sections_ping_pong(rig):
    """The paper's ping-pong scheme with a simulation on a stream of its own:
    per frame, mm_prepare_views, the simulation writes buffer W from buffer R
    on its stream while the view of R is rendered, then mm_update_views;
    every rendered frame and both buffers match the oracle."""
    say("case: compute sections, two buffers of 2^20 points, 640x360, 12 frames")
    torch, mm = rig.torch, rig.mm
    n, w, h, seed = 1 << 20, 640, 360, 5
    pts = synth.uniform_cube(n, seed=11)
    bufs = [rig.cloud(pts)[0], rig.cloud(pts)[0]]
    allocs = [mm.mm_alloc_wrap(rig.inst, b.data_ptr(), b.numel() * 4) for b in bufs]
    views = [rig.view(a, n, 3, w, h, 1, seed, 0.0, False, synth.orbit_camera(0, w, h))
             for a in allocs]
    for v in views:
        mm.mm_set_tuning(v, mm.MM_SPLAT_BINNED)
    sim = torch.cuda.Stream()
    # the simulation's step k: every coordinate += 2^-10 (k + 1), exact in binary32
    host = [pts.copy(), pts.copy()]
    for k in range(12):
        r, wr = k % 2, (k + 1) % 2
        cam = synth.orbit_camera(k, w, h)
        mm.mm_prepare_views(rig.inst, sim.cuda_stream)
        with torch.cuda.stream(sim):
            torch.add(bufs[r], (k + 1) * 2.0**-10, out=bufs[wr])
        mm.mm_set_camera(views[r], cam)
        mm.mm_render(views[r])  # reads buffer r beside the simulation
        mm.mm_update_views(rig.inst, sim.cuda_stream)
        want = oracle.render(host[r], seed, cam, w, h, 1)
        host[wr] = (host[r] + np.float32((k + 1) * 2.0**-10)).astype(np.float32)
        got = mm.mm_read_frame(views[r], w, h)
        assert np.array_equal(got, want), f"frame {k}: {first_diff(got, want)}"
    torch.cuda.synchronize()
    for b, ref in zip(bufs, host):
        assert same_bits(rig.positions(b), ref)


def test_overlap_frames_per_launch_and_marks(rig):
    """With frame overlap, mm_step_render_frames enqueues its frames one by
    one (the same frames, the buffer one frame behind until the flush), and
    the frame marks, stored by each frame's bin kernel, cover every frame."""
    say("case: overlap + mm_step_render_frames + marks, 3D uniform, 150001 points, 480x320")
    mm = rig.mm
    n, w, h, seed, amp = 150001, 480, 320, 21, 0.002
    pts = synth.uniform_cube(n, seed=seed)
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, n, 3, w, h, 1, seed, amp, False, synth.orbit_camera(0, w, h))
    mm.mm_set_frame_overlap(view, True)
    ref = pts.copy()
    mm.mm_mark_begin(view, 12 + 1)
    cams = [synth.orbit_camera(7 * f, w, h) for f in range(12)]
    mm.mm_step_render_frames(view, 0, 5, cams[:5])
    mm.mm_step_render_frames(view, 5, 7, cams[5:])
    for f in range(12):
        oracle.displace(ref, seed, f, amp, False)
    mm.mm_mark_end(view)  # draws the pending frame first
    iv = mm.mm_mark_read(view, 13)
    assert iv.shape == (12,) and np.all(iv > 0), iv
    want = oracle.render(ref, seed, cams[-1], w, h, 1)
    got = mm.mm_read_frame(view, w, h)
    assert np.array_equal(got, want), first_diff(got, want)
    assert same_bits(rig.positions(dev), ref)
    mm.mm_destroy_view(view)
    mm.mm_free(alloc)
