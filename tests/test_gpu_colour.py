"""GPU parity of the colour property (mm_set_colour): a palette read through
a per-point index buffer or by point index must give the oracle's frames bit
for bit, for the direct and the binned splat and both footprints."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import Rig, first_diff, say

pytestmark = pytest.mark.gpu

ST = 0xFFFFFFFF
MODES = [(1, 0, 0, 0, 0, 0), (2, 32, 8, 2, 1024, ST), (2, 64, 8, 0, 512, 4096),
         (2, 32, 8, 1, 1024, ST)]
IDS = ["direct", "binned-t32-z2", "binned-t64-balanced", "binned-t32-fused"]


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


def _alloc(rig, arr: np.ndarray):
    t = rig.torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    rig.keep.append(t)
    return rig.mm.mm_alloc_wrap(rig.inst, t.data_ptr(), t.numel() * t.element_size())


@pytest.mark.parametrize("mode", MODES, ids=IDS)
@pytest.mark.parametrize("foot", [1, 3])
def test_palette_through_indices_of_each_width(rig, mode, foot):
    say(f"case: palette, 3D mixture 150001 points, 400x300, footprint {foot}")
    mm = rig.mm
    w, h, seed, amp = 400, 300, 11, 0.001
    pts = synth.gaussian_mixture(150001, seed=4, sigma=0.05)
    n = pts.shape[0]
    dev, alloc = rig.cloud(pts)
    cam = synth.orbit_camera(20, w, h)
    view = rig.view(alloc, n, 3, w, h, foot, seed, amp, False, cam)
    mm.mm_set_tuning(view, *mode)
    rng = np.random.default_rng(foot)
    pal = rng.integers(0, 2**32, size=200, dtype=np.uint64).astype(np.uint32)
    pal_alloc = _alloc(rig, pal)
    ref = pts.copy()
    step = 0
    for dt in (np.uint8, np.uint16, np.uint32):
        idx = rng.integers(0, 256, size=n).astype(dt)  # 200..255 are past the palette
        idx_alloc = _alloc(rig, idx)
        mm.mm_set_colour(view, pal_alloc, pal.shape[0], idx_alloc, np.dtype(dt).itemsize)
        mm.mm_step_render(view, step)
        oracle.displace(ref, seed, step, amp, False)
        want = oracle.render_palette(ref, cam, w, h, foot, pal, idx)
        got = mm.mm_read_frame(view, w, h)
        assert np.array_equal(got, want), f"{np.dtype(dt).name}: {first_diff(got, want)}"
        step += 1
    # per-point palette (no index buffer)
    per_point = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    mm.mm_set_colour(view, _alloc(rig, per_point), n)
    mm.mm_step_render(view, step)
    oracle.displace(ref, seed, step, amp, False)
    want = oracle.render_palette(ref, cam, w, h, foot, per_point)
    assert np.array_equal(mm.mm_read_frame(view, w, h), want)
    step += 1
    # back to the default hash colour
    mm.mm_set_colour(view, None)
    mm.mm_step_render(view, step)
    want = oracle.step_render(ref, seed, step, amp, False, cam, w, h, foot)
    assert np.array_equal(mm.mm_read_frame(view, w, h), want)
    mm.mm_destroy_view(view)


def test_palette_with_frame_overlap_and_moving_camera(rig):
    say("case: palette + frame overlap, 2^18 points, 640x360, 5 frames")
    mm = rig.mm
    w, h, seed, amp = 640, 360, 3, 0.002
    pts = synth.uniform_cube(1 << 18, seed=3)
    n = pts.shape[0]
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, n, 3, w, h, 1, seed, amp, False, synth.orbit_camera(0, w, h))
    pal = np.arange(1, 65, dtype=np.uint32) * 0x01030507
    idx = (np.arange(n) % 64).astype(np.uint8)
    mm.mm_set_colour(view, _alloc(rig, pal), 64, _alloc(rig, idx), 1)
    mm.mm_set_frame_overlap(view, True)
    ref = pts.copy()
    for s in range(5):
        cam = synth.orbit_camera(7 * s, w, h)
        mm.mm_set_camera(view, cam)
        mm.mm_step_render(view, s)
        oracle.displace(ref, seed, s, amp, False)
        want = oracle.render_palette(ref, cam, w, h, 1, pal, idx)
    mm.mm_flush_frame(view)
    assert np.array_equal(mm.mm_read_frame(view, w, h), want)
    mm.mm_destroy_view(view)


def test_palette_validation_and_allocs_in_use(rig):
    say("case: mm_set_colour validation")
    mm = rig.mm
    n = 1000
    pts = synth.uniform_cube(n, seed=1)
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, n, 3, 64, 64, 1, 0, 0.0, False, synth.orbit_camera(0, 64, 64))
    pal = _alloc(rig, np.arange(16, dtype=np.uint32))
    idx4 = _alloc(rig, np.zeros(n, dtype=np.uint32))
    small_idx = _alloc(rig, np.zeros(n // 2, dtype=np.uint32))
    for args in [(pal, 17, idx4, 4),        # more entries than the alloc holds
                 (pal, 0, idx4, 4),         # empty palette
                 (pal, 16, idx4, 3),        # index width
                 (pal, 16, small_idx, 4),   # too few indices for the points
                 (pal, 16, None, 0)]:       # per-point palette smaller than the cloud
        with pytest.raises(mm.MMError) as e:
            mm.mm_set_colour(view, *args)
        assert e.value.status == mm.MM_ERR_INVALID_ARG, args
    mm.mm_set_colour(view, pal, 16, idx4, 4)
    with pytest.raises(mm.MMError) as e:
        mm.mm_free(pal)
    assert e.value.status == mm.MM_ERR_IN_USE
    mm.mm_set_colour(view, None)
    mm.mm_free(pal)
    mm.mm_destroy_view(view)
