"""GPU parity: positions and frames from the HIP path through the C ABI must
equal the CPU oracle bit for bit (the frame is the unique min over a total
order of keys, and positions follow a deterministic binary32 recurrence)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import Rig, first_diff, hip, same_bits, say, HIP_D2H, HIP_H2D

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


# splat strategies and shapes: (splat, tile, points_per_thread, splits, bin_threads,
# piece_records); 0 = auto. piece_records 1024 .. 2^20 balances the depth test by
# load; MM_PIECES_STATIC (and auto) gives `splits` workgroups per tile.
ST = 0xFFFFFFFF
DIRECT = (1, 0, 0, 0, 0, 0)
BINNED = (2, 0, 0, 0, 0, 0)
MODES = [DIRECT, BINNED]
SHAPES = [DIRECT, (2, 16, 4, 1, 256, ST), (2, 32, 8, 4, 256, ST), (2, 64, 16, 2, 256, ST),
          (2, 32, 4, 8, 256, ST), (2, 32, 16, 2, 512, ST), (2, 32, 16, 0, 1024, 1024),
          (2, 64, 8, 0, 1024, 8192), (2, 16, 4, 0, 512, 2048), (2, 32, 8, 0, 256, 4096),
          (2, 32, 8, 1, 1024, ST), (2, 64, 8, 1, 1024, ST)]


def _ids(modes):
    return ["direct" if m[0] == 1 else
            f"binned-t{m[1]}-p{m[2]}-n{m[4]}-" + (f"z{m[3]}" if m[5] == ST else f"r{m[5]}")
            + ("-nocull" if len(m) > 6 and m[6] == 2 else "-cull" if len(m) > 6 and m[6] == 1 else "")
            for m in modes]


# the occlusion cull (on by default where it applies: 3D, 1x1 footprint, one
# static split) against the same shape with every record kept
CULL_ON, CULL_OFF = 1, 2
CULL_SHAPES = [(2, 32, 16, 1, 512, ST, CULL_ON), (2, 32, 8, 1, 1024, ST, CULL_OFF),
               (2, 16, 4, 1, 256, ST, CULL_ON), (2, 64, 16, 1, 512, ST, CULL_ON),
               (2, 32, 8, 1, 1024, ST, CULL_ON)]


def _run(rig, pts, dim, w, h, foot, seed, amp, wrap, frames, cam_fn, check_every=1,
         split=False, mode=None):
    mm = rig.mm
    n = pts.shape[0]
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, n, dim, w, h, foot, seed, amp, wrap, cam_fn(0))
    if mode is not None:
        mm.mm_set_tuning(view, *mode)
        got_mode = mm.mm_get_tuning(view)
        assert got_mode[0] == mode[0]
        say(f"  tuning {got_mode}")
    ref = pts.copy()
    for s in range(frames):
        cam = cam_fn(s)
        mm.mm_set_camera(view, cam)
        if split:
            mm.mm_step(view, s)
            mm.mm_render(view)
        else:
            mm.mm_step_render(view, s)
        want = oracle.step_render(ref, seed, s, amp, wrap, cam, w, h, foot)
        if s % check_every == 0 or s == frames - 1:
            got = mm.mm_read_frame(view, w, h)
            assert np.array_equal(got, want), f"frame {s}: {first_diff(got, want)}"
            pos = rig.positions(dev)
            assert same_bits(pos, ref), f"positions after step {s}: {first_diff(pos, ref)}"
    mm.mm_destroy_view(view)
    mm.mm_free(alloc)
    return ref


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_2d_65536_points_512sq_100_steps(rig, mode):
    say("case: 2D uniform, 65536 points, 512x512, a=0.005, wrap, 100 steps, every step")
    pts = synth.uniform_square(65536, seed=0)
    _run(rig, pts, 2, 512, 512, 1, 0, 0.005, True, 100, lambda s: synth.IDENTITY, mode=mode)


@pytest.mark.parametrize("mode", SHAPES, ids=_ids(SHAPES))
def test_3d_uniform_ragged_small(rig, mode):
    say("case: 3D uniform, 65613 points (ragged), 320x240, 12 frames")
    pts = synth.uniform_cube(65536 + 77, seed=3)
    _run(rig, pts, 3, 320, 240, 1, 3, 0.001, False, 12,
         lambda s: synth.orbit_camera(s, 320, 240), mode=mode)


# 1x1 footprint with several static splits per tile (a merge pass resolves)
PART_SHAPES = [(2, 32, 8, 8, 1024, ST), (2, 16, 8, 4, 512, ST), (2, 64, 8, 2, 1024, ST),
               (2, 32, 4, 8, 256, ST)]


@pytest.mark.parametrize("mode", PART_SHAPES, ids=_ids(PART_SHAPES))
def test_3d_dense_tiles_in_splits(rig, mode):
    """Clustered points give tiles of 10^4 records and more, shared by the
    splits; the camera jumps every third frame, so tiles appear and leave."""
    say(f"case: 3D mixture, 2^18 points, 640x360, 1x1 in splits, 9 frames, jumping camera, mode {mode}")
    pts = synth.gaussian_mixture(1 << 18, seed=7)
    _run(rig, pts, 3, 640, 360, 1, 7, 0.001, False, 9,
         lambda s: synth.orbit_camera(70 * (s // 3), 640, 360), mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_3d_split_step_render_matches(rig, mode):
    say("case: 3D uniform, mm_step + mm_render, 30001 points, 200x100, 5 frames")
    pts = synth.uniform_cube(30001, seed=4)
    _run(rig, pts, 3, 200, 100, 1, 4, 0.001, False, 5,
         lambda s: synth.orbit_camera(3 * s, 200, 100), split=True, mode=mode)


@pytest.mark.parametrize("mode", SHAPES, ids=_ids(SHAPES))
def test_3d_footprint3_mixture(rig, mode):
    say("case: 3D mixture sigma 0.02, 3x3 footprint, 2^18 points, 640x360, 4 frames")
    pts = synth.gaussian_mixture(1 << 18, seed=0)
    _run(rig, pts, 3, 640, 360, 3, 0, 0.001, False, 4,
         lambda s: synth.orbit_camera(s, 640, 360), mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_2d_footprint3_ties(rig, mode):
    say("case: 2D grid points with heavy ties, 3x3 footprint, 20000 points, 64x64")
    rng = np.random.default_rng(0)
    pts = (rng.integers(-32, 32, size=(20000, 2)) / 32.0).astype(np.float32)
    _run(rig, pts, 2, 64, 64, 3, 9, 0.0, False, 2, lambda s: synth.IDENTITY, mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_3d_2p20_points_1080p(rig, mode):
    say("case: 3D uniform, 2^20 points, 1920x1080, 3 frames")
    pts = synth.uniform_cube(1 << 20, seed=0)
    _run(rig, pts, 3, 1920, 1080, 1, 0, 0.001, False, 3,
         lambda s: synth.orbit_camera(s, 1920, 1080), mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_3d_2p24_points_1080p_full_size(rig, mode):
    say("case: 3D uniform, 2^24 points, 1920x1080, 2 frames (full benchmark size)")
    pts = synth.uniform_cube(1 << 24, seed=0)
    _run(rig, pts, 3, 1920, 1080, 1, 0, 0.001, False, 2,
         lambda s: synth.orbit_camera(s, 1920, 1080), mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_3d_mixture_4k_footprint3(rig, mode):
    say("case: 3D mixture, 2^22 points, 3840x2160, 3x3 footprint, 2 frames")
    pts = synth.gaussian_mixture(1 << 22, seed=0)
    _run(rig, pts, 3, 3840, 2160, 3, 0, 0.001, False, 2,
         lambda s: synth.orbit_camera(s, 3840, 2160), mode=mode)


def test_3d_mixture_2p28_4k_footprint3_full_size(rig):
    """The 4K benchmark at its full size, in the launch configuration the
    benchmark times (default tuning: 64-pixel tiles, the tile pass balanced
    by load): one frame and every position."""
    say("case: 3D mixture, 2^28 points, 3840x2160, 3x3 footprint, 1 frame (full benchmark size)")
    pts = synth.gaussian_mixture(1 << 28, seed=0)
    _run(rig, pts, 3, 3840, 2160, 3, 0, 0.001, False, 1,
         lambda s: synth.orbit_camera(s, 3840, 2160))


@pytest.mark.parametrize("mode", SHAPES, ids=_ids(SHAPES))
@pytest.mark.parametrize("n", [1, 2, 255, 256, 257, 511, 1025, 4097])
def test_tiny_and_ragged_counts(rig, n, mode):
    say(f"case: 3D uniform, {n} points, 16x8 and 2D {n} points 8x8, mode {mode}")
    _run(rig, synth.uniform_cube(n, seed=n), 3, 16, 8, 3, n, 0.001, False, 3,
         lambda s: synth.orbit_camera(10 * s, 16, 8), mode=mode)
    _run(rig, synth.uniform_square(n, seed=n), 2, 8, 8, 1, n, 0.005, True, 3,
         lambda s: synth.IDENTITY, mode=mode)
    # a screen that is not a whole number of tiles
    _run(rig, synth.uniform_cube(n, seed=n + 1), 3, 70, 38, 3, n, 0.001, False, 2,
         lambda s: synth.orbit_camera(20 * s, 70, 38), mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_smallest_screen_and_everything_culled(rig, mode):
    say("case: 2x2 screen; camera looking away (all culled)")
    pts = synth.uniform_cube(4096, seed=1)
    _run(rig, pts, 3, 2, 2, 3, 1, 0.001, False, 2, lambda s: synth.orbit_camera(s, 2, 2),
         mode=mode)
    away = synth.look_at_perspective((0.5, 0.5, 3.0), (0.5, 0.5, 6.0), (0, 1, 0), 60.0, 1.0)
    mm = rig.mm
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, 4096, 3, 32, 32, 1, 1, 0.001, False, away)
    mm.mm_set_tuning(view, *mode)
    mm.mm_step_render(view, 0)
    assert not mm.mm_read_frame(view, 32, 32).any()


CLEAR_MODES = [DIRECT, BINNED, (2, 32, 8, 1, 1024, ST), (2, 32, 8, 2, 1024, ST),
               (2, 64, 8, 0, 512, 4096)]


@pytest.mark.parametrize("mode", CLEAR_MODES, ids=_ids(CLEAR_MODES))
def test_tiles_drawn_then_empty_are_cleared(rig, mode):
    say("case: draw, look away (nothing drawn: an empty frame), look back; 2^18 points 640x360")
    mm = rig.mm
    n, w, h, seed = 1 << 18, 640, 360, 4
    pts = synth.uniform_cube(n, seed=8)
    dev, alloc = rig.cloud(pts)
    cam = synth.orbit_camera(0, w, h)
    away = synth.look_at_perspective((0.5, 0.5, 3.0), (0.5, 0.5, 6.0), (0, 1, 0), 60.0, w / h)
    view = rig.view(alloc, n, 3, w, h, 1, seed, 0.001, False, cam)
    mm.mm_set_tuning(view, *mode)
    ref = pts.copy()
    for s, m in enumerate([cam, away, away, cam]):
        mm.mm_set_camera(view, m)
        mm.mm_step_render(view, s)
        want = oracle.step_render(ref, seed, s, 0.001, False, m, w, h, 1)
        got = mm.mm_read_frame(view, w, h)
        assert np.array_equal(got, want), f"frame {s}: {first_diff(got, want)}"
        if m is away:
            assert not got.any()
    assert same_bits(rig.positions(dev), ref)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_2d_points_on_pixel_edges_and_borders(rig, mode):
    say("case: 2D points on pixel edges, corners and just inside/outside the box")
    w, h = 64, 32
    xs = np.array([-1.0, 1.0 - 2.0**-23, 1.0 - 2.0**-24, 0.0, -0.5, 2.0 / 64 - 1.0],
                  dtype=np.float32)
    pts = np.array([[x, y] for x in xs for y in xs], dtype=np.float32)
    _run(rig, pts, 2, w, h, 3, 5, 0.0, False, 1, lambda s: synth.IDENTITY, mode=mode)


def test_view_sharing_one_cloud(rig):
    say("case: two views over one cloud: one steps, the other renders only")
    mm = rig.mm
    pts = synth.uniform_cube(50000, seed=2)
    dev, alloc = rig.cloud(pts)
    va = rig.view(alloc, 50000, 3, 160, 120, 1, 2, 0.001, False, synth.orbit_camera(0, 160, 120))
    camb = synth.orbit_camera(90, 256, 256)
    vb = rig.view(alloc, 50000, 3, 256, 256, 3, 2, 0.001, False, camb)
    mm.mm_set_tuning(va, *BINNED)
    mm.mm_set_tuning(vb, *DIRECT)
    ref = pts.copy()
    for s in range(3):
        mm.mm_step_render(va, s)
        mm.mm_render(vb)
        fa = oracle.step_render(ref, 2, s, 0.001, False, synth.orbit_camera(0, 160, 120),
                                160, 120, 1)
        assert np.array_equal(mm.mm_read_frame(va, 160, 120), fa)
        assert np.array_equal(mm.mm_read_frame(vb, 256, 256),
                              oracle.render(ref, 2, camb, 256, 256, 3))
    with pytest.raises(mm.MMError) as e:
        mm.mm_free(alloc)
    assert e.value.status == mm.MM_ERR_IN_USE
    mm.mm_destroy_view(va)
    mm.mm_destroy_view(vb)
    mm.mm_free(alloc)


def test_alloc_linear_owned_memory(rig):
    say("case: mm_alloc_linear memory, host copies through hipMemcpy")
    mm = rig.mm
    n = 10007
    pts = synth.uniform_cube(n, seed=12)
    ptr, alloc = mm.mm_alloc_linear(rig.inst, n * 12)
    assert ptr % 256 == 0
    H = hip()
    assert H.hipMemcpy(ptr, pts.ctypes.data, n * 12, HIP_H2D) == 0
    cam = synth.orbit_camera(7, 128, 96)
    view = rig.view(alloc, n, 3, 128, 96, 1, 12, 0.001, False, cam)
    mm.mm_step_render(view, 0)
    ref = pts.copy()
    want = oracle.step_render(ref, 12, 0, 0.001, False, cam, 128, 96, 1)
    assert np.array_equal(mm.mm_read_frame(view, 128, 96), want)
    back = np.empty_like(pts)
    assert H.hipMemcpy(back.ctypes.data, ptr, n * 12, HIP_D2H) == 0
    assert same_bits(back, ref)
    mm.mm_destroy_view(view)
    mm.mm_free(alloc)


def test_resume_from_snapshot(rig):
    say("case: checkpoint at step 50 of the 2D workload and resume")
    mm = rig.mm
    pts = synth.uniform_square(65536, seed=0)
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, 65536, 2, 512, 512, 1, 0, 0.005, True)
    for s in range(50):
        mm.mm_step_render(view, s)
    snap = rig.positions(dev).copy()
    dev2, alloc2 = rig.cloud(snap)
    view2 = rig.view(alloc2, 65536, 2, 512, 512, 1, 0, 0.005, True)
    ref = snap.copy()
    for s in range(50, 60):
        mm.mm_step_render(view, s)
        mm.mm_step_render(view2, s)
        want = oracle.step_render(ref, 0, s, 0.005, True, synth.IDENTITY, 512, 512, 1)
        got = mm.mm_read_frame(view2, 512, 512)
        assert np.array_equal(got, want), f"resumed frame {s}: {first_diff(got, want)}"
        assert np.array_equal(mm.mm_read_frame(view, 512, 512), got)
    assert same_bits(rig.positions(dev), rig.positions(dev2))
    assert same_bits(rig.positions(dev2), ref)


@pytest.mark.parametrize("mode", CULL_SHAPES, ids=_ids(CULL_SHAPES))
def test_cull_orbit_many_frames(rig, mode):
    """A dense cube under the orbit camera for 16 frames: from the second
    frame on, the previous frame's winners rule out most records; every frame
    and position equals the oracle's."""
    say("case: occlusion cull, 3D uniform, 2^20 points, 480x270, 16 frames")
    pts = synth.uniform_cube(1 << 20, seed=21)
    _run(rig, pts, 3, 480, 270, 1, 21, 0.001, False, 16,
         lambda s: synth.orbit_camera(s, 480, 270), mode=mode)


@pytest.mark.parametrize("mode", CULL_SHAPES, ids=_ids(CULL_SHAPES))
def test_cull_equal_depths_keep_the_smallest_index(rig, mode):
    """Many copies of a few points (equal depth at one pixel, amplitude 0): a
    record as deep as its pixel's bound is never ruled out, so the smallest
    index still wins every frame."""
    say("case: occlusion cull, 64 points repeated 500 times each, 128x96, 4 frames")
    base = synth.uniform_cube(64, seed=22)
    pts = np.ascontiguousarray(np.tile(base, (500, 1)))
    _run(rig, pts, 3, 128, 96, 1, 22, 0.0, False, 4,
         lambda s: synth.orbit_camera(0, 128, 96), mode=mode)


@pytest.mark.parametrize("mode", CULL_SHAPES[:2], ids=_ids(CULL_SHAPES[:2]))
def test_cull_wrap_3d(rig, mode):
    say("case: occlusion cull with the 3D fold into [-1, 1)^3, a = 0.02, 200000 points, 320x240")
    pts = (synth.uniform_cube(200000, seed=23) * 2.0 - 1.0).astype(np.float32)
    cam = lambda s: synth.look_at_perspective((2.0 * np.sin(s * 0.05), 0.3, 2.0 * np.cos(s * 0.05)),
                                              (0, 0, 0), (0, 1, 0), 60.0, 320 / 240)
    _run(rig, pts, 3, 320, 240, 1, 23, 0.02, True, 6, cam, mode=mode)


@pytest.mark.parametrize("mode", CULL_SHAPES[:1], ids=_ids(CULL_SHAPES[:1]))
def test_cull_positions_rewritten_between_frames(rig, mode):
    """The caller overwrites the positions between frames (a simulation of
    its own): the hints then name points that are somewhere else entirely,
    and the frames must still equal the oracle's."""
    say("case: occlusion cull, positions replaced between frames, 300000 points, 400x300")
    mm = rig.mm
    n, w, h = 300000, 400, 300
    pts = synth.uniform_cube(n, seed=24)
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, n, 3, w, h, 1, 24, 0.001, False, synth.orbit_camera(0, w, h))
    mm.mm_set_tuning(view, *mode)
    assert mm.mm_get_tuning(view)[6] == mm.MM_CULL_ON
    ref = pts.copy()
    for s in range(6):
        cam = synth.orbit_camera(3 * s, w, h)
        if s in (2, 4):
            new = synth.gaussian_mixture(n, seed=100 + s, sigma=0.05)
            rig.torch.cuda.synchronize()
            dev.copy_(rig.torch.from_numpy(new))
            rig.torch.cuda.synchronize()
            ref = new.copy()
        mm.mm_set_camera(view, cam)
        mm.mm_step_render(view, s)
        want = oracle.step_render(ref, 24, s, 0.001, False, cam, w, h, 1)
        got = mm.mm_read_frame(view, w, h)
        assert np.array_equal(got, want), f"frame {s}: {first_diff(got, want)}"
    mm.mm_destroy_view(view)


def _subnormal_cloud(n, seed):
    """A 3D cloud with subnormal, signed-zero and normal coordinates mixed."""
    rng = np.random.default_rng(seed)
    pts = synth.uniform_cube(n, seed)
    bits = pts.view(np.uint32)
    # a third of the coordinates become subnormal (exponent field 0, mantissa
    # non-zero), some negative; a few become -0.0
    sub = rng.random(pts.shape) < 1 / 3
    mant = rng.integers(1, 1 << 23, size=pts.shape, dtype=np.uint64).astype(np.uint32)
    sign = (rng.random(pts.shape) < 0.5).astype(np.uint32) << 31
    bits[sub] = (mant | sign)[sub]
    negz = rng.random(pts.shape) < 0.01
    bits[negz] = np.uint32(0x80000000)
    assert np.count_nonzero((bits & 0x7F800000) == 0) > n // 2
    return pts


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
@pytest.mark.parametrize("amp", [0.0, 0.001])
def test_subnormal_coordinates_kept(rig, mode, amp):
    """binary32 with subnormals (no flush to zero, no denormals-are-zero): with
    amplitude 0 a subnormal coordinate is stored back unchanged (x + (+-0) = x),
    and with a non-zero amplitude x + d rounds as IEEE arithmetic does."""
    say(f"case: 3D cloud with subnormal coordinates, 40000 points, 256x192, amplitude {amp}")
    pts = _subnormal_cloud(40000, 11)
    _run(rig, pts, 3, 256, 192, 1, 5, amp, False, 3,
         lambda s: synth.orbit_camera(s, 256, 192), mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_subnormal_coordinates_2d_wrap(rig, mode):
    say("case: 2D cloud with subnormal coordinates, wrap, amplitude 0, 30000 points, 128x128")
    pts = synth.uniform_square(30000, 12)
    rng = np.random.default_rng(12)
    bits = pts.view(np.uint32)
    sub = rng.random(pts.shape) < 0.5
    mant = rng.integers(1, 1 << 23, size=pts.shape, dtype=np.uint64).astype(np.uint32)
    bits[sub] = mant[sub] | ((rng.random(pts.shape) < 0.5).astype(np.uint32) << 31)[sub]
    _run(rig, pts, 2, 128, 128, 1, 6, 0.0, True, 2, lambda s: synth.IDENTITY, mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
@pytest.mark.parametrize("seed", [(1 << 32) + 7, 0xFEDCBA9876543210])
def test_seed_above_2p32(rig, mode, seed):
    """The key's high word is the seed's upper 32 bits: a seed of 2^32 or more
    changes both the displacement draw and the colour hash."""
    say(f"case: 3D uniform, seed {seed:#x}, 50001 points, 320x200, 3 frames")
    pts = synth.uniform_cube(50001, seed=13)
    _run(rig, pts, 3, 320, 200, 1, seed, 0.002, False, 3,
         lambda s: synth.orbit_camera(2 * s, 320, 200), mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_profile_records_kernel_times(rig, mode):
    say("case: mm_profile_begin/end around 20 frames, 2^20 points 1080p")
    mm = rig.mm
    pts = synth.uniform_cube(1 << 20, seed=0)
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, 1 << 20, 3, 1920, 1080, 1, 0, 0.001, False,
                    synth.orbit_camera(0, 1920, 1080))
    mm.mm_set_tuning(view, *mode)
    mm.mm_profile_begin(view, 20)
    ref = pts.copy()
    for s in range(25):  # 5 beyond capacity run untimed
        mm.mm_set_camera(view, synth.orbit_camera(s, 1920, 1080))
        mm.mm_step_render(view, s)
    sp, rs, fr = mm.mm_profile_end(view, 20)
    assert sp.shape == (20,) and np.all(sp > 0) and np.all(rs > 0)
    assert np.all(fr >= sp) and np.all(fr >= rs)
    # the timed graph computes the same frames
    for s in range(25):
        want = oracle.step_render(ref, 0, s, 0.001, False, synth.orbit_camera(s, 1920, 1080),
                                  1920, 1080, 1)
    assert np.array_equal(mm.mm_read_frame(view, 1920, 1080), want)
    assert same_bits(rig.positions(dev), ref)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_profile_sampling_records_one_frame_in_every(rig, mode):
    say("case: mm_profile_every 3, capacity 4, 14 frames, 2^18 points 640x480")
    mm = rig.mm
    pts = synth.uniform_cube(1 << 18, seed=5)
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, 1 << 18, 3, 640, 480, 1, 7, 0.002, True,
                    synth.orbit_camera(0, 640, 480))
    mm.mm_set_tuning(view, *mode)
    with pytest.raises(RuntimeError):
        mm.mm_profile_every(view, 0)
    with pytest.raises(RuntimeError):
        mm.mm_profile_every(view, 1001)
    mm.mm_profile_every(view, 3)
    mm.mm_profile_begin(view, 4)
    ref = pts.copy()
    for s in range(14):  # frames 0, 3, 6, 9 are recorded; 12 finds the buffer full
        mm.mm_set_camera(view, synth.orbit_camera(s, 640, 480))
        mm.mm_step_render(view, s)
        want = oracle.step_render(ref, 7, s, 0.002, True, synth.orbit_camera(s, 640, 480),
                                  640, 480, 1)
        if s in (2, 3, 13):  # a plain frame, a timed frame, a frame past capacity
            assert np.array_equal(mm.mm_read_frame(view, 640, 480), want), s
    sp, rs, fr = mm.mm_profile_end(view, 4)
    assert sp.shape == (4,) and np.all(sp > 0) and np.all(rs > 0) and np.all(fr >= sp)
    assert same_bits(rig.positions(dev), ref)
    # back to every frame: a new profile of 3 frames records 3
    mm.mm_profile_every(view, 1)
    mm.mm_profile_begin(view, 3)
    for s in range(14, 17):
        mm.mm_step_render(view, s)
    sp, _, _ = mm.mm_profile_end(view, 3)
    assert sp.shape == (3,)


@pytest.mark.parametrize("mode", MODES, ids=_ids(MODES))
def test_frame_marks_time_every_frame(rig, mode):
    say("case: mm_mark_begin/end around 12 frames (capacity 10), 2^18 points 640x480")
    mm = rig.mm
    pts = synth.uniform_cube(1 << 18, seed=6)
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, 1 << 18, 3, 640, 480, 1, 8, 0.002, False,
                    synth.orbit_camera(0, 640, 480))
    mm.mm_set_tuning(view, *mode)
    with pytest.raises(RuntimeError):
        mm.mm_mark_begin(view, 1)
    with pytest.raises(RuntimeError):
        mm.mm_mark_end(view)
    mm.mm_mark_begin(view, 10)
    mm.mm_profile_every(view, 4)
    mm.mm_profile_begin(view, 3)
    ref = pts.copy()
    for s in range(12):  # frames 0..8 are marked; 9..11 find the marks full
        cam = synth.orbit_camera(s, 640, 480)
        mm.mm_set_camera(view, cam)
        mm.mm_step_render(view, s)
        want = oracle.step_render(ref, 8, s, 0.002, False, cam, 640, 480, 1)
    with pytest.raises(RuntimeError):
        mm.mm_mark_read(view, 10)  # still marking
    mm.mm_mark_end(view)
    iv = mm.mm_mark_read(view, 10)
    sp, _, fr = mm.mm_profile_end(view, 3)
    assert iv.shape == (9,) and np.all(iv > 0), iv
    assert sp.shape == (3,)
    # the marks span the frames they bracket: their sum is at least the
    # graph time of the profiled frames among them
    assert iv.sum() >= fr[:3].sum() * 0.99
    assert np.array_equal(mm.mm_read_frame(view, 640, 480), want)
    assert same_bits(rig.positions(dev), ref)


@pytest.mark.parametrize("mode", [DIRECT, (2, 32, 8, 1, 1024, ST), (2, 16, 4, 2, 256, ST),
                                  (2, 32, 16, 1, 512, ST, CULL_ON)],
                         ids=["direct", "binned-fused", "binned-z2", "binned-cull"])
def test_step_render_frames_matches_the_oracle(rig, mode):
    """Several frames per graph launch: after each launch the frame buffer and
    the positions equal the oracle's after the same steps and cameras (tiles
    left by the cloud between frames of one launch are cleared), for counts
    1, 7, 16 and 3, with per-frame cameras and with the view's own; frame
    marks cover every frame of every launch."""
    say(f"case: mm_step_render_frames, 100003 points, 320x240, mode {mode}")
    mm = rig.mm
    n, w, h, seed, amp = 100003, 320, 240, 11, 0.002
    pts = synth.uniform_cube(n, seed=seed)
    dev, alloc = rig.cloud(pts)
    view = rig.view(alloc, n, 3, w, h, 1, seed, amp, False, synth.orbit_camera(0, w, h))
    mm.mm_set_tuning(view, *mode)
    ref, step, cam = pts.copy(), 0, synth.orbit_camera(0, w, h)
    plan = [(7, True), (1, True), (16, False), (3, True)]
    total = sum(c for c, _ in plan)
    mm.mm_mark_begin(view, total + 1)
    for count, with_cams in plan:
        cams = [synth.orbit_camera(13 * (step + i), w, h) for i in range(count)] if with_cams else None
        mm.mm_step_render_frames(view, step, count, cams)
        for i in range(count):
            oracle.displace(ref, seed, step + i, amp, False)
        if with_cams:
            cam = cams[-1]
        want = oracle.render(ref, seed, cam, w, h, 1)
        got = mm.mm_read_frame(view, w, h)
        assert np.array_equal(got, want), f"after steps {step}..{step + count - 1}: {first_diff(got, want)}"
        assert same_bits(rig.positions(dev), ref), f"positions after step {step + count - 1}"
        step += count
    mm.mm_mark_end(view)
    iv = mm.mm_mark_read(view, total + 1)
    assert iv.shape == (total,) and np.all(iv > 0), iv
    with pytest.raises(mm.MMError):
        mm.mm_step_render_frames(view, 0, 65, None)
    with pytest.raises(mm.MMError):
        mm.mm_step_render_frames(view, 0, 0, None)


def test_invalid_descriptions_are_rejected(rig):
    say("case: invalid view descriptions and wraps")
    mm = rig.mm
    pts = synth.uniform_cube(1000, seed=0)
    dev, alloc = rig.cloud(pts)
    base = dict(alloc=alloc, n=1000, dim=3, w=64, h=64)

    def expect(status, **kw):
        args = {**base, **kw}
        with pytest.raises(mm.MMError) as e:
            rig.view(args["alloc"], args["n"], args["dim"], args["w"], args["h"],
                     kw.get("foot", 1), 0, kw.get("amp", 0.001), kw.get("wrap", False))
        assert e.value.status == status, str(e.value)

    expect(mm.MM_ERR_INVALID_ARG, n=1001)          # overruns the alloc
    expect(mm.MM_ERR_INVALID_ARG, n=0)
    expect(mm.MM_ERR_INVALID_ARG, w=63)            # odd width
    expect(mm.MM_ERR_INVALID_ARG, h=0)
    expect(mm.MM_ERR_INVALID_ARG, w=16386)
    expect(mm.MM_ERR_INVALID_ARG, foot=2)
    expect(mm.MM_ERR_INVALID_ARG, amp=float("nan"))
    expect(mm.MM_ERR_INVALID_ARG, amp=-0.001)
    expect(mm.MM_ERR_INVALID_ARG, amp=2.0, wrap=True)
    # float3 data described as 2D
    d = mm.make_view_desc(alloc, 1000, 3, 64, 64)
    d.domain = mm.MM_DOMAIN_2D
    with pytest.raises(mm.MMError) as e:
        mm.mm_create_view(rig.inst, d)
    assert e.value.status == mm.MM_ERR_UNSUPPORTED
    # wrapping more bytes than the device allocation holds (torch's caching
    # allocator carves tensors out of larger segments, so overrun by far more
    # than any segment)
    with pytest.raises(mm.MMError) as e:
        mm.mm_alloc_wrap(rig.inst, dev.data_ptr(), 1 << 40)
    assert e.value.status == mm.MM_ERR_INVALID_ARG
    # a host pointer is not device memory
    host = np.zeros(16, dtype=np.float32)
    with pytest.raises(mm.MMError):
        mm.mm_alloc_wrap(rig.inst, host.ctypes.data, 64)
    # a non-finite camera
    view = rig.view(alloc, 1000, 3, 64, 64)
    bad = np.eye(4, dtype=np.float32)
    bad[0, 0] = np.inf
    with pytest.raises(mm.MMError):
        mm.mm_set_camera(view, bad)
    with pytest.raises(mm.MMError):
        mm.mm_read_frame(view, 32, 32)  # too small a host buffer


def test_tuning_choices_and_validation(rig):
    say("case: tuning resolution and rejection")
    mm = rig.mm
    pts = synth.uniform_cube(5000, seed=0)
    dev, alloc = rig.cloud(pts)
    cam = synth.orbit_camera(0, 1920, 1080)
    view = rig.view(alloc, 5000, 3, 1920, 1080, 1, 0, 0.001, False, cam)
    # 5000 points on a 1080p screen: the direct splat (a small cloud)
    OFF, ON = mm.MM_CULL_OFF, mm.MM_CULL_ON
    assert mm.mm_get_tuning(view) == (mm.MM_SPLAT_DIRECT, 0, 0, 0, 0, 0, OFF)
    # binned by request: one bin workgroup, so one workgroup per tile in the depth test
    mm.mm_set_tuning(view, mm.MM_SPLAT_BINNED)
    assert mm.mm_get_tuning(view) == (mm.MM_SPLAT_BINNED, 32, 8, 1, 1024, ST, OFF)
    # the occlusion cull asked for: 512 threads of 16 points by default
    mm.mm_set_tuning(view, mm.MM_SPLAT_BINNED, 0, 0, 0, 0, 0, ON)
    assert mm.mm_get_tuning(view) == (mm.MM_SPLAT_BINNED, 32, 16, 1, 512, ST, ON)
    # 2^21 points (256 bin workgroups): the 1x1 footprint keeps one workgroup per
    # tile (which resolves the tile itself), the 3x3 footprint takes two splits
    n2 = 1 << 21
    dev2, alloc2 = rig.cloud(synth.uniform_cube(n2, seed=1))
    v1 = rig.view(alloc2, n2, 3, 1920, 1080, 1, 0, 0.001, False, cam)
    assert mm.mm_get_tuning(v1) == (mm.MM_SPLAT_BINNED, 32, 8, 1, 1024, ST, OFF)
    v3 = rig.view(alloc2, n2, 3, 1920, 1080, 3, 0, 0.001, False, cam)
    assert mm.mm_get_tuning(v3) == (mm.MM_SPLAT_BINNED, 32, 8, 2, 1024, ST, OFF)
    for bad, status in [((2, 128, 16, 0, 0, 0), mm.MM_ERR_INVALID_ARG),
                        ((2, 32, 3, 0, 0, 0), mm.MM_ERR_INVALID_ARG),
                        ((2, 32, 16, 3, 0, ST), mm.MM_ERR_INVALID_ARG),
                        ((2, 32, 16, 0, 384, 0), mm.MM_ERR_INVALID_ARG),
                        ((2, 32, 16, 0, 256, 512), mm.MM_ERR_INVALID_ARG),
                        ((7, 0, 0, 0, 0, 0), mm.MM_ERR_INVALID_ARG),
                        ((2, 16, 16, 0, 0, 0), mm.MM_ERR_UNSUPPORTED),
                        ((2, 32, 8, 1, 1024, ST, 3), mm.MM_ERR_INVALID_ARG),
                        ((1, 0, 0, 0, 0, 0, ON), mm.MM_ERR_UNSUPPORTED),
                        ((2, 32, 8, 2, 1024, ST, ON), mm.MM_ERR_UNSUPPORTED),
                        ((2, 32, 8, 0, 1024, 4096, ON), mm.MM_ERR_UNSUPPORTED),
                        ((2, 32, 16, 1, 1024, ST, ON), mm.MM_ERR_UNSUPPORTED)]:
        with pytest.raises(mm.MMError) as e:
            mm.mm_set_tuning(view, *bad)
        assert e.value.status == status, (bad, str(e.value))
    # a rejected tuning leaves the previous one working
    mm.mm_step_render(view, 0)
    ref = pts.copy()
    assert np.array_equal(mm.mm_read_frame(view, 1920, 1080),
                          oracle.step_render(ref, 0, 0, 0.001, False, cam, 1920, 1080, 1))
    mm.mm_set_tuning(view, 2, 64, 4, 8, 512, ST)
    assert mm.mm_get_tuning(view) == (2, 64, 4, 8, 512, ST, OFF)
    mm.mm_step_render(view, 1)
    assert np.array_equal(mm.mm_read_frame(view, 1920, 1080),
                          oracle.step_render(ref, 0, 1, 0.001, False, cam, 1920, 1080, 1))
    mm.mm_set_tuning(view, 2, 32, 8, 1, 1024, ST, OFF)
    assert mm.mm_get_tuning(view) == (2, 32, 8, 1, 1024, ST, OFF)
    mm.mm_set_tuning(view, 1, 0, 0, 0, 0, 0)
    assert mm.mm_get_tuning(view) == (1, 0, 0, 0, 0, 0, OFF)


def test_largest_screen_falls_back_to_direct(rig):
    say("case: 16384x16384 screen, 3x3 footprint, 6000 points (direct only)")
    mm = rig.mm
    n, w = 6000, 16384
    pts = synth.gaussian_mixture(n, seed=5, sigma=0.2)
    dev, alloc = rig.cloud(pts)
    cam = synth.orbit_camera(30, w, w)
    view = rig.view(alloc, n, 3, w, w, 3, 5, 0.001, False, cam)
    assert mm.mm_get_tuning(view)[0] == mm.MM_SPLAT_DIRECT
    mm.mm_step_render(view, 0)
    got = mm.mm_read_frame(view, w, w)
    ref = pts.copy()
    want = oracle.step_render(ref, 5, 0, 0.001, False, cam, w, w, 3)
    assert np.array_equal(got, want)
    mm.mm_destroy_view(view)


@pytest.mark.parametrize("foot", [1, 3])
@pytest.mark.parametrize("mode", SHAPES, ids=_ids(SHAPES))
def test_frames_whose_tile_sets_change(rig, mode, foot):
    _tile_sets_change(rig, mode, foot)


CULL_ON_SHAPES = [m for m in CULL_SHAPES if m[6] == CULL_ON]


@pytest.mark.parametrize("mode", CULL_ON_SHAPES, ids=_ids(CULL_ON_SHAPES))
def test_cull_frames_whose_tile_sets_change(rig, mode):
    """Camera jumps and render-only frames between culled frames: the hints
    then name points far from where they land, or come from a frame drawn
    without displacement."""
    _tile_sets_change(rig, mode, 1)


@pytest.mark.parametrize("mode", CULL_ON_SHAPES, ids=_ids(CULL_ON_SHAPES))
def test_cull_uniform_ragged_small(rig, mode):
    say("case: occlusion cull, 3D uniform, 65613 points (ragged), 320x240, 12 frames")
    pts = synth.uniform_cube(65536 + 77, seed=3)
    _run(rig, pts, 3, 320, 240, 1, 3, 0.001, False, 12,
         lambda s: synth.orbit_camera(s, 320, 240), mode=mode)


def _tile_sets_change(rig, mode, foot):
    say(f"case: consecutive frames drawing different tiles, footprint {foot}, mode {mode}")
    mm = rig.mm
    w, h = 640, 360
    pts = synth.gaussian_mixture(60000, seed=11, sigma=0.03)
    dev, alloc = rig.cloud(pts)
    away = synth.look_at_perspective((0.5, 0.5, 3.0), (0.5, 0.5, 6.0), (0, 1, 0), 60.0, w / h)
    zoom = synth.look_at_perspective((0.5, 0.5, 1.2), (0.5, 0.5, 0.5), (0, 1, 0), 60.0, w / h)
    cams = [synth.orbit_camera(0, w, h), away, synth.orbit_camera(90, w, h),
            synth.orbit_camera(90, w, h), zoom, away, away, synth.orbit_camera(200, w, h)]
    view = rig.view(alloc, 60000, 3, w, h, foot, 11, 0.001, False, cams[0])
    mm.mm_set_tuning(view, *mode)
    ref = pts.copy()
    for s, cam in enumerate(cams):
        mm.mm_set_camera(view, cam)
        if s % 3 == 2:
            mm.mm_render(view)
            want = oracle.render(ref, 11, cam, w, h, foot)
        else:
            mm.mm_step_render(view, s)
            want = oracle.step_render(ref, 11, s, 0.001, False, cam, w, h, foot)
        got = mm.mm_read_frame(view, w, h)
        assert np.array_equal(got, want), f"frame {s}: {first_diff(got, want)}"
