"""GPU parity of batches: every (cloud, view) frame of a batch, and every
cloud's positions, equal the CPU oracle bit for bit: the plain single-view
frame of that cloud and view after the same steps."""
import numpy as np
import pytest

import oracle
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


class Batch:
    """A batch over host clouds, with the oracle's copy of every cloud beside it."""

    def __init__(self, rig, clouds, views, dim=3, foot=1):
        # clouds: [(pts, seed, amp, wrap)]; views: [(cloud, w, h, cam)]
        mm = rig.mm
        self.rig, self.mm, self.dim, self.foot = rig, mm, dim, foot
        self.clouds, self.views = clouds, views
        self.devs, descs = [], []
        for pts, seed, amp, wrap in clouds:
            dev, alloc = rig.cloud(pts)
            self.devs.append(dev)
            descs.append(mm.make_cloud_desc(alloc, pts.shape[0], dim, seed, amp, wrap))
        vds = [mm.make_batch_view_desc(c, w, h, cam) for c, w, h, cam in views]
        self.b = mm.mm_create_batch(rig.inst, dim, foot, descs, vds)
        self.ref = [pts.copy() for pts, _, _, _ in clouds]

    def step_render(self, step, check=True):
        self.mm.mm_batch_step_render(self.b, step)
        for j, (_, seed, amp, wrap) in enumerate(self.clouds):
            oracle.displace(self.ref[j], seed, step, amp, wrap)
        if check:
            self.check(f"step {step}")

    def render(self):
        self.mm.mm_batch_render(self.b)
        self.check("render only")

    def check_positions(self, what):
        for j, dev in enumerate(self.devs):
            pos = self.rig.positions(dev)
            assert same_bits(pos, self.ref[j]), f"{what}, cloud {j} positions: {first_diff(pos, self.ref[j])}"

    def check(self, what, views=None):
        for k in (range(len(self.views)) if views is None else views):
            c, w, h, cam = self.views[k]
            seed = self.clouds[c][1]
            want = oracle.render(self.ref[c], seed, cam, w, h, self.foot)
            got = self.mm.mm_batch_read_frame(self.b, k, w, h)
            assert np.array_equal(got, want), f"{what}, view {k} (cloud {c}, {w}x{h}): {first_diff(got, want)}"
        for j, dev in enumerate(self.devs):
            pos = self.rig.positions(dev)
            assert same_bits(pos, self.ref[j]), f"{what}, cloud {j} positions: {first_diff(pos, self.ref[j])}"

    def set_camera(self, k, cam):
        c, w, h, _ = self.views[k]
        self.views[k] = (c, w, h, cam)
        self.mm.mm_batch_set_camera(self.b, k, cam)

    def close(self):
        self.mm.mm_destroy_batch(self.b)


def _mixed_3d(seed=0):
    """Five 3D clouds: ragged sizes (one point up to a few chunks), uniform and
    mixture, 0 to 3 views each at assorted screens (views listed out of
    cloud order)."""
    sizes = [1, 4097, 70001, 300000, 5000]
    clouds = []
    for j, n in enumerate(sizes):
        pts = synth.uniform_cube(n, 7 + j) if j % 2 == 0 else synth.gaussian_mixture(n, 7 + j)
        clouds.append((pts, 100 + j, 0.001 if j != 3 else 0.004, False))
    screens = [(256, 256), (512, 384), (70, 38), (1024, 1024), (128, 96), (300, 200)]
    views = []
    for k, (c, s) in enumerate([(3, 0), (1, 1), (3, 2), (0, 4), (1, 3), (3, 5), (2, 0)]):
        w, h = screens[s]
        views.append((c, w, h, synth.orbit_camera(0, w, h, start_deg=37.0 * k)))
    # cloud 4 has no view: it is only displaced
    return clouds, views


TUNINGS = [(0, 0, 0, 0, 0), (16, 4, 1, 0, 256), (32, 8, 2, 0, 256), (64, 16, 4, 0, 256),
           (32, 16, 0, 256, 256), (32, 8, 8, 8, 256), (32, 16, 0, 0, 1024), (64, 8, 1, 64, 512),
           (16, 16, 2, 0, 1024)]


@pytest.mark.parametrize("tuning", TUNINGS,
                         ids=[f"t{t[0]}-p{t[1]}-z{t[2]}-g{t[3]}-n{t[4]}" for t in TUNINGS])
def test_batch_3d_mixed_clouds_and_screens(rig, tuning):
    say(f"case: batch 3D, 5 clouds (1..300000 points), 7 views, tuning {tuning}")
    clouds, views = _mixed_3d()
    b = Batch(rig, clouds, views)
    rig.mm.mm_batch_set_tuning(b.b, *tuning)
    got = rig.mm.mm_batch_get_tuning(b.b)
    assert all(g != 0 for g in got[:2]) and (tuning[3] == got[3])
    say(f"  tuning in use {got}")
    for s in range(3):
        for k in range(len(views)):
            c, w, h, _ = views[k]
            b.set_camera(k, synth.orbit_camera(s, w, h, start_deg=37.0 * k))
        b.step_render(s)
    b.close()


def test_batch_render_only_and_camera_change(rig):
    say("case: batch render-only, then step_render after a camera change")
    clouds, views = _mixed_3d()
    b = Batch(rig, clouds, views)
    b.render()
    c, w, h, _ = views[0]
    b.set_camera(0, synth.orbit_camera(90, w, h))
    b.render()
    b.step_render(5)
    b.render()
    b.close()


def test_batch_3x3_footprint(rig):
    say("case: batch 3D mixture, 3x3 footprint, 3 clouds, 5 views, 3 frames")
    clouds = [(synth.gaussian_mixture(200000, 3), 11, 0.002, False),
              (synth.uniform_cube(50000, 4), 12, 0.001, False),
              (synth.gaussian_mixture(9000, 5), 13, 0.003, False)]
    views = [(0, 640, 360, synth.orbit_camera(0, 640, 360)),
             (0, 256, 256, synth.orbit_camera(0, 256, 256, start_deg=120.0)),
             (1, 330, 130, synth.orbit_camera(0, 330, 130, start_deg=200.0)),
             (2, 96, 64, synth.orbit_camera(0, 96, 64, start_deg=10.0)),
             (2, 512, 512, synth.orbit_camera(0, 512, 512, start_deg=300.0))]
    for tuning in [(0, 0, 0, 0, 0), (16, 8, 2, 64, 256), (32, 16, 1, 0, 1024)]:
        b = Batch(rig, clouds, views, foot=3)
        rig.mm.mm_batch_set_tuning(b.b, *tuning)
        for s in range(3):
            b.step_render(s)
        b.close()


def test_batch_2d_wrap_and_free_clouds(rig):
    say("case: batch 2D, a wrapped and a free cloud, 20 steps")
    clouds = [(synth.uniform_square(65536, 0), 0, 0.005, True),
              (synth.uniform_square(10000, 1) * np.float32(0.5), 5, 0.01, False)]
    views = [(0, 512, 512, synth.IDENTITY), (1, 256, 128, synth.IDENTITY),
             (0, 64, 64, synth.IDENTITY)]
    b = Batch(rig, clouds, views, dim=2)
    for s in range(20):
        b.step_render(s, check=(s % 5 == 4))
    b.close()


def test_batch_matches_plain_views(rig):
    say("case: batch frames equal plain-view frames on the GPU (same clouds, steps)")
    clouds, views = _mixed_3d()
    b = Batch(rig, clouds, views)
    plain = [rig.cloud(pts) for pts, _, _, _ in clouds]
    pv = []
    for k, (c, w, h, cam) in enumerate(views):
        _, seed, amp, wrap = clouds[c]
        pv.append(rig.view(plain[c][1], clouds[c][0].shape[0], 3, w, h, 1, seed, amp, wrap, cam))
    for s in range(2):
        b.step_render(s, check=False)
        # plain views: step each cloud once (first view of the cloud), render all
        stepped = set()
        for k, (c, w, h, cam) in enumerate(views):
            if c not in stepped:
                rig.mm.mm_step(pv[k], s)
                stepped.add(c)
        for k in range(len(views)):
            rig.mm.mm_render(pv[k])
        for k, (c, w, h, cam) in enumerate(views):
            got = rig.mm.mm_batch_read_frame(b.b, k, w, h)
            want = rig.mm.mm_read_frame(pv[k], w, h)
            assert np.array_equal(got, want), f"step {s} view {k}: {first_diff(got, want)}"
    b.check("after 2 frames", views=[0, 3])
    for v in pv:
        rig.mm.mm_destroy_view(v)
    b.close()


def test_batch_workload_64_clouds(rig):
    say("case: 64 clouds of 2^12..2^22 points, 1-4 views at 256/512/1024, 2 frames; "
        "every view of frame 1 checked, sampled views of frame 0")
    specs = synth.batched_set(64, seed=0)
    clouds, views = [], []
    for j, sp in enumerate(specs):
        clouds.append((synth.cloud_points(sp), sp.seed, 0.001, False))
        for (w, h, deg) in sp.views:
            views.append((j, w, h, synth.orbit_camera(0, w, h, start_deg=deg)))
    total = sum(c[0].shape[0] for c in clouds)
    say(f"  {len(clouds)} clouds, {total} points, {len(views)} views")
    b = Batch(rig, clouds, views)
    # check the views of the smallest clouds fully and two large ones
    order = sorted(range(len(views)), key=lambda k: clouds[views[k][0]][0].shape[0])
    sample = order[:6] + order[-2:]
    b.step_render(0, check=False)
    b.check("step 0", views=sample)
    b.step_render(1, check=False)
    b.check("step 1, every view")
    b.close()


def test_batch_invalid_descriptions(rig):
    mm = rig.mm
    pts = synth.uniform_cube(1000, 0)
    dev, alloc = rig.cloud(pts)
    dev2, alloc2 = rig.cloud(pts)
    good = mm.make_cloud_desc(alloc, 1000, 3, 0, 0.001)
    v = mm.make_batch_view_desc(0, 64, 64, synth.orbit_camera(0, 64, 64))

    def status(clouds, views, dim=3, foot=1):
        try:
            b = mm.mm_create_batch(rig.inst, dim, foot, clouds, views)
        except mm.MMError as e:
            return e.status
        mm.mm_destroy_batch(b)
        return mm.MM_OK

    assert status([good], [v]) == mm.MM_OK
    assert status([good, good], [v]) == mm.MM_ERR_INVALID_ARG           # shared alloc
    assert status([good], [mm.make_batch_view_desc(1, 64, 64)]) == mm.MM_ERR_INVALID_ARG
    assert status([good], [mm.make_batch_view_desc(0, 63, 64)]) == mm.MM_ERR_INVALID_ARG
    assert status([good], [mm.make_batch_view_desc(0, 8192, 4160)]) == mm.MM_ERR_UNSUPPORTED
    assert status([good], [v], foot=2) == mm.MM_ERR_INVALID_ARG
    assert status([good], [v], dim=2) == mm.MM_ERR_UNSUPPORTED          # float3 cloud, 2D
    assert status([mm.make_cloud_desc(alloc2, 2000, 3)], [v]) == mm.MM_ERR_INVALID_ARG
    assert status([], [v]) == mm.MM_ERR_INVALID_ARG
    bad_cam = np.full(16, np.nan, dtype=np.float32)
    assert status([good], [mm.make_batch_view_desc(0, 64, 64, bad_cam)]) == mm.MM_ERR_INVALID_ARG
    b = mm.mm_create_batch(rig.inst, 3, 1, [good], [v])
    for t in [(48, 0, 0, 0), (32, 3, 0, 0), (32, 16, 3, 0), (32, 16, 0, 12)]:
        with pytest.raises(mm.MMError) as e:
            mm.mm_batch_set_tuning(b, *t)
        assert e.value.status == mm.MM_ERR_INVALID_ARG, t
    with pytest.raises(mm.MMError):
        mm.mm_batch_read_frame(b, 1, 64, 64)
    with pytest.raises(mm.MMError) as e:
        mm.mm_free(alloc)
    assert e.value.status == mm.MM_ERR_IN_USE
    mm.mm_destroy_batch(b)
    mm.mm_free(alloc)
    mm.mm_free(alloc2)


def test_batch_profile(rig):
    clouds, views = _mixed_3d()
    b = Batch(rig, clouds, views)
    rig.mm.mm_batch_profile_begin(b.b, 4)
    for s in range(6):
        b.step_render(s, check=False)
    t = rig.mm.mm_batch_profile_end(b.b, 4)
    assert t.shape == (4,) and np.all(t > 0) and np.all(t < 1000)
    b.check("after profiled frames")
    b.close()


def test_autotune_restores_positions_and_keeps_parity(rig, tmp_path, monkeypatch):
    mm = rig.mm
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("MM_TUNE_CACHE", str(cache))
    say("case: autotune of a plain view (3D, 60000 points, 640x360) and of a batch")
    pts = synth.gaussian_mixture(60000, 8)
    dev, alloc = rig.cloud(pts)
    cam = synth.orbit_camera(0, 640, 360)
    view = rig.view(alloc, 60000, 3, 640, 360, 1, 4, 0.002, False, cam)
    t = mm.mm_autotune(view, 2)
    assert t == mm.mm_get_tuning(view) and t[0] in (mm.MM_SPLAT_DIRECT, mm.MM_SPLAT_BINNED)
    assert np.array_equal(rig.positions(dev).view(np.uint32), pts.view(np.uint32))
    assert cache.read_text().count("view:") == 1
    t2 = mm.mm_autotune(view, 2)           # from the cache, no timing
    assert t2 == t and cache.read_text().count("view:") == 1
    ref = pts.copy()
    mm.mm_step_render(view, 0)
    want = oracle.step_render(ref, 4, 0, 0.002, False, cam, 640, 360, 1)
    assert np.array_equal(mm.mm_read_frame(view, 640, 360), want)
    mm.mm_destroy_view(view)

    clouds, views = _mixed_3d()
    b = Batch(rig, clouds, views)
    bt = mm.mm_batch_autotune(b.b, 1)
    assert bt == mm.mm_batch_get_tuning(b.b)
    # the frames hold the last timed frame; the positions are as before
    b.check_positions("after batch autotune")
    b.step_render(0)
    assert cache.read_text().count("batch:") == 1
    b.close()
