"""GPU parity of the edges view: frames equal the oracle's bit for bit for
vertex pairs and triangles, 2D and 3D, long and off-screen segments, index
values past the vertex count, and camera changes between renders."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import Rig, first_diff, say

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


def _u32_alloc(rig, arr):
    t = rig.torch.from_numpy(np.ascontiguousarray(arr, dtype=np.uint32).view(np.int32)).cuda()
    rig.keep.append(t)
    return rig.mm.mm_alloc_wrap(rig.inst, t.data_ptr(), t.numel() * 4)


@pytest.mark.parametrize("prim", [2, 3])
@pytest.mark.parametrize("dim", [2, 3])
def test_edges_match_oracle(rig, prim, dim):
    say(f"case: edges, dim {dim}, {prim} vertices per primitive")
    mm = rig.mm
    w, h, seed = 640, 360, 5
    rng = np.random.default_rng(prim * 10 + dim)
    nv = 20000
    if dim == 2:
        pos = rng.uniform(-1.2, 1.2, size=(nv, 2)).astype(np.float32)  # some off screen
        cams = [synth.IDENTITY]
    else:
        pos = synth.gaussian_mixture(nv, 3, sigma=0.08)
        cams = [synth.orbit_camera(a, w, h) for a in (0, 50, 200)]
    nprim = 30000
    # mostly short segments between nearby indices, some long ones, a few past the end
    base = rng.integers(0, nv - 8, nprim)
    idx = np.stack([base + rng.integers(0, 8, nprim) for _ in range(prim)], axis=1).astype(np.uint32)
    idx[rng.integers(0, nprim, 200)] = rng.integers(0, nv, (200, prim))
    idx[rng.integers(0, nprim, 20), 0] = nv + 5
    dev, alloc = rig.cloud(pos)
    ia = _u32_alloc(rig, idx.reshape(-1))
    v = mm.mm_create_edges(rig.inst, alloc, nv, dim, ia, nprim, prim, w, h, seed, cams[0])
    for cam in cams:
        mm.mm_edges_set_camera(v, cam)
        mm.mm_edges_render(v)
        want = oracle.render_edges(pos, idx.reshape(-1), prim, seed, cam, w, h)
        got = mm.mm_edges_read_frame(v, w, h)
        assert np.array_equal(got, want), first_diff(got, want)
    mm.mm_destroy_edges(v)


def test_edges_follow_moving_vertices(rig):
    say("case: edges over a displaced cloud (a view and an edges view on one alloc)")
    mm = rig.mm
    w, h, seed, amp = 320, 240, 2, 0.01
    pos = synth.uniform_cube(5000, seed=2)
    dev, alloc = rig.cloud(pos)
    rng = np.random.default_rng(1)
    idx = rng.integers(0, 5000, (4000, 2)).astype(np.uint32)
    ia = _u32_alloc(rig, idx.reshape(-1))
    cam = synth.orbit_camera(15, w, h)
    view = rig.view(alloc, 5000, 3, w, h, 1, seed, amp, False, cam)
    e = mm.mm_create_edges(rig.inst, alloc, 5000, 3, ia, 4000, 2, w, h, seed, cam)
    ref = pos.copy()
    for s in range(3):
        mm.mm_step(view, s)
        oracle.displace(ref, seed, s, amp, False)
        mm.mm_edges_render(e)
        want = oracle.render_edges(ref, idx.reshape(-1), 2, seed, cam, w, h)
        assert np.array_equal(mm.mm_edges_read_frame(e, w, h), want)
    mm.mm_destroy_edges(e)
    mm.mm_destroy_view(view)


def test_edges_validation(rig):
    say("case: edges validation")
    mm = rig.mm
    pos = synth.uniform_cube(100, seed=0)
    dev, alloc = rig.cloud(pos)
    ia = _u32_alloc(rig, np.zeros(60, np.uint32))
    cam = synth.orbit_camera(0, 64, 64)
    for args, what in [((alloc, 100, 3, ia, 31, 2, 64, 64, 0, cam), "more indices than the alloc"),
                       ((alloc, 100, 3, ia, 21, 3, 64, 64, 0, cam), "more triangle indices than the alloc"),
                       ((alloc, 100, 3, ia, 10, 4, 64, 64, 0, cam), "vertices per primitive"),
                       ((alloc, 100, 3, ia, 0, 2, 64, 64, 0, cam), "no primitives"),
                       ((alloc, 101, 3, ia, 10, 2, 64, 64, 0, cam), "more vertices than the alloc"),
                       ((alloc, 100, 3, ia, 10, 2, 65, 64, 0, cam), "odd screen")]:
        with pytest.raises(mm.MMError) as e:
            mm.mm_create_edges(rig.inst, *args)
        assert e.value.status == mm.MM_ERR_INVALID_ARG, what
    v = mm.mm_create_edges(rig.inst, alloc, 100, 3, ia, 30, 2, 64, 64, 0, cam)
    with pytest.raises(mm.MMError) as e:
        mm.mm_free(ia)
    assert e.value.status == mm.MM_ERR_IN_USE
    bad = cam.copy().reshape(-1)
    bad[3] = np.nan
    with pytest.raises(mm.MMError):
        mm.mm_edges_set_camera(v, bad)
    mm.mm_destroy_edges(v)
    mm.mm_free(ia)
