"""Error-path contract of the C ABI under allocation failure (GPU).

mm_debug_fail_allocations(k) lets k of the library's device or pinned host
allocations succeed and fails the next one. For every k up to the number of
allocations a call makes, each test checks that the failing call
 - returns MM_ERR_OUT_OF_MEMORY,
 - leaves its out-parameters untouched (a sentinel survives),
 - gives back what it allocated: device memory free, by hipMemGetInfo, is
   back to where it was within 2 MiB, while the frame, key and record
   buffers of these sizes are 8 MiB or more each (a leak of one of the
   small tables would go unseen),
 - leaves the objects it was called on as they were: their next frames equal
   the oracle's bit for bit.
Then the call succeeds with no failure planted and is checked the same way.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from gpu_util import Rig, first_diff, say

pytestmark = pytest.mark.gpu

N, W, H = 1 << 20, 1920, 1080      # 8 MiB of records, 8 MiB frames, 16 MiB of direct keys
SEED, AMP = 77, 0.002
SLACK = 2 << 20                    # bytes of free-memory drift tolerated per check
SENTINEL = 0x5EC0_0001_D00D_F00D
MAX_ALLOCS = 64                    # no call here makes more allocations than this


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
    r.mm.mm_debug_fail_allocations(-1)
    r.close()


def _free(rig) -> int:
    rig.torch.cuda.synchronize()
    return rig.torch.cuda.mem_get_info(0)[0]


def _sentinel():
    return C.c_void_p(SENTINEL)


def _fail_each(rig, attempt, what):
    """Runs attempt() with the k-th allocation failing for k = 0, 1, ... until
    it succeeds with none failing; returns (allocations made, its result)."""
    mm = rig.mm
    for k in range(MAX_ALLOCS):
        before = _free(rig)
        mm.mm_debug_fail_allocations(k)
        st, out = attempt()
        mm.mm_debug_fail_allocations(-1)
        if st == mm.MM_OK:
            say(f"{what}: succeeds with {k} allocations")
            return k, out
        assert st == mm.MM_ERR_OUT_OF_MEMORY, f"{what}, failing allocation {k}: status {st} ({mm.mm_last_error()})"
        assert out == SENTINEL, f"{what}, failing allocation {k}: out-parameter written ({out:#x})"
        assert "fail" in mm.mm_last_error().lower() or "memory" in mm.mm_last_error().lower()
        drift = before - _free(rig)
        assert drift <= SLACK, f"{what}, failing allocation {k}: {drift} bytes not given back"
    raise AssertionError(f"{what}: still failing after {MAX_ALLOCS} allocations")


def _view_desc(rig, alloc, foot=1):
    return rig.mm.make_view_desc(alloc, N, 3, W, H, foot, SEED, AMP, False, synth.orbit_camera(0, W, H))


def _check_view(rig, view, dev, ref, step, what, overlap=False, foot=1):
    mm = rig.mm
    mm.mm_step_render(view, step)
    oracle.displace(ref, SEED, step, AMP, False)
    if overlap:
        mm.mm_flush_frame(view)
    got = mm.mm_read_frame(view, W, H)
    want = oracle.render(ref, SEED, synth.orbit_camera(0, W, H), W, H, foot)
    assert np.array_equal(got, want), f"{what}: {first_diff(got, want)}"
    assert np.array_equal(rig.positions(dev).view(np.uint32), ref.view(np.uint32)), f"{what}: positions"


def test_alloc_linear_failure(rig):
    mm, L = rig.mm, rig.mm.lib()
    ptr, out = _sentinel(), _sentinel()

    def attempt():
        ptr.value, out.value = SENTINEL, SENTINEL
        st = L.mm_alloc_linear(rig.inst, 64 << 20, C.byref(ptr), C.byref(out))
        assert st != mm.MM_OK or ptr.value != SENTINEL
        if st != mm.MM_OK:
            assert ptr.value == SENTINEL, "dev_ptr written on failure"
        return st, out.value

    k, alloc = _fail_each(rig, attempt, "mm_alloc_linear")
    assert k == 1
    mm.mm_free(alloc)


@pytest.mark.parametrize("splat,foot", [(2, 1), (1, 1), (2, 3)], ids=["binned", "direct", "binned-foot3"])
def test_create_view_failure(rig, splat, foot):
    mm, L = rig.mm, rig.mm.lib()
    pts = synth.uniform_cube(N, 5)
    dev, alloc = rig.cloud(pts)
    d = _view_desc(rig, alloc, foot)
    out = _sentinel()

    def attempt():
        out.value = SENTINEL
        return L.mm_create_view(rig.inst, C.byref(d), C.byref(out)), out.value

    k, view = _fail_each(rig, attempt, f"mm_create_view ({foot=})")
    assert k >= 2
    # the alloc must not count a user for any failed view: it can be freed
    # once the one view made is gone (checked at the end)
    ref = pts.copy()
    mm.mm_set_tuning(view, splat)
    _check_view(rig, view, dev, ref, 0, "view made after failures", foot=foot)
    mm.mm_destroy_view(view)
    mm.mm_free(alloc)


def test_set_tuning_failure_keeps_the_tuning(rig):
    mm, L = rig.mm, rig.mm.lib()
    pts = synth.gaussian_mixture(N, 6)
    dev, alloc = rig.cloud(pts)
    view = mm.mm_create_view(rig.inst, _view_desc(rig, alloc))
    mm.mm_set_tuning(view, mm.MM_SPLAT_BINNED, 32, 8, 1, 1024)
    had = mm.mm_get_tuning(view)
    ref = pts.copy()
    step = [0]

    def attempt(t):
        def run():
            st = L.mm_set_tuning(view, C.byref(mm.mm_tuning(*t)))
            if st != mm.MM_OK:
                assert mm.mm_get_tuning(view) == had, "tuning changed by a failed call"
                _check_view(rig, view, dev, ref, step[0], f"after failed set_tuning {t}")
                step[0] += 1
            return st, SENTINEL
        return run

    for t in [(mm.MM_SPLAT_BINNED, 64, 4, 1, 512, 0, 0), (mm.MM_SPLAT_DIRECT, 0, 0, 0, 0, 0, 0),
              (mm.MM_SPLAT_BINNED, 32, 8, 2, 1024, 0, 0), (mm.MM_SPLAT_BINNED, 32, 16, 1, 512, mm.MM_PIECES_STATIC, mm.MM_CULL_ON)]:
        _fail_each(rig, attempt(t), f"mm_set_tuning {t}")
        got = mm.mm_get_tuning(view)
        _check_view(rig, view, dev, ref, step[0], f"after set_tuning {t}")
        step[0] += 1
        mm.mm_set_tuning(view, *had)  # back, for the next shape's failures
        assert mm.mm_get_tuning(view) == had
        assert got != had
    mm.mm_destroy_view(view)


def test_frame_overlap_failure_keeps_the_mode(rig):
    mm, L = rig.mm, rig.mm.lib()
    pts = synth.uniform_cube(N, 7)
    dev, alloc = rig.cloud(pts)
    view = mm.mm_create_view(rig.inst, _view_desc(rig, alloc))
    ref = pts.copy()
    step = [0]
    for on in (1, 0):
        def run():
            st = L.mm_set_frame_overlap(view, on)
            if st != mm.MM_OK:  # still in the other mode: frames lag only when overlapped
                _check_view(rig, view, dev, ref, step[0], f"after failed overlap {on}", overlap=bool(1 - on))
                step[0] += 1
            return st, SENTINEL
        k, _ = _fail_each(rig, run, f"mm_set_frame_overlap({on})")
        assert k >= 1
        _check_view(rig, view, dev, ref, step[0], f"overlap {on}", overlap=bool(on))
        step[0] += 1
    mm.mm_destroy_view(view)


def test_autotune_failure_leaves_the_cloud(rig):
    mm, L = rig.mm, rig.mm.lib()
    pts = synth.uniform_cube(N, 8)
    dev, alloc = rig.cloud(pts)
    view = mm.mm_create_view(rig.inst, _view_desc(rig, alloc))
    had = mm.mm_get_tuning(view)
    out = mm.mm_tuning(*[0xDEAD] * 7)
    mm.mm_debug_fail_allocations(0)  # the positions' backup
    st = L.mm_autotune(view, 1, C.byref(out))
    mm.mm_debug_fail_allocations(-1)
    assert st == mm.MM_ERR_OUT_OF_MEMORY, mm.mm_last_error()
    assert mm._tuning_tuple(out) == (0xDEAD,) * 7
    assert mm.mm_get_tuning(view) == had
    ref = pts.copy()
    _check_view(rig, view, dev, ref, 0, "after failed autotune")
    mm.mm_destroy_view(view)


def _batch_parts(rig):
    mm = rig.mm
    clouds, descs = [], []
    for j in range(2):
        pts = synth.uniform_cube(N // 2, 40 + j) if j == 0 else synth.gaussian_mixture(N // 2, 40 + j)
        dev, alloc = rig.cloud(pts)
        clouds.append((pts, dev))
        descs.append(mm.make_cloud_desc(alloc, N // 2, 3, SEED + j, AMP))
    views = [(0, W, H, synth.orbit_camera(0, W, H)), (1, 640, 480, synth.orbit_camera(30, 640, 480)),
             (0, 512, 512, synth.orbit_camera(90, 512, 512))]
    vds = [mm.make_batch_view_desc(c, w, h, cam) for c, w, h, cam in views]
    return clouds, descs, views, vds


def _check_batch(rig, b, clouds, refs, views, step, what):
    mm = rig.mm
    mm.mm_batch_step_render(b, step)
    for j in range(len(clouds)):
        oracle.displace(refs[j], SEED + j, step, AMP, False)
    for k, (c, w, h, cam) in enumerate(views):
        got = mm.mm_batch_read_frame(b, k, w, h)
        want = oracle.render(refs[c], SEED + c, cam, w, h, 1)
        assert np.array_equal(got, want), f"{what}, view {k}: {first_diff(got, want)}"


def test_create_batch_and_set_tuning_failures(rig):
    mm, L = rig.mm, rig.mm.lib()
    clouds, descs, views, vds = _batch_parts(rig)
    ca = (mm.mm_cloud_desc * len(descs))(*descs)
    va = (mm.mm_batch_view_desc * len(vds))(*vds)
    d = mm.mm_batch_desc()
    d.domain, d.footprint = mm.MM_DOMAIN_3D, 1
    d.n_clouds, d.clouds, d.n_views, d.views = len(descs), ca, len(vds), va
    out = _sentinel()

    def create():
        out.value = SENTINEL
        return L.mm_create_batch(rig.inst, C.byref(d), C.byref(out)), out.value

    k, b = _fail_each(rig, create, "mm_create_batch")
    assert k >= len(vds) + 2
    refs = [c[0].copy() for c in clouds]
    _check_batch(rig, b, clouds, refs, views, 0, "batch made after failures")
    had = mm.mm_batch_get_tuning(b)
    step = [1]

    def retune():
        st = L.mm_batch_set_tuning(b, C.byref(mm.mm_batch_tuning(64, 4, 2, 0, 512)))
        if st != mm.MM_OK:
            assert mm.mm_batch_get_tuning(b) == had
            _check_batch(rig, b, clouds, refs, views, step[0], "after failed batch_set_tuning")
            step[0] += 1
        return st, SENTINEL

    _fail_each(rig, retune, "mm_batch_set_tuning")
    assert mm.mm_batch_get_tuning(b) != had
    _check_batch(rig, b, clouds, refs, views, step[0], "after batch_set_tuning")
    mm.mm_destroy_batch(b)


def _server(rig):
    mm, L = rig.mm, rig.mm.lib()
    d = mm.mm_server_desc()
    d.fb_budget_bytes = 64 << 20
    d.streams, d.max_batch = 2, 16
    d.domain, d.footprint = mm.MM_DOMAIN_3D, 1
    d.tuning = mm.mm_batch_tuning(0, 0, 0, 0, 0)
    out = _sentinel()

    def create():
        out.value = SENTINEL
        return L.mm_create_server(rig.inst, C.byref(d), C.byref(out)), out.value

    k, srv = _fail_each(rig, create, "mm_create_server")
    assert k >= 1
    pts = synth.uniform_cube(N, 9)
    dev, alloc = rig.cloud(pts)
    cloud = mm.mm_server_add_cloud(srv, mm.make_cloud_desc(alloc, N, 3, SEED, AMP))
    return srv, cloud, pts


def _refused(rig, srv, cloud, cam):
    mm, L = rig.mm, rig.mm.lib()
    rid = C.c_uint64(SENTINEL)
    m = np.ascontiguousarray(cam, dtype=np.float32).reshape(16)
    st = L.mm_server_submit(srv, 1, cloud, mm._fptr(m), W, H, None, C.byref(rid))
    assert st != mm.MM_OK and rid.value == SENTINEL, (st, rid.value)


def test_server_recovers_by_eviction(rig):
    """A frame buffer that cannot be had is found by evicting an idle session."""
    mm = rig.mm
    srv, cloud, pts = _server(rig)
    cam = synth.orbit_camera(0, W, H)
    cam2 = synth.orbit_camera(40, 512, 512)
    rid = mm.mm_server_submit(srv, 1, cloud, cam, W, H)
    mm.mm_server_wait(srv, rid)
    ref = pts.copy()
    oracle.displace(ref, SEED, 0, AMP, False)
    got = mm.mm_server_read_frame(srv, 1, W, H)
    want = oracle.render(ref, SEED, cam, W, H, 1)
    assert np.array_equal(got, want), first_diff(got, want)
    mm.mm_debug_fail_allocations(0)       # session 2's buffer: fails once
    rid2 = mm.mm_server_submit(srv, 2, cloud, cam2, 512, 512)
    mm.mm_server_wait(srv, rid2)
    mm.mm_debug_fail_allocations(-1)
    oracle.displace(ref, SEED, 1, AMP, False)
    got = mm.mm_server_read_frame(srv, 2, 512, 512)
    want = oracle.render(ref, SEED, cam2, 512, 512, 1)
    assert np.array_equal(got, want), first_diff(got, want)
    st = mm.mm_server_stats_get(srv)
    assert st["evictions"] >= 1 and st["dropped"] == 0, st
    mm.mm_destroy_server(srv)


@pytest.mark.parametrize("after,what", [(0, "frame buffer"), (1, "staging of the launch")])
def test_server_stops_when_memory_cannot_be_had(rig, after, what):
    """Nothing to evict and nothing in flight (the frame buffer), or a launch
    that cannot go out (its staging buffer): the requests are dropped, their
    waiters return with an error, and the server takes no more work."""
    mm = rig.mm
    srv, cloud, _ = _server(rig)
    cam = synth.orbit_camera(0, W, H)
    mm.mm_debug_fail_allocations(after)
    rids = []
    for s in (1, 2, 3):
        try:
            rids.append(mm.mm_server_submit(srv, s, cloud, cam, W, H))
        except mm.MMError:  # the server stopped before this submit
            break
    assert rids
    for rid in rids:
        with pytest.raises(mm.MMError):
            mm.mm_server_wait(srv, rid)
    mm.mm_debug_fail_allocations(-1)
    st = mm.mm_server_stats_get(srv)
    assert st["dropped"] == len(rids) and st["completed"] == 0, (what, st)
    _refused(rig, srv, cloud, cam)
    mm.mm_destroy_server(srv)


def test_static_frame_allocates_nothing(rig):
    """The entry point for callers that cannot allocate makes no allocation
    through the library: every allocation failing changes nothing."""
    mm, torch = rig.mm, rig.torch
    pts = synth.uniform_cube(N, 10)
    dev = torch.from_numpy(pts.copy()).cuda()
    rgba = torch.empty((H, W), dtype=torch.int32, device="cuda")
    cam = synth.orbit_camera(0, W, H)
    mm.mm_debug_fail_allocations(0)
    mm.mm_step_render_static(dev.data_ptr(), N, 3, W, H, rgba.data_ptr(), 0, 1, SEED, AMP, False, cam,
                             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    # the planted failure is still pending: nothing consumed it
    pl = mm.mm_alloc_linear
    with pytest.raises(mm.MMError):
        pl(rig.inst, 1 << 20)
    mm.mm_debug_fail_allocations(-1)
    ref = pts.copy()
    oracle.displace(ref, SEED, 0, AMP, False)
    want = oracle.render(ref, SEED, cam, W, H, 1)
    got = rgba.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want), first_diff(got, want)
