"""GPU parity of the served form: each request's frame equals the frame of its
cloud rendered alone after the same steps (the k-th request on a cloud
displaces it with step k), whatever else was queued or in flight, under any
batching, stream count and memory budget."""
import time

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


def _clouds(rig, sizes, seed0=20):
    out = []
    for j, n in enumerate(sizes):
        pts = synth.uniform_cube(n, seed0 + j) if j % 2 == 0 else synth.gaussian_mixture(n, seed0 + j)
        dev, alloc = rig.cloud(pts)
        out.append((pts, dev, alloc, 300 + j, 0.002))
    return out


def _expected(clouds, reqs, foot):
    """reqs in submission order: (cloud, cam, w, h). Replays each cloud's steps."""
    refs = [c[0].copy() for c in clouds]
    steps = [0] * len(clouds)
    want = []
    for c, cam, w, h in reqs:
        _, _, _, seed, amp = clouds[c]
        oracle.displace(refs[c], seed, steps[c], amp, False)
        steps[c] += 1
        want.append(oracle.render(refs[c], seed, cam, w, h, foot))
    return want, refs


def _serve(rig, clouds, sessions, order, budget, streams, max_batch, foot=1,
           tuning=(0, 0, 0, 0, 0), gate=0):
    """order: [(session, cloud, frame)]; every request renders into its own
    buffer. gate: each of the first `gate` requests has gone to the device in
    a launch of its own before the next one is submitted."""
    mm, torch = rig.mm, rig.torch
    srv = mm.mm_create_server(rig.inst, budget, streams, max_batch, 3, foot, *tuning)
    ids = [mm.mm_server_add_cloud(srv, mm.make_cloud_desc(c[2], c[0].shape[0], 3, c[3], c[4]))
           for c in clouds]
    assert ids == list(range(len(clouds)))
    reqs, outs, rids = [], [], []
    for s, c, f in order:
        w, h, deg = sessions[s]
        reqs.append((c, synth.orbit_camera(f, w, h, start_deg=deg), w, h))
        outs.append(torch.zeros((h, w), dtype=torch.int32, device="cuda"))
    # outputs ready before the first submission; no device-wide wait between
    # submissions, so requests arrive while earlier launches run
    torch.cuda.synchronize()
    for k, ((s, _, _), (c, cam, w, h), out) in enumerate(zip(order, reqs, outs)):
        rids.append(mm.mm_server_submit(srv, s, c, cam, w, h, out.data_ptr()))
        if k < gate:
            t0 = time.perf_counter()
            while mm.mm_server_stats_get(srv)["launches"] < k + 1:
                assert time.perf_counter() - t0 < 10.0, f"request {k} was not launched"
    lat = [mm.mm_server_wait(srv, r) for r in rids]
    stats = mm.mm_server_stats_get(srv)
    mm.mm_destroy_server(srv)
    return reqs, outs, lat, stats


SESSIONS = {0: (64, 48, 0.0), 1: (256, 256, 40.0), 2: (640, 360, 80.0), 3: (128, 96, 120.0),
            4: (300, 200, 160.0), 5: (512, 512, 200.0), 6: (70, 38, 240.0), 7: (1024, 576, 280.0)}


@pytest.mark.parametrize("streams,max_batch", [(1, 1), (2, 4), (4, 64)])
def test_server_results_equal_each_request_alone(rig, streams, max_batch):
    say(f"case: server, 5 clouds, 8 sessions, 48 interleaved requests, streams {streams}, "
        f"max_batch {max_batch}")
    clouds = _clouds(rig, [5000, 70001, 1, 200000, 4097])
    rng = np.random.default_rng(5)
    order = [(int(rng.integers(0, 8)), int(rng.integers(0, 5)), f) for f in range(48)]
    reqs, outs, lat, stats = _serve(rig, clouds, SESSIONS, order, 1 << 34, streams, max_batch)
    want, refs = _expected(clouds, reqs, 1)
    for k, (got, exp) in enumerate(zip(outs, want)):
        g = got.cpu().numpy().view(np.uint32)
        assert np.array_equal(g, exp), f"request {k} {order[k]}: {first_diff(g, exp)}"
    for j, c in enumerate(clouds):
        pos = rig.positions(c[1])
        assert np.array_equal(pos.view(np.uint32), refs[j].view(np.uint32)), f"cloud {j} positions"
    assert stats["completed"] == 48 and stats["submitted"] == 48
    assert all(x > 0 for x in lat)
    say(f"  launches {stats['launches']}, p50 latency {np.median(lat) * 1e3:.2f} ms")


def test_server_served_screens_and_large_clouds(rig):
    """The served workload's own screens (1280x720, 1920x1080, 3840x2160) and
    clouds from the upper half of the batched set's sizes (2^20, 2^22
    points), so that launches take two splits per tile and the merge, at
    4K tile tables; every request against the oracle's replay of its cloud.
    Requests arrive while launches are on the device: some launches carry
    several requests, and two launches are in flight at once."""
    clouds = _clouds(rig, [1 << 20, 1 << 22, 70000, (1 << 22) - 333])
    sessions = {0: (1280, 720, 10.0), 1: (1920, 1080, 50.0), 2: (3840, 2160, 95.0),
                3: (1280, 720, 140.0), 4: (1920, 1080, 185.0), 5: (3840, 2160, 230.0)}
    rng = np.random.default_rng(17)
    # a 4K request on a 2^22-point cloud first (about a millisecond on the
    # device) in a launch of its own, then one on another cloud, which goes
    # out on the second stream beside it (nothing is queued behind the first
    # cloud yet, so it does not wait for it); the rest arrive while those run
    # and pack into launches
    order = [(2, 1, 0), (0, 0, 1)] + [(int(rng.integers(0, 6)), int(rng.integers(0, 4)), f)
                                      for f in range(2, 30)]
    say(f"case: server, 4 clouds (2^20, 2^22, 70000, 2^22-333 points), 6 sessions at "
        f"720p/1080p/4K, 30 requests, 2 streams, max_batch 8")
    reqs, outs, lat, stats = _serve(rig, clouds, sessions, order, 1 << 36, 2, 8, gate=2)
    say(f"  stats {stats}")
    want, refs = _expected(clouds, reqs, 1)
    for k, (got, exp) in enumerate(zip(outs, want)):
        g = got.cpu().numpy().view(np.uint32)
        assert np.array_equal(g, exp), f"request {k} {order[k]}: {first_diff(g, exp)}"
    for j, c in enumerate(clouds):
        pos = rig.positions(c[1])
        assert np.array_equal(pos.view(np.uint32), refs[j].view(np.uint32)), f"cloud {j} positions"
    assert stats["completed"] == 30 and stats["dropped"] == 0
    # continuous batching: fewer launches than requests, several requests in
    # one launch, and a second launch sent while another was in flight
    assert stats["launches"] < stats["completed"], stats
    assert stats["max_batch"] >= 2, stats
    assert stats["max_in_flight"] >= 2, stats


def test_server_one_buffer_two_sessions_one_cloud(rig):
    """Two sessions share a cloud under a budget of one frame buffer, with
    submissions A0, B0, A1: after A0, B0 needs A's buffer while A still has
    A1 queued. A must be evicted for B0 all the same, or the served loop has
    nothing to run. Polled against a host deadline, so that a stall fails
    the test instead of hanging it."""
    mm = rig.mm
    clouds = _clouds(rig, [20000])
    w, h = 256, 256
    # the budget: exactly one 256x256 frame buffer of this server's shape
    # (RGBA8, two splits of 64x64-pixel u64 partial tiles, one stamp per tile)
    budget = 256 * 256 * 4 + 16 * 2 * 64 * 64 * 8 + 256
    srv = mm.mm_create_server(rig.inst, budget, 1, 8, 3, 1)
    c = clouds[0]
    mm.mm_server_add_cloud(srv, mm.make_cloud_desc(c[2], c[0].shape[0], 3, c[3], c[4]))
    cams = [synth.orbit_camera(f, w, h, start_deg=30.0 * f) for f in range(3)]
    say("case: server, budget of one 256x256 buffer, sessions A, B on one cloud: A0, B0, A1")
    rids = [mm.mm_server_submit(srv, s, 0, cams[k], w, h) for k, s in enumerate([0, 1, 0])]
    deadline = time.monotonic() + 30.0
    while True:
        done = [mm.mm_server_poll(srv, r)[0] for r in rids]
        if all(done):
            break
        assert time.monotonic() < deadline, f"served loop stalled: done {done}, " \
            f"stats {mm.mm_server_stats_get(srv)}"
        time.sleep(0.002)
    # the last request drew session A's frame: the cloud after steps 0, 1, 2
    ref = c[0].copy()
    for k in range(3):
        oracle.displace(ref, c[3], k, c[4], False)
    want = oracle.render(ref, c[3], cams[2], w, h, 1)
    got = mm.mm_server_read_frame(srv, 0, w, h)
    assert np.array_equal(got, want), first_diff(got, want)
    st = mm.mm_server_stats_get(srv)
    assert st["completed"] == 3 and st["evictions"] >= 2 and st["fb_bytes_in_use"] <= budget
    mm.mm_destroy_server(srv)


def test_server_small_budget_queues_and_evicts(rig):
    mm = rig.mm
    clouds = _clouds(rig, [30000, 60000, 9000])
    # about two 512x512 sessions: RGBA8 frame, two splits of 64x64-pixel u64
    # partial tiles, one stamp per tile
    budget = 2 * (512 * 512 * 4 + 64 * 2 * 64 * 64 * 8 + 64 * 4) + 4096
    say(f"case: server, budget {budget} B, 6 sessions of 256^2..512^2, 36 requests")
    sessions = {0: (256, 256, 0.0), 1: (512, 512, 60.0), 2: (384, 256, 120.0),
                3: (256, 384, 180.0), 4: (512, 512, 240.0), 5: (128, 128, 300.0)}
    rng = np.random.default_rng(9)
    order = [(int(rng.integers(0, 6)), int(rng.integers(0, 3)), f) for f in range(36)]
    reqs, outs, lat, stats = _serve(rig, clouds, sessions, order, budget, 2, 16)
    want, _ = _expected(clouds, reqs, 1)
    for k, (got, exp) in enumerate(zip(outs, want)):
        g = got.cpu().numpy().view(np.uint32)
        assert np.array_equal(g, exp), f"request {k} {order[k]}: {first_diff(g, exp)}"
    say(f"  stats {stats}")
    assert stats["evictions"] > 0 and stats["fb_bytes_in_use"] <= budget


def test_server_frame_buffer_holds_the_last_request(rig):
    mm = rig.mm
    say("case: server, requests drawn into session frame buffers, read back")
    clouds = _clouds(rig, [50000, 8000])
    srv = mm.mm_create_server(rig.inst, 1 << 32, 2, 8, 3, 1)
    for c in clouds:
        mm.mm_server_add_cloud(srv, mm.make_cloud_desc(c[2], c[0].shape[0], 3, c[3], c[4]))
    sessions = {0: (320, 240, 0.0), 1: (160, 120, 90.0), 2: (320, 240, 180.0)}
    refs = [c[0].copy() for c in clouds]
    steps = [0, 0]
    for f in range(3):
        for s, c in [(0, 0), (1, 1), (2, 0), (1, 0)]:
            w, h, deg = sessions[s]
            cam = synth.orbit_camera(f, w, h, start_deg=deg)
            r = mm.mm_server_submit(srv, s, c, cam, w, h)
            mm.mm_server_wait(srv, r)
            _, _, _, seed, amp = clouds[c]
            oracle.displace(refs[c], seed, steps[c], amp, False)
            steps[c] += 1
            want = oracle.render(refs[c], seed, cam, w, h, 1)
            got = mm.mm_server_read_frame(srv, s, w, h)
            assert np.array_equal(got, want), f"frame {f} session {s}: {first_diff(got, want)}"
    mm.mm_server_close_session(srv, 1)
    with pytest.raises(mm.MMError) as e:
        mm.mm_server_read_frame(srv, 1, 160, 120)
    assert e.value.status == mm.MM_ERR_NOT_READY
    st = mm.mm_server_stats_get(srv)
    assert st["completed"] == 12 and st["admitted_sessions"] == 2
    mm.mm_destroy_server(srv)


def test_server_session_frames_clear_what_the_last_frame_drew(rig):
    """A session's frame buffer clears only the tiles its previous frame drew
    and this one does not. A dense cloud (60,000 points) and a sparse one
    (12 points) alternate in one session's buffer, so most tiles go from
    drawn to clear and back. With a budget of one buffer, two sessions of one
    screen then hand the buffer back and forth through the pool, each frame
    drawn over the other session's. Every frame is read back and compared
    with the oracle's."""
    mm = rig.mm
    say("case: server, session frames over dense and sparse clouds, one-buffer pool")
    clouds = _clouds(rig, [60000, 12])
    refs = [c[0].copy() for c in clouds]
    steps = [0, 0]

    def serve(srv, s, c, f, w, h, deg):
        cam = synth.orbit_camera(f, w, h, start_deg=deg)
        r = mm.mm_server_submit(srv, s, c, cam, w, h)
        mm.mm_server_wait(srv, r)
        _, _, _, seed, amp = clouds[c]
        oracle.displace(refs[c], seed, steps[c], amp, False)
        steps[c] += 1
        want = oracle.render(refs[c], seed, cam, w, h, 1)
        got = mm.mm_server_read_frame(srv, s, w, h)
        assert np.array_equal(got, want), f"session {s} cloud {c} frame {f}: {first_diff(got, want)}"

    srv = mm.mm_create_server(rig.inst, 1 << 32, 2, 4, 3, 1)
    for c in clouds:
        mm.mm_server_add_cloud(srv, mm.make_cloud_desc(c[2], c[0].shape[0], 3, c[3], c[4]))
    for f, c in enumerate([0, 1, 1, 0, 1, 0, 0, 1]):
        serve(srv, 0, c, f, 320, 200, 30.0)
    mm.mm_destroy_server(srv)
    # one 256x192 frame buffer (under 1 MB with its tile scratch) fits the budget, two do not;
    # a new server counts each cloud's steps from 0 again (on the positions reached so far)
    steps[:] = [0, 0]
    srv = mm.mm_create_server(rig.inst, 1 << 20, 1, 4, 3, 1)
    for c in clouds:
        mm.mm_server_add_cloud(srv, mm.make_cloud_desc(c[2], c[0].shape[0], 3, c[3], c[4]))
    for f in range(6):
        serve(srv, f % 2, f % 2, 8 + f, 256, 192, 60.0 * (f % 2))
    st = mm.mm_server_stats_get(srv)
    assert st["evictions"] >= 4 and st["admitted_sessions"] == 1, st
    mm.mm_destroy_server(srv)
    # a frame into the caller's buffer between two into the session's own: the
    # session's buffer still holds the frame before it, so the frame after it
    # clears every tile it does not draw
    steps[:] = [0, 0]
    torch = rig.torch
    srv = mm.mm_create_server(rig.inst, 1 << 32, 2, 4, 3, 1)
    for c in clouds:
        mm.mm_server_add_cloud(srv, mm.make_cloud_desc(c[2], c[0].shape[0], 3, c[3], c[4]))
    serve(srv, 3, 0, 20, 200, 160, 10.0)
    out = torch.zeros((160, 200), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    cam = synth.orbit_camera(21, 200, 160, start_deg=10.0)
    mm.mm_server_wait(srv, mm.mm_server_submit(srv, 3, 1, cam, 200, 160, out.data_ptr()))
    _, _, _, seed, amp = clouds[1]
    oracle.displace(refs[1], seed, steps[1], amp, False)
    steps[1] += 1
    got = out.cpu().numpy().view(np.uint32)
    want = oracle.render(refs[1], seed, cam, 200, 160, 1)
    assert np.array_equal(got, want), f"frame into the caller's buffer: {first_diff(got, want)}"
    serve(srv, 3, 1, 22, 200, 160, 10.0)
    serve(srv, 3, 0, 23, 200, 160, 10.0)
    mm.mm_destroy_server(srv)


def test_server_3x3_footprint(rig):
    say("case: server, 3x3 footprint, 3 clouds, 4 sessions, 20 requests")
    clouds = _clouds(rig, [40000, 9000, 120000])
    sessions = {0: (256, 192, 0.0), 1: (330, 130, 70.0), 2: (96, 64, 140.0), 3: (640, 480, 210.0)}
    rng = np.random.default_rng(3)
    order = [(int(rng.integers(0, 4)), int(rng.integers(0, 3)), f) for f in range(20)]
    reqs, outs, lat, stats = _serve(rig, clouds, sessions, order, 1 << 33, 2, 8, foot=3,
                                    tuning=(16, 8, 0, 0, 512))
    want, _ = _expected(clouds, reqs, 3)
    for k, (got, exp) in enumerate(zip(outs, want)):
        g = got.cpu().numpy().view(np.uint32)
        assert np.array_equal(g, exp), f"request {k} {order[k]}: {first_diff(g, exp)}"


def test_server_rejects_invalid_requests(rig):
    mm = rig.mm
    clouds = _clouds(rig, [1000])
    srv = mm.mm_create_server(rig.inst, 64 * 64 * 40, 1, 4, 3, 1)
    mm.mm_server_add_cloud(srv, mm.make_cloud_desc(clouds[0][2], 1000, 3, 1, 0.001))
    cam = synth.orbit_camera(0, 64, 64)

    def status(fn):
        try:
            fn()
        except mm.MMError as e:
            return e.status
        return mm.MM_OK

    assert status(lambda: mm.mm_server_submit(srv, 0, 0, cam, 1024, 1024)) == mm.MM_ERR_BUDGET
    assert status(lambda: mm.mm_server_submit(srv, 0, 1, cam, 64, 64)) == mm.MM_ERR_INVALID_ARG
    assert status(lambda: mm.mm_server_submit(srv, 0, 0, cam, 63, 64)) == mm.MM_ERR_INVALID_ARG
    r = mm.mm_server_submit(srv, 0, 0, cam, 64, 64)
    assert status(lambda: mm.mm_server_submit(srv, 0, 0, cam, 32, 32)) == mm.MM_ERR_INVALID_ARG
    # a 1 MiB allocation cannot hold a 1024x1024 frame (4 MiB); the frame buffer
    # of such a session would also exceed this server's budget, so the request
    # is refused either way
    ptr, small = mm.mm_alloc_linear(rig.inst, 1 << 20)
    assert status(lambda: mm.mm_server_submit(srv, 1, 0, cam, 1024, 1024, ptr)) == \
        mm.MM_ERR_INVALID_ARG
    mm.mm_free(small)
    host = np.zeros(64 * 64, dtype=np.uint32)
    assert status(lambda: mm.mm_server_submit(srv, 1, 0, cam, 64, 64, host.ctypes.data)) == \
        mm.MM_ERR_INVALID_ARG
    mm.mm_server_wait(srv, r)
    assert status(lambda: mm.mm_server_poll(srv, 999999)) == mm.MM_ERR_INVALID_ARG
    assert mm.mm_server_poll(srv, r)[0] is True
    with pytest.raises(mm.MMError) as e:
        mm.mm_free(clouds[0][2])
    assert e.value.status == mm.MM_ERR_IN_USE
    mm.mm_destroy_server(srv)
    mm.mm_free(clouds[0][2])
