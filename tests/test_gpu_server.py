"""GPU parity of the served form: each request's frame equals the frame of its
cloud rendered alone after the same steps (the k-th request on a cloud
displaces it with step k), whatever else was queued or in flight, under any
batching, stream count and memory budget."""
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
           tuning=(0, 0, 0, 0, 0)):
    """order: [(session, cloud, frame)]; every request renders into its own buffer."""
    mm, torch = rig.mm, rig.torch
    srv = mm.mm_create_server(rig.inst, budget, streams, max_batch, 3, foot, *tuning)
    ids = [mm.mm_server_add_cloud(srv, mm.make_cloud_desc(c[2], c[0].shape[0], 3, c[3], c[4]))
           for c in clouds]
    assert ids == list(range(len(clouds)))
    reqs, outs, rids = [], [], []
    for s, c, f in order:
        w, h, deg = sessions[s]
        cam = synth.orbit_camera(f, w, h, start_deg=deg)
        out = torch.zeros((h, w), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        rids.append(mm.mm_server_submit(srv, s, c, cam, w, h, out.data_ptr()))
        outs.append(out)
        reqs.append((c, cam, w, h))
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
