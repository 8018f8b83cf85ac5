"""Benchmark of the displace+render frame on one MI355X.

Workload (default): 2^24 float3 points uniform in [0,1)^3 (seed 0), each
frame displaces every point by a Philox draw of +-0.001 per coordinate, then
splats it at 1920x1080 with a camera orbiting the cube centre (radius 2.5,
fov 60 deg, 1 deg per frame), then resolves RGBA8. One hipGraph launch per
frame; the line also gives, beside it, the same frames at 8 per launch
(mm_step_render_frames). Positions start resident in HBM; nothing crosses
PCIe in the timed region.

Prints ONE JSON line: throughput in Gpoints/s (value), frames/s, p50/p99
frame time from the device clock stored by each timed frame's first kernel
(and after the last), the roofline of the dominant kernel (the bin kernel,
timed by events inside the frame graph on one frame in 32), the whole frame's
roofline, the host it ran on, and the CPU oracle timed on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "displace+render Gpoints/s & frames/s @2^24 pts 1080p; p99 frame latency"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2504_20937_amd", "csrc")

# HBM traffic of the dominant kernel per launch, from rocprofv3 --pmc runs of
# this benchmark's default workload (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch, mean of the last 25 dispatches), scaled by what the same counters read for a plain 256 MiB device
# copy (FETCH_SIZE reads half the copied bytes: x2; WRITE_SIZE reads them
# all: x1). Keyed by a digest of the sources the kernel is built from: any
# change to them makes the entry stale and the reported traffic null until it
# is measured again.
KERNEL_SOURCES = {
    "bin_kernel": ["mm_bin_plain.hip", "mm_bin_dev.h", "mm_device.h", "mm_internal.h"],
}
TRAFFIC = {
    "bin_kernel": {"workload": "3d-uniform-2^24pts-1920x1080-orbit-1deg",
                   "tuning": [2, 32, 8, 1, 1024, 0xFFFFFFFF, 2],
                   "digest": "6d0bd9d98184e02d", "fetch_kib": 98394.9, "write_kib": 335988.3,
                   "fetch_scale": 2.0, "write_scale": 1.0},
}
FRAMES_PER_LAUNCH = 1  # frames per graph launch: the workload is one hipGraph per frame
MULTI_FRAMES = 8       # the extra measurement of several frames per launch
# Frames per profiled frame: the profiled frame launches a second graph with
# event-record nodes around the bin kernel, which costs that frame about
# 35 us; one in 32 keeps that under 1.5 us per frame on average (measured:
# 4.5 us per frame at one in 8) and still gives 31 samples in 1000 frames.
PROFILE_EVERY = 32
POINT_BYTES = 24   # float3 read + write per point and frame
PIXEL_BYTES = 20   # key read + empty-key write (8 + 8) and RGBA8 write (4)


def kernel_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sorted(KERNEL_SOURCES[kernel]):
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, tuning):
    """HBM bytes per launch from the counters, for the workload, tuning and
    kernel sources they were taken on; None otherwise."""
    e = TRAFFIC.get(kernel)
    if (not e or e["workload"] != workload or tuple(e["tuning"]) != tuple(tuning)
            or e["digest"] != kernel_digest(kernel)):
        return None
    return (e["fetch_kib"] * e["fetch_scale"] + e["write_kib"] * e["write_scale"]) * 1024.0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_info() -> dict:
    """The host the line was measured on: cores this process may use, the
    machine's logical CPUs, and the CPU model."""
    return {"cores_available": len(os.sched_getaffinity(0)), "logical_cpus": os.cpu_count(),
            "cpu_model": cpu_model()}


MIN_P99_SAMPLES = 100


LATENCY_FRAMES = 1000
SETTLE_S = 0.3           # seconds of untimed frames before the timed ones
SETTLE_BLOCK = 64        # frames per host synchronisation while settling
MAX_SETTLE_FRAMES = 20000


FRAME_MARKS = "the device clock stored by each frame's first kernel as it starts, and after the last"


def latency_fields(spans_ms, source: str = "timed frames",
                   how: str = "HIP events on the frame stream before every frame and after the last") -> dict:
    """p50 / p99 of per-frame spans, one per frame; p99 is null with fewer
    than MIN_P99_SAMPLES frames, where it would be little more than the
    largest sample."""
    spans = np.asarray(spans_ms, dtype=np.float64)
    return {"p50_frame_ms": float(np.percentile(spans, 50)) if spans.size else None,
            "p99_frame_ms": (float(np.percentile(spans, 99)) if spans.size >= MIN_P99_SAMPLES
                             else None),
            "max_frame_ms": float(spans.max()) if spans.size else None,
            "latency_samples": int(spans.size),
            "latency_source": f"{source}: {how}"}


def make_points(n: int, dist: str) -> np.ndarray:
    import synth
    if dist == "square":
        return synth.uniform_square(n, 0)
    return synth.uniform_cube(n, 0) if dist == "uniform" else synth.gaussian_mixture(n, 0)


def frame_setup(dist: str):
    """(dim, amplitude, wrap) of a frame workload: the 2D square folds its
    points into [-1, 1)^2 with steps of up to 0.005; the 3D clouds move freely
    by up to 0.001 per step."""
    return (2, 0.005, True) if dist == "square" else (3, 0.001, False)


def frame_camera(dist: str, f: int, w: int, h: int):
    import synth
    return synth.IDENTITY if dist == "square" else synth.orbit_camera(f, w, h)


def cpu_baseline(n, w, h, frames, dist="uniform", footprint=1):
    """The oracle as it stands, single-threaded, on `frames` frames of the
    workload (for more than 2^24 points, of its first 2^24 points)."""
    import oracle
    import synth

    m = min(n, 1 << 24)
    pts = make_points(n, dist)[:m].copy() if m < n else make_points(n, dist)
    depth = oracle.new_depth(w, h)
    _, amp, wrap = frame_setup(dist)
    cams = [frame_camera(dist, f, w, h) for f in range(frames)]
    oracle.lib()
    t0 = time.perf_counter()
    for f in range(frames):
        oracle.step_render(pts, 0, f, amp, wrap, cams[f], w, h, footprint, depth)
    dt = time.perf_counter() - t0
    what = "full frames" if m == n else f"frames of the first 2^24 of the 2^{int(np.log2(n))} points"
    return {"value": m * frames / dt / 1e9, "unit": "Gpoints/s", "cores": 1, "kind": "oracle",
            "cpu": cpu_model(), "host_cores_available": len(os.sched_getaffinity(0)),
            "sample": f"{frames} {what} ({dist}, {w}x{h}, footprint {footprint}), "
                      f"{dt:.1f} s on one host core",
            "ms_per_frame": dt / frames * 1e3}


def stream_copy_GBps(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Measured device copy ceiling: bytes read + written per second."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del src, dst
    return 2.0 * nbytes * reps / dt / 1e9


def batch_workload(seed: int = 0):
    """64 clouds of round(2^U[12,22]) points (uniform if even, Gaussian mixture
    if odd), each with 1-4 square views at 256, 512 or 1024 px and its own
    orbit start angle."""
    import synth
    specs = synth.batched_set(64, seed=seed)
    return specs, [synth.cloud_points(sp) for sp in specs]


def bench_batched(args) -> dict:
    """One batch frame (every cloud displaced, every view rendered) per graph
    launch, against the same work as plain views: per cloud, mm_step_render
    on its first view and mm_render on its other views."""
    import torch

    import paper_2504_20937_amd as mm
    import synth

    specs, pts = batch_workload()
    K, W = args.steps, args.warmup
    stream = torch.cuda.current_stream()
    inst = mm.mm_create_instance(0, stream.cuda_stream)
    devs, allocs, clouds, views, vinfo = [], [], [], [], []
    for j, (sp, p) in enumerate(zip(specs, pts)):
        d = torch.from_numpy(p).cuda()
        a = mm.mm_alloc_wrap(inst, d.data_ptr(), d.numel() * 4)
        devs.append(d)
        allocs.append(a)
        clouds.append(mm.make_cloud_desc(a, p.shape[0], 3, sp.seed, 0.001, False))
        for (vw, vh, deg) in sp.views:
            views.append(mm.make_batch_view_desc(j, vw, vh, synth.orbit_camera(0, vw, vh, start_deg=deg)))
            vinfo.append((j, vw, vh, deg))
    total_pts = sum(p.shape[0] for p in pts)
    total_px = sum(vw * vh for _, vw, vh, _ in vinfo)
    del pts

    def cams(f):
        return [synth.orbit_camera(f, vw, vh, start_deg=deg) for _, vw, vh, deg in vinfo]

    frames_cams = [np.ascontiguousarray(np.stack(cams(f)), dtype=np.float32) for f in range(W + K)]
    b = mm.mm_create_batch(inst, 3, 1, clouds, views)
    if args.autotune:
        mm.mm_batch_autotune(b, 5)
    elif args.tile or args.ppt or args.splits or args.grid or args.bin_threads:
        mm.mm_batch_set_tuning(b, args.tile, args.ppt, args.splits, args.grid, args.bin_threads)
    tuning = mm.mm_batch_get_tuning(b)
    print(f"bench batched: {len(clouds)} clouds, {total_pts} points, {len(views)} views, "
          f"{total_px} px, tuning {tuning}", file=sys.stderr, flush=True)

    # raw library calls with the cameras converted before the timed region
    # (inputs, like the points); each frame still hands all its cameras to
    # mm_batch_set_cameras, and each call's status is checked
    Lb = mm.lib()
    nviews = len(views)
    cam_ptrs_b = [mm._fptr(c) for c in frames_cams]  # frames_cams keeps the memory alive

    def batch_frame(f):
        st = (Lb.mm_batch_set_cameras(b, 0, nviews, cam_ptrs_b[f])
              or Lb.mm_batch_step_render(b, f))
        if st:
            raise mm.MMError(st, "batch frame loop", mm.mm_last_error())

    for f in range(W):
        batch_frame(f)
    mm.mm_batch_profile_begin(b, K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        batch_frame(W + k)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    frame_ms = mm.mm_batch_profile_end(b, K)
    mm.mm_destroy_batch(b)

    # the same frames as plain views: a graph per cloud (displace + first
    # view) and a render per further view
    pv = []
    for k, (j, vw, vh, deg) in enumerate(vinfo):
        d = mm.make_view_desc(allocs[j], devs[j].shape[0], 3, vw, vh, 1, specs[j].seed, 0.001,
                              False, frames_cams[0][k])
        v = mm.mm_create_view(inst, d)
        mm.mm_set_tuning(v, mm.MM_SPLAT_BINNED)
        pv.append(v)
    first = {}
    for k, (j, _, _, _) in enumerate(vinfo):
        first.setdefault(j, k)

    # raw library calls with prepared arguments: the host loop costs about what
    # a C caller's would
    L = mm.lib()
    import ctypes as C
    fp = C.POINTER(C.c_float)
    cam_ptrs = [[frames_cams[f][k].ctypes.data_as(fp) for k in range(len(pv))]
                for f in range(W + K)]
    is_first = [first[vinfo[k][0]] == k for k in range(len(pv))]

    def plain_frame(f):
        cp = cam_ptrs[f]
        for k, v in enumerate(pv):
            L.mm_set_camera(v, cp[k])
            if is_first[k]:
                L.mm_step_render(v, f)
            else:
                L.mm_render(v)

    for f in range(min(W, 5)):
        plain_frame(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        plain_frame(W + k)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for v in pv:
        mm.mm_destroy_view(v)
    for a in allocs:
        mm.mm_free(a)
    mm.mm_destroy_instance(inst)
    # the frame's byte model: positions read and written, and per pixel a key
    # clear, a key read and an RGBA8 write (as for the plain frame)
    point_bytes = POINT_BYTES * total_pts
    batch_bytes = point_bytes + PIXEL_BYTES * total_px
    return {
        "metric": "batched displace+render Gpoints/s & frames/s, 64 clouds (2^12..2^22 pts), "
                  "1-4 views each; vs plain launches",
        "value": total_pts * K / t_batch / 1e9,
        "unit": "Gpoints/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": t_batch / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched-64-clouds-2^12..2^22-1..4-views-256/512/1024",
                   "clouds": len(clouds), "points": total_pts, "views": len(views),
                   "pixels": total_px, "tile": tuning[0], "points_per_thread": tuning[1],
                   "splits": tuning[2], "grid_blocks": tuning[3], "bin_threads": tuning[4]},
        "frames_per_s": K / t_batch,
        "views_per_s": K * len(views) / t_batch,
        **{k: v for k, v in latency_fields(frame_ms).items() if k != "latency_source"},
        "latency_source": "HIP events before each batch frame's upload and after its graph "
                          "(every timed frame)",
        "plain": {"value": total_pts * K / t_plain / 1e9, "unit": "Gpoints/s",
                  "ms_per_step": t_plain / K * 1e3, "frames_per_s": K / t_plain,
                  "launches_per_frame": len(views)},
        "speedup_vs_plain": t_plain / t_batch,
        "frame_roofline": {"bytes_per_frame": batch_bytes,
                           "byte_model": "24 B per point + 20 B per pixel",
                           "achieved_GBps": batch_bytes / (t_batch / K) / 1e9,
                           "frac": batch_bytes / (t_batch / K) / 1e9 / HBM_PEAK_GBS},
        "host": host_info(),
    }


SERVED_SCREENS = [(1280, 720), (1920, 1080), (3840, 2160)]


def bench_served(args) -> dict:
    """Poisson arrivals of displace+render requests from 256 sessions on the 64
    clouds of the batched workload; each session has one screen (720p, 1080p
    or 4K); the server batches them continuously. Reports latency from
    submission to completion and the throughput, at the given rate and with
    every request submitted at once (saturation)."""
    import torch

    import paper_2504_20937_amd as mm
    import synth

    specs, pts = batch_workload()
    stream = torch.cuda.current_stream()
    inst = mm.mm_create_instance(0, stream.cuda_stream)
    devs, allocs = [], []
    for sp, p in zip(specs, pts):
        d = torch.from_numpy(p).cuda()
        devs.append(d)
        allocs.append(mm.mm_alloc_wrap(inst, d.data_ptr(), d.numel() * 4))
    sizes = [p.shape[0] for p in pts]
    del pts
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    n_sessions = 256
    screens = [SERVED_SCREENS[int(rng.integers(0, 3))] for _ in range(n_sessions)]

    def run(rate, count, budget, seed):
        srv = mm.mm_create_server(inst, budget, args.streams, args.max_batch, 3, 1,
                                  args.tile, args.ppt, args.splits, args.grid, args.bin_threads)
        for j, sp in enumerate(specs):
            mm.mm_server_add_cloud(srv, mm.make_cloud_desc(allocs[j], sizes[j], 3, sp.seed, 0.001))
        r = np.random.default_rng(seed)
        sess = r.integers(0, n_sessions, count)
        cl = r.integers(0, len(specs), count)
        deg = r.uniform(0.0, 360.0, count)
        cams = [synth.orbit_camera(0, screens[s][0], screens[s][1], start_deg=float(a))
                for s, a in zip(sess, deg)]
        arrivals = (synth.poisson_arrivals(rate, count, seed) if np.isfinite(rate)
                    else np.zeros(count))
        ids = []
        t0 = time.perf_counter()
        for k in range(count):
            while time.perf_counter() - t0 < arrivals[k]:
                pass
            w, h = screens[sess[k]]
            ids.append(mm.mm_server_submit(srv, int(sess[k]), int(cl[k]), cams[k], w, h))
        lat = np.array([mm.mm_server_wait(srv, i) for i in ids])
        t1 = time.perf_counter()
        st = mm.mm_server_stats_get(srv)
        mm.mm_destroy_server(srv)
        pts_done = float(sum(sizes[c] for c in cl))
        px_done = float(sum(screens[s][0] * screens[s][1] for s in sess))
        return {"rate_per_s": None if not np.isfinite(rate) else rate, "requests": count,
                "budget_bytes": budget, "wall_s": t1 - t0,
                "frames_per_s": count / (t1 - t0), "Gpoints_per_s": pts_done / (t1 - t0) / 1e9,
                "Gpixels_per_s": px_done / (t1 - t0) / 1e9,
                "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
                "launches": st["launches"], "mean_batch": count / max(1, st["launches"]),
                "evictions": st["evictions"], "admissions": st["admissions"]}

    def served_vs_batched(rounds):
        """One request set run both ways from the same initial positions:
        session c renders cloud c at screen SERVED_SCREENS[c % 3], and round r
        asks every cloud for its frame at step r with the orbit camera of
        frame r (the clouds' start angles). Served: every request submitted
        at once (saturation). Batched offline: one batch of the 64 (cloud,
        screen) views, one batch frame per round. The last frame of every
        session is compared between the two (bit for bit)."""
        nc = len(specs)
        scr = [SERVED_SCREENS[c % 3] for c in range(nc)]
        start = [float(specs[c].views[0][2]) for c in range(nc)]
        cams = np.ascontiguousarray(np.stack([np.stack(
            [synth.orbit_camera(r, scr[c][0], scr[c][1], start_deg=start[c]) for c in range(nc)])
            for r in range(rounds)]), dtype=np.float32)          # (rounds, clouds, 4, 4)
        saved = [d.clone() for d in devs]
        torch.cuda.synchronize()
        # served, saturated
        srv = mm.mm_create_server(inst, 64 << 30, args.streams, args.max_batch, 3, 1,
                                  args.tile, args.ppt, args.splits, args.grid, args.bin_threads)
        for j, sp in enumerate(specs):
            mm.mm_server_add_cloud(srv, mm.make_cloud_desc(allocs[j], sizes[j], 3, sp.seed, 0.001))
        t0 = time.perf_counter()
        ids = [mm.mm_server_submit(srv, c, c, cams[r, c], scr[c][0], scr[c][1])
               for r in range(rounds) for c in range(nc)]
        for i in ids:
            mm.mm_server_wait(srv, i)
        t_served = time.perf_counter() - t0
        last_served = [mm.mm_server_read_frame(srv, c, scr[c][0], scr[c][1]) for c in range(nc)]
        st = mm.mm_server_stats_get(srv)
        mm.mm_destroy_server(srv)
        # batched offline, from the same initial positions
        for d, s0 in zip(devs, saved):
            d.copy_(s0)
        torch.cuda.synchronize()
        clouds = [mm.make_cloud_desc(allocs[j], sizes[j], 3, sp.seed, 0.001, False)
                  for j, sp in enumerate(specs)]
        vds = [mm.make_batch_view_desc(c, scr[c][0], scr[c][1], cams[0, c]) for c in range(nc)]
        b = mm.mm_create_batch(inst, 3, 1, clouds, vds)
        Lb = mm.lib()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(rounds):
            s = (Lb.mm_batch_set_cameras(b, 0, nc, mm._fptr(cams[r]))
                 or Lb.mm_batch_step_render(b, r))
            if s:
                raise mm.MMError(s, "offline batch", mm.mm_last_error())
        torch.cuda.synchronize()
        t_batched = time.perf_counter() - t0
        same = all(np.array_equal(mm.mm_batch_read_frame(b, c, scr[c][0], scr[c][1]), last_served[c])
                   for c in range(nc))
        mm.mm_destroy_batch(b)
        for d, s0 in zip(devs, saved):
            d.copy_(s0)
        torch.cuda.synchronize()
        n_req = rounds * nc
        pts_round = float(sum(sizes))
        return {"request_set": f"{rounds} rounds x {nc} clouds (session c: cloud c at "
                               f"{'/'.join(f'{w}x{h}' for w, h in SERVED_SCREENS)} by c mod 3)",
                "requests": n_req,
                "served": {"frames_per_s": n_req / t_served,
                           "Gpoints_per_s": pts_round * rounds / t_served / 1e9,
                           "wall_s": t_served, "launches": st["launches"],
                           "max_in_flight": st["max_in_flight"], "max_batch": st["max_batch"]},
                "batched_offline": {"frames_per_s": n_req / t_batched,
                                    "Gpoints_per_s": pts_round * rounds / t_batched / 1e9,
                                    "wall_s": t_batched, "launches": rounds},
                "served_over_batched": t_batched / t_served,
                "last_frames_identical": bool(same)}

    count = args.requests
    print(f"bench served: 256 sessions, {len(specs)} clouds, {count} requests per run",
          file=sys.stderr, flush=True)
    runs = [run(args.rate, count, 64 << 30, 1), run(args.rate, count, 1 << 30, 2)]
    for rate in (4 * args.rate, 16 * args.rate, float("inf")):
        runs.append(run(rate, count, 64 << 30, 3))
        print(f"  rate {rate}: {runs[-1]['frames_per_s']:.0f} frames/s", file=sys.stderr, flush=True)
    vs = served_vs_batched(40)
    print(f"  same request set: served {vs['served']['frames_per_s']:.0f} frames/s, batched offline "
          f"{vs['batched_offline']['frames_per_s']:.0f} frames/s", file=sys.stderr, flush=True)
    for a in allocs:
        mm.mm_free(a)
    mm.mm_destroy_instance(inst)
    main_run = runs[0]
    return {
        "metric": "served displace+render: p50/p99 request latency and frames/s, 256 sessions, "
                  "Poisson arrivals, 64 clouds (2^12..2^22 pts), 720p/1080p/4K",
        "value": main_run["frames_per_s"], "unit": "frames/s",
        "n_gpus": 1, "steps": count, "warmup": 0,
        "ms_per_step": main_run["wall_s"] / count * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served-256-sessions-poisson-{args.rate:g}-per-s",
                   "streams": args.streams, "max_batch": args.max_batch},
        "p50_latency_ms": main_run["p50_latency_ms"],
        "p99_latency_ms": main_run["p99_latency_ms"],
        "runs": runs,
        "served_vs_batched_offline": vs,
    }


def bench_grid(args) -> dict:
    """Structured-grid view: a 4096 x 4096 lattice of 1-byte cell states
    (a Potts-like q = 256 field) drawn through a 256-entry palette at the
    given screen size, rendered every frame."""
    import torch

    import paper_2504_20937_amd as mm

    L = 4096
    w, h = args.width, args.height
    K, W = args.steps, args.warmup
    rng = np.random.default_rng(0)
    pal_t = torch.from_numpy(rng.integers(0, 2**32, 256, dtype=np.uint64).astype(np.uint32)).cuda()
    cells_t = torch.from_numpy(rng.integers(0, 256, L * L, dtype=np.uint8)).cuda()
    # an explicit stream: the instance launches on it and the events time it
    # (torch's default stream handle is null, for which an instance makes its own)
    stream = torch.cuda.Stream()
    inst = mm.mm_create_instance(0, stream.cuda_stream)
    pal_a = mm.mm_alloc_wrap(inst, pal_t.data_ptr(), pal_t.numel() * 4)
    cells_a = mm.mm_alloc_wrap(inst, cells_t.data_ptr(), cells_t.numel())
    g = mm.mm_create_grid(inst, L, L, w, h, pal_a, 256, cells_a, 1)
    for _ in range(W):
        mm.mm_grid_render(g)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(K):
        mm.mm_grid_render(g)
    end.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gpu_ms = start.elapsed_time(end) / K
    mm.mm_destroy_grid(g)
    mm.mm_destroy_instance(inst)
    bytes_per_frame = w * h * (4 + 1)  # RGBA8 write + one 1-byte cell read per pixel
    achieved = bytes_per_frame / (gpu_ms * 1e-3) / 1e9
    return {
        "metric": "structured-grid view: frames/s, 4096x4096 lattice of 1-byte states, 256-entry palette",
        "value": K / elapsed, "unit": "frames/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": elapsed / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"grid-4096x4096-u8-{w}x{h}", "cells": L * L, "width": w, "height": h},
        "gpu_ms_per_frame": gpu_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "grid_kernel",
                     "bytes_per_launch": bytes_per_frame},
    }


def bench_edges(args) -> dict:
    """Edges view: a 1024 x 1024 vertex lattice jittered in 2D and cut into
    two triangles per cell (about 2.1 M triangles, 6.3 M edges, like the
    paper's Delaunay edge views), drawn at the given screen size."""
    import torch

    import paper_2504_20937_amd as mm

    L = 1024
    w, h = args.width, args.height
    K, W = args.steps, args.warmup
    rng = np.random.default_rng(0)
    g = (np.arange(L, dtype=np.float64) + 0.5) / L * 2.0 - 1.0
    xy = np.stack(np.meshgrid(g, g, indexing="xy"), axis=-1).reshape(-1, 2)
    pos = (xy + rng.uniform(-0.3, 0.3, xy.shape) * (2.0 / L)).astype(np.float32)
    v = np.arange(L * L, dtype=np.uint32).reshape(L, L)
    a, b, c, d = v[:-1, :-1], v[:-1, 1:], v[1:, :-1], v[1:, 1:]
    tri = np.concatenate([np.stack([a, b, d], -1).reshape(-1, 3),
                          np.stack([a, d, c], -1).reshape(-1, 3)]).reshape(-1)
    stream = torch.cuda.Stream()  # explicit, so the events time the instance's stream
    inst = mm.mm_create_instance(0, stream.cuda_stream)
    pos_t = torch.from_numpy(pos).cuda()
    tri_t = torch.from_numpy(tri.view(np.int32)).cuda()
    pa = mm.mm_alloc_wrap(inst, pos_t.data_ptr(), pos_t.numel() * 4)
    ta = mm.mm_alloc_wrap(inst, tri_t.data_ptr(), tri_t.numel() * 4)
    ntri = tri.shape[0] // 3
    e = mm.mm_create_edges(inst, pa, L * L, 2, ta, ntri, 3, w, h, 0)
    for _ in range(W):
        mm.mm_edges_render(e)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(K):
        mm.mm_edges_render(e)
    end.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gpu_ms = start.elapsed_time(end) / K
    mm.mm_destroy_edges(e)
    mm.mm_destroy_instance(inst)
    return {
        "metric": "edges view: frames/s and Gedges/s, 1024^2-vertex triangulated lattice, 2D",
        "value": K / elapsed, "unit": "frames/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": elapsed / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"edges-lattice-1024^2-2d-{w}x{h}", "vertices": L * L,
                   "triangles": ntri, "edges": 3 * ntri, "width": w, "height": h},
        "gpu_ms_per_frame": gpu_ms, "Gedges_per_s": 3 * ntri / (gpu_ms * 1e-3) / 1e9,
    }


def bench_cobound(args) -> dict:
    """The co-bounds of the two passes: `mm_cobound` (built beside the
    library) times the per-point Philox draw, and the draw with the
    displacement and projection, in the bin kernel's launch shape without the
    position traffic, and the launch with only its index arithmetic and one
    store per thread (the bin pass's ALU co-bound); and one tile workgroup
    per CU streaming a tile's worth of 8-byte records with nothing else (the
    tile pass's co-bound: what one CU reads of a dense tile per second)."""
    import subprocess

    from paper_2504_20937_amd import build as mmbuild

    if not os.path.exists(mmbuild.COBOUND_EXE):
        raise SystemExit(f"{mmbuild.COBOUND_EXE} is not built: run __graft_entry__.build()")
    r = subprocess.run([mmbuild.COBOUND_EXE, str(args.log2n), "50"], capture_output=True,
                       text=True, timeout=120)
    if r.returncode != 0:
        raise SystemExit(f"mm_cobound failed ({r.returncode}): {r.stderr.strip()}")
    probe = json.loads(r.stdout.strip().splitlines()[-1])
    n = probe["points"]
    alu_us = probe["displace_project_us"] - probe["index_store_us"]
    # the tile pass's co-bound: one 1024-thread workgroup per CU streaming
    # 8-byte words (the mean and the heaviest active tile's records at 2^24
    # points and 1080p), durations from the device clock at each workgroup's
    # start and end
    st = probe["stream"]
    mean_b, heavy_b = 8 * st["mean_words"], 8 * st["heavy_words"]
    tile_stream = {
        "mean_tile_bytes": mean_b,
        "heavy_tile_bytes": heavy_b,
        "every_cu_streaming_us": st["even_u12"]["wg_mean_us"],
        "every_cu_streaming_GBps_per_cu": mean_b / st["even_u12"]["wg_mean_us"] / 1e3,
        "heavy_workgroup_us": st["heavy_u12"]["wg0_us"],
        "heavy_workgroup_GBps": heavy_b / st["heavy_u12"]["wg0_us"] / 1e3,
        "heavy_workgroup_us_24_windows": st["heavy_u24"]["wg0_us"],
        # every CU reading the heaviest tile's words: contiguously, and in the
        # tile pass's layout (runs of 73 at misaligned or 1 KB-aligned offsets)
        "every_cu_heavy_contiguous_us": st["contiguous_wg_us"],
        "every_cu_heavy_runs_us": st["runs_wg_us"],
        "every_cu_heavy_aligned_runs_us": st["aligned_runs_wg_us"],
    }
    return {
        "metric": "bin pass ALU co-bound: per-point displace + project time without memory traffic (with the pass's memory co-bound and one CU's record stream beside it)",
        "value": alu_us,
        "unit": "us per launch",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "u32 Philox + f32",
        "data": "synthetic",
        "config": {"workload": f"cobound-2^{args.log2n}pts-1024x8", "points": n},
        "philox_us": probe["philox_us"] - probe["index_store_us"],
        "displace_project_us": alu_us,
        "launch_and_store_us": probe["index_store_us"],
        # the bin pass's bytes alone (12 B read + 12 B written in place + an
        # 8 B record per point), the memory co-bound of the bin kernel
        "bin_traffic_us": probe["traffic_us"],
        "bin_traffic_TBps": probe["traffic_bytes"] / probe["traffic_us"] / 1e6,
        "tile_stream": tile_stream,
        "probe": probe,
    }


def bench_hostcopy(args) -> dict:
    """The comparison the paper draws: per frame the device displaces the
    cloud, the positions are copied to host memory, and the host renders
    them on all its cores. Beside it, the device path on the same workload."""
    import torch

    import paper_2504_20937_amd as mm
    from paper_2504_20937_amd import hostcopy
    import synth

    n, w, h = 1 << args.log2n, args.width, args.height
    K = max(1, args.hostcopy_frames)

    def dev_free() -> int:  # hipMemGetInfo
        torch.cuda.synchronize()
        return torch.cuda.mem_get_info(0)[0]

    pts = synth.uniform_cube(n, 0)
    torch.zeros(1, device="cuda")            # the runtime's own set-up, before any delta
    f0 = dev_free()
    dev = torch.from_numpy(pts).cuda()
    dev_positions = f0 - dev_free()          # both paths keep the positions on the device
    del pts
    host = torch.empty((n, 3), dtype=torch.float32, pin_memory=True)
    frame = np.empty((h, w), dtype=np.uint32)
    frame.fill(0)
    stream = torch.cuda.current_stream()
    inst = mm.mm_create_instance(0, stream.cuda_stream)
    alloc = mm.mm_alloc_wrap(inst, dev.data_ptr(), dev.numel() * 4)
    f1 = dev_free()
    view = mm.mm_create_view(inst, mm.make_view_desc(alloc, n, 3, w, h, 1, 0, 0.001, False,
                                                     synth.orbit_camera(0, w, h)))
    dev_view = f1 - dev_free()               # the device path's frame and splat buffers
    threads = hostcopy.max_threads()
    hostcopy.render(np.zeros((1, 3), np.float32), 0, synth.orbit_camera(0, w, h), w, h)  # warm
    t_disp = t_copy = t_render = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(K):
        a = time.perf_counter()
        mm.mm_step(view, f)
        torch.cuda.synchronize()
        b = time.perf_counter()
        host.copy_(dev)            # device -> pinned host, 12 B per point
        c = time.perf_counter()
        hostcopy.render(host.numpy(), 0, synth.orbit_camera(f, w, h), w, h, 1, threads, frame)
        d = time.perf_counter()
        t_disp += b - a
        t_copy += c - b
        t_render += d - c
    elapsed = time.perf_counter() - t0
    # the device path on the same workload, for the ratio
    G = 200
    for f in range(20):
        mm.mm_set_camera(view, synth.orbit_camera(f, w, h))
        mm.mm_step_render(view, K + f)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for f in range(G):
        mm.mm_set_camera(view, synth.orbit_camera(f, w, h))
        mm.mm_step_render(view, K + 20 + f)
    torch.cuda.synchronize()
    g_elapsed = time.perf_counter() - g0
    mm.mm_destroy_view(view)
    mm.mm_free(alloc)
    mm.mm_destroy_instance(inst)
    fps = K / elapsed
    gpu_fps = G / g_elapsed
    return {
        "metric": "host-copy path (device displace, copy to host, render on all host cores) "
                  "vs device path, 2^24 pts 1080p",
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": K, "warmup": 0,
        "ms_per_step": elapsed / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"3d-uniform-2^{args.log2n}pts-{w}x{h}-orbit-1deg-hostcopy",
                   "host_threads": threads, "cpus": len(os.sched_getaffinity(0))},
        "displace_ms": t_disp / K * 1e3, "copy_ms": t_copy / K * 1e3,
        "render_ms": t_render / K * 1e3,
        "pcie_GBps": 12.0 * n * K / t_copy / 1e9,
        "memory": {"how": "device: hipMemGetInfo free bytes before and after each allocation "
                          "(after the runtime's own set-up); host: the sizes allocated (pinned "
                          "positions, frame, the render's per-thread depth buffers)",
                   "hostcopy_device_bytes": dev_positions,
                   "hostcopy_host_bytes": 12 * n + 4 * w * h + 8 * w * h * threads,
                   "device_path_bytes": dev_positions + dev_view,
                   "device_path_view_bytes": dev_view,
                   "device_path_over_hostcopy_device": (dev_positions + dev_view) / dev_positions},
        "Gpoints_per_s": n * K / elapsed / 1e9,
        "device_path_frames_per_s": gpu_fps,
        "device_over_hostcopy": gpu_fps / fps,
        "cpu": cpu_model(),
        "paper": {"framerate_ratio": "up to 9x", "total_time_ratio": "up to 12x lower",
                  "gpu_memory_ratio": "1.5x less",
                  "hardware": "AMD Ryzen 7 3700X, 16 GB RAM; NVIDIA GeForce RTX 2070 SUPER 8 GB; "
                              "CUDA 12.2; Vulkan 1.3.236; 1920x1080 at 144 Hz",
                  "workload": "N and resolution not stated"},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--cpu-frames", type=int, default=48)
    ap.add_argument("--dist", choices=["uniform", "mixture", "square"], default="uniform",
                    help="frame: uniform cube, mixture of 32 Gaussians (sigma 0.02), or the 2D "
                         "square [-1, 1)^2 with wrap (orthographic)")
    ap.add_argument("--footprint", type=int, choices=[1, 3], default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--splat", choices=["auto", "direct", "binned"], default="auto")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--ppt", type=int, default=0)
    ap.add_argument("--splits", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0, help="batched: persistent grid blocks")
    ap.add_argument("--bin-threads", type=int, default=0, help="threads per bin workgroup")
    ap.add_argument("--piece-records", type=int, default=0,
                    help="frame: records per balanced tile piece (0 auto or -1: static splits)")
    ap.add_argument("--cull", choices=["auto", "on", "off"], default="auto",
                    help="frame: the occlusion cull of the binned 3D 1x1 pass (auto: where it applies)")
    ap.add_argument("--autotune", action="store_true", help="time the shapes, keep the fastest")
    ap.add_argument("--frames-per-launch", type=int, default=FRAMES_PER_LAUNCH,
                    help="frames per graph launch (1: one mm_step_render call per frame)")
    ap.add_argument("--palette", action="store_true",
                    help="frame: colour through a 256-entry palette and 1-byte indices (mm_set_colour)")
    ap.add_argument("--overlap", action="store_true",
                    help="frame: bin frame f while frame f - 1 is drawn (mm_set_frame_overlap)")
    ap.add_argument("--hostcopy-frames", type=int, default=10, help="hostcopy: frames timed")
    ap.add_argument("--workload", choices=["frame", "batched", "served", "hostcopy", "grid", "edges",
                                           "cobound"],
                    default="frame",
                    help="frame: the 2^24-point 1080p frame (default); batched: 64 clouds "
                         "with 1-4 views each in one launch per pass; served: Poisson "
                         "requests from 256 sessions through the server; hostcopy: device "
                         "displace, copy to host, render on the host cores; cobound: the "
                         "bin pass's per-point ALU work without memory traffic")
    ap.add_argument("--rate", type=float, default=2000.0, help="served: requests per second")
    ap.add_argument("--requests", type=int, default=4000, help="served: requests per run")
    ap.add_argument("--streams", type=int, default=2, help="served: streams")
    ap.add_argument("--max-batch", type=int, default=256, help="served: requests per launch")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run 10 plain device copies of BYTES (for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the displace+render path is built and "
              "measured on a single MI355X (multi-GPU sharding is a design note, not "
              "built); run with --gpus 1", file=sys.stderr)
        return 2

    if args.workload == "cobound":  # before this process touches the GPU
        print(json.dumps(bench_cobound(args)), flush=True)
        return 0

    import torch

    import paper_2504_20937_amd as mm
    import synth

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n4 = args.calibrate_copy // 4
        src = torch.ones(n4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n4 * 4, "launches": 10}), flush=True)
        return 0
    if args.workload == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return 0
    if args.workload == "served":
        print(json.dumps(bench_served(args)), flush=True)
        return 0
    if args.workload == "edges":
        print(json.dumps(bench_edges(args)), flush=True)
        return 0
    if args.workload == "grid":
        print(json.dumps(bench_grid(args)), flush=True)
        return 0
    if args.workload == "hostcopy":
        print(json.dumps(bench_hostcopy(args)), flush=True)
        return 0
    n, w, h = 1 << args.log2n, args.width, args.height
    K, W = args.steps, args.warmup
    copy_ceiling = stream_copy_GBps()
    pts = make_points(n, args.dist)
    dev = torch.from_numpy(pts).cuda()
    del pts
    dim, amp, wrap = frame_setup(args.dist)
    stream = torch.cuda.current_stream()
    inst = mm.mm_create_instance(0, stream.cuda_stream)
    alloc = mm.mm_alloc_wrap(inst, dev.data_ptr(), dev.numel() * 4)
    view = mm.mm_create_view(inst, mm.make_view_desc(alloc, n, dim, w, h, args.footprint, 0, amp,
                                                     wrap, frame_camera(args.dist, 0, w, h)))
    splat = {"auto": mm.MM_SPLAT_AUTO, "direct": mm.MM_SPLAT_DIRECT,
             "binned": mm.MM_SPLAT_BINNED}[args.splat]
    if args.autotune:
        mm.mm_autotune(view, 10)
    elif (splat != mm.MM_SPLAT_AUTO or args.tile or args.ppt or args.splits or args.bin_threads
          or args.piece_records or args.cull != "auto"):
        pieces = mm.MM_PIECES_STATIC if args.piece_records < 0 else args.piece_records
        cull = {"auto": mm.MM_CULL_AUTO, "on": mm.MM_CULL_ON, "off": mm.MM_CULL_OFF}[args.cull]
        mm.mm_set_tuning(view, splat, args.tile, args.ppt, args.splits, args.bin_threads, pieces,
                         cull)
    tuning = mm.mm_get_tuning(view)
    mode = "direct" if tuning[0] == mm.MM_SPLAT_DIRECT else "binned"
    if args.palette:
        rng = np.random.default_rng(1)
        pal_t = torch.from_numpy(rng.integers(0, 2**32, 256, dtype=np.uint64).astype(np.uint32)).cuda()
        idx_t = torch.from_numpy(rng.integers(0, 256, n, dtype=np.uint8)).cuda()
        pal_alloc = mm.mm_alloc_wrap(inst, pal_t.data_ptr(), pal_t.numel() * 4)
        idx_alloc = mm.mm_alloc_wrap(inst, idx_t.data_ptr(), idx_t.numel())
        mm.mm_set_colour(view, pal_alloc, 256, idx_alloc, 1)
    if args.overlap:
        mm.mm_set_frame_overlap(view, True)
    print(f"bench: {n} points, {w}x{h}, warmup {W}, timed {K}, splat {mode} {tuning}",
          file=sys.stderr, flush=True)
    # Frames go B = --frames-per-launch to a graph launch (mm_step_render_frames:
    # each frame its own step and camera, the same frames as B single calls)
    B = max(1, min(64, args.frames_per_launch))
    L = mm.lib()

    def cameras(first, count):
        return np.ascontiguousarray(
            np.stack([frame_camera(args.dist, first + k, w, h) for k in range(count)]),
            dtype=np.float32).reshape(-1)

    def frames(cam_all, first, count, what, per=B):
        # cam_all: count * 16 floats; the C entry points directly, so Python
        # adds as little as possible to the host side of a launch
        for k0 in range(0, count, per):
            c = min(per, count - k0)
            ptr = C.cast(cam_all.ctypes.data + 64 * k0, C.POINTER(C.c_float))
            st = (L.mm_set_camera(view, ptr) or L.mm_step_render(view, first + k0)) if c == 1 \
                else L.mm_step_render_frames(view, first + k0, c, ptr)
            if st:
                raise mm.MMError(st, what, mm.mm_last_error())

    # W warm-up frames as asked, then further untimed frames of the same loop
    # until SETTLE_S seconds of them have run back to back: a few frames after
    # set-up still run at a lower rate (about 17% at 2^24 points, 1080p) until
    # the device settles under sustained load
    frames(cameras(0, W), 0, W, "warm-up")
    torch.cuda.synchronize()
    f, t_settle = W, time.perf_counter()
    while time.perf_counter() - t_settle < SETTLE_S and f < W + MAX_SETTLE_FRAMES:
        frames(cameras(f, SETTLE_BLOCK), f, SETTLE_BLOCK, "settle")
        f += SETTLE_BLOCK
        torch.cuda.synchronize()
    F0, settle_frames = f, f - W
    # HIP events inside the frame graph (on the first frame of a launch) on
    # one frame in PROFILE_EVERY: the kernel durations of the roofline
    every = max(B, PROFILE_EVERY // B * B)
    mm.mm_profile_every(view, every)
    prof_cap = (K + every - 1) // every
    # the cameras of the timed frames are inputs, like the points: converted
    # before the timed region
    cam_all = cameras(F0, K)
    mm.mm_profile_begin(view, prof_cap)  # synchronises
    # the device clock at the start of every frame (stored by its first
    # kernel) and after the last: the per-frame spans for p50 / p99
    mm.mm_mark_begin(view, K + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    frames(cam_all, F0, K, "frame loop")
    # with overlap, the last frame is drawn inside the timed region; the
    # closing mark follows it
    mm.mm_mark_end(view)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    frame_spans = mm.mm_mark_read(view, K + 1)
    splat_ms, resolve_ms, frame_ms = mm.mm_profile_end(view, prof_cap)
    elapsed = t1 - t0
    # p99 from fewer than MIN_P99_SAMPLES frames is little more than the
    # largest one: then a latency run of LATENCY_FRAMES further frames of the
    # same loop (after the timed region) gives the distribution
    lat_spans, lat_source = frame_spans, "timed frames"
    if K < MIN_P99_SAMPLES:
        R = LATENCY_FRAMES
        lat_cams = cameras(F0 + K, R)
        mm.mm_mark_begin(view, R + 1)
        frames(lat_cams, F0 + K, R, "latency loop")
        mm.mm_mark_end(view)
        lat_spans = mm.mm_mark_read(view, R + 1)
        lat_source = f"a latency run of {R} frames after the {K} timed ones"
    # beside the timed loop: the next frames at MULTI_FRAMES per graph launch
    multi = None
    if B == 1 and not args.overlap:
        Fm = F0 + K + (LATENCY_FRAMES if K < MIN_P99_SAMPLES else 0)
        M = max(MULTI_FRAMES, min(K, 1000) // MULTI_FRAMES * MULTI_FRAMES)
        cam_m = cameras(Fm, M)
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        frames(cam_m, Fm, M, "multi-frame loop", MULTI_FRAMES)
        torch.cuda.synchronize()
        tm = time.perf_counter() - tm0
        multi = {"frames_per_launch": MULTI_FRAMES, "frames": M, "ms_per_step": tm / M * 1e3,
                 "value": n * M / tm / 1e9, "unit": "Gpoints/s",
                 "note": "the same frames, several per graph launch (mm_step_render_frames); "
                         "not the one-graph-per-frame workload"}
    mm.mm_destroy_view(view)
    mm.mm_free(alloc)
    mm.mm_destroy_instance(inst)

    point_bytes = (8 if dim == 2 else 12) * 2 * n  # read + write of each position
    frame_bytes = point_bytes + PIXEL_BYTES * w * h
    splat_avg = float(np.mean(splat_ms))
    achieved = point_bytes / (splat_avg * 1e-3) / 1e9
    workload = ((f"2d-square-2^{args.log2n}pts-{w}x{h}-wrap" if dim == 2 else
                 f"3d-{args.dist}-2^{args.log2n}pts-{w}x{h}-orbit-1deg")
                + (f"-{args.footprint}x{args.footprint}" if args.footprint != 1 else ""))
    out = {
        "metric": METRIC,
        "value": n * K / elapsed / 1e9,
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "settle_frames": settle_frames,
        "settle": f"untimed frames after the {W} warm-up ones until {SETTLE_S} s of frames had run",
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload,
                   "points": n, "width": w, "height": h, "footprint": args.footprint,
                   "amplitude": amp, "wrap": wrap,
                   "graph": ("bin of frame f beside the draw of frame f - 1 (two streams)"
                             if args.overlap else f"{B} frames per hipGraph launch"),
                   "colour": "256-entry palette, 1-byte indices" if args.palette else "index hash",
                   "splat": mode, "tile": tuning[1], "points_per_thread": tuning[2],
                   "splits": tuning[3], "bin_threads": tuning[4], "piece_records": tuning[5],
                   "occlusion_cull": "on" if tuning[6] == mm.MM_CULL_ON else "off",
                   "frames_per_launch": 1 if args.overlap else B},
        "frames_per_s": K / elapsed,
        **latency_fields(lat_spans, lat_source, FRAME_MARKS),
        "timed_frames_p50_ms": float(np.percentile(frame_spans, 50)),
        "timed_frames_max_ms": float(np.max(frame_spans)),
        "kernel_profiled_frames": f"{len(frame_ms)} (1 in {every} of the timed frames)",
        "graph_ms_profiled_mean": float(np.mean(frame_ms)),
        "point_kernel_ms": splat_avg,
        "rest_of_frame_ms": float(np.mean(resolve_ms)),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic("bin_kernel", workload, tuning)
                                 if mode == "binned" else None),
                     "kernel": ("bin_kernel (displace+project+tile sort)" if mode == "binned"
                                else "point_kernel (displace+project+splat)"),
                     "bytes_per_launch": point_bytes},
        "frame_roofline": {"bytes_per_frame": frame_bytes,
                           "achieved_GBps": frame_bytes / (elapsed / K) / 1e9,
                           "frac": frame_bytes / (elapsed / K) / 1e9 / HBM_PEAK_GBS},
        "stream_copy_GBps": copy_ceiling,
        "host": host_info(),
    }
    if multi:
        multi["frame_roofline_frac"] = frame_bytes / (multi["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS
        out["multi_frame_launch"] = multi
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, w, h, args.cpu_frames, args.dist, args.footprint)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
