"""Seeded synthetic inputs for the displace+render workloads.

This module is shared by the CPU oracle's tests and by the GPU path's tests
and benchmark. It draws inputs only: initial point positions, camera
matrices, cloud/view sets and request arrival times. It holds none of the
displacement, projection, splat or resolve arithmetic.

The Mimir paper's benchmark starts from randomly generated points and moves
them every timestep (section "Performance Benchmark"); its setup is not
timed, so the initial positions are plain input data here, drawn on the
host with numpy's PCG64 and handed identically to both sides.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_square(n: int, seed: int = 0) -> np.ndarray:
    """n float32 points (x, y) uniform on the grid k * 2^-23 - 1 of [-1, 1)^2.

    Every value is exactly representable, so the float32 array is the same
    on every platform. Shape (n, 2), C-contiguous (AoS float2)."""
    k = _rng(seed).integers(0, 1 << 24, size=(n, 2), dtype=np.uint32)
    return (k.astype(np.float64) * 2.0**-23 - 1.0).astype(np.float32)


def uniform_cube(n: int, seed: int = 0) -> np.ndarray:
    """n float32 points uniform on the grid k * 2^-24 of [0, 1)^3 (AoS float3)."""
    k = _rng(seed).integers(0, 1 << 24, size=(n, 3), dtype=np.uint32)
    return (k.astype(np.float64) * 2.0**-24).astype(np.float32)


def gaussian_mixture(n: int, seed: int = 0, components: int = 32,
                     sigma: float = 0.02, chunk: int = 1 << 22) -> np.ndarray:
    """n float32 points from an equal-weight mixture of isotropic Gaussians.

    Centres uniform in [0, 1)^3, each point's component drawn i.i.d., so
    consecutive indices land in unrelated clusters. Drawn in float64 and
    rounded once to float32. Generated in chunks to bound host memory."""
    rng = _rng(seed)
    centres = rng.random((components, 3))
    out = np.empty((n, 3), dtype=np.float32)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        comp = rng.integers(0, components, size=hi - lo)
        pts = centres[comp] + sigma * rng.standard_normal((hi - lo, 3))
        out[lo:hi] = pts.astype(np.float32)
    return out


def look_at_perspective(eye, centre, up, fov_y_deg: float, aspect: float,
                        near: float = 0.1, far: float = 100.0) -> np.ndarray:
    """Row-major float32 view-projection P @ V, built in float64, rounded once.

    V is a right-handed look-at (camera looks down -z); P is the usual
    OpenGL-style perspective, so clip w equals the distance along the view
    axis."""
    eye = np.asarray(eye, dtype=np.float64)
    centre = np.asarray(centre, dtype=np.float64)
    up = np.asarray(up, dtype=np.float64)
    f = centre - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, up)
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    view = np.eye(4)
    view[0, :3], view[1, :3], view[2, :3] = s, u, -f
    view[0, 3], view[1, 3], view[2, 3] = -s @ eye, -u @ eye, f @ eye
    t = 1.0 / math.tan(math.radians(fov_y_deg) / 2.0)
    proj = np.zeros((4, 4))
    proj[0, 0] = t / aspect
    proj[1, 1] = t
    proj[2, 2] = (far + near) / (near - far)
    proj[2, 3] = 2.0 * far * near / (near - far)
    proj[3, 2] = -1.0
    return (proj @ view).astype(np.float32)


def orbit_camera(frame: int, width: int, height: int, radius: float = 2.5,
                 deg_per_frame: float = 1.0, fov_y_deg: float = 60.0,
                 centre=(0.5, 0.5, 0.5), start_deg: float = 0.0) -> np.ndarray:
    """Camera of the 3D workloads: orbits the cube centre in the x-z plane."""
    theta = math.radians(start_deg + deg_per_frame * frame)
    c = np.asarray(centre, dtype=np.float64)
    eye = c + radius * np.array([math.sin(theta), 0.0, math.cos(theta)])
    return look_at_perspective(eye, c, (0.0, 1.0, 0.0), fov_y_deg, width / height)


IDENTITY = np.eye(4, dtype=np.float32)


@dataclass
class CloudSpec:
    """One cloud of the batched workload."""
    n: int
    seed: int
    kind: str                       # "uniform" or "mixture"
    views: list = field(default_factory=list)   # [(width, height, start_deg)]


def batched_set(count: int = 64, seed: int = 0, lo_log2: float = 12.0,
                hi_log2: float = 22.0, resolutions=(256, 512, 1024),
                max_views: int = 4) -> list[CloudSpec]:
    """Cloud sizes log-uniform in [2^lo, 2^hi]; 1..max_views square views."""
    rng = _rng(seed)
    out = []
    for j in range(count):
        n = int(round(2.0 ** rng.uniform(lo_log2, hi_log2)))
        kind = "uniform" if j % 2 == 0 else "mixture"
        nv = int(rng.integers(1, max_views + 1))
        views = []
        for _ in range(nv):
            r = int(resolutions[int(rng.integers(0, len(resolutions)))])
            views.append((r, r, float(rng.uniform(0.0, 360.0))))
        out.append(CloudSpec(n=n, seed=1000 + j, kind=kind, views=views))
    return out


def cloud_points(spec: CloudSpec) -> np.ndarray:
    if spec.kind == "uniform":
        return uniform_cube(spec.n, spec.seed)
    return gaussian_mixture(spec.n, spec.seed)


def poisson_arrivals(rate_hz: float, count: int, seed: int = 0) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process."""
    gaps = _rng(seed).exponential(1.0 / rate_hz, size=count)
    return np.cumsum(gaps)
