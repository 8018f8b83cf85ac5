"""The host-copy comparison renderer draws the oracle's frame bit for bit,
at any thread count (per-thread key buffers merged by minimum)."""
import numpy as np
import pytest

import oracle
import synth
from paper_2504_20937_amd import hostcopy


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_3d_uniform_matches_oracle(threads):
    pts = synth.uniform_cube(20011, 4)
    for f in (0, 33):
        cam = synth.orbit_camera(f, 320, 200)
        want = oracle.render(pts, 17, cam, 320, 200, 1)
        got = hostcopy.render(pts, 17, cam, 320, 200, 1, threads)
        assert np.array_equal(got, want)


def test_3d_mixture_3x3_matches_oracle():
    pts = synth.gaussian_mixture(30000, 2)
    cam = synth.orbit_camera(10, 257 * 2, 130)
    want = oracle.render(pts, 5, cam, 514, 130, 3)
    assert np.array_equal(hostcopy.render(pts, 5, cam, 514, 130, 3, 5), want)


def test_2d_ties_resolve_to_the_smallest_index():
    # many points on few pixels: depth 0 everywhere, so the index decides
    pts = (synth.uniform_square(5000, 1) * np.float32(0.01)).astype(np.float32)
    pts = np.concatenate([pts, pts, pts])
    want = oracle.render(pts, 3, synth.IDENTITY, 64, 64, 1)
    for threads in (1, 4, 7):
        assert np.array_equal(hostcopy.render(pts, 3, synth.IDENTITY, 64, 64, 1, threads), want)


def test_after_steps_equals_oracle_step_render():
    pts = synth.uniform_square(4099, 0)
    ref = pts.copy()
    for s in range(3):
        want = oracle.step_render(ref, 9, s, 0.005, True, synth.IDENTITY, 96, 48, 3)
        got = hostcopy.render(ref, 9, synth.IDENTITY, 96, 48, 3, 2)
        assert np.array_equal(got, want)


def test_invalid_arguments():
    with pytest.raises(RuntimeError):
        hostcopy.render(np.zeros((4, 3), np.float32), 0, synth.IDENTITY, 1, 8)
    with pytest.raises(RuntimeError):
        hostcopy.render(np.zeros((4, 3), np.float32), 0, synth.IDENTITY, 8, 8, footprint=2)
