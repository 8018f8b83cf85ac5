"""Pin the oracle's displacement step (offset map, wrap, per-point law).

* The 24-bit offset map is checked exhaustively against the exact value of
  (k * 2^-23 - 1) * a, which float64 holds exactly and rounds once.
* Wrapping keeps 2D points in [-1, 1) at every step.
* Amplitude 0 leaves positions unchanged.
* Unwrapped 3D drift equals the float64 sum of the drawn offsets within the
  accumulated rounding bound.
* The per-point law: the offset of point i at step s uses Philox word c of
  counter (s, 0, i, 0) under key seed, checked against directly drawn words.
* Statistics: mean ~0, variance a^2/3 (uniform on [-a, a)).
"""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("a", [0.005, 0.001, 1.0, 0.0, 1e-30])
def test_offset_map_exhaustive(a):
    a32 = np.float32(a)
    k = np.arange(1 << 24, dtype=np.uint64)
    exact = ((k.astype(np.float64) * 2.0**-23 - 1.0) * np.float64(a32)).astype(np.float32)
    words = (k << np.uint64(8)).astype(np.uint32)
    got = oracle.offset_many(words, float(a32))
    assert np.array_equal(got.view(np.uint32), exact.view(np.uint32))
    # the low 8 bits of the word never matter
    got_low = oracle.offset_many(words | np.uint32(0xFF), float(a32))
    assert np.array_equal(got_low.view(np.uint32), got.view(np.uint32))
    # bounds: never beyond a; the grid reaches -a exactly
    assert np.all(np.abs(exact) <= a32)
    assert exact.min() == -a32
    assert float(oracle.offset(0x80000000, float(a32))) == 0.0


def test_offset_map_all_codes_through_displace():
    # Every one of the 2^24 codes, through the full displacement path: points
    # at 0 with a fixed key pick up exactly the offsets of their Philox words.
    n = 1 << 20
    pos = np.zeros((n, 3), dtype=np.float32)
    oracle.displace(pos, seed=99, step=3, a=0.005, wrap=False)
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = 3
    ctr[:, 2] = np.arange(n, dtype=np.uint32)
    key = np.tile(np.array([[99, 0]], dtype=np.uint32), (n, 1))
    r = oracle.philox4x32_10(ctr, key)[:, :3]
    k = (r >> np.uint32(8)).astype(np.float64)
    exact = ((k * 2.0**-23 - 1.0) * np.float64(np.float32(0.005))).astype(np.float32)
    assert np.array_equal(pos.view(np.uint32), exact.view(np.uint32))


def test_wrap_keeps_square_points_in_box():
    pos = synth.uniform_square(1 << 16, seed=0)
    # push many points near the edges to exercise both folds
    pos[:4096, 0] = np.float32(0.9999)
    pos[4096:8192, 1] = np.float32(-1.0)
    for s in range(40):
        oracle.displace(pos, seed=0, step=s, a=0.005, wrap=True)
        assert pos.min() >= -1.0 and pos.max() < 1.0


def test_wrap_folds_exactly():
    for x in [1.0, 1.004, 1.0049999, -1.0000001, -1.005, 0.5, -1.0, 0.99999994]:
        x32 = np.float32(x)
        w = np.float32(oracle.wrap(float(x32)))
        if x32 >= 1.0:
            assert float(w) == float(x32) - 2.0  # exact in float64 too
        elif x32 < -1.0:
            assert float(w) == float(x32) + 2.0
        else:
            assert w == x32


def test_zero_amplitude_is_identity():
    pos = synth.uniform_cube(4096, seed=5)
    before = pos.copy()
    oracle.displace(pos, seed=1, step=7, a=0.0, wrap=False)
    # -1 * 0 gives -0.0 and x + -0.0 == x bit for bit for x != 0
    assert np.array_equal(pos.view(np.uint32), before.view(np.uint32))


def test_unwrapped_drift_matches_float64_sum():
    n, steps, a = 4096, 50, np.float32(0.001)
    pos = synth.uniform_cube(n, seed=3)
    p0 = pos.astype(np.float64)
    total = np.zeros((n, 3))
    for s in range(steps):
        oracle.displace(pos, seed=8, step=s, a=float(a), wrap=False)
        ctr = np.zeros((n, 4), dtype=np.uint32)
        ctr[:, 0] = s
        ctr[:, 2] = np.arange(n, dtype=np.uint32)
        key = np.tile(np.array([[8, 0]], dtype=np.uint32), (n, 1))
        k = (oracle.philox4x32_10(ctr, key)[:, :3] >> np.uint32(8)).astype(np.float64)
        total += (k * 2.0**-23 - 1.0) * np.float64(a)
    # each step rounds the offset (<= ulp(a)/2) and the sum (<= ulp(2)/2)
    bound = steps * (2.0**-24 * 2 + 2.0**-24 * float(a) * 2)
    assert np.max(np.abs(pos.astype(np.float64) - (p0 + total))) <= bound


def test_displacement_statistics():
    n, a = 1 << 18, 0.005
    pos = np.zeros((n, 3), dtype=np.float32)
    oracle.displace(pos, seed=2024, step=0, a=a, wrap=False)
    d = pos.astype(np.float64)
    assert abs(d.mean()) < 4 * a / np.sqrt(3 * 3 * n)
    assert abs(d.var() / (a * a / 3.0) - 1.0) < 0.01
    # coordinates uncorrelated
    c = np.corrcoef(d.T)
    assert np.all(np.abs(c - np.eye(3)) < 0.01)


def test_steps_seeds_and_indices_decorrelate():
    n = 1 << 14
    base = np.zeros((n, 2), dtype=np.float32)
    a = base.copy(); oracle.displace(a, seed=1, step=0, a=0.005, wrap=False)
    b = base.copy(); oracle.displace(b, seed=1, step=1, a=0.005, wrap=False)
    c = base.copy(); oracle.displace(c, seed=2, step=0, a=0.005, wrap=False)
    for x, y in [(a, b), (a, c), (b, c)]:
        assert abs(np.corrcoef(x[:, 0], y[:, 0])[0, 1]) < 0.05
    # a point's step does not depend on where it sits in the array
    sub = base[100:200].copy()
    oracle.displace(sub, seed=1, step=0, a=0.005, wrap=False)
    assert np.array_equal(sub, a[:100])        # index, not memory, keys the draw
    assert not np.array_equal(sub, a[100:200])
