"""Pins of the oracle's edges view (segments between indexed vertices):
closed-form pixel runs, depth order at a crossing, the degenerate segment,
triangles as their three sides, skipped indices, and connectivity."""
import numpy as np

import oracle
import synth

EMPTY = 0xFFFFFFFFFFFFFFFF


def _keys(pos, idx, prim, m, w, h):
    d = oracle.new_depth(w, h)
    oracle.lib().oracle_splat_edges(
        oracle._ptr(pos, oracle.C.c_float), pos.shape[0], pos.shape[1],
        oracle._ptr(np.ascontiguousarray(idx, dtype=np.uint32), oracle.C.c_uint32),
        len(idx) // prim, prim, oracle._ptr(oracle._mat(m), oracle.C.c_float), w, h,
        oracle._ptr(d, oracle.C.c_uint64))
    return d.reshape(h, w)


def _x2d(sx, w):  # 2D coordinate whose screen x is sx (exact at these sizes)
    return np.float32(sx / (w / 2) - 1.0)


def test_horizontal_and_diagonal_runs_in_2d():
    w, h = 64, 32
    # from screen (10.5, 16.5) to (40.5, 16.5): 30 steps of one pixel
    pos = np.array([[_x2d(10.5, w), _x2d(16.5, h)], [_x2d(40.5, w), _x2d(16.5, h)],
                    [_x2d(5.5, w), _x2d(5.5, h)], [_x2d(25.5, w), _x2d(25.5, h)]], np.float32)
    k = _keys(pos, [0, 1], 2, synth.IDENTITY, w, h)
    drawn = np.argwhere(k != EMPTY)
    assert sorted(map(tuple, drawn)) == [(h - 1 - 16, x) for x in range(10, 41)]
    assert np.all(k[k != EMPTY] == 0)  # 2D: depth bits 0, edge 0
    k = _keys(pos, [2, 3], 2, synth.IDENTITY, w, h)
    assert sorted(map(tuple, np.argwhere(k != EMPTY))) == sorted((h - 1 - (5 + j), 5 + j) for j in range(21))


def test_degenerate_segment_is_its_vertex_pixel():
    w, h = 96, 64
    m = synth.orbit_camera(30, w, h)
    rng = np.random.default_rng(0)
    for _ in range(50):
        p = (0.5 + 0.2 * rng.standard_normal((1, 3))).astype(np.float32)
        k = _keys(p, [0, 0], 2, m, w, h)
        r = oracle.project(p[0], m, w, h)
        if r is None:
            assert np.all(k == EMPTY)
        else:
            px, py, bits = r
            assert np.argwhere(k != EMPTY).tolist() == [[py, px]]
            assert int(k[py, px]) == (bits << 32)


def test_nearer_segment_wins_the_crossing():
    w, h = 64, 64
    # camera: screen x = (x / z + 1) W/2, screen y = (y / z + 1) H/2, clip w = z
    m = np.zeros(16, np.float32)
    m[0], m[5], m[14] = 1.0, 1.0, 1.0
    near = np.array([[-0.5, 0.0, 1.0], [0.5, 0.0, 1.0]], np.float32)    # w = 1, horizontal
    far = np.array([[0.0, -1.0, 2.0], [0.0, 1.0, 2.0]], np.float32)     # w = 2, vertical
    pos = np.concatenate([far, near])
    k = _keys(pos, [0, 1, 2, 3], 2, m, w, h)
    cross = (h - 1 - 32, 32)
    assert int(k[cross]) == (int(np.float32(1.0).view(np.uint32)) << 32) | 1
    # elsewhere on the far segment its own key
    assert int(k[h - 1 - 20, 32]) == (int(np.float32(2.0).view(np.uint32)) << 32) | 0


def test_triangles_are_their_three_sides():
    w, h = 80, 60
    m = synth.orbit_camera(10, w, h)
    pos = synth.gaussian_mixture(300, 2, sigma=0.1)
    rng = np.random.default_rng(3)
    tri = rng.integers(0, 300, size=(40, 3)).astype(np.uint32)
    pairs = np.stack([tri, np.roll(tri, -1, axis=1)], axis=2).reshape(-1)  # side j: (v_j, v_{j+1})
    assert np.array_equal(_keys(pos, tri.reshape(-1), 3, m, w, h), _keys(pos, pairs, 2, m, w, h))


def test_out_of_range_vertex_skips_the_segment():
    w, h = 32, 32
    pos = np.array([[-0.5, 0.0], [0.5, 0.0]], np.float32)
    assert np.all(_keys(pos, [0, 2], 2, synth.IDENTITY, w, h) == EMPTY)
    assert np.any(_keys(pos, [0, 1], 2, synth.IDENTITY, w, h) != EMPTY)


def test_segment_pixels_are_8_connected_and_start_at_the_vertex():
    w, h = 128, 96
    m = synth.orbit_camera(45, w, h)
    rng = np.random.default_rng(7)
    for _ in range(100):
        p = (0.5 + 0.3 * rng.standard_normal((2, 3))).astype(np.float32)
        k = _keys(p, [0, 1], 2, m, w, h)
        pts = {tuple(x) for x in np.argwhere(k != EMPTY)}
        a = oracle.project(p[0], m, w, h)
        b, sa = oracle.project(p[1], m, w, h), oracle.screen(p[0], m, w, h)
        if a is not None and b is not None:
            assert (a[1], a[0]) in pts
            # 8-connected: a walk from the start reaches every drawn pixel
            seen, todo = {(a[1], a[0])}, [(a[1], a[0])]
            while todo:
                y, x = todo.pop()
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        q = (y + dy, x + dx)
                        if q in pts and q not in seen:
                            seen.add(q)
                            todo.append(q)
            assert seen == pts
