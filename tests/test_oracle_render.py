"""Pin the oracle's projection, splat and resolve.

* Closed-form pixels: points placed (in float64) at known pixel centres must
  land on exactly that pixel; 2D grid centres and edges; 3D points solved
  from the matrix rows so that their projection is >= 0.25 px inside the
  target pixel. A transposed matrix, a missing row flip or a dropped term
  moves them.
* Depth order: on one ray the nearer point wins; equal keys go to the
  smaller index; points behind the near plane or off screen write nothing.
* Processing-order invariance: the splat in any permuted order gives the
  same depth buffer.
* Brute force in gather form on tiny clouds (1000 seeds): per pixel, the
  minimum key over all points whose footprint covers it.
* Resolve: covered pixels carry colour(argmin index) with alpha 0xFF,
  uncovered pixels are 0, and the depth buffer is left empty.
"""
import numpy as np
import pytest

import oracle
import synth

EMPTY = 0xFFFFFFFFFFFFFFFF


def _screen_xy(m64, p32, w, h):
    p = np.append(p32.astype(np.float64), 1.0)
    c = m64 @ p
    return (c[0] / c[3] + 1.0) * (w / 2), (c[1] / c[3] + 1.0) * (h / 2), c[3]


def _solve_point(m32, u, v, depth, w, h):
    """World point whose projection is the centre of pixel (u, v) at clip w
    = depth, solved in float64 from rows 0, 1, 3 of the float32 matrix."""
    m = m32.astype(np.float64)
    sx, sy = u + 0.5, (h - 1 - v) + 0.5
    nx, ny = sx / (w / 2) - 1.0, sy / (h / 2) - 1.0
    a = m[[0, 1, 3], :3]
    b = np.array([nx * depth - m[0, 3], ny * depth - m[1, 3], depth - m[3, 3]])
    return np.linalg.solve(a, b).astype(np.float32)


def test_2d_pixel_centres_and_edges():
    w = h = 512
    eye = synth.IDENTITY
    for k in [0, 1, 17, 255, 256, 510, 511]:
        for j in [0, 3, 256, 511]:
            x = np.float32((2 * k + 1) / w - 1.0)
            y = np.float32((2 * j + 1) / h - 1.0)
            assert oracle.project([x, y], eye, w, h) == (k, h - 1 - j, 0)
    # left/bottom edge is inside, exactly; the last float below 1 is inside
    assert oracle.project([-1.0, -1.0], eye, w, h) == (0, h - 1, 0)
    below_one = np.float32(1.0 - 2.0**-23)
    assert oracle.project([below_one, below_one], eye, w, h) == (w - 1, 0, 0)
    # 1 - 2^-24 + 1 rounds (to even) to 2.0, so x maps to sx == W: culled
    assert oracle.project([np.float32(1.0 - 2.0**-24), 0.0], eye, w, h) is None
    assert oracle.project([np.float32(1.0), 0.0], eye, w, h) is None


def test_2d_non_square_screen():
    w, h = 64, 16
    for k in range(w):
        x = np.float32((2 * k + 1) / w - 1.0)
        assert oracle.project([x, np.float32(-1.0)], synth.IDENTITY, w, h) == (k, h - 1, 0)
    for j in range(h):
        y = np.float32((2 * j + 1) / h - 1.0)
        assert oracle.project([np.float32(-1.0), y], synth.IDENTITY, w, h) == (0, h - 1 - j, 0)


@pytest.mark.parametrize("frame", [0, 37, 90, 211])
@pytest.mark.parametrize("res", [(1920, 1080), (3840, 2160), (512, 512)])
def test_3d_closed_form_pixels(frame, res):
    w, h = res
    m32 = synth.orbit_camera(frame, w, h)
    rng = np.random.default_rng(frame * 7 + w)
    checked = 0
    for _ in range(300):
        u, v = int(rng.integers(0, w)), int(rng.integers(0, h))
        depth = float(rng.choice([1.6, 2.5, 3.4]))
        p = _solve_point(m32, u, v, depth, w, h)
        sx, sy, cw = _screen_xy(m32.astype(np.float64), p, w, h)
        fx, fy = sx - np.floor(sx), sy - np.floor(sy)
        if min(fx, 1 - fx, fy, 1 - fy) < 0.25:
            continue  # rounding of p moved it too close to an edge
        got = oracle.project(p, m32, w, h)
        assert got is not None
        assert got[:2] == (u, v)
        dw = np.array([got[2]], dtype=np.uint32).view(np.float32)[0]
        assert abs(float(dw) - cw) <= 4e-7 * cw
        checked += 1
    assert checked > 250


def test_3d_cube_centre_near_screen_centre():
    # Camera sanity (the camera is a host-side input, not pinned further).
    for f in [0, 45, 180]:
        m = synth.orbit_camera(f, 1920, 1080)
        px, py, bits = oracle.project(np.float32([0.5, 0.5, 0.5]), m, 1920, 1080)
        assert abs(px - 960) <= 1 and abs(py - 540) <= 1
        d = np.array([bits], dtype=np.uint32).view(np.float32)[0]
        assert abs(float(d) - 2.5) < 1e-5


def test_3d_culling():
    w, h = 320, 240
    m = synth.orbit_camera(0, w, h)
    # camera at (0.5, 0.5, 3.0) looking at -z: a point behind it, one at the
    # camera, one between the camera and the near plane
    for z in [3.5, 3.0, 2.95]:
        assert oracle.project(np.float32([0.5, 0.5, z]), m, w, h) is None
    # just past the near plane (distance 0.2) is kept
    assert oracle.project(np.float32([0.5, 0.5, 2.8]), m, w, h) is not None
    # far off to the side: off screen
    assert oracle.project(np.float32([50.0, 0.5, 0.5]), m, w, h) is None


def test_depth_order_on_one_ray():
    w, h = 256, 128
    m = synth.orbit_camera(10, w, h)
    u, v = 100, 50
    near = _solve_point(m, u, v, 1.6, w, h)
    far = _solve_point(m, u, v, 3.4, w, h)
    pos = np.stack([far, near]).astype(np.float32)  # far has the smaller index
    d = oracle.new_depth(w, h)
    oracle.splat(pos, m, w, h, 1, d)
    assert int(d[v * w + u]) & 0xFFFFFFFF == 1  # the nearer point wins
    # equal keys: two copies of one point, the smaller index wins
    pos2 = np.stack([near, near, far]).astype(np.float32)
    d2 = oracle.new_depth(w, h)
    oracle.splat(pos2, m, w, h, 1, d2)
    assert int(d2[v * w + u]) & 0xFFFFFFFF == 0
    assert np.count_nonzero(d2 != oracle.EMPTY) == 1


def test_footprint_3x3_clips_at_borders():
    w = h = 16
    eye = synth.IDENTITY
    corner = np.float32([[-1.0, -1.0]])  # pixel (0, 15): bottom-left
    d = oracle.new_depth(w, h)
    oracle.splat(corner, eye, w, h, 3, d)
    hit = np.argwhere(d.reshape(h, w) != oracle.EMPTY)
    assert sorted(map(tuple, hit)) == [(14, 0), (14, 1), (15, 0), (15, 1)]
    mid = np.float32([[(2 * 7 + 1) / w - 1.0, (2 * 7 + 1) / h - 1.0]])
    d = oracle.new_depth(w, h)
    oracle.splat(mid, eye, w, h, 3, d)
    hit = np.argwhere(d.reshape(h, w) != oracle.EMPTY)
    assert sorted(map(tuple, hit)) == [(r, c) for r in (7, 8, 9) for c in (6, 7, 8)]


@pytest.mark.parametrize("dim,footprint", [(2, 1), (3, 1), (3, 3), (2, 3)])
def test_splat_is_invariant_under_processing_order(dim, footprint):
    w, h = 96, 64
    n = 20000
    pos = (synth.uniform_square(n, 4) if dim == 2 else synth.gaussian_mixture(n, 4, sigma=0.05))
    m = synth.IDENTITY if dim == 2 else synth.orbit_camera(3, w, h)
    ref = oracle.new_depth(w, h)
    oracle.splat(pos, m, w, h, footprint, ref)
    rng = np.random.default_rng(9)
    for _ in range(3):
        d = oracle.new_depth(w, h)
        oracle.splat(pos, m, w, h, footprint, d, order=rng.permutation(n))
        assert np.array_equal(d, ref)


def test_memory_permutation_relabels_indices():
    # Permuting memory order relabels the points; with no depth ties the
    # same point wins each pixel, under its new index.
    w, h = 80, 60
    n = 5000
    pos = synth.uniform_cube(n, 6)
    m = synth.orbit_camera(0, w, h)
    d0 = oracle.new_depth(w, h)
    oracle.splat(pos, m, w, h, 1, d0)
    perm = np.random.default_rng(1).permutation(n)      # new slot j holds old perm[j]
    d1 = oracle.new_depth(w, h)
    oracle.splat(np.ascontiguousarray(pos[perm]), m, w, h, 1, d1)
    cov = d0 != oracle.EMPTY
    assert np.array_equal(cov, d1 != oracle.EMPTY)
    assert np.array_equal(d0[cov] >> np.uint64(32), d1[cov] >> np.uint64(32))
    old_idx = (d0[cov] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    new_idx = (d1[cov] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert np.array_equal(perm[new_idx], old_idx)


def _gather(pos, m, w, h, footprint):
    """Gather form: per pixel, the min key over all covering points."""
    reach = footprint // 2
    n = pos.shape[0]
    px = np.full(n, -10**6)
    py = np.full(n, -10**6)
    keys = np.zeros(n, dtype=np.uint64)
    for i in range(n):
        r = oracle.project(pos[i], m, w, h)
        if r is not None:
            px[i], py[i] = r[0], r[1]
            keys[i] = (np.uint64(r[2]) << np.uint64(32)) | np.uint64(i)
    qy, qx = np.mgrid[0:h, 0:w]
    cover = ((np.abs(qx.reshape(-1, 1) - px) <= reach)
             & (np.abs(qy.reshape(-1, 1) - py) <= reach))
    big = np.where(cover, keys, np.uint64(EMPTY))
    return big.min(axis=1)


def test_gather_brute_force_tiny_clouds():
    for seed in range(1000):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(1, 33))
        w = 2 * int(rng.integers(1, 9))
        h = 2 * int(rng.integers(1, 9))
        footprint = 1 if seed % 2 == 0 else 3
        if seed % 3 == 0:
            # 2D, points on a coarse grid so ties are frequent
            pos = (rng.integers(-4, 4, size=(n, 2)) / 4.0).astype(np.float32)
            m = synth.IDENTITY
        else:
            pos = (0.5 + 0.2 * rng.standard_normal((n, 3))).astype(np.float32)
            if seed % 5 == 0:
                pos[n // 2:] = pos[: n - n // 2]  # duplicated points: depth ties
            m = synth.orbit_camera(int(rng.integers(0, 360)), w, h)
        d = oracle.new_depth(w, h)
        oracle.splat(pos, m, w, h, footprint, d)
        assert np.array_equal(d, _gather(pos, m, w, h, footprint)), seed


def test_resolve_definition():
    w, h = 64, 48
    pos = synth.gaussian_mixture(3000, 2, sigma=0.1)
    m = synth.orbit_camera(5, w, h)
    d = oracle.new_depth(w, h)
    oracle.splat(pos, m, w, h, 3, d)
    keys = d.copy()
    c = oracle.resolve(d, seed=77)
    assert np.all(d == oracle.EMPTY)
    cov = keys != oracle.EMPTY
    assert np.all(c[~cov] == 0)
    assert np.count_nonzero(c) == np.count_nonzero(cov)
    for q in np.flatnonzero(cov):
        i = int(keys[q]) & 0xFFFFFFFF
        assert int(c[q]) == oracle.colour(i, 77)
        assert int(c[q]) >> 24 == 0xFF
    # the colour hash is the first Philox word of the colour-tagged counter
    for i in [0, 1, 12345, 2**31 + 5]:
        r = oracle.philox4x32_10(np.array([[0, 2, i, 0]]), np.array([[77, 0]]))
        assert oracle.colour(i, 77) == int(r[0, 0]) | 0xFF000000


def test_step_render_is_displace_then_render():
    w, h = 128, 128
    pos = synth.uniform_square(5000, 0)
    a = pos.copy()
    frame = oracle.step_render(a, 0, 4, 0.005, True, synth.IDENTITY, w, h, 1)
    b = pos.copy()
    oracle.displace(b, 0, 4, 0.005, True)
    assert np.array_equal(a, b)
    assert np.array_equal(frame, oracle.render(b, 0, synth.IDENTITY, w, h, 1))


def test_palette_of_hash_colours_is_the_default_render():
    """Special case that reduces to the pinned hash colour: a per-point
    palette holding each point's hash colour gives the default frame."""
    w, h = 96, 64
    pos = synth.uniform_cube(4000, 3)
    m = synth.orbit_camera(40, w, h)
    pal = np.array([oracle.colour(i, 5) for i in range(pos.shape[0])], dtype=np.uint32)
    assert np.array_equal(oracle.render_palette(pos, m, w, h, 3, pal),
                          oracle.render(pos, 5, m, w, h, 3))
    # the same through an identity index buffer of each width
    for dt in (np.uint16, np.uint32):
        idx = np.arange(pos.shape[0], dtype=dt)
        assert np.array_equal(oracle.render_palette(pos, m, w, h, 3, pal, idx),
                              oracle.render(pos, 5, m, w, h, 3))


def test_palette_single_entry_covers_exactly_the_drawn_pixels():
    w, h = 80, 60
    pos = synth.gaussian_mixture(3000, 1, sigma=0.05)
    m = synth.orbit_camera(10, w, h)
    idx = np.zeros(pos.shape[0], dtype=np.uint8)
    got = oracle.render_palette(pos, m, w, h, 1, np.array([0x11223344], np.uint32), idx)
    drawn = oracle.render(pos, 0, m, w, h, 1) != 0  # hash colours are never 0 (opaque)
    assert np.all(got[drawn] == 0x11223344) and np.all(got[~drawn] == 0)


def test_palette_brute_force_with_indices_past_the_end():
    """Gather form: per pixel the winning point by brute force, then its
    palette entry through its index; indices at or past the end give 0."""
    for seed in range(200):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(1, 33))
        w, h = 2 * int(rng.integers(1, 9)), 2 * int(rng.integers(1, 9))
        footprint = 1 if seed % 2 == 0 else 3
        pos = (0.5 + 0.2 * rng.standard_normal((n, 3))).astype(np.float32)
        m = synth.orbit_camera(int(rng.integers(0, 360)), w, h)
        pal = rng.integers(1, 2**32, size=int(rng.integers(1, 9)), dtype=np.uint64).astype(np.uint32)
        idx = rng.integers(0, pal.shape[0] + 3, size=n).astype(np.uint8)
        keys = _gather(pos, m, w, h, footprint)
        want = np.zeros(w * h, dtype=np.uint32)
        for q in range(w * h):
            if keys[q] != EMPTY:
                j = int(idx[int(keys[q]) & 0xFFFFFFFF])
                want[q] = pal[j] if j < pal.shape[0] else 0
        got = oracle.render_palette(pos, m, w, h, footprint, pal, idx)
        assert np.array_equal(got.reshape(-1), want), seed


def test_grid_one_pixel_per_cell_is_the_flipped_lattice():
    """Closed form: with one pixel per cell the frame is the lattice of
    palette colours with its rows flipped (cell row 0 at the bottom)."""
    rng = np.random.default_rng(0)
    cols, rows = 12, 8
    pal = rng.integers(0, 2**32, 10, dtype=np.uint64).astype(np.uint32)
    cells = rng.integers(0, 12, cols * rows).astype(np.uint16)  # 10, 11 past the palette
    want = np.where(cells < 10, pal[np.minimum(cells, 9)], 0).astype(np.uint32).reshape(rows, cols)[::-1]
    assert np.array_equal(oracle.render_grid(cols, rows, cols, rows, pal, cells), want)


def test_grid_integer_magnification_replicates_cells():
    rng = np.random.default_rng(1)
    cols, rows, k = 6, 4, 3
    pal = rng.integers(0, 2**32, 8, dtype=np.uint64).astype(np.uint32)
    cells = rng.integers(0, 8, cols * rows).astype(np.uint8)
    base = oracle.render_grid(cols, rows, cols, rows, pal, cells)
    want = np.repeat(np.repeat(base, k, axis=0), k, axis=1)
    assert np.array_equal(oracle.render_grid(cols, rows, k * cols, k * rows, pal, cells), want)


def test_grid_cell_of_pixel_centre_in_float64():
    """The integer cell rule equals the cell holding the pixel centre,
    computed in float64 (exact at these sizes), for non-divisible sizes."""
    for cols, width in [(7, 10), (10, 7), (1, 2), (33, 64), (64, 34), (5, 2)]:
        for px in range(width):
            centre = (px + 0.5) * cols / width
            assert (2 * px + 1) * cols // (2 * width) == int(np.floor(centre))
