"""GPU parity of the structured-grid view: frames equal the oracle's bit for
bit, for magnified, reduced and non-divisible lattice-to-screen ratios, each
index width, values past the palette, and cell values rewritten between
renders (as a simulation updating its lattice)."""
import numpy as np
import pytest

import oracle
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


def _tensor_alloc(rig, arr):
    t = rig.torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    rig.keep.append(t)
    return t, rig.mm.mm_alloc_wrap(rig.inst, t.data_ptr(), t.numel() * t.element_size())


@pytest.mark.parametrize("cols,rows,w,h", [(512, 512, 1920, 1080), (1000, 700, 640, 480),
                                           (3, 5, 64, 32), (4096, 4096, 1024, 1024),
                                           (1, 1, 2, 2), (65536, 3, 256, 2)])
@pytest.mark.parametrize("dt", [np.uint8, np.uint16, np.uint32])
def test_grid_matches_oracle(rig, cols, rows, w, h, dt):
    say(f"case: grid {cols}x{rows} on {w}x{h}, {np.dtype(dt).name} cells")
    mm = rig.mm
    rng = np.random.default_rng(cols + rows + w)
    pal = rng.integers(0, 2**32, 200, dtype=np.uint64).astype(np.uint32)
    cells = rng.integers(0, 256, cols * rows).astype(dt)  # values 200..255 are past the palette
    _, pal_a = _tensor_alloc(rig, pal)
    cells_t, cells_a = _tensor_alloc(rig, cells)
    g = mm.mm_create_grid(rig.inst, cols, rows, w, h, pal_a, 200, cells_a, np.dtype(dt).itemsize)
    mm.mm_grid_render(g)
    want = oracle.render_grid(cols, rows, w, h, pal, cells)
    got = mm.mm_grid_read_frame(g, w, h)
    assert np.array_equal(got, want), first_diff(got, want)
    # the simulation rewrites its lattice; the next render shows the new values
    cells2 = rng.integers(0, 200, cols * rows).astype(dt)
    cells_t.copy_(rig.torch.from_numpy(cells2))
    mm.mm_grid_render(g)
    want = oracle.render_grid(cols, rows, w, h, pal, cells2)
    assert np.array_equal(mm.mm_grid_read_frame(g, w, h), want)
    mm.mm_destroy_grid(g)


def test_grid_validation(rig):
    say("case: grid validation")
    mm = rig.mm
    _, pal_a = _tensor_alloc(rig, np.arange(8, dtype=np.uint32))
    _, cells_a = _tensor_alloc(rig, np.zeros(100, dtype=np.uint8))
    for args, what in [((10, 10, 64, 64, pal_a, 9, cells_a, 1), "palette larger than its alloc"),
                       ((11, 10, 64, 64, pal_a, 8, cells_a, 1), "more cells than the alloc holds"),
                       ((10, 10, 64, 64, pal_a, 8, cells_a, 3), "index width"),
                       ((10, 10, 63, 64, pal_a, 8, cells_a, 1), "odd screen"),
                       ((0, 10, 64, 64, pal_a, 8, cells_a, 1), "empty lattice"),
                       ((10, 10, 64, 64, pal_a, 0, cells_a, 1), "empty palette")]:
        with pytest.raises(mm.MMError) as e:
            mm.mm_create_grid(rig.inst, *args)
        assert e.value.status == mm.MM_ERR_INVALID_ARG, what
    g = mm.mm_create_grid(rig.inst, 10, 10, 64, 64, pal_a, 8, cells_a, 1)
    with pytest.raises(mm.MMError) as e:
        mm.mm_free(pal_a)
    assert e.value.status == mm.MM_ERR_IN_USE
    mm.mm_destroy_grid(g)
    mm.mm_free(pal_a)
