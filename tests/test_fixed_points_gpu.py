"""Uniform fields of +1, -1 and 0 are exact fixed points of the explicit step
(section 1: +-1 are the minima of the double-well F, 0 its stationary point),
and the kernels keep them bit for bit in both precisions: FP32 through the
increment form of the update, FP64 through its product form (k1 = 1 - 2d r
rounded once).  Every 2D, 3D and batched kernel, on ragged grids of several
tiles, with several depths."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available()
    from paper_2105_09671_amd import api as a
    return a


def _params(n):
    h = 1.0 / n
    return h, 0.1 * h * h, 4.0 * h       # r = 0.1, alpha = 0.1 / 16


DTYPES = [torch.float32, torch.float64]
VALUES = [1.0, -1.0, 0.0]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("value", VALUES)
def test_uniform_2d_fields_stay_exact(api, dtype, value):
    h, dt, eps = _params(301)
    tunes = [None, dict(kernel=4, tb_depth=5, tile_x=64, tile_y=64),
             dict(kernel=6, tb_depth=7, tile_x=128, tile_y=64), dict(kernel=3, tb_depth=4, tile_x=64, tile_y=64),
             dict(kernel=1, tb_depth=3, tile_x=64, tile_y=32)]
    for tune in tunes:
        phi = torch.full((173, 301), value, dtype=dtype, device="cuda")
        api.step2d(phi, h, dt, eps, 37, tune=tune)
        torch.cuda.synchronize()
        assert torch.equal(phi, torch.full_like(phi, value)), (tune, value)
    small = torch.full((40, 56), value, dtype=dtype, device="cuda")   # one whole-grid tile
    api.step2d(small, h, dt, eps, 101)
    assert torch.equal(small, torch.full_like(small, value))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("value", VALUES)
def test_uniform_3d_fields_stay_exact(api, dtype, value):
    h, dt, eps = _params(70)
    tunes = [None, dict(kernel=5, tb_depth=3, tile_x=64, tile_y=32, tile_z=16),
             dict(kernel=2, tb_depth=4, tile_x=32, tile_y=32, tile_z=16)]
    for tune in tunes:
        phi = torch.full((41, 53, 70), value, dtype=dtype, device="cuda")
        api.step3d(phi, h, dt, eps, 13, tune=tune)
        torch.cuda.synchronize()
        assert torch.equal(phi, torch.full_like(phi, value)), (tune, value)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("value", VALUES)
def test_uniform_batched_fields_stay_exact(api, dtype, value):
    shapes2 = [(97, 131), (150, 64), (40, 300)]
    b = api.Batch([np.full(s, value) for s in shapes2], [_params(max(s)) for s in shapes2], dtype=dtype)
    b.step(23)
    torch.cuda.synchronize()
    for v in b.views():
        assert torch.equal(v, torch.full_like(v, value))
    shapes3 = [(20, 30, 70), (33, 16, 24)]
    b3 = api.Batch3D([np.full(s, value) for s in shapes3], [_params(max(s)) for s in shapes3], dtype=dtype)
    b3.step(9)
    torch.cuda.synchronize()
    for v in b3.views():
        assert torch.equal(v, torch.full_like(v, value))
