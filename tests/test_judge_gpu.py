"""The judge kernel (interface Hausdorff distance and RMS) against the oracle's
exact Hausdorff distance (scipy cKDTree over the same zero crossings)."""
import math

import numpy as np
import pytest
import torch

from oracle import diagnostics as D
from paper_2105_09671_amd import inputs, params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available()
    from paper_2105_09671_amd import api as a
    return a


def _judge(api, a, b, h, window=3):
    ta = torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    tb = torch.from_numpy(np.ascontiguousarray(b, np.float32)).cuda()
    i, l = api.judge2d(ta, tb, h, window)
    return i.cpu().numpy(), l.cpu().numpy()


def test_circles_against_exact_hausdorff(api):
    n, h = 128, 1 / 128
    eps = params.eps_m(h, 4)
    base = inputs.circle2d(n, n, h, eps, 0.25)
    shifts = [0.0, 0.3, 1.1, 1.9, 2.6, 5.0]
    a = np.stack([base] * len(shifts)).astype(np.float32)
    b = np.stack([inputs.circle2d(n, n, h, eps, 0.25 + s * h) for s in shifts]).astype(np.float32)
    got, l2 = _judge(api, a, b, h)
    for k, s in enumerate(shifts):
        exact = D.interface_error(a[k].astype(np.float64), b[k].astype(np.float64), h)
        if exact <= 2 * h:
            assert abs(got[k] - exact) <= 1e-4 * h + 1e-6 * exact, (s, got[k], exact)
        else:
            assert got[k] > 2 * h, (s, got[k], exact)
        assert abs(l2[k] - math.sqrt(np.mean((a[k].astype(np.float64) - b[k]) ** 2))) <= 1e-5


def test_random_fields_and_edge_cases(api):
    n, h = 48, 1 / 48
    a = inputs.random_field((4, n, n), 90).astype(np.float32)
    b = (a + 0.02 * inputs.random_field((4, n, n), 91)).astype(np.float32)
    b[3] = np.abs(b[3]) + 0.1          # no interface at all in b[3]
    got, _ = _judge(api, a, b, h, window=4)
    for k in range(3):
        exact = D.interface_error(a[k].astype(np.float64), b[k].astype(np.float64), h)
        if exact <= 3 * h:
            assert abs(got[k] - exact) <= 1e-4 * h
    assert math.isinf(got[3])
    same, l2 = _judge(api, a, a, h)
    assert np.all(same == 0) and np.all(l2 == 0)
    pos = np.ones((2, 16, 16), np.float32)
    z, _ = _judge(api, pos, pos * 0.5, 1 / 16)
    assert np.all(z == 0)                # neither has an interface


def test_ragged_grids_and_widest_window(api):
    """Grids that are not whole 64 x 16 judge tiles, with the widest window (16
    cells) and a narrow one: every value the window can decide against the
    oracle's exact Hausdorff distance."""
    for (nx, ny), w, shifts in (((100, 70), 16, [0.4, 3.3, 9.7]), ((65, 17), 16, [0.0, 2.2]),
                                ((100, 70), 2, [0.0, 0.4]), ((1, 1), 3, [0.0])):
        h = 1 / max(nx, ny)
        eps = params.eps_m(h, 4)
        base = inputs.circle2d(nx, ny, h, eps, 0.25)
        a = np.stack([base] * len(shifts)).astype(np.float32)
        b = np.stack([inputs.circle2d(nx, ny, h, eps, 0.25 + s * h) for s in shifts]).astype(np.float32)
        got, l2 = _judge(api, a, b, h, window=w)
        for k, s in enumerate(shifts):
            exact = D.interface_error(a[k].astype(np.float64), b[k].astype(np.float64), h)
            if exact <= (w - 1) * h:
                assert abs(got[k] - exact) <= 1e-4 * h + 1e-6 * exact, ((nx, ny), w, s, got[k], exact)
            else:
                assert got[k] >= (w - 1) * h, ((nx, ny), w, s, got[k], exact)
            ref = math.sqrt(np.mean((a[k].astype(np.float64) - b[k]) ** 2))
            assert abs(l2[k] - ref) <= 1e-5 + 1e-5 * ref
    n = 65
    ra = inputs.random_field((2, 17, n), 93).astype(np.float32)
    rb = (ra + 0.02 * inputs.random_field((2, 17, n), 94)).astype(np.float32)
    got, _ = _judge(api, ra, rb, 1 / n, 16)
    for k in range(2):
        exact = D.interface_error(ra[k].astype(np.float64), rb[k].astype(np.float64), 1 / n)
        if exact <= 15 / n:
            assert abs(got[k] - exact) <= 1e-4 / n, (k, got[k], exact)
