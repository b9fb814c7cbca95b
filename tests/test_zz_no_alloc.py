"""The allocation-free judge entry point (ac_judge_2d_noalloc) against the
workspace variant (ac_judge_2d), through the C ABI: two calls in a row, the
second on a smaller batch of smaller grids (the static scratch keeps the first
call's contents, which the second must not see)."""
import math

import numpy as np
import pytest
import torch

from oracle import diagnostics as D
from paper_2105_09671_amd import _lib as L
from paper_2105_09671_amd import inputs, params

pytestmark = pytest.mark.gpu


def _fields(batch, ny, nx, seed):
    h = 1.0 / max(nx, ny)
    eps = params.eps_m(h, 4)
    a = np.stack([inputs.circle2d(nx, ny, h, eps, 0.22 + 0.01 * k) for k in range(batch)])
    b = np.stack([inputs.circle2d(nx, ny, h, eps, 0.22 + 0.01 * k + (0.2 + 0.25 * k) * h)
                  for k in range(batch)])
    b[-1] = inputs.random_field((ny, nx), seed, amp=0.9)        # a ragged interface
    return (torch.from_numpy(a.astype(np.float32)).cuda(),
            torch.from_numpy(b.astype(np.float32)).cuda(), h)


def _both(lib, a, b, h, window):
    n, ny, nx = a.shape
    st = torch.cuda.current_stream().cuda_stream
    i1, l1 = (torch.full((n,), float("nan"), device="cuda") for _ in range(2))
    ws = torch.empty(int(lib.ac_judge_workspace_bytes(n)), dtype=torch.uint8, device="cuda")
    L.check(lib.ac_judge_2d(a.data_ptr(), b.data_ptr(), n, nx, ny, h, window, i1.data_ptr(),
                            l1.data_ptr(), ws.data_ptr(), st), "ac_judge_2d")
    i2, l2 = (torch.full((n,), float("nan"), device="cuda") for _ in range(2))
    L.check(lib.ac_judge_2d_noalloc(a.data_ptr(), b.data_ptr(), n, nx, ny, h, window, i2.data_ptr(),
                                    l2.data_ptr(), st), "ac_judge_2d_noalloc")
    torch.cuda.synchronize()
    return i1.cpu().numpy(), l1.cpu().numpy(), i2.cpu().numpy(), l2.cpu().numpy()


def test_noalloc_judge_matches_workspace_judge():
    assert torch.cuda.is_available()
    lib = L.lib()
    cases = [(7, 160, 144, 11, 3), (3, 48, 40, 12, 4)]       # second: smaller batch and grids
    for batch, ny, nx, seed, window in cases:
        a, b, h = _fields(batch, ny, nx, seed)
        print("noalloc judge: batch %d, %d x %d, window %d" % (batch, ny, nx, window), flush=True)
        i1, l1, i2, l2 = _both(lib, a, b, h, window)
        # the distance is a max of per-crossing minima (order-free): bit for bit;
        # the RMS sums FP32 atomics in arrival order: to FP32 rounding
        assert np.array_equal(i1, i2), (i1, i2)
        assert np.all(np.isfinite(l2)) and np.allclose(l1, l2, rtol=1e-6, atol=0)
        an, bn = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
        for k in range(batch - 1):
            exact = D.interface_error(an[k], bn[k], h)
            assert exact <= (window - 1) * h and abs(i2[k] - exact) <= 1e-4 * h, (k, i2[k], exact)
            assert abs(l2[k] - math.sqrt(np.mean((an[k] - bn[k]) ** 2))) <= 1e-5


def test_noalloc_judge_allocates_nothing_and_rejects_oversize():
    lib = L.lib()
    a, b, h = _fields(4, 64, 64, 13)
    st = torch.cuda.current_stream().cuda_stream
    iface = torch.empty(4, device="cuda")
    l2 = torch.empty(4, device="cuda")
    L.check(lib.ac_judge_2d_noalloc(a.data_ptr(), b.data_ptr(), 4, 64, 64, h, 3, iface.data_ptr(),
                                    l2.data_ptr(), st), "warm-up")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        L.check(lib.ac_judge_2d_noalloc(a.data_ptr(), b.data_ptr(), 4, 64, 64, h, 3, iface.data_ptr(),
                                        l2.data_ptr(), st), "ac_judge_2d_noalloc")
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert lib.ac_judge_2d_noalloc(a.data_ptr(), b.data_ptr(), 16385, 64, 64, h, 3, iface.data_ptr(),
                                   l2.data_ptr(), st) == L.AC_ERR_INVALID_ARG
    assert b"16384" in lib.ac_last_error()
