"""Precision trace (the paper's Err, Eq. ERReq, FP32 against FP64) on the GPU.

The fused kernel's FP64 path equals the FP64 oracle, its FP32 path equals the
FP32 product stepper bit for bit, and its per-step RMS equals the RMS of the
difference between those two, computed independently, at sampled steps.
The Table-3 analogue: Err of the FP32 path against FP64 on the paper's own
workloads stays within the largest error the paper reports for its FP32 GPU
code against its FP64 CPU code (Table 3: 3.36e-6); the ratios to the table's
entries are printed."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import diagnostics as D
from paper_2105_09671_amd import api, inputs, paper_suite
from paper_2105_09671_amd.params import dt_of, eps_m

pytestmark = pytest.mark.gpu

THREADS = min(32, max(1, oracle.cpus_available()))

TABLE3 = paper_suite.TABLE3   # Err of the paper's FP32 GPU code against its FP64 CPU code


def _rms(a, b):
    return math.sqrt(float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2)))


@pytest.mark.parametrize("shape,nsteps", [((50, 70), 301), ((12, 20, 17), 61)])
def test_trace_matches_product_and_oracle(shape, nsteps):
    n = shape[-1]
    h = 1.0 / n
    dt, eps = dt_of(h), eps_m(h, 3)
    p0 = inputs.random_field(shape, 77, amp=0.6).astype(np.float32)
    p32 = torch.from_numpy(p0).cuda()
    p64 = torch.from_numpy(p0.astype(np.float64)).cuda()
    rms, err = api.err_trace(p32, p64, h, dt, eps, nsteps)
    step = oracle.step2d if len(shape) == 2 else oracle.step3d
    prod = api.step2d if len(shape) == 2 else api.step3d
    # FP64 path = oracle; FP32 path = the product stepper, bit for bit
    assert D.rel_linf(p64.cpu().numpy(), step(p0.astype(np.float64), h, dt, eps, nsteps)) <= 1e-12
    q = torch.from_numpy(p0).cuda()
    prod(q, h, dt, eps, nsteps)
    assert torch.equal(p32, q)
    # per-step RMS at sampled steps against the independent difference
    r = rms.cpu().numpy()
    assert r.shape == (nsteps,)
    for t in (1, 2, 17, nsteps):
        q = torch.from_numpy(p0).cuda()
        prod(q, h, dt, eps, t)
        ref = _rms(q.cpu().numpy(), step(p0.astype(np.float64), h, dt, eps, t))
        assert abs(r[t - 1] - ref) <= 1e-9 * ref + 1e-15, (t, r[t - 1], ref)
    assert abs(err - float(np.mean(r))) <= 1e-12 * max(err, 1e-30)
    assert 0 < err < 1e-5


def test_zero_steps():
    p32 = torch.zeros(8, 8, device="cuda")
    p64 = torch.zeros(8, 8, dtype=torch.float64, device="cuda")
    rms, err = api.err_trace(p32, p64, 1 / 8, dt_of(1 / 8), eps_m(1 / 8, 4), 0)
    assert rms.numel() == 0 and err == 0.0


def test_table3_analogue():
    out = {}
    for name, ref in TABLE3.items():
        c = paper_suite.CASES[name]
        p0 = np.ascontiguousarray(c.initial()).astype(np.float32)
        p32 = torch.from_numpy(p0).cuda()
        p64 = torch.from_numpy(p0.astype(np.float64)).cuda()
        _, err = api.err_trace(p32, p64, c.h, c.dt, c.eps, c.steps)
        out[name] = err
        print("%-13s Err %.3g   paper %.3g   ratio %.2f" % (name, err, ref, err / ref))
        assert 0 < err <= 3.36e-6
