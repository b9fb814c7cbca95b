"""Batched 3D stepping on the GPU: every instance of a persistent launch is
stepped exactly as ac_step_3d steps it (bit for bit), and in FP64 equals the
oracle; step counts that leave a shorter remainder phase and an odd number of
phases (a final copy phase) are covered, as is the 64-grid workload."""
import numpy as np
import pytest
import torch

import oracle
from oracle import diagnostics as D
from paper_2105_09671_amd import api, inputs, workloads
from paper_2105_09671_amd.params import dt_of, eps_m

pytestmark = pytest.mark.gpu

THREADS = min(32, max(1, oracle.cpus_available()))
NP = {torch.float32: np.float32, torch.float64: np.float64}


@pytest.fixture(params=[False, True], ids=["phase-graph", "persistent"])
def mode(request):
    api.batched_persistent(request.param)
    yield request.param
    api.batched_persistent(False)


def _small_batch():
    # (nz, ny, nx); in FP32 the grids at least 64 wide run on register tiles
    shapes = [(5, 1, 1), (9, 40, 7), (33, 33, 33), (20, 17, 61), (2, 70, 45), (40, 8, 3),
              (64, 64, 24), (1, 1, 30), (26, 29, 31), (12, 37, 70), (7, 50, 130), (35, 33, 64),
              (3, 1, 66)]
    fields, prm = [], []
    for i, (nz, ny, nx) in enumerate(shapes):
        h = 1.0 / max(8, min(nx, ny, nz))
        fields.append(inputs.random_field((nz, ny, nx), 300 + i, amp=0.6))
        prm.append((h, dt_of(h), eps_m(h, 3 + i % 4)))
    return fields, prm


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nsteps,tune", [(7, None), (9, None), (4, None), (1, None),
                                         (11, dict(tb_depth=3, tile_x=32, tile_y=16, tile_z=16)),
                                         (6, dict(tb_depth=2, tile_x=16, tile_y=16, tile_z=8)),
                                         (9, dict(kernel=2)), (10, dict(kernel=5, tb_depth=4))])
def test_batch3d_matches_single_and_oracle(mode, dtype, nsteps, tune):
    fields, prm = _small_batch()
    fields = [f.astype(NP[dtype]) for f in fields]
    b = api.Batch3D(fields, prm, dtype=dtype)
    info = b.step(nsteps, tune=tune)
    api.check()
    for v, f, (h, dt, eps) in zip(b.views(), fields, prm):
        single = torch.from_numpy(f).cuda()
        api.step3d(single, h, dt, eps, nsteps)
        assert torch.equal(v, single)
        if dtype == torch.float64:
            ref = oracle.step3d(f, h, dt, eps, nsteps, THREADS)
            assert D.rel_linf(v.cpu().numpy(), ref) <= 1e-12
    print(nsteps, tune, info)


def test_batch3d_replay_and_workload(mode):
    insts = workloads.batch3d_instances(64)
    fields = [g.initial().astype(np.float32) for g in insts]
    prm = [(g.h, g.dt, g.eps) for g in insts]
    b = api.Batch3D(fields, prm)
    b.step(250)
    b.step(250)                                    # replay of the cached graph
    api.check()
    for i in range(0, 64, 9):
        g = insts[i]
        single = torch.from_numpy(fields[i]).cuda()
        api.step3d(single, g.h, g.dt, g.eps, 500)
        assert torch.equal(b.views()[i], single), i
    # FP64 sample against the oracle
    sample = list(range(0, 64, 16))
    b64 = api.Batch3D([g.initial() for g in insts], prm, dtype=torch.float64)
    b64.step(200)
    for i in sample:
        g = insts[i]
        ref = oracle.step3d(g.initial(), g.h, g.dt, g.eps, 200, THREADS)
        assert D.rel_linf(b64.views()[i].cpu().numpy(), ref) <= 1e-12, i


def test_long_3d_call_runs_as_bounded_graphs():
    fields, prm = _small_batch()
    fields = [f.astype(np.float32) for f in fields[:3]]
    prm = prm[:3]
    n = 2048 * 4 + 5
    b = api.Batch3D(fields, prm)
    b.step(n)
    api.check()
    for v, f, (h, dt, eps) in zip(b.views(), fields, prm):
        one = torch.from_numpy(f).cuda()
        api.step3d(one, h, dt, eps, n)
        assert torch.equal(v, one)
