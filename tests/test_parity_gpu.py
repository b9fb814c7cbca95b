"""GPU parity: libac (through the C ABI) against the FP64 CPU oracle.

Bars: FP64 rel L_inf <= 1e-12; FP32 rel L_inf <= 1e-5 against the FP64 oracle
started from the same FP32-rounded initial state.  Temporal-blocking depths
and tile shapes must agree bitwise with each other (every cell is always
updated by the same expression from the same neighbour values).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import diagnostics as D
from paper_2105_09671_amd import inputs, params, workloads

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
NP = {torch.float64: np.float64, torch.float32: np.float32}


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2105_09671_amd import api as a
    return a


def _run2d(api, phi0, h, dt, eps, n, dtype, tune=None):
    t = torch.from_numpy(np.ascontiguousarray(phi0, dtype=NP[dtype])).cuda()
    api.step2d(t, h, dt, eps, n, tune=tune)
    api.check()
    return t.cpu().numpy()


def _run3d(api, phi0, h, dt, eps, n, dtype, tune=None):
    t = torch.from_numpy(np.ascontiguousarray(phi0, dtype=NP[dtype])).cuda()
    api.step3d(t, h, dt, eps, n, tune=tune)
    api.check()
    return t.cpu().numpy()


def _par(n, m):
    h = 1.0 / n
    return h, params.dt_of(h), params.eps_m(h, m)


# ------------------------------------------------------------------- 2D ----
def test_phase64_fp64_resident(api):
    """64x64 FP64 random start, 500 steps: the whole grid as one register tile,
    all steps in one launch."""
    p = api.plan2d(64, 64, 500, torch.float64)
    assert p["kernel"] == 4 and p["tb_depth"] == 0 and p["launches"] == 1, p
    g = workloads.phase64()
    phi0 = g.initial()
    got = _run2d(api, phi0, g.h, g.dt, g.eps, 500, torch.float64)
    ref = oracle.step2d(phi0, g.h, g.dt, g.eps, 500)
    assert D.rel_linf(got, ref) <= 1e-12


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_2d_tiled_all_depths(api, dtype):
    """300x211 grid (ragged against every tile), 37 steps, depths 1..8."""
    h, dt, eps = _par(256, 4)
    phi0 = inputs.random_field((211, 300), seed=21).astype(NP[dtype])
    ref = oracle.step2d(phi0.astype(np.float64), h, dt, eps, 37)
    outs = {}
    for k in range(1, 9):
        outs[k] = _run2d(api, phi0, h, dt, eps, 37, dtype, tune=dict(tb_depth=k, tile_x=-1))
        assert D.rel_linf(outs[k], ref) <= TOL[dtype], "depth %d" % k
    for k in range(2, 9):
        assert np.array_equal(outs[k], outs[1]), "depth %d differs bitwise from depth 1" % k


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_2d_tile_shapes_bitwise(api, dtype):
    h, dt, eps = _par(128, 5)
    phi0 = inputs.random_field((150, 170), seed=22).astype(NP[dtype])
    base = _run2d(api, phi0, h, dt, eps, 20, dtype, tune=dict(tb_depth=1, tile_x=-1))
    # kernel 0: the plan's choice; 4: registers, 6: registers two columns per
    # lane, 3: in place in LDS, 1: two LDS buffers
    for tx, ty, k, kern in [(64, 64, 4, 0), (128, 32, 3, 0), (256, 16, 2, 0), (96, 40, 8, 0),
                            (64, 17, 8, 0), (64, 16, 7, 4), (64, 48, 5, 4), (64, 256, 8, 4),
                            (64, 128, 1, 4), (128, 64, 7, 6), (128, 8, 1, 6), (128, 24, 3, 6),
                            (128, 128, 8, 6), (64, 64, 4, 3), (64, 64, 4, 1)]:
        tune = dict(tb_depth=k, tile_x=tx, tile_y=ty, kernel=kern)
        if kern:
            assert api.plan2d(170, 150, 20, dtype, tune)["kernel"] == kern
        got = _run2d(api, phi0, h, dt, eps, 20, dtype, tune=tune)
        assert np.array_equal(got, base), (tx, ty, k, kern)
    res = _run2d(api, phi0, h, dt, eps, 20, dtype)       # LDS-resident path
    assert np.array_equal(res, base)


@pytest.mark.parametrize("shape", [(1, 1), (1, 50), (50, 1), (3, 200), (200, 3), (65, 63),
                                   (1, 129), (130, 2)])
@pytest.mark.parametrize("nsteps", [0, 1, 2, 5])
def test_2d_edge_shapes(api, shape, nsteps):
    h, dt, eps = _par(64, 4)
    phi0 = inputs.random_field(shape, seed=23, amp=0.8)
    ref = oracle.step2d(phi0, h, dt, eps, nsteps)
    for tune in (None, dict(tb_depth=3, tile_x=-1)):
        got = _run2d(api, phi0, h, dt, eps, nsteps, torch.float64, tune=tune)
        assert D.rel_linf(got, ref) <= 1e-12, tune


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_2d_register_tiling_sizes(api, dtype):
    """Register tiles sit flush against the domain edges: the first tile starts
    at 0, the last ends at n, the ones between step by L - 2K.  Sizes around
    every change of the tile count (depth 7, 64 x 32 tiles: 50 x 18 outputs),
    with 19 steps so the last launch is shorter: bitwise the two-buffer LDS
    kernel (uniform tiling) and the oracle."""
    h, dt, eps = _par(64, 4)
    for ny, nx in [(32, 64), (33, 65), (31, 63), (50, 114), (51, 115), (64, 128), (46, 164),
                   (47, 165), (32, 200), (200, 64), (18, 70), (100, 1)]:
        phi0 = inputs.random_field((ny, nx), seed=35 + nx + ny, amp=0.9).astype(NP[dtype])
        ref = oracle.step2d(phi0.astype(np.float64), h, dt, eps, 19)
        reg = _run2d(api, phi0, h, dt, eps, 19, dtype,
                     tune=dict(tb_depth=7, tile_x=64, tile_y=32, kernel=4))
        lds = _run2d(api, phi0, h, dt, eps, 19, dtype,
                     tune=dict(tb_depth=7, tile_x=64, tile_y=32, kernel=1))
        assert np.array_equal(reg, lds), (ny, nx)
        assert D.rel_linf(reg, ref) <= TOL[dtype], (ny, nx)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_2d_wide_register_tiling_sizes(api, dtype):
    """128-wide register tiles (two adjacent columns per lane) sit flush against
    the domain edges like the 64-wide ones.  Widths around every change of the
    tile count (depth 7: 114 output columns per middle tile), odd widths (rows
    then move one value at a time instead of pairs), heights below one tile
    and the single-tile width 128; 19 steps so the last launch is shorter:
    bitwise the 64-wide register kernel, and the oracle."""
    h, dt, eps = _par(64, 4)
    for ny, nx in [(32, 128), (33, 129), (31, 241), (50, 242), (51, 243), (64, 300), (17, 301),
                   (8, 356), (100, 357), (200, 130)]:
        phi0 = inputs.random_field((ny, nx), seed=41 + nx + ny, amp=0.9).astype(NP[dtype])
        ref = oracle.step2d(phi0.astype(np.float64), h, dt, eps, 19)
        wide = _run2d(api, phi0, h, dt, eps, 19, dtype,
                      tune=dict(tb_depth=7, tile_x=128, tile_y=32, kernel=6))
        narrow = _run2d(api, phi0, h, dt, eps, 19, dtype,
                        tune=dict(tb_depth=7, tile_x=64, tile_y=32, kernel=4))
        assert np.array_equal(wide, narrow), (ny, nx)
        assert D.rel_linf(wide, ref) <= TOL[dtype], (ny, nx)
    # one wave per tile up to sixteen, depth 1 to 8
    phi0 = inputs.random_field((90, 250), seed=43, amp=0.9).astype(NP[dtype])
    narrow = _run2d(api, phi0, h, dt, eps, 17, dtype, tune=dict(tb_depth=1, tile_x=-1))
    for k, ly in [(1, 8), (3, 16), (5, 40), (8, 128)]:
        wide = _run2d(api, phi0, h, dt, eps, 17, dtype,
                      tune=dict(tb_depth=k, tile_x=128, tile_y=ly, kernel=6))
        assert np.array_equal(wide, narrow), (k, ly)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_2d_whole_grid_register_tile(api, dtype):
    """Grids up to 64 wide and 256 tall run as one register tile with every
    step in one launch: the oracle, and bitwise the forced tiled plan."""
    h, dt, eps = _par(64, 4)
    for ny, nx in [(64, 64), (1, 1), (37, 50), (256, 64), (200, 3), (17, 64), (16, 1)]:
        phi0 = inputs.random_field((ny, nx), seed=37 + nx + ny, amp=0.9).astype(NP[dtype])
        for n in (1, 2, 33):
            assert api.plan2d(nx, ny, n, dtype)["tb_depth"] == 0
            got = _run2d(api, phi0, h, dt, eps, n, dtype)
            ref = oracle.step2d(phi0.astype(np.float64), h, dt, eps, n)
            assert D.rel_linf(got, ref) <= TOL[dtype], (ny, nx, n)
            tiled = _run2d(api, phi0, h, dt, eps, n, dtype, tune=dict(tb_depth=3, tile_x=-1))
            assert np.array_equal(got, tiled), (ny, nx, n)


def test_2d_plan_kernels(api):
    from paper_2105_09671_amd import _lib as L
    # large grids default to a register kernel: 64 wide (16 rows per wave) or
    # 128 wide (two columns per lane, 8 rows per wave), whichever the measured
    # rates predict faster; the streaming regime of 16384^2 FP32 takes 128
    for dt_ in (torch.float32, torch.float64):
        p = api.plan2d(2048, 2048, 100, dt_)
        assert p["kernel"] in (4, 6), p
        rows = 16 if p["kernel"] == 4 else 8
        assert p["tile_x"] == (64 if p["kernel"] == 4 else 128) and p["tile_y"] % rows == 0, p
        assert p["threads"] == 64 * p["tile_y"] // rows
    assert api.plan2d(16384, 16384, 100, torch.float32)["kernel"] == 6
    assert api.plan2d(127, 2048, 100, torch.float32)["kernel"] == 4
    # grids up to 64 x 256: one register tile, all steps in one launch; wider
    # small grids: one LDS-resident workgroup
    assert api.plan2d(64, 256, 10, torch.float32)["tb_depth"] == 0
    assert api.plan2d(64, 257, 10, torch.float32)["kernel"] != 4 or \
        api.plan2d(64, 257, 10, torch.float32)["tb_depth"] > 0
    assert api.plan2d(100, 60, 10, torch.float32)["kernel"] == 0
    assert api.plan2d(50, 50, 10, torch.float32, dict(tb_depth=3))["kernel"] == 0
    # 64-wide tiles whose height is not whole 16-row waves fall back to LDS
    assert api.plan2d(2048, 2048, 100, torch.float32, dict(tb_depth=4, tile_y=40))["kernel"] == 3
    with pytest.raises(L.AcError):
        api.plan2d(2048, 2048, 100, torch.float32, dict(tb_depth=4, tile_y=40, kernel=4))
    with pytest.raises(L.AcError):
        api.plan2d(2048, 2048, 100, torch.float32, dict(tb_depth=4, tile_x=128, kernel=4))
    with pytest.raises(L.AcError):
        api.plan2d(2048, 2048, 100, torch.float32, dict(kernel=2))
    # 128-wide register tiles: whole 8-row waves, grids at least 128 wide
    p = api.plan2d(300, 200, 100, torch.float32, dict(kernel=6, tb_depth=5, tile_y=40))
    assert p["kernel"] == 6 and p["tile_x"] == 128 and p["threads"] == 64 * 5, p
    for bad in (dict(kernel=6, tb_depth=4, tile_y=36), dict(kernel=6, tb_depth=4, tile_y=136),
                dict(kernel=6, tb_depth=4, tile_x=64)):
        with pytest.raises(L.AcError):
            api.plan2d(300, 200, 100, torch.float32, bad)
    with pytest.raises(L.AcError):
        api.plan2d(127, 200, 100, torch.float32, dict(kernel=6))


def test_2d_split_equals_single_call(api):
    h, dt, eps = _par(200, 4)
    phi0 = inputs.random_field((200, 200), seed=24).astype(np.float32)
    tune = dict(tb_depth=4, tile_x=-1)
    once = _run2d(api, phi0, h, dt, eps, 50, torch.float32, tune)
    a = _run2d(api, phi0, h, dt, eps, 21, torch.float32, tune)
    both = _run2d(api, a, h, dt, eps, 29, torch.float32, tune)
    assert np.array_equal(once, both)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_2d_invariants(api, dtype):
    h, dt, eps = _par(160, 3)            # m = 3: the largest alpha accepted
    for tune in (dict(tb_depth=5, tile_x=-1), dict(tb_depth=5, tile_x=128, tile_y=64, kernel=6)):
        for v in (1.0, -1.0, 0.0):
            c = np.full((170, 140), v, dtype=NP[dtype])
            assert np.array_equal(_run2d(api, c, h, dt, eps, 30, dtype, tune), c)
        phi0 = inputs.random_field((170, 140), seed=25, amp=1.0).astype(NP[dtype])
        out = _run2d(api, phi0, h, dt, eps, 60, dtype, tune)
        assert np.max(np.abs(out)) <= 1.0 + 4 * np.finfo(NP[dtype]).eps
        assert np.array_equal(_run2d(api, -phi0, h, dt, eps, 60, dtype, tune), -out)
        assert np.array_equal(_run2d(api, phi0[:, ::-1], h, dt, eps, 60, dtype, tune), out[:, ::-1])
        assert np.array_equal(_run2d(api, phi0[::-1], h, dt, eps, 60, dtype, tune), out[::-1])
        assert np.array_equal(_run2d(api, phi0.T, h, dt, eps, 60, dtype, tune), out.T)


def test_2d_energy_decreases(api):
    h, dt, eps = _par(256, 4)
    phi = inputs.random_field((256, 256), seed=26)
    E = D.energy(phi, h, eps)
    t = torch.from_numpy(phi).cuda()
    for _ in range(20):
        api.step2d(t, h, dt, eps, 25)
        E2 = D.energy(t.cpu().numpy(), h, eps)
        assert E2 <= E * (1 + 1e-13)
        E = E2


# ------------------------------------------------------------------- 3D ----
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_3d_all_depths(api, dtype):
    """37x29x23 grid, z segments of 8 planes, 13 steps, depths 1..8."""
    h, dt, eps = _par(64, 4)
    phi0 = inputs.random_field((23, 29, 37), seed=31).astype(NP[dtype])
    ref = oracle.step3d(phi0.astype(np.float64), h, dt, eps, 13)
    outs = {}
    for k in range(1, 9):
        lx = 2 * k + 16
        outs[k] = _run3d(api, phi0, h, dt, eps, 13, dtype,
                         tune=dict(tb_depth=k, tile_x=lx, tile_y=2 * k + 9, tile_z=8))
        assert D.rel_linf(outs[k], ref) <= TOL[dtype], "depth %d" % k
    for k in range(2, 9):
        assert np.array_equal(outs[k], outs[1]), "depth %d differs bitwise" % k
    default = _run3d(api, phi0, h, dt, eps, 13, dtype)
    assert np.array_equal(default, outs[1])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_3d_register_kernel(api, dtype):
    """The register-resident 3D kernel (64-wide tiles, 4 rows per wave) at depths
    1..8 (FP64 1..6) and 1..8 waves, on a grid ragged against every tile and z
    segment: bitwise the LDS kernel, and the oracle to the usual bar."""
    h, dt, eps = _par(64, 4)
    phi0 = inputs.random_field((37, 45, 70), seed=34).astype(NP[dtype])
    ref = oracle.step3d(phi0.astype(np.float64), h, dt, eps, 13)
    base = _run3d(api, phi0, h, dt, eps, 13, dtype,
                  tune=dict(tb_depth=2, tile_x=24, tile_y=24, tile_z=8, kernel=2))
    assert D.rel_linf(base, ref) <= TOL[dtype]
    cases = [(1, 4, 5), (2, 16, 8), (3, 8, 16), (4, 32, 8), (4, 12, 64), (3, 32, 37), (5, 32, 8),
             (6, 16, 12)]
    if dtype == torch.float32:
        cases += [(7, 32, 20), (8, 20, 9), (8, 32, 64)]
    for k, ly, lz in cases:
        tune = dict(tb_depth=k, tile_x=64, tile_y=ly, tile_z=lz, kernel=5)
        p = api.plan3d(70, 45, 37, 13, dtype, tune)
        assert p["kernel"] == 5 and p["threads"] == 64 * ly // 4, p
        got = _run3d(api, phi0, h, dt, eps, 13, dtype, tune=tune)
        assert np.array_equal(got, base), (k, ly, lz)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_3d_register_tiling_sizes(api, dtype):
    """3D register tiles sit flush against the x and y domain edges like the 2D
    ones.  Depth 3, 64 x 16 tiles (58 x 10 outputs), z segments of 4 planes,
    sizes around the tile-count thresholds, 7 steps (a shorter last launch):
    bitwise the LDS kernel and the oracle."""
    h, dt, eps = _par(48, 4)
    for nz, ny, nx in [(5, 16, 64), (6, 17, 65), (4, 15, 63), (5, 22, 122), (3, 23, 123),
                       (7, 9, 70), (9, 1, 100), (2, 60, 1), (5, 26, 131)]:
        phi0 = inputs.random_field((nz, ny, nx), seed=36 + nx + ny + nz, amp=0.9).astype(NP[dtype])
        ref = oracle.step3d(phi0.astype(np.float64), h, dt, eps, 7)
        reg = _run3d(api, phi0, h, dt, eps, 7, dtype,
                     tune=dict(tb_depth=3, tile_x=64, tile_y=16, tile_z=4, kernel=5))
        lds = _run3d(api, phi0, h, dt, eps, 7, dtype,
                     tune=dict(tb_depth=3, tile_x=16, tile_y=16, tile_z=4, kernel=2))
        assert np.array_equal(reg, lds), (nz, ny, nx)
        assert D.rel_linf(reg, ref) <= TOL[dtype], (nz, ny, nx)


def test_3d_plan_kernels(api):
    from paper_2105_09671_amd import _lib as L
    # large grids run on register tiles, grids of too few 64-wide tiles on LDS
    for dt_ in (torch.float32, torch.float64):
        assert api.plan3d(1024, 1024, 1024, 100, dt_)["kernel"] == 5
        assert api.plan3d(96, 96, 96, 100, dt_)["kernel"] == 2
        assert api.plan3d(96, 96, 96, 100, dt_, dict(kernel=5))["kernel"] == 5
        assert api.plan3d(1024, 1024, 1024, 100, dt_, dict(kernel=2))["kernel"] == 2
    for bad in (dict(kernel=5, tb_depth=9), dict(kernel=5, tile_x=32), dict(kernel=5, tile_y=36),
                dict(kernel=5, tile_y=30), dict(kernel=4)):
        with pytest.raises(L.AcError):
            api.plan3d(256, 256, 256, 100, torch.float32, bad)
    # register depth limits: FP32 8, FP64 6
    assert api.plan3d(256, 256, 256, 100, torch.float32, dict(kernel=5, tb_depth=8))["tb_depth"] == 8
    assert api.plan3d(256, 256, 256, 100, torch.float64, dict(kernel=5, tb_depth=6))["tb_depth"] == 6
    with pytest.raises(L.AcError):
        api.plan3d(256, 256, 256, 100, torch.float64, dict(kernel=5, tb_depth=7))


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 9), (9, 1, 1), (1, 7, 1), (2, 3, 4),
                                   (5, 70, 3), (40, 2, 66)])
@pytest.mark.parametrize("nsteps", [1, 4])
def test_3d_edge_shapes(api, shape, nsteps):
    h, dt, eps = _par(32, 4)
    phi0 = inputs.random_field(shape, seed=32, amp=0.8)
    ref = oracle.step3d(phi0, h, dt, eps, nsteps)
    for tune in (None, dict(tb_depth=2, tile_x=12, tile_y=12, tile_z=2),
                 dict(tb_depth=3, tile_x=64, tile_y=8, tile_z=2, kernel=5)):
        got = _run3d(api, phi0, h, dt, eps, nsteps, torch.float64, tune)
        assert D.rel_linf(got, ref) <= 1e-12, tune


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_3d_invariants(api, dtype):
    h, dt, eps = _par(48, 3)
    tune = dict(tb_depth=3, tile_x=24, tile_y=20, tile_z=16)
    reg = dict(tb_depth=3, tile_x=64, tile_y=16, tile_z=16, kernel=5)
    for v in (1.0, -1.0, 0.0):
        c = np.full((20, 30, 40), v, dtype=NP[dtype])
        assert np.array_equal(_run3d(api, c, h, dt, eps, 9, dtype, reg), c)
        assert np.array_equal(_run3d(api, c, h, dt, eps, 9, dtype, tune), c)
    phi0 = inputs.random_field((20, 30, 40), seed=33, amp=1.0).astype(NP[dtype])
    out = _run3d(api, phi0, h, dt, eps, 12, dtype, tune)
    assert np.max(np.abs(out)) <= 1.0 + 4 * np.finfo(NP[dtype]).eps
    assert np.array_equal(_run3d(api, -phi0, h, dt, eps, 12, dtype, tune), -out)
    for ax in range(3):
        f = [slice(None)] * 3
        f[ax] = slice(None, None, -1)
        f = tuple(f)
        assert np.array_equal(_run3d(api, phi0[f], h, dt, eps, 12, dtype, tune), out[f])
    assert np.array_equal(_run3d(api, phi0, h, dt, eps, 12, dtype, reg), out)


def test_api_rejects_cpu_tensor(api):
    with pytest.raises(TypeError):
        api.step2d(torch.zeros(4, 4), 0.1, 0.001, 0.1, 1)
