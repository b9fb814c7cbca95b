"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formula: each checks an independent fact
(fixed points, the maximum principle, energy decay, the closed-form linear
modes of the Neumann Laplacian, the stationary tanh profile, the mean-curvature
radius law, a dense-matrix brute force, symmetries), chosen so that a dropped
term, a wrong sign or index, or a transposed operand fails at least one.
"""
import math

import numpy as np
import pytest

from oracle import brute
from oracle import diagnostics as D
from paper_2105_09671_amd import inputs, params


def _par(n, m, dim=2):
    h = 1.0 / n
    dt = 0.1 * h * h
    import oracle
    return h, dt, oracle.eps_m(h, m)


def _step(oracle_mod, phi, h, dt, eps, n, threads=1):
    if phi.ndim == 2:
        return oracle_mod.step2d(phi, h, dt, eps, n, threads)
    return oracle_mod.step3d(phi, h, dt, eps, n, threads)


# ---------------------------------------------------------------- P7 brute ----
@pytest.mark.parametrize("shape", [(8, 8), (5, 7), (1, 9), (9, 1), (1, 1), (2, 3),
                                   (4, 4, 4), (2, 3, 4), (1, 1, 5), (1, 1, 1), (3, 1, 2)])
def test_brute_force_matches(oracle_mod, shape):
    """Oracle loops == explicit dense graph-Laplacian stepping (section 2.1 scheme,
    section 2 Neumann boundary), including degenerate 1xN and 1x1 grids."""
    h, dt, eps = 1.0 / 8, 0.1 / 64, oracle_mod.eps_m(1.0 / 8, 3)
    phi0 = inputs.random_field(shape, seed=11, amp=0.9)
    got = _step(oracle_mod, phi0, h, dt, eps, 25)
    ref = brute.step(phi0, h, dt, eps, 25)
    assert np.max(np.abs(got - ref)) <= 1e-14


def test_zero_steps_is_identity(oracle_mod):
    phi0 = inputs.random_field((6, 7), seed=2)
    assert np.array_equal(oracle_mod.step2d(phi0, 0.1, 0.001, 0.05, 0), phi0)


# ------------------------------------------------------------ P1 fixed pts ----
@pytest.mark.parametrize("value", [1.0, -1.0, 0.0])
@pytest.mark.parametrize("m", [3, 4, 8])
def test_constant_states_fixed_bitwise(oracle_mod, value, m):
    """+-1 (minima of F) and 0 (F'(0) = 0) are exact fixed points (section 1, F)."""
    h, dt, eps = _par(16, m)
    for shape in [(16, 12), (6, 5, 7)]:
        phi = np.full(shape, value)
        out = _step(oracle_mod, phi, h, dt, eps, 50)
        assert np.array_equal(out, phi)


# --------------------------------------------------------- P2 max principle ---
@pytest.mark.parametrize("shape", [(48, 40), (20, 18, 16)])
def test_max_principle(oracle_mod, shape):
    """|phi0| <= 1 keeps |phi^n| <= 1 when r <= 1/(2d) and alpha <= (1-2dr)/2;
    the worst configuration used here is m = 3 (alpha = 0.1927)."""
    n = shape[-1]
    h, dt, eps = _par(n, 3)
    alpha, r, d = dt / eps ** 2, dt / h ** 2, len(shape)
    assert r <= 1.0 / (2 * d) and alpha <= (1 - 2 * d * r) / 2
    phi = inputs.random_field(shape, seed=5, amp=1.0)
    for _ in range(10):
        phi = _step(oracle_mod, phi, h, dt, eps, 20)
        assert np.max(np.abs(phi)) <= 1.0 + 4 * np.finfo(np.float64).eps


# -------------------------------------------------------------- P3 energy -----
@pytest.mark.parametrize("shape,m", [((64, 64), 4), ((40, 56), 3), ((16, 16, 16), 4)])
def test_energy_non_increasing(oracle_mod, shape, m):
    """The scheme is explicit gradient descent on E_h (phi' = phi - dt h^-d grad E_h),
    so E_h does not increase while 2 alpha + 4 d r <= 2."""
    n = shape[-1]
    h, dt, eps = _par(n, m)
    phi = inputs.random_field(shape, seed=1)
    E = D.energy(phi, h, eps)
    for _ in range(60):
        phi = _step(oracle_mod, phi, h, dt, eps, 5)
        E2 = D.energy(phi, h, eps)
        assert E2 <= E * (1 + 1e-13)
        E = E2


def test_energy_gradient_matches_step(oracle_mod):
    """One step equals phi - dt h^-d grad E_h, grad E_h taken by central
    differences of the energy functional (no Laplacian code involved)."""
    h, dt, eps = _par(6, 4)
    phi = inputs.random_field((5, 6), seed=9, amp=0.8)
    g = np.zeros_like(phi)
    s = 1e-6
    for idx in np.ndindex(phi.shape):
        p, q = phi.copy(), phi.copy()
        p[idx] += s
        q[idx] -= s
        g[idx] = (D.energy(p, h, eps) - D.energy(q, h, eps)) / (2 * s)
    expect = phi - dt * g / h ** 2
    got = oracle_mod.step2d(phi, h, dt, eps, 1)
    assert np.max(np.abs(got - expect)) < 1e-9


# ------------------------------------------------------- P4 linear modes ------
@pytest.mark.parametrize("shape,kl", [((9, 6), (2, 1)), ((9, 6), (0, 5)), ((7, 10), (3, 3)),
                                      ((4, 5, 6), (1, 2, 3)), ((4, 5, 6), (3, 0, 1))])
def test_dct_modes_closed_form(oracle_mod, shape, kl):
    """DCT-II modes prod cos(pi k (i + 1/2)/N) are eigenvectors of the Neumann
    Laplacian with eigenvalue -(4/h^2) sum sin^2(pi k / 2N); a small multiple
    grows by (1 + alpha + dt lambda) per step up to O(delta^3)."""
    h, dt, eps = 1.0 / 10, 0.1 / 100, 0.05
    alpha = dt / eps ** 2
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    mode = np.ones(shape)
    lam = 0.0
    for ax, k in enumerate(kl):
        N = shape[ax]
        mode = mode * np.cos(np.pi * k * (grids[ax] + 0.5) / N)
        lam += -(4.0 / h ** 2) * np.sin(np.pi * k / (2 * N)) ** 2
    delta = 1e-8
    g = 1.0 + alpha + dt * lam
    for nsteps in (1, 7):
        out = _step(oracle_mod, delta * mode, h, dt, eps, nsteps)
        expect = delta * mode * g ** nsteps
        assert np.max(np.abs(out - expect)) <= 1e-12 * delta * max(1.0, abs(g) ** nsteps)


# -------------------------------------------------------- P5 tanh profile -----
def _front(n, m, ny=2):
    h = 1.0 / n
    eps = params.eps_m(h, m)
    x = inputs.centres(n, h)
    prof = np.tanh((x - 0.5) / (math.sqrt(2) * eps))
    return h, 0.1 * h * h, eps, np.tile(prof, (ny, 1))


def test_tanh_front_antisymmetric_bitwise(oracle_mod):
    """A planar front centred on a cell face stays exactly antisymmetric, so the
    zero crossing cannot drift (reflection symmetry of the 5-point stencil)."""
    h, dt, eps, phi = _front(256, 4)
    out = oracle_mod.step2d(phi, h, dt, eps, 400)
    assert np.array_equal(out[:, ::-1], -out)


def test_tanh_front_relaxes_to_stationary_profile(oracle_mod):
    """tanh(x/(sqrt2 eps)) solves eps^2 phi'' = phi^3 - phi exactly; the discrete
    front relaxes to a profile within O((h/eps)^2) of it and then stops."""
    devs = []
    for m in (4, 8, 16):
        h, dt, eps, phi = _front(256, m)
        out = oracle_mod.step2d(phi, h, dt, eps, 6000)
        nxt = oracle_mod.step2d(out, h, dt, eps, 1)
        assert np.max(np.abs(nxt - out)) <= 1e-13
        devs.append(np.max(np.abs(out - phi)))
    assert devs[0] / devs[1] > 3.0 and devs[1] / devs[2] > 3.0
    assert devs[2] < 5e-3


def test_tanh_front_3d(oracle_mod):
    h, dt, eps, row = _front(128, 4, ny=1)
    phi = np.broadcast_to(row[0], (2, 3, 128)).copy()
    out = oracle_mod.step3d(phi, h, dt, eps, 300)
    assert np.array_equal(out[..., ::-1], -out)
    out2 = oracle_mod.step2d(row.reshape(1, 128), h, dt, eps, 300)
    assert np.max(np.abs(out[1, 1] - out2[0])) <= 1e-15


# ------------------------------------------------------- P6 radius law --------
def _radius_run(oracle_mod, phi, h, dt, eps, chunks, per, threads):
    ts, R2 = [0.0], [D.volume_radius(phi, h) ** 2]
    for c in range(chunks):
        phi = _step(oracle_mod, phi, h, dt, eps, per, threads)
        ts.append((c + 1) * per * dt)
        R2.append(D.volume_radius(phi, h) ** 2)
    return np.array(ts), np.array(R2), phi


def test_circle_shrinks_by_mean_curvature(oracle_mod):
    """2D: R^2 = R0^2 - 2t (Eq. exactradiusEQ, d = 2); 256^2, R0 = 0.25, m = 4."""
    n, R0 = 256, 0.25
    h, dt, eps = _par(n, 4)
    phi = inputs.circle2d(n, n, h, eps, R0)
    ts, R2, _ = _radius_run(oracle_mod, phi, h, dt, eps, 10, 250, 4)
    R_end = math.sqrt(R2[-1])
    assert abs(R_end - D.radius_law(R0, ts[-1], 2)) <= h
    slope = np.polyfit(ts[2:], R2[2:], 1)[0]
    assert abs(slope - (-2.0)) <= 0.2


def test_sphere_shrinks_by_mean_curvature(oracle_mod):
    """3D: R^2 = R0^2 - 4t (Eq. exactradiusEQ, d = 3); 128^3, R0 = 0.3, m = 4."""
    n, R0 = 128, 0.3
    h, dt, eps = _par(n, 4)
    phi = inputs.sphere3d(n, n, n, h, eps, R0)
    threads = min(8, oracle_mod.cpus_available())
    ts, R2, _ = _radius_run(oracle_mod, phi, h, dt, eps, 5, 200, threads)
    assert abs(math.sqrt(R2[-1]) - D.radius_law(R0, ts[-1], 3)) <= h
    slope = np.polyfit(ts[1:], R2[1:], 1)[0]
    assert abs(slope - (-4.0)) <= 0.4


# ------------------------------------------------------------ P8 symmetry -----
def test_symmetries_2d(oracle_mod):
    h, dt, eps = _par(32, 4)
    phi = inputs.random_field((24, 32), seed=3, amp=0.6)
    out = oracle_mod.step2d(phi, h, dt, eps, 30)
    assert np.array_equal(oracle_mod.step2d(-phi, h, dt, eps, 30), -out)
    assert np.array_equal(oracle_mod.step2d(phi[:, ::-1], h, dt, eps, 30), out[:, ::-1])
    assert np.array_equal(oracle_mod.step2d(phi[::-1, :], h, dt, eps, 30), out[::-1, :])
    assert np.array_equal(oracle_mod.step2d(phi.T, h, dt, eps, 30), out.T)


def test_symmetries_3d(oracle_mod):
    h, dt, eps = _par(12, 4)
    phi = inputs.random_field((8, 10, 12), seed=4, amp=0.6)
    out = oracle_mod.step3d(phi, h, dt, eps, 20)
    assert np.array_equal(oracle_mod.step3d(-phi, h, dt, eps, 20), -out)
    for ax in range(3):
        flip = [slice(None)] * 3
        flip[ax] = slice(None, None, -1)
        f = tuple(flip)
        assert np.array_equal(oracle_mod.step3d(phi[f], h, dt, eps, 20), out[f])
    tr = np.transpose(phi, (2, 0, 1)).copy()
    got = oracle_mod.step3d(tr, h, dt, eps, 20)
    assert np.max(np.abs(got - np.transpose(out, (2, 0, 1)))) <= 1e-14


# --------------------------------------------------------- eps_m, batched -----
@pytest.mark.parametrize("m", [3, 4, 5, 10, 12])
def test_eps_m_spans_m_cells(oracle_mod, m):
    """Eq. emvalue: with eps_m the profile tanh(x/(sqrt2 eps)) goes from -0.9 to
    +0.9 across a width of m cells."""
    h = 1.0 / 200
    eps = oracle_mod.eps_m(h, m)
    assert math.isclose(math.tanh((m * h / 2) / (math.sqrt(2) * eps)), 0.9, rel_tol=1e-14)
    assert math.isclose(params.eps_m(h, m), eps, rel_tol=1e-15)


def test_batched_equals_independent_runs(oracle_mod):
    shapes = [(9, 13), (16, 16), (1, 7), (12, 5)]
    fields = [inputs.random_field(s, seed=20 + i) for i, s in enumerate(shapes)]
    hs = [1 / 13, 1 / 16, 1 / 7, 1 / 5]
    dts = [0.1 * h * h for h in hs]
    es = [oracle_mod.eps_m(h, m) for h, m in zip(hs, [3, 4, 5, 6])]
    outs = oracle_mod.step_batched2d(fields, hs, dts, es, 40, threads=3)
    for f, h, dt, e, o in zip(fields, hs, dts, es, outs):
        assert np.array_equal(o, oracle_mod.step2d(f, h, dt, e, 40))


def test_thread_count_does_not_change_result(oracle_mod):
    h, dt, eps = _par(40, 4)
    phi = inputs.random_field((40, 40), seed=8)
    a = oracle_mod.step2d(phi, h, dt, eps, 50, 1)
    b = oracle_mod.step2d(phi, h, dt, eps, 50, 4)
    assert np.array_equal(a, b)
    phi3 = inputs.random_field((10, 12, 14), seed=8)
    assert np.array_equal(oracle_mod.step3d(phi3, h, dt, eps, 10, 1),
                          oracle_mod.step3d(phi3, h, dt, eps, 10, 4))


def test_crop_locality(oracle_mod):
    """After n steps a cell depends only on cells within n of it (one cell per
    step along each axis): running on a crop that extends a window by n cells
    gives the window exactly.  The full-size GPU checks rely on this."""
    n = 7
    p2 = inputs.random_field((40, 44), seed=21, amp=0.6)
    full = oracle_mod.step2d(p2, 1 / 44, 0.1 / 44 ** 2, params.eps_m(1 / 44, 3), n)
    crop = oracle_mod.step2d(np.ascontiguousarray(p2[3:32, 10:30]), 1 / 44, 0.1 / 44 ** 2,
                             params.eps_m(1 / 44, 3), n)
    assert np.array_equal(full[10:25, 17:23], crop[7:22, 7:13])
    # one cell fewer of margin is not enough
    crop1 = oracle_mod.step2d(np.ascontiguousarray(p2[4:31, 11:29]), 1 / 44, 0.1 / 44 ** 2,
                              params.eps_m(1 / 44, 3), n)
    assert not np.array_equal(full[10:25, 17:23], crop1[6:21, 6:12])
    p3 = inputs.random_field((20, 21, 22), seed=22, amp=0.6)
    h = 1 / 22
    full3 = oracle_mod.step3d(p3, h, 0.1 * h * h, params.eps_m(h, 3), n)
    crop3 = oracle_mod.step3d(np.ascontiguousarray(p3[0:15, 5:20, 8:22]), h, 0.1 * h * h,
                              params.eps_m(h, 3), n)
    assert np.array_equal(full3[0:8, 12:13, 15:22], crop3[0:8, 7:8, 7:14])


# ----------------------------------------------------------------------------
# Interface diagnostics (the reading of "interface error": zero crossings on
# the edges between cell centres, located by linear interpolation; the error
# is the symmetric Hausdorff distance between the two crossing sets).  Pinned
# to geometry, not to the code's own formulas.

def _centres(n, h):
    return (np.arange(n) + 0.5) * h


@pytest.mark.parametrize("x0", [0.3141, 0.5, 0.515625, 0.7773])
def test_crossings_of_linear_field_are_exact(x0):
    """Linear interpolation is exact on a linear field: phi = x - x0 crosses
    zero at x = x0 on every row (one crossing per row, on a horizontal edge,
    none on vertical ones); phi = y - y0 likewise on every column.  A wrong
    interpolation weight or a half-cell offset on either axis moves these
    points.  x0 = 0.515625 sits exactly on a cell centre (phi = 0 there): the
    crossing is that centre."""
    nx, ny, h = 64, 40, 1 / 64
    X, Y = np.meshgrid(_centres(nx, h), _centres(ny, h))       # shape (ny, nx)
    p = D.crossings(X - x0, h)
    assert p.shape == (ny, 2)
    assert np.max(np.abs(p[:, 0] - x0)) <= 1e-14
    assert np.max(np.abs(np.sort(p[:, 1]) - _centres(ny, h))) <= 1e-14
    y0 = x0 * 40 / 64 + 0.1
    Xt, Yt = np.meshgrid(_centres(ny, h), _centres(nx, h))     # shape (nx, ny): 64 rows
    q = D.crossings(Yt - y0, h)
    assert q.shape == (ny, 2)
    assert np.max(np.abs(q[:, 1] - y0)) <= 1e-14
    assert np.max(np.abs(np.sort(q[:, 0]) - _centres(ny, h))) <= 1e-14


def test_crossings_of_oblique_linear_field_lie_on_the_line():
    """phi = (x - x0) + 2 (y - y0): every crossing, on horizontal and vertical
    edges alike, lies exactly on the line, and there is one per sign-changing
    edge."""
    n, h, x0, y0 = 48, 1 / 48, 0.41, 0.57
    X, Y = np.meshgrid(_centres(n, h), _centres(n, h))
    phi = (X - x0) + 2 * (Y - y0)
    p = D.crossings(phi, h)
    edges = int(np.sum((phi[:, :-1] > 0) != (phi[:, 1:] > 0)) + np.sum((phi[:-1] > 0) != (phi[1:] > 0)))
    assert len(p) == edges and edges > n
    assert np.max(np.abs((p[:, 0] - x0) + 2 * (p[:, 1] - y0))) <= 1e-14


def test_interface_error_of_parallel_fronts():
    """Two straight fronts x = x0 and x = x1 on the same rows: every crossing of
    one has its nearest crossing of the other on its own row, |x1 - x0| away."""
    n, h = 64, 1 / 64
    X, _ = np.meshgrid(_centres(n, h), _centres(n, h))
    for x0, x1 in ((0.3, 0.3 + 0.37 / 64), (0.25, 0.61), (0.5, 0.5)):
        assert abs(D.interface_error(X - x0, X - x1, h) - abs(x1 - x0)) <= 1e-15


@pytest.mark.parametrize("s", [1, 2, 5])
def test_interface_error_of_front_shifted_by_whole_cells(s):
    """A tanh front and the same front moved by s whole cells: the sampled
    values are the same numbers s cells over, so every crossing moves by
    exactly s h and the distance is s h."""
    n, h = 96, 1 / 96
    eps = params.eps_m(h, 4)
    X, _ = np.meshgrid(_centres(n, h), _centres(n, h))
    a = np.tanh((X - 0.4) / (math.sqrt(2) * eps))
    b = np.tanh((X - 0.4 - s * h) / (math.sqrt(2) * eps))
    assert abs(D.interface_error(a, b, h) - s * h) <= 1e-13


@pytest.mark.parametrize("n,R", [(128, 0.25), (256, 0.3)])
def test_interface_error_of_concentric_circles(n, R):
    """Crossings of a sampled circle lie on the circle to O(h^2) (the
    interpolation error of a smooth front: measured below 1.3 h^2 / R for
    these tanh profiles, bound 2 h^2 / R).  For circles R and R + d the two
    crossing sets are discrete: a crossing of one circle is at least d - 2h^2/R
    from every crossing of the other, and within sqrt(d^2 + h^2/2) + 2h^2/R of
    one (consecutive crossings along a front lie on the boundary of one cell,
    at most sqrt(2) h apart, so the nearest is at most h/sqrt(2) along the front
    from the foot of the normal)."""
    h = 1 / n
    eps = params.eps_m(h, 4)
    X, Y = np.meshgrid(_centres(n, h), _centres(n, h))
    r = np.hypot(X - 0.5, Y - 0.5)
    f = lambda RR: np.tanh((RR - r) / (math.sqrt(2) * eps))
    p = D.crossings(f(R), h)
    slack = 2 * h * h / R
    assert np.max(np.abs(np.hypot(p[:, 0] - 0.5, p[:, 1] - 0.5) - R)) <= slack
    for d in (0.37 * h, 1.5 * h, 3.0 * h):
        e = D.interface_error(f(R), f(R + d), h)
        assert d - slack <= e <= math.sqrt(d * d + h * h / 2) + slack, (d / h, e / h)


def test_hausdorff_against_brute_force():
    """cKDTree queries against the full distance matrix (max of row minima and
    of column minima) on random sets, including one set inside the other,
    where the two directed distances differ."""
    rng = np.random.RandomState(3)
    for na, nb in ((7, 11), (30, 5), (1, 1)):
        A, B = rng.rand(na, 2), rng.rand(nb, 2)
        M = np.sqrt(((A[:, None, :] - B[None, :, :]) ** 2).sum(-1))
        assert abs(D.hausdorff(A, B) - max(M.min(1).max(), M.min(0).max())) <= 1e-15
    A = rng.rand(6, 2)
    B = np.concatenate([A, [[5.0, 5.0]]])
    far = np.min(np.hypot(A[:, 0] - 5.0, A[:, 1] - 5.0))
    assert abs(D.hausdorff(A, B) - far) <= 1e-15 and abs(D.hausdorff(B, A) - far) <= 1e-15


def test_interface_error_empty_cases():
    n, h = 16, 1 / 16
    pos = np.ones((n, n))
    X, _ = np.meshgrid(_centres(n, h), _centres(n, h))
    assert D.interface_error(pos, 0.5 * pos, h) == 0.0
    assert math.isinf(D.interface_error(pos, X - 0.5, h))
    assert math.isinf(D.interface_error(X - 0.5, -pos, h))


def test_err_metric_closed_forms():
    """Eq. ERReq's Err is the time average of the per-snapshot RMS difference.
    A constant difference c_t has RMS |c_t|; a checkerboard of +-a has RMS a.
    Differences 1 and 3 average to 2 (an RMS over time would give sqrt(5), a
    sum 4)."""
    a = [np.zeros((5, 7)), np.zeros((5, 7))]
    assert D.err_metric(a, [x + 1.0 for x in a[:1]] + [a[1] - 3.0]) == 2.0
    chk = np.where((np.add.outer(np.arange(6), np.arange(8)) % 2) == 0, 0.25, -0.25)
    assert D.err_metric([np.zeros((6, 8))], [chk]) == 0.25
    assert D.err_metric(a, a) == 0.0
