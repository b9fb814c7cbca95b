"""The paper's own workloads (section 3): its grids, interface widths and the
step counts of Tables 1-2, each with a coarse check of what the paper says
the run shows.

2D: 200^2 on the unit square, eps_10, dt = 0.1 h^2 (section 3.2); the
dumbbell on (0,2) x (0,1) with 400 x 200 cells.  3D: 100^3 on the unit cube,
eps_12 (section 3.3); the dumbbell on (0,2) x (0,1)^2 with 200 x 100 x 100.
Step counts are the tables' iteration counts minus one (they count the
initial state).  Readings where the paper is silent or inconsistent:

* circle / sphere radius R0: not stated; 0.3 (2D) and 0.4 (3D).
* 2D dumbbell: 15000 steps reach the stated T = 0.0094 only with
  dt = 0.1 / 400^2 (h taken as 1/Nx for the time step) while the shape lives
  on (0,2) x (0,1) (h = 1/200 for space); that is the reading here.
* 3D dumbbell: neither the stated T = 0.0025 nor the table's 2000 steps
  shows the figure's state (handle pinched off, end spheres still there);
  1000 steps with dt = 0.1 h^2 (T = 0.01) does.
* the maze (its code is in a missing appendix) and the 3D star and torus
  (garbled formulas) are left out.

The checks read the fields with plain measurements defined here: the radius
of the disc/ball with the phase volume, the zero crossing along a ray from
the centre, the fraction of separated cells.

    python -m paper_2105_09671_amd.paper_suite      # GPU times at the tables' counts
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field
from typing import Callable

import numpy as np
import torch

from . import api, inputs
from .params import eps_m, radius_law


def volume_radius(phi: np.ndarray, h: float) -> float:
    d = phi.ndim
    V = h ** d * float(np.sum(0.5 * (1.0 + phi.astype(np.float64))))
    return math.sqrt(V / math.pi) if d == 2 else (V / (4.0 / 3.0 * math.pi)) ** (1.0 / 3.0)


def ray_crossing(phi: np.ndarray, h: float, angle: float, centre=(0.5, 0.5)) -> float:
    """Distance from the centre to the first sign change of a 2D field along
    the ray at `angle` (nearest-cell sampling every h/4)."""
    ny, nx = phi.shape
    for k in range(1, int(0.5 / h * 4)):
        r = k * h / 4
        i = int(round((centre[0] + r * math.cos(angle)) / h - 0.5))
        j = int(round((centre[1] + r * math.sin(angle)) / h - 0.5))
        if not (0 <= i < nx and 0 <= j < ny) or phi[j, i] < 0:
            return r
    return 0.5


def separated(phi: np.ndarray) -> float:
    return float(np.mean(np.abs(phi) > 0.9))


def dumbbell3d(nx, ny, nz, h, eps, R0=0.25) -> np.ndarray:
    """Eq. 3Ddumbellini on (0, nx h) x (0, ny h) x (0, nz h)."""
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    z = (np.arange(nz) + 0.5) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    YZ = (Y - 0.5) ** 2 + (Z - 0.5) ** 2
    s2e = math.sqrt(2.0) * eps
    phi = (1.0 + np.tanh((R0 - np.sqrt((X - 0.3) ** 2 + YZ)) / s2e)
           + np.tanh((R0 - np.sqrt((X - 1.7) ** 2 + YZ)) / s2e))
    bar = (X > 0.4) & (X < 1.6) & (Y > 0.4) & (Y < 0.6) & (Z > 0.4) & (Z < 0.6)
    phi[bar] = 1.0
    return phi


@dataclass
class Case:
    name: str
    shape: tuple            # (ny, nx) or (nz, ny, nx)
    h: float
    dt: float
    m: int
    steps: int              # table iterations - 1 (or the reading above)
    table_steps: int        # the table's iterations - 1
    paper_gpu_s: float      # GPU:Pytorch seconds of Table 1 / 2 (RTX 2080 Super)
    initial: Callable[[], np.ndarray]
    # check(step -> field) at the listed steps; returns a dict of measurements
    checkpoints: tuple = ()
    check: Callable[[dict], dict] = field(default=lambda snaps: {})

    @property
    def eps(self) -> float:
        return eps_m(self.h, self.m)

    @property
    def dim(self) -> int:
        return len(self.shape)


def _cases() -> list[Case]:
    h2, h3 = 1 / 200, 1 / 100
    e2, e3 = eps_m(h2, 10), eps_m(h3, 12)
    d2, d3 = 0.1 * h2 * h2, 0.1 * h3 * h3

    def circle_check(s):
        R = volume_radius(s[12000], h2)
        return {"R_T": R, "R_law": radius_law(0.3, 12000 * d2, 2), "ok": abs(R - radius_law(0.3, 12000 * d2, 2)) <= h2}

    def dumbbell_check(s):
        a0, a1 = float((s[0] > 0).sum()) * h2 * h2, float((s[15000] > 0).sum()) * h2 * h2
        f = s[15000]
        lobes = f[100, 60] > 0.9 and f[100, 340] > 0.9 and f[100, 200] > 0.9
        mirror = float(np.max(np.abs(f - f[:, ::-1]))) <= 1e-9   # symmetric about x = 1
        return {"area0": a0, "area_T": a1, "lobes_and_bar": bool(lobes), "mirror": mirror,
                "ok": a1 < a0 and lobes and mirror}

    def star_check(s):
        tip0, gap0 = ray_crossing(s[0], h2, 0.0), ray_crossing(s[0], h2, math.pi / 6)
        tip1, gap1 = ray_crossing(s[2000], h2, 0.0), ray_crossing(s[2000], h2, math.pi / 6)
        tip2, gap2 = ray_crossing(s[6000], h2, 0.0), ray_crossing(s[6000], h2, math.pi / 6)
        return {"tip": [tip0, tip1, tip2], "gap": [gap0, gap1, gap2],
                "ok": tip1 < tip0 and gap1 > gap0 and abs(tip2 - gap2) <= 2 * h2}

    def torus_check(s):
        f = s[23000]
        hole_closed = f[100, 100] > 0.9
        R = ray_crossing(f, h2, 0.3) if hole_closed else -1.0
        law = radius_law(0.4, 23000 * d2, 2)
        # the hole (R2 = 0.3) closes at t = 0.045: still open at 16000 steps (t = 0.04)
        hole_open_before = s[16000][100, 100] < -0.9
        return {"outer_R_T": R, "outer_law": law, "hole_open_at_t0.04": bool(hole_open_before),
                "ok": hole_closed and hole_open_before and abs(R - law) <= 2 * h2}

    def sep2d_check(s):
        fr = separated(s[12000])
        return {"separated": fr, "ok": fr >= 0.85}

    def sphere_check(s):
        R = volume_radius(s[2000], h3)
        law = radius_law(0.4, 2000 * d3, 3)
        return {"R_T": R, "R_law": law, "ok": abs(R - law) <= h3}

    def dumbbell3d_check(s):
        f = s[1000]
        broken = f[50, 50, 100] < -0.9
        spheres = f[50, 50, 30] > 0.9 and f[50, 50, 170] > 0.9
        intact_early = s[250][50, 50, 100] > 0.5
        return {"handle_broken": bool(broken), "spheres_remain": bool(spheres),
                "handle_intact_at_250": bool(intact_early), "ok": broken and spheres and intact_early}

    def sep3d_check(s):
        fr = separated(s[2000])
        return {"separated": fr, "ok": fr >= 0.6}

    return [
        Case("circle", (200, 200), h2, d2, 10, 12000, 12000, 3.67,
             lambda: inputs.circle2d(200, 200, h2, e2, 0.3), (12000,), circle_check),
        Case("dumbbell", (200, 400), h2, 0.1 / 400 ** 2, 10, 15000, 15000, 6.90,
             lambda: inputs.dumbbell2d(400, 200, h2, e2, 0.2), (0, 15000), dumbbell_check),
        Case("star", (200, 200), h2, d2, 10, 13000, 13000, 5.68,
             lambda: inputs.star2d(200, 200, h2, e2, 0.25, 0.1), (0, 2000, 6000, 13000), star_check),
        Case("torus", (200, 200), h2, d2, 10, 23000, 23000, 8.01,
             lambda: inputs.torus2d(200, 200, h2, e2, 0.4, 0.3), (16000, 23000), torus_check),
        Case("separation", (200, 200), h2, d2, 10, 12000, 12000, 5.64,
             lambda: inputs.random_field((200, 200), 1), (12000,), sep2d_check),
        Case("sphere3d", (100, 100, 100), h3, d3, 12, 2000, 2000, 1.02,
             lambda: inputs.sphere3d(100, 100, 100, h3, e3, 0.4), (2000,), sphere_check),
        Case("dumbbell3d", (100, 100, 200), h3, d3, 12, 1000, 2000, 1.97,
             lambda: dumbbell3d(200, 100, 100, h3, e3, 0.25), (250, 1000), dumbbell3d_check),
        Case("separation3d", (100, 100, 100), h3, d3, 12, 2000, 2000, 1.03,
             lambda: inputs.random_field((100, 100, 100), 3), (2000,), sep3d_check),
    ]


CASES = {c.name: c for c in _cases()}


def _step(case: Case, phi: torch.Tensor, n: int) -> None:
    if n <= 0:
        return
    if case.dim == 2:
        api.step2d(phi, case.h, case.dt, case.eps, n)
    else:
        api.step3d(phi, case.h, case.dt, case.eps, n)


def run(case: Case, dtype=torch.float64, phi0: np.ndarray | None = None) -> dict:
    """Advance the case through its checkpoints on the GPU; returns the
    snapshots (numpy, by step), the final field and the check's result."""
    p0 = case.initial() if phi0 is None else phi0
    phi = torch.from_numpy(np.ascontiguousarray(p0)).to(dtype).cuda()
    snaps, done = {}, 0
    for cp in sorted(set(case.checkpoints) | {case.steps}):
        _step(case, phi, cp - done)
        done = cp
        if cp in case.checkpoints:
            snaps[cp] = phi.cpu().numpy().astype(np.float64)
    return {"snapshots": snaps, "final": phi, "initial": p0, "check": case.check(snaps)}


def time_table_count(case: Case, dtype=torch.float32, reps: int = 3) -> float:
    """Median seconds of the table's step count on the GPU (state in HBM)."""
    phi = torch.from_numpy(np.ascontiguousarray(case.initial())).to(dtype).cuda()
    _step(case, phi, case.table_steps)
    ts = []
    for _ in range(reps):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        _step(case, phi, case.table_steps)
        e.record()
        torch.cuda.synchronize()
        ts.append(s.elapsed_time(e) / 1e3)
    return sorted(ts)[len(ts) // 2]


def timings(dtype=torch.float32) -> dict:
    """GPU seconds at the tables' step counts next to the paper's GPU:Pytorch
    seconds (other hardware: context, not a target)."""
    out = {}
    for c in CASES.values():
        t = time_table_count(c, dtype)
        cells = int(np.prod(c.shape))
        out[c.name] = {"steps": c.table_steps, "ms": round(t * 1e3, 3),
                       "GLUPS": round(cells * c.table_steps / t / 1e9, 2),
                       "paper_gpu_s": c.paper_gpu_s, "ratio_vs_paper": round(c.paper_gpu_s / t, 1)}
    return out


# Table 3 of the paper: Err (Eq. ERReq) of its FP32 GPU code against its FP64
# CPU code, by workload (maze omitted: its start is not reproducible)
TABLE3 = {"separation": 1.75e-6, "dumbbell": 7.03e-7, "circle": 5.51e-7, "star": 6.55e-7,
          "torus": 7.52e-7, "separation3d": 3.01e-6, "dumbbell3d": 1.20e-6, "sphere3d": 1.11e-6}


def err_table() -> dict:
    """Err between the FP32 and FP64 runs of each Table-3 workload (fused
    on-device trace), next to the paper's value."""
    out = {}
    for name, ref in TABLE3.items():
        c = CASES[name]
        p0 = np.ascontiguousarray(c.initial()).astype(np.float32)
        p32 = torch.from_numpy(p0).cuda()
        p64 = torch.from_numpy(p0.astype(np.float64)).cuda()
        _, err = api.err_trace(p32, p64, c.h, c.dt, c.eps, c.steps)
        out[name] = {"Err": float("%.4g" % err), "paper": ref, "ratio": round(err / ref, 3)}
    return out


def main():
    print(json.dumps(timings()))
    print(json.dumps(err_table()))


if __name__ == "__main__":
    main()
