"""The synthetic workloads the stepper is tested and measured on.

Every input is seeded and formula-defined (section 3.1 shapes); no dataset is
involved.  Sizes follow the configurations this implementation is measured on:

* ``phase64``   2D 64x64, h=1/64, m=4, random phi0 (seed 1), FP64, 500 steps
* ``circle2048`` 2D 2048x2048, h=1/2048, m=4, circle R0=0.25, 20000 steps
* ``sep256c``   3D 256^3, h=1/256, m=4, random phi0 (seed 3), FP32, 2000 steps;
                ``sphere256`` the same grid with a sphere of R0=0.3
* ``batch512``  512 independent 2D grids (seed 4), sides from
                {96,128,192,256,384,512,768,1024}, m in {3..8}, mixed
                random / circle (R0=0.25) / star (0.3 + 0.08 cos 6θ), 5000 steps
* ``sur256``    2D 256x256 grids for the learned K=100-step surrogate
* ``hbm16k`` / ``hbm1024c``  HBM-resident sizes well past the last-level
                cache: 2D 16384^2 (1 GiB per FP32 buffer, seed 5) and 3D 1024^3
                (4 GiB per FP32 buffer, seed 6), m=4, random phi0, 200 steps
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import inputs
from .params import dt_of, eps_m

SIDES = (96, 128, 192, 256, 384, 512, 768, 1024)
IC_KINDS = ("random", "circle", "star")


@dataclass
class Grid2D:
    nx: int
    ny: int
    h: float
    dt: float
    eps: float
    m: int
    kind: str
    seed: int
    stream: int = 0

    def initial(self, dtype=np.float64) -> np.ndarray:
        if self.kind == "random":
            return inputs.random_field((self.ny, self.nx), self.seed, self.stream, dtype=dtype)
        if self.kind == "circle":
            return inputs.circle2d(self.nx, self.ny, self.h, self.eps, 0.25)
        if self.kind == "star":
            return inputs.star2d(self.nx, self.ny, self.h, self.eps, 0.3, 0.08)
        raise ValueError(self.kind)


def unit_grid2d(n: int, m: int, kind: str, seed: int = 0, ny: int | None = None) -> Grid2D:
    h = 1.0 / n
    return Grid2D(n, ny or n, h, dt_of(h), eps_m(h, m), m, kind, seed)


def phase64() -> Grid2D:
    return unit_grid2d(64, 4, "random", seed=1)


def circle2048(n: int = 2048) -> Grid2D:
    return unit_grid2d(n, 4, "circle")


@dataclass
class Grid3D:
    nx: int
    ny: int
    nz: int
    h: float
    dt: float
    eps: float
    kind: str
    seed: int
    R0: float = 0.3

    def initial(self, dtype=np.float64) -> np.ndarray:
        if self.kind == "random":
            return inputs.random_field((self.nz, self.ny, self.nx), self.seed, 0, dtype=dtype)
        if self.kind == "sphere":
            return inputs.sphere3d(self.nx, self.ny, self.nz, self.h, self.eps, self.R0)
        raise ValueError(self.kind)


def unit_grid3d(n: int, m: int, kind: str, seed: int = 3) -> Grid3D:
    h = 1.0 / n
    return Grid3D(n, n, n, h, dt_of(h), eps_m(h, m), kind, seed)


def sep256c(n: int = 256) -> Grid3D:
    return unit_grid3d(n, 4, "random", seed=3)


def sphere256(n: int = 256) -> Grid3D:
    return unit_grid3d(n, 4, "sphere")


HBM_STEPS = 200

SIDES3D = (24, 32, 48, 64, 96, 128)


def batch3d_instances(n_inst: int = 64, seed: int = 8, sides=SIDES3D,
                      m_range=(3, 8)) -> list[Grid3D]:
    """Seeded table of independent 3D instances: nx, ny, nz drawn from
    ``sides``, m uniform on ``m_range``, random (stream 2000 + b) or a sphere
    of radius 0.3 centred in (0, nx h) x (0, ny h) x (0, nz h), h = 1 / min side."""
    out = []
    for b in range(n_inst):
        nx, ny, nz = (sides[inputs.draw_int(seed, b, k, 0, len(sides) - 1)] for k in range(3))
        m = inputs.draw_int(seed, b, 3, m_range[0], m_range[1])
        kind = ("random", "sphere")[inputs.draw_int(seed, b, 4, 0, 1)]
        h = 1.0 / min(nx, ny, nz)
        out.append(Grid3D(nx, ny, nz, h, dt_of(h), eps_m(h, m), kind, seed * 1000 + b))
    return out


def hbm16k(n: int = 16384) -> Grid2D:
    return unit_grid2d(n, 4, "random", seed=5)


def hbm1024c(n: int = 1024) -> Grid3D:
    return unit_grid3d(n, 4, "random", seed=6)


def batch_instances(n_inst: int = 512, seed: int = 4, sides=SIDES,
                    m_range=(3, 8)) -> list[Grid2D]:
    """Seeded table of independent 2D instances.

    Each instance ``b`` draws (from stream ``b`` of ``seed``): nx, ny from
    ``sides``; m uniform on ``m_range``; the initial kind uniform over
    random / circle / star.  Non-square grids use h = 1/min(nx, ny) on
    (0, nx h) x (0, ny h), shapes centred in the domain; random fields use
    stream ``1000 + b``.
    """
    out = []
    for b in range(n_inst):
        nx = sides[inputs.draw_int(seed, b, 0, 0, len(sides) - 1)]
        ny = sides[inputs.draw_int(seed, b, 1, 0, len(sides) - 1)]
        m = inputs.draw_int(seed, b, 2, m_range[0], m_range[1])
        kind = IC_KINDS[inputs.draw_int(seed, b, 3, 0, 2)]
        h = 1.0 / min(nx, ny)
        out.append(Grid2D(nx, ny, h, dt_of(h), eps_m(h, m), m, kind, seed, 1000 + b))
    return out


def surrogate_grid(seed: int, n: int = 256) -> Grid2D:
    """One 256x256 surrogate trajectory: kind uniform over random / circle /
    star, m uniform on {4, 5, 6}; circles draw R0 uniform on [0.15, 0.35]."""
    m = inputs.draw_int(seed, 7, 0, 4, 6)
    kind = IC_KINDS[inputs.draw_int(seed, 7, 1, 0, 2)]
    return unit_grid2d(n, m, kind, seed=seed)


def surrogate_initial(g: Grid2D) -> np.ndarray:
    if g.kind == "circle":
        R0 = inputs.draw_uniform(g.seed, 7, 2, 0.15, 0.35)
        return inputs.circle2d(g.nx, g.ny, g.h, g.eps, R0)
    if g.kind == "star":
        return inputs.star2d(g.nx, g.ny, g.h, g.eps, 0.3, 0.08)
    return inputs.random_field((g.ny, g.nx), g.seed, 0)
