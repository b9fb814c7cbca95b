"""Dense-matrix brute force of the explicit Allen-Cahn step, for tiny grids.

TEST INFRASTRUCTURE ONLY (part of the oracle).

The zero-Neumann 5-point (2D) / 7-point (3D) Laplacian of section 2 is the
graph Laplacian of the grid graph divided by h^2: a ghost cell equal to the
cell beside it contributes (phi_c - phi_c) = 0, so only in-grid neighbours
appear.  This module builds that matrix explicitly,
    L[c, c] = -(number of in-grid neighbours of c) / h^2,
    L[c, n] = 1 / h^2 for each in-grid neighbour n,
and steps  phi <- phi + dt (phi - phi^3) / eps^2 + dt L phi  (Eq. pytorchACeq).
It shares nothing with the loop oracle except the problem statement.
"""
from __future__ import annotations

import itertools

import numpy as np


def neumann_laplacian(shape, h: float) -> np.ndarray:
    """Dense Laplacian matrix for a grid of the given (row-major) shape."""
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    L = np.zeros((n, n), dtype=np.float64)
    idx = np.arange(n).reshape(shape)
    for pos in itertools.product(*[range(s) for s in shape]):
        c = idx[pos]
        for axis in range(len(shape)):
            for d in (-1, 1):
                q = list(pos)
                q[axis] += d
                if 0 <= q[axis] < shape[axis]:
                    L[c, idx[tuple(q)]] += 1.0
                    L[c, c] -= 1.0
    return L / (h * h)


def step(phi0, h: float, dt: float, eps: float, nsteps: int) -> np.ndarray:
    phi = np.array(phi0, dtype=np.float64).ravel()
    L = neumann_laplacian(np.shape(phi0), h)
    for _ in range(nsteps):
        phi = phi + dt * (phi - phi ** 3) / eps ** 2 + dt * (L @ phi)
    return phi.reshape(np.shape(phi0))
