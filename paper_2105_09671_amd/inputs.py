"""Seeded synthetic initial states for the Allen-Cahn stepper.

This module only *draws inputs*: it holds none of the time-stepping arithmetic.
Both the GPU path and the CPU oracle are fed the arrays it returns.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: output ``i`` of stream ``(seed, stream)`` is ``mix(key + (i+1)*G)``
with ``G = 0x9E3779B97F4A7C15`` and ``key = mix(seed*G + stream)``.  A uniform
double in [0, 1) is ``(x >> 11) * 2**-53``.

Initial shapes follow section 3.1 of the paper (cell centres at
``a + (i + 1/2) h`` for 0-based ``i``, section 2):

* random:  phi0 = 0.1 * rand, rand uniform on [-1, 1)   (Eqs. 2Dtrnadini, 3Drandini)
* circle / sphere: tanh((R0 - |x - c|) / (sqrt(2) eps))  (Eqs. 2Dcircleini, 3Dsphereini)
* star:    tanh((r0 + a cos(6 theta) - |x - c|) / (sqrt(2) eps)), theta = atan2
           (Eq. 2Dstarini; the piecewise arctan there is atan2 up to 2*pi)
* dumbbell: Eq. 2Ddumbellini;  torus: Eq. 2Dtorusini.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (the finaliser applied to the counter)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs ``start .. start+n-1`` of SplitMix64 stream ``(seed, stream)``."""
    with np.errstate(over="ignore"):
        key = _mix64(np.array([np.uint64(seed) * GOLDEN + np.uint64(stream)],
                              dtype=np.uint64))[0]
        idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        return _mix64(key + idx * GOLDEN)


def uniform01(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits each."""
    x = splitmix64(seed, stream, n, start)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def draw_int(seed: int, stream: int, index: int, lo: int, hi: int) -> int:
    """One integer uniform on [lo, hi] from counter ``index`` of the stream."""
    u = uniform01(seed, stream, 1, start=index)[0]
    return lo + min(int(u * (hi - lo + 1)), hi - lo)


def draw_uniform(seed: int, stream: int, index: int, lo: float, hi: float) -> float:
    u = uniform01(seed, stream, 1, start=index)[0]
    return lo + (hi - lo) * u


# ---------------------------------------------------------------- grids ----

def centres(n: int, h: float, a: float = 0.0) -> np.ndarray:
    """Cell centres a + (i + 1/2) h, i = 0..n-1 (section 2)."""
    return a + (np.arange(n, dtype=np.float64) + 0.5) * h


def _mesh2d(nx, ny, h, origin=(0.0, 0.0)):
    x = centres(nx, h, origin[0])
    y = centres(ny, h, origin[1])
    return np.meshgrid(x, y, indexing="xy")  # arrays of shape (ny, nx)


def _mesh3d(nx, ny, nz, h, origin=(0.0, 0.0, 0.0)):
    x = centres(nx, h, origin[0])
    y = centres(ny, h, origin[1])
    z = centres(nz, h, origin[2])
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")  # shape (nz, ny, nx)
    return xx, yy, zz


# ------------------------------------------------------- initial states ----

def random_field(shape, seed: int, stream: int = 0, amp: float = 0.1,
                 dtype=np.float64, chunk: int = 1 << 24) -> np.ndarray:
    """amp * rand with rand uniform on [-1, 1), i.i.d. per cell, row-major order.

    The value of cell ``i`` is counter ``i`` of the stream, computed in double
    precision; ``dtype=np.float32`` rounds each value once.  Large fields are
    drawn ``chunk`` cells at a time, with the same result.
    """
    n = int(np.prod(shape))
    out = np.empty(n, dtype=dtype)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        u = uniform01(seed, stream, m, start=s)
        out[s:s + m] = amp * (2.0 * u - 1.0)
    return out.reshape(shape)


def _signed(c: int) -> int:
    """A 64-bit constant as the signed integer with the same bits."""
    return c - (1 << 64) if c >= (1 << 63) else c


def random_field_torch(shape, seed: int, stream: int = 0, amp: float = 0.1, dtype=None,
                       device="cpu", chunk: int = 1 << 26):
    """``random_field`` drawn with torch on ``device`` (bit-identical values).

    SplitMix64 runs on int64 tensors: products wrap modulo 2**64 as for
    uint64, and a logical right shift is an arithmetic shift with the copied
    sign bits masked off.  Meant for fields too large to draw quickly on the
    host (a 1024^3 grid).
    """
    import torch
    dtype = dtype or torch.float64
    G, M1, M2 = _signed(int(GOLDEN)), _signed(int(_M1)), _signed(int(_M2))

    def shr(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)

    def mix(z):
        z = (z ^ shr(z, 30)) * M1
        z = (z ^ shr(z, 27)) * M2
        return z ^ shr(z, 31)

    with np.errstate(over="ignore"):
        key = _signed(int(_mix64(np.array([np.uint64(seed) * GOLDEN + np.uint64(stream)],
                                          dtype=np.uint64))[0]))
    n = int(np.prod(shape))
    out = torch.empty(n, dtype=dtype, device=device)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        idx = torch.arange(s + 1, s + m + 1, dtype=torch.int64, device=device)
        x = mix(key + idx * G)
        u = shr(x, 11).to(torch.float64) * (2.0 ** -53)
        out[s:s + m] = (amp * (2.0 * u - 1.0)).to(dtype)
    return out.reshape(shape)


def circle2d(nx, ny, h, eps, R0, centre=None) -> np.ndarray:
    if centre is None:
        centre = (0.5 * nx * h, 0.5 * ny * h)
    X, Y = _mesh2d(nx, ny, h)
    r = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2)
    return np.tanh((R0 - r) / (np.sqrt(2.0) * eps))


def sphere3d(nx, ny, nz, h, eps, R0, centre=None) -> np.ndarray:
    if centre is None:
        centre = (0.5 * nx * h, 0.5 * ny * h, 0.5 * nz * h)
    X, Y, Z = _mesh3d(nx, ny, nz, h)
    r = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2)
    return np.tanh((R0 - r) / (np.sqrt(2.0) * eps))


def star2d(nx, ny, h, eps, r0=0.3, amp=0.08, centre=None) -> np.ndarray:
    """Six-pointed star.  Defaults are the batched workload's r = 0.3 + 0.08 cos 6θ;
    the paper's own star is r0=0.25, amp=0.1 (Eq. 2Dstarini)."""
    if centre is None:
        centre = (0.5 * nx * h, 0.5 * ny * h)
    X, Y = _mesh2d(nx, ny, h)
    dx, dy = X - centre[0], Y - centre[1]
    theta = np.arctan2(dy, dx)
    r = np.sqrt(dx ** 2 + dy ** 2)
    return np.tanh((r0 + amp * np.cos(6.0 * theta) - r) / (np.sqrt(2.0) * eps))


def dumbbell2d(nx, ny, h, eps, R0=0.2) -> np.ndarray:
    """Eq. 2Ddumbellini on (0, nx h) x (0, ny h) (the paper: (0,2) x (0,1))."""
    X, Y = _mesh2d(nx, ny, h)
    Yt = (Y - 0.5) ** 2
    s2e = np.sqrt(2.0) * eps
    phi = (1.0 + np.tanh((R0 - np.sqrt((X - 0.3) ** 2 + Yt)) / s2e)
           + np.tanh((R0 - np.sqrt((X - 1.7) ** 2 + Yt)) / s2e))
    bar = (X > 0.4) & (X < 1.6) & (Y > 0.4) & (Y < 0.6)
    phi[bar] = 1.0
    return phi


def torus2d(nx, ny, h, eps, R1=0.4, R2=0.3) -> np.ndarray:
    """Eq. 2Dtorusini: an annulus between radii R2 < R1 about (0.5, 0.5)."""
    X, Y = _mesh2d(nx, ny, h)
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2)
    s2e = np.sqrt(2.0) * eps
    return -1.0 + np.tanh((R1 - r) / s2e) - np.tanh((R2 - r) / s2e)
