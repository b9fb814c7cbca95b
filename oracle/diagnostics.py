"""Diagnostics on phase fields (oracle side; TEST INFRASTRUCTURE ONLY).

* ``energy`` -- discrete Ginzburg-Landau energy whose explicit gradient
  descent is the scheme of section 2.1:
  E_h = h^d [ sum_cells F(phi)/eps^2 + 1/2 sum_interior-faces ((phi_a - phi_b)/h)^2 ],
  F(phi) = (phi^2 - 1)^2 / 4 (section 1).  With the zero-Neumann boundary no
  boundary face contributes.
* ``volume_radius`` -- radius of the disc / ball with the volume of {phi > 0},
  measured as V = h^d sum (1 + phi)/2.
* ``crossings`` -- zero crossings of phi on grid edges by linear interpolation.
* ``hausdorff`` -- symmetric Hausdorff distance between two point sets.
* ``rel_linf`` -- max |a - b| / max |b|.
* ``err_metric`` -- the paper's Err: mean over time of the RMS difference
  (Eq. ERReq).
"""
from __future__ import annotations

import math

import numpy as np


def energy(phi, h: float, eps: float) -> float:
    phi = np.asarray(phi, dtype=np.float64)
    d = phi.ndim
    bulk = np.sum(0.25 * (phi * phi - 1.0) ** 2) / (eps * eps)
    grad = 0.0
    for ax in range(d):
        diff = np.diff(phi, axis=ax) / h
        grad += 0.5 * np.sum(diff * diff)
    return float(h ** d * (bulk + grad))


def volume_radius(phi, h: float) -> float:
    phi = np.asarray(phi, dtype=np.float64)
    d = phi.ndim
    V = h ** d * np.sum(0.5 * (1.0 + phi))
    if d == 2:
        return math.sqrt(V / math.pi)
    if d == 3:
        return (V / (4.0 / 3.0 * math.pi)) ** (1.0 / 3.0)
    raise ValueError("2D or 3D field expected")


def radius_law(R0: float, t: float, dim: int) -> float:
    """r(t) = sqrt(r0^2 + 2(1 - d) t) (Eq. exactradiusEQ)."""
    v = R0 * R0 + 2.0 * (1 - dim) * t
    return math.sqrt(v) if v > 0 else 0.0


def crossings(phi, h: float) -> np.ndarray:
    """Points (x, y) where phi changes sign along a horizontal or vertical edge
    between cell centres, located by linear interpolation.  Cell (j, i) sits at
    ((i + 1/2) h, (j + 1/2) h)."""
    phi = np.asarray(phi, dtype=np.float64)
    pts = []
    # horizontal edges (i, j) -- (i+1, j)
    a, b = phi[:, :-1], phi[:, 1:]
    jj, ii = np.nonzero((a > 0) != (b > 0))
    if jj.size:
        fa, fb = a[jj, ii], b[jj, ii]
        t = fa / (fa - fb)
        pts.append(np.stack([(ii + 0.5 + t) * h, (jj + 0.5) * h], axis=1))
    a, b = phi[:-1, :], phi[1:, :]
    jj, ii = np.nonzero((a > 0) != (b > 0))
    if jj.size:
        fa, fb = a[jj, ii], b[jj, ii]
        t = fa / (fa - fb)
        pts.append(np.stack([(ii + 0.5) * h, (jj + 0.5 + t) * h], axis=1))
    if not pts:
        return np.zeros((0, 2))
    return np.concatenate(pts, axis=0)


def hausdorff(A, B) -> float:
    """Symmetric Hausdorff distance; inf if exactly one set is empty, 0 if both are."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if len(A) == 0 and len(B) == 0:
        return 0.0
    if len(A) == 0 or len(B) == 0:
        return math.inf
    from scipy.spatial import cKDTree
    dab = cKDTree(B).query(A)[0].max()
    dba = cKDTree(A).query(B)[0].max()
    return float(max(dab, dba))


def interface_error(phi_a, phi_b, h: float) -> float:
    """Hausdorff distance between the zero-crossing sets of two 2D fields.

    The sets are discrete (about one point per cell the front passes through):
    for two smooth fronts a distance d apart the value lies between d and
    sqrt(d^2 + h^2/2), up to the O(h^2) interpolation error of the crossings."""
    return hausdorff(crossings(phi_a, h), crossings(phi_b, h))


def rel_linf(a, ref) -> float:
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(a - ref))) if ref.size else 0.0
    return num / den if den > 0 else num


def err_metric(traj_a, traj_b) -> float:
    """Err = (1/n) sum_t sqrt(avg((a_t - b_t)^2)) over snapshots t (Eq. ERReq)."""
    vals = [math.sqrt(float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2)))
            for a, b in zip(traj_a, traj_b)]
    return float(np.mean(vals)) if vals else 0.0
