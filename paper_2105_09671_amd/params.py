"""Host-side parameter derivation (section 2).

* h = 1 / N_x on the unit domain (grid definition, section 2);
* dt = 0.1 h^2 (section 2);
* eps_m = h m / (2 sqrt(2) atanh(0.9)), m = cells across the transition layer
  (Eq. emvalue).

The C library derives alpha = dt/eps^2 and r = dt/h^2 from these itself.
"""
from __future__ import annotations

import math


def eps_m(h: float, m: float) -> float:
    """Interface thickness spanning m cells (Eq. emvalue)."""
    return h * m / (2.0 * math.sqrt(2.0) * math.atanh(0.9))


def dt_of(h: float) -> float:
    """Time step dt = 0.1 h^2 (section 2)."""
    return 0.1 * h * h


def radius_law(R0: float, t: float, dim: int) -> float:
    """Sharp-interface radius r(t) = sqrt(r0^2 + 2(1 - d) t) (Eq. exactradiusEQ)."""
    v = R0 * R0 + 2.0 * (1 - dim) * t
    return math.sqrt(v) if v > 0 else 0.0
