"""Fixed synthetic potential at the quadrature points.

The paper's effective potential (LDA + electrostatics, Sec. II) is replaced by
the external potential of erf-smeared nuclei,
    V(x) = sum_I -Z_I erf(r_I / sigma) / r_I,
with r_I the distance from x to the nearest periodic image of atom I (the
nearest-image convention of eqnUOEFEAtomic).  r -> 0 limit: -2 Z / (sigma sqrt(pi)).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def erf_over_r(r: np.ndarray, sigma: float) -> np.ndarray:
    """erf(r / sigma) / r, with the Taylor series 2/(sigma sqrt(pi)) (1 - x^2/3 + x^4/10), x = r/sigma, near 0."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    small = r < 1e-6 * sigma
    x = r[small] / sigma
    out[small] = 2.0 / (sigma * np.sqrt(np.pi)) * (1.0 - x * x / 3.0 + x ** 4 / 10.0)
    rs = r[~small]
    out[~small] = erf(rs / sigma) / rs
    return out


def min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def nuclear_potential(points: np.ndarray, pos: np.ndarray, Z: np.ndarray, sigma: float, L: float) -> np.ndarray:
    """V at an array of points [..., 3]."""
    V = np.zeros(points.shape[:-1])
    for I in range(pos.shape[0]):
        d = min_image(points - pos[I], L)
        r = np.sqrt((d * d).sum(-1))
        V -= Z[I] * erf_over_r(r, sigma)
    return V
