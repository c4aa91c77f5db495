"""Occupations, Fermi level, band energy and electron density from Ritz pairs (Sec. II).

* Fermi-Dirac occupancy of a state of energy eps at Fermi level mu and smearing
  temperature T (eqnfd): f = 1 / (1 + exp((eps - mu) / (k_B T))).
* The Fermi level fixes the number of electrons (eqnne):
  2 sum_k w_k sum_alpha f(eps_{alpha,k}, mu) = N_e.  The paper does not say how mu is
  found; here it is bisection on mu (the count is increasing in mu), from the bracket
  [min eps - 50 kT, max eps + 50 kT], halving until the bracket is at rounding level
  (4 u max(1, |mu|)) or after 200 halvings, mu = the bracket's midpoint.
* Band energy (the E_band of Sec. II): 2 sum_k w_k sum_alpha f eps.
* Electron density at the quadrature points (eqnrho):
  rho(x) = 2 sum_k w_k sum_alpha f |u_{alpha,k}(x)|^2, with |u| = |psi| for the Bloch
  functions of the phase-twisted basis; psi at the quadrature points as in adjoint.py.
"""
from __future__ import annotations

import numpy as np

from . import adjoint

K_BOLTZMANN_HA_PER_K = 3.166811563e-6  # Hartree per kelvin


def fermi_dirac(eps, mu: float, kT: float) -> np.ndarray:
    """f(eps, mu) of eqnfd, elementwise (float64)."""
    x = (np.asarray(eps, dtype=np.float64) - mu) / kT
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(x))


def electron_count(thetas, wk, mu: float, kT: float) -> float:
    """2 sum_k w_k sum_alpha f(eps_{alpha,k}, mu) (eqnne); thetas: one array of Ritz values per k-point."""
    return float(sum(2.0 * w * np.sum(fermi_dirac(th, mu, kT)) for th, w in zip(thetas, wk)))


def fermi_level(thetas, wk, n_elec: float, kT: float, max_halvings: int = 200):
    """mu with electron_count(mu) = n_elec by bisection; returns (mu, halvings)."""
    lo = min(float(np.min(t)) for t in thetas) - 50.0 * kT
    hi = max(float(np.max(t)) for t in thetas) + 50.0 * kT
    if not (0.0 < n_elec < electron_count(thetas, wk, hi, kT)):
        raise ValueError("the electron count cannot be reached with these states")
    it = 0
    while it < max_halvings:
        mid = 0.5 * (lo + hi)
        if hi - lo <= 4.0 * np.finfo(float).eps * max(1.0, abs(mid)):
            break
        if electron_count(thetas, wk, mid, kT) < n_elec:
            lo = mid
        else:
            hi = mid
        it += 1
    return 0.5 * (lo + hi), it


def band_energy(thetas, wk, occ) -> float:
    """E_band = 2 sum_k w_k sum_alpha f eps."""
    return float(sum(2.0 * w * np.sum(f * th) for th, w, f in zip(thetas, wk, occ)))


def density(op, X: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """sum_alpha weights_alpha |psi_alpha(x_{e,q})|^2 at the quadrature points, [n_cells, nq];
    with weights = 2 w_k f this is one k-point's term of eqnrho."""
    psi = adjoint.fields_at_quad(op, X)
    return np.einsum("eqv,v->eq", np.abs(psi) ** 2, weights)
