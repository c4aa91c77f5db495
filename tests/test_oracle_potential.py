"""Pins of the oracle's synthetic potential (oracle/potential.py).

V(x) = sum_I -Z_I erf(r_I / sigma) / r_I with r_I the distance to the nearest
periodic image of atom I.  Each check compares against a fact fixed by the
mathematics rather than by the same formula:

* far field: erf(6) rounds to 1 in float64, so V is the bare Coulomb -Z / r;
* r -> 0: the limit 2 / (sigma sqrt(pi)) of erf(r / sigma) / r, and continuity
  where the code switches from its series to the erf branch;
* Poisson: the 7-point finite-difference Laplacian of erf(r/sigma)/r equals
  -4 pi times the unit Gaussian charge (pi sigma^2)^(-3/2) exp(-r^2/sigma^2),
  which fixes the sigma convention (a sigma sqrt(2) or sigma^2 slip fails);
* the nearest image equals a brute-force minimum over the 27 neighbouring
  images; V is periodic; V of two atoms is the sum of the one-atom potentials.
"""
import itertools

import numpy as np
import pytest

from oracle.potential import erf_over_r, min_image, nuclear_potential

SIGMA = 0.5


def test_far_field_is_bare_coulomb():
    r = np.array([6.0, 7.5, 10.0, 25.0]) * SIGMA
    np.testing.assert_allclose(erf_over_r(r, SIGMA), 1.0 / r, rtol=1e-15, atol=0)
    pts = np.array([[r_, 0.0, 0.0] for r_ in r])
    V = nuclear_potential(pts, np.zeros((1, 3)), np.array([3.0]), SIGMA, 100.0)
    np.testing.assert_allclose(V, -3.0 / r, rtol=1e-15, atol=0)


def test_limit_at_the_nucleus_and_continuity_at_the_series_switch():
    lim = 2.0 / (SIGMA * np.sqrt(np.pi))
    assert abs(erf_over_r(np.array([0.0]), SIGMA)[0] - lim) <= 1e-15 * lim
    V0 = nuclear_potential(np.zeros((1, 3)), np.zeros((1, 3)), np.array([14.0]), SIGMA, 10.0)
    assert abs(V0[0] + 14.0 * lim) <= 1e-14 * 14.0 * lim
    # the two branches meet at r = 1e-6 sigma: values on either side agree to the size of
    # the next series term (x^6 / 42 ~ 1e-38) plus rounding
    sw = 1e-6 * SIGMA
    below = erf_over_r(np.array([sw * (1 - 1e-9)]), SIGMA)[0]
    above = erf_over_r(np.array([sw * (1 + 1e-9)]), SIGMA)[0]
    assert abs(below - above) <= 4e-16 * lim
    # monotone decreasing away from the nucleus
    r = np.linspace(0.0, 4.0, 400)
    assert np.all(np.diff(erf_over_r(r, SIGMA)) < 0)


@pytest.mark.parametrize("x", [[0.21, 0.05, -0.13], [0.4, 0.3, 0.1], [0.0, 0.75, 0.2], [0.9, -0.2, 0.35]])
def test_laplacian_is_minus_four_pi_gaussian_charge(x):
    """Central differences of V of one unit charge (Z = 1 gives V = -erf(r/sigma)/r) against Poisson."""
    x = np.array(x)
    hh = 2e-3
    pos = np.zeros((1, 3))
    Z = np.array([1.0])
    pts = [x]
    for d in range(3):
        for s in (1.0, -1.0):
            e = np.zeros(3)
            e[d] = s * hh
            pts.append(x + e)
    V = nuclear_potential(np.array(pts), pos, Z, SIGMA, 50.0)
    lap = (V[1:].sum() - 6.0 * V[0]) / hh ** 2
    r2 = float(x @ x)
    rho = (np.pi * SIGMA ** 2) ** -1.5 * np.exp(-r2 / SIGMA ** 2)
    # -grad^2 V = -4 pi rho for V = -phi, i.e. grad^2 V = 4 pi rho (unit positive charge)
    np.testing.assert_allclose(lap, 4.0 * np.pi * rho, rtol=2e-5)


def test_gaussian_charge_normalization_of_the_poisson_pin():
    # the charge density of the Poisson pin integrates to one (radial quadrature)
    r = np.linspace(0.0, 8.0 * SIGMA, 20001)
    f = 4.0 * np.pi * r ** 2 * (np.pi * SIGMA ** 2) ** -1.5 * np.exp(-(r / SIGMA) ** 2)
    assert abs(np.trapezoid(f, r) - 1.0) < 1e-9


def test_nearest_image_is_the_closest_of_all_images():
    rng = np.random.default_rng(7)
    L = 10.26
    d = rng.uniform(-1.5 * L, 1.5 * L, size=(200, 3))
    m = min_image(d, L)
    assert np.all(np.abs(m) <= 0.5 * L + 1e-12)
    shifts = np.array(list(itertools.product((-2, -1, 0, 1, 2), repeat=3)), dtype=float) * L
    brute = np.min(np.linalg.norm(d[:, None, :] + shifts[None, :, :], axis=-1), axis=1)
    np.testing.assert_allclose(np.linalg.norm(m, axis=-1), brute, rtol=1e-13, atol=1e-13)


def test_periodic_and_additive():
    rng = np.random.default_rng(11)
    L = 10.26
    pos = rng.uniform(0.0, L, size=(2, 3))
    Z = np.array([14.0, 6.0])
    pts = rng.uniform(0.0, L, size=(50, 3))
    V = nuclear_potential(pts, pos, Z, SIGMA, L)
    for d in range(3):
        e = np.zeros(3)
        e[d] = L
        np.testing.assert_allclose(nuclear_potential(pts + e, pos, Z, SIGMA, L), V, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(nuclear_potential(pts - 2 * e, pos, Z, SIGMA, L), V, rtol=1e-12, atol=1e-12)
    V1 = nuclear_potential(pts, pos[:1], Z[:1], SIGMA, L)
    V2 = nuclear_potential(pts, pos[1:], Z[1:], SIGMA, L)
    np.testing.assert_allclose(V, V1 + V2, rtol=1e-14, atol=1e-14)
    # each one-atom potential is the charge times the unit-charge potential of the nearest image
    d = min_image(pts - pos[0], L)
    r = np.linalg.norm(d, axis=-1)
    from scipy.special import erf
    np.testing.assert_allclose(V1, -14.0 * erf(r / SIGMA) / r, rtol=1e-14)
