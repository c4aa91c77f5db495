"""Pins of the oracle's occupations, Fermi level, band energy and density (oracle/occupations.py).

* Fermi-Dirac against scipy's logistic function, f(mu) = 1/2 and f(mu + x) = 1 - f(mu - x);
* the Fermi level satisfies the electron-count constraint to rounding, for one and several
  k-points with weights;
* the zero-temperature limit: with a gap at the Fermi level the occupations become the
  aufbau step (the lowest N_e / 2 states full), and the band energy 2 sum of their energies;
* the band energy from Ritz pairs equals the Rayleigh quotients' weighted sum computed by the
  adjoint module's independent route (x^* Ht x with the same weights);
* the density integrates to the weighted sum of the states' quadrature norms, and for the
  exact eigenvectors of a tiny operator to N_e within the Gauss-vs-lumped-mass quadrature
  difference.
"""
import numpy as np
import pytest
from scipy.special import expit

from oracle import adjoint as adj
from oracle import occupations as occ
from oracle.operator import OEFEOperator
from paper_2010_09701_amd import workloads as wl

KT = 500.0 * occ.K_BOLTZMANN_HA_PER_K


def test_fermi_dirac_closed_form_and_symmetry():
    eps = np.linspace(-1.0, 1.0, 2001)
    np.testing.assert_allclose(occ.fermi_dirac(eps, 0.1, KT), expit(-(eps - 0.1) / KT), rtol=1e-15, atol=1e-300)
    assert occ.fermi_dirac(np.array([0.3]), 0.3, KT)[0] == 0.5
    x = np.linspace(0, 20 * KT, 50)
    np.testing.assert_allclose(occ.fermi_dirac(0.2 + x, 0.2, KT), 1.0 - occ.fermi_dirac(0.2 - x, 0.2, KT), atol=1e-15)
    assert occ.fermi_dirac(np.array([1e3]), 0.0, KT)[0] == 0.0


@pytest.mark.parametrize("nk", [1, 3])
def test_fermi_level_meets_electron_count(nk):
    rng = np.random.default_rng(nk)
    thetas = [np.sort(rng.uniform(-40.0, 2.0, size=30 + 7 * k)) for k in range(nk)]
    wk = rng.uniform(0.5, 1.0, size=nk)
    wk = wk / wk.sum()
    for n_elec in (10.0, 33.3, 47.0):
        mu, it = occ.fermi_level(thetas, wk, n_elec, KT)
        assert it < 200
        assert abs(occ.electron_count(thetas, wk, mu, KT) - n_elec) <= 1e-12 * n_elec
    with pytest.raises(ValueError):
        occ.fermi_level(thetas, wk, 2.0 * sum(w * t.size for t, w in zip(thetas, wk)) + 1.0, KT)


def test_zero_temperature_limit_is_aufbau():
    rng = np.random.default_rng(4)
    th = np.sort(rng.uniform(-5.0, 5.0, size=40))
    th[20:] += 1.0  # a gap of at least 1 Ha between states 19 and 20
    kT = 1e-4
    mu, _ = occ.fermi_level([th], [1.0], 40.0, kT)
    assert th[19] < mu < th[20]
    f = occ.fermi_dirac(th, mu, kT)
    np.testing.assert_allclose(f, (np.arange(40) < 20).astype(float), atol=1e-12)
    assert abs(occ.band_energy([th], [1.0], [f]) - 2.0 * th[:20].sum()) <= 1e-10 * abs(th[:20]).sum()


def test_band_energy_equals_rayleigh_quotients_of_ritz_pairs():
    sysm = wl.single_atom()
    op = OEFEOperator(sysm)
    lam, U = np.linalg.eigh(op.dense())
    X = U[:, :12]
    th = np.array([x @ op.apply(x[:, None])[:, 0] for x in X.T])
    mu, _ = occ.fermi_level([th], [1.0], 9.0, KT)
    f = occ.fermi_dirac(th, mu, KT)
    e1 = occ.band_energy([th], [1.0], [f])
    e2 = adj.band_energy(op, X, 2.0 * f)
    assert abs(e1 - e2) <= 1e-11 * abs(e1)


def test_density_integrates_to_the_electron_count():
    sysm = wl.tiny_system(nc=2, p=2, n_atoms=1, seed=5)
    op = OEFEOperator(sysm)
    lam, U = np.linalg.eigh(op.dense())
    nv = 6
    X = U[:, :nv]
    mu, _ = occ.fermi_level([lam[:nv]], [1.0], 5.0, KT)
    wts = 2.0 * occ.fermi_dirac(lam[:nv], mu, KT)
    rho = occ.density(op, X, wts)
    assert np.all(rho >= 0.0)
    W = op.mesh.Wcell[None, :]
    # the quadrature integral of each |psi|^2 is its Gauss norm: the weighted sum of those norms
    gnorm = np.einsum("eqv,eq->v", np.abs(adj.fields_at_quad(op, X)) ** 2, np.broadcast_to(W, rho.shape))
    assert abs(np.sum(W * rho) - np.sum(wts * gnorm)) <= 1e-12 * np.sum(wts)
    # ... which differs from N_e only by the Gauss vs lumped (GLL) mass of the basis
    assert abs(np.sum(W * rho) - 5.0) < 0.05 * 5.0
