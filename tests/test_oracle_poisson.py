"""Pins of the oracle's auxiliary-potential Poisson problem (oracle/poisson.py).

* The unit smeared charge integrates to one; v_g solves the radial Poisson equation
  -(1/4 pi) (1/r^2) (r^2 v')' = g inside rc (central differences) and joins 1/r at rc with its
  derivative; the model Hartree potential solves it for the model density and tends to Z/r.
* The smearing radii: half the nearest distance, including periodic images.
* A second route: A and c assembled from the values and gradients of every basis function at
  every quadrature point equal the cell-wise sparse assembly.
* A annihilates the constants (1 on the FE part), and the neutralized force vector sums to zero
  on the FE part; the solution satisfies A phi = c.
* The enriched problem contains the classical one, so its minimum of 1/2 phi^T A phi - c^T phi is
  no larger (a sign error in A^co or c^O breaks this).
* The discrete potential converges to the exact periodic potential (the absolutely convergent
  lattice sum of the atoms' neutral potentials) as the mesh is refined.
"""
import dataclasses

import numpy as np
import pytest

from oracle import poisson as po
from paper_2010_09701_amd import workloads as wl


def test_smeared_charge_normalization_and_potential():
    rc = 1.7
    x, w = np.polynomial.legendre.leggauss(60)
    r = 0.5 * rc * (x + 1.0)
    assert abs(np.sum(0.5 * rc * w * 4.0 * np.pi * r * r * po.g_smeared(r, rc)) - 1.0) < 1e-14
    assert po.g_smeared(np.array([rc * 1.0001]), rc)[0] == 0.0
    # -(1/4 pi) (1/r^2) d/dr (r^2 dv/dr) = g inside, from the analytic derivative by differences
    rr = np.linspace(0.2, rc - 0.05, 15)
    hh = 1e-5
    flux = lambda s: s * s * po.v_g(s, rc)[1]
    lap = (flux(rr + hh) - flux(rr - hh)) / (2 * hh) / rr ** 2
    np.testing.assert_allclose(-lap / (4 * np.pi), po.g_smeared(rr, rc), rtol=1e-7, atol=1e-9)
    # value and derivative continuous at rc, 1/r outside
    v_in, d_in = po.v_g(np.array([rc * (1 - 1e-13)]), rc)
    assert abs(v_in[0] - 1.0 / rc) < 1e-12 and abs(d_in[0] + 1.0 / rc ** 2) < 1e-11
    v_out, _ = po.v_g(np.array([2.5 * rc]), rc)
    assert abs(v_out[0] - 1.0 / (2.5 * rc)) < 1e-15
    # the derivative is the derivative of the value
    rr = np.linspace(0.1, 3.0, 30)
    num = (po.v_g(rr + 1e-6, rc)[0] - po.v_g(rr - 1e-6, rc)[0]) / 2e-6
    np.testing.assert_allclose(num, po.v_g(rr, rc)[1], rtol=1e-6, atol=1e-8)


def test_model_hartree_potential():
    Z, a = 14.0, po.model_alpha(14.0)
    rr = np.linspace(0.05, 6.0, 40)
    hh = 1e-5
    flux = lambda s: s * s * po.hartree_model(s, Z, a)[1]
    lap = (flux(rr + hh) - flux(rr - hh)) / (2 * hh) / rr ** 2
    np.testing.assert_allclose(-lap / (4 * np.pi), po.model_density(rr, Z, a), rtol=1e-6, atol=1e-9)
    num = (po.hartree_model(rr + 1e-6, Z, a)[0] - po.hartree_model(rr - 1e-6, Z, a)[0]) / 2e-6
    np.testing.assert_allclose(num, po.hartree_model(rr, Z, a)[1], rtol=1e-6, atol=1e-8)
    # far field Z/r, finite limit Z alpha / 2 at the nucleus (series branch)
    assert abs(po.hartree_model(np.array([12.0]), Z, a)[0][0] - Z / 12.0) < 1e-12
    assert abs(po.hartree_model(np.array([0.0]), Z, a)[0][0] - Z * a / 2) < 1e-12
    v_s = po.hartree_model(np.array([0.999e-3 / a]), Z, a)[0][0]
    v_c = po.hartree_model(np.array([1.001e-3 / a]), Z, a)[0][0]
    assert abs(v_s - v_c) < 1e-9 * Z * a


def test_smear_radii():
    pos = np.array([[1.0, 1.0, 1.0], [2.0, 1.0, 1.0], [5.5, 5.5, 5.5]])
    rc = po.smear_radii(pos, 6.0)
    np.testing.assert_allclose(rc, [0.5, 0.5, 0.5 * np.sqrt(3 * 1.5 ** 2)])
    assert po.smear_radii(np.array([[3.0, 3.0, 3.0]]), 6.0)[0] == 3.0  # own image at L


def _global_route(P, f):
    """A and c from the values / gradients of all basis functions at all quadrature points."""
    mesh = P.mesh
    nq, nd = mesh.nq, mesh.nd
    nrow = mesh.n_cells * nq
    val = np.zeros((nrow, P.n_tot))
    grad = np.zeros((3, nrow, P.n_tot))
    s = 2.0 / mesh.h
    for e in range(mesh.n_cells):
        rows = e * nq + np.arange(nq)
        for a in range(nd):
            g = mesh.cell_dofs[e, a]
            val[rows, g] += mesh.B[:, a]
            for d in range(3):
                grad[d, rows, g] += s * mesh.Gref[d][:, a]
    for I, (cells, Phi, gPhi) in enumerate(P.atoms):
        for ci, e in enumerate(cells):
            rows = e * nq + np.arange(nq)
            val[rows, P.N + I] = Phi[ci]
            for d in range(3):
                grad[d, rows, P.N + I] = gPhi[ci, :, d]
    Wr = np.tile(mesh.Wcell, mesh.n_cells)
    A = sum(grad[d].T @ (Wr[:, None] * grad[d]) for d in range(3)) / (4 * np.pi)
    c = val.T @ (Wr * f.ravel())
    return A, c


def _tiny(nc, p=2, Z=2.0):
    s = wl.tiny_system(nc=nc, p=p, n_atoms=2, seed=5, L=6.0, r0=1.0, r1=2.0)
    return dataclasses.replace(s, Z=np.full(2, Z))


def test_assembly_second_route_and_null_space():
    P = po.PoissonOEFE(_tiny(3, p=2))
    f = P.neutral_charge(P.model_electron_density())
    A2, c2 = _global_route(P, f)
    A = P.matrix().toarray()
    c = P.force_vector(f)
    assert np.abs(A - A2).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(c - c2).max() <= 1e-13 * np.abs(c).max()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    one = np.concatenate([np.ones(P.N), np.zeros(P.n_enr)])
    assert np.abs(A @ one).max() <= 1e-12 * np.abs(A).max()
    assert abs(c[:P.N].sum()) <= 1e-12 * np.abs(c).sum()
    phi = P.solve(f)
    assert np.linalg.norm(A @ phi - c) <= 1e-11 * np.linalg.norm(c)
    assert abs((P.m * phi[:P.N]).sum()) <= 1e-12 * np.abs(phi).sum()


@pytest.mark.parametrize("Z", [2.0, 14.0])
def test_enriched_energy_not_above_classical(Z):
    sysm = _tiny(4, p=3, Z=Z)
    e = []
    for enr in (True, False):
        P = po.PoissonOEFE(sysm, enrich=enr)
        f = P.neutral_charge(P.model_electron_density())
        phi = P.solve(f)
        c = P.force_vector(f)
        e.append(0.5 * phi @ (P.matrix() @ phi) - c @ phi)
    assert e[0] <= e[1] + 1e-12 * abs(e[1])
    assert e[0] < e[1]  # the enrichment adds something


def test_converges_to_exact_periodic_potential():
    errs = []
    for nc in (2, 3, 4, 6):
        sysm = _tiny(nc, p=4)
        P = po.PoissonOEFE(sysm)
        phi = P.solve(P.neutral_charge(P.model_electron_density()))
        fq = P.field_at_quad(phi)
        ex = po.exact_potential(P.mesh.quad_points(), sysm, P.rc, P.alpha)
        W = P.mesh.Wcell[None, :]
        vol = W.sum() * P.mesh.n_cells
        e = (fq - (W * fq).sum() / vol) - (ex - (W * ex).sum() / vol)
        errs.append(np.sqrt((W * e * e).sum() / vol))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3 and errs[-1] < errs[0] / 20
