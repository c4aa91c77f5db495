"""Pins of the oracle's adaptive quadrature for the enrichment integrals (oracle/adaptive.py).

* The radial whole-space integrals (the refinement's scales) against closed forms: with the
  cutoff far outside the function, int exp(-2 zeta r) = pi / zeta^3, int |grad exp(-zeta r)|^2
  = pi / zeta, int (x exp(-zeta r))^2 = pi / zeta^5, int |grad (x exp(-zeta r))|^2 = pi / zeta^3.
* The leaves of every cell tile the cell (volumes and weights sum to h^3; a polynomial of
  degree 2q - 1 per direction is integrated exactly), and every point lies in its cell.
* The total of each trial integral over the rule equals the radial whole-space integral (the
  supports cover the function) ever more closely as the tolerance and depth grow, while the
  plain Gauss rule misses it by tens of percent for a sharp function.
* max_depth = 0: one leaf per cell, and the operator's enrichment blocks and its N^O at the
  Gauss points equal those of the Gauss-rule operator (oracle/enrichment.py) at Gamma and at a
  Bloch k.
* With refinement: M^oo, H^oo, H^co approach those of the rule with tol = 0 (every box where
  the functions do not vanish split to the same depth) as tol falls: at tol = 1e-7 to 1e-8 with
  V = 0 (the trial integrals cover every integrand), to 2e-6 with the nuclear potential (V is
  not among the trial integrals); M^oo stays Hermitian positive definite.
* The periodic-function k-point form on the rule: max_depth = 0 gives the blocks of
  oracle/uform.py; at k = 0 the blocks equal the Gamma-point operator's on the same rule; M^oo
  and H^oo are Hermitian.
* The auxiliary-potential Poisson problem on a rule built from its own enrichment functions:
  max_depth = 0 gives oracle/poisson.py's A^co, A^oo and force vector; A stays symmetric and
  annihilates the FE constant; A^co, A^oo and the enrichment rows of the force vector converge to
  the fully refined rule's as tol falls (1e-6 at tol 1e-8: the charge is not among the trial
  integrals), and the solution with them.
"""
import dataclasses

import numpy as np
import pytest

from oracle import adaptive as ad
from oracle.mesh import Mesh
from oracle.operator import OEFEOperator
from oracle.enrichment import atomic_function
from oracle.potential import min_image
from paper_2010_09701_amd import workloads as wl

K = np.array([0.21, -0.13, 0.07])


def _sharp(nc=3, p=3, seed=3):
    s = wl.tiny_system(nc=nc, p=p, n_atoms=1, seed=seed, L=6.0, r0=1.0, r1=2.0)
    return dataclasses.replace(s, enr=[wl.EnrichmentFn(0, 0, 6.0, -1), wl.EnrichmentFn(0, 1, 3.0, 0)])


def test_radial_scales_closed_forms():
    z = 2.0
    for fn, A, B in ((wl.EnrichmentFn(0, 0, z, -1), np.pi / z ** 3, np.pi / z),
                     (wl.EnrichmentFn(0, 0, z, 0), np.pi / z ** 5, np.pi / z ** 3)):
        a, b = ad.radial_scales(fn, 29.0, 30.0)
        assert abs(a / A - 1) < 1e-12 and abs(b / B - 1) < 1e-12


def test_leaves_tile_the_cells():
    s = _sharp()
    mesh = Mesh(s.L, s.nc, s.p)
    R = ad.AdaptiveRule(mesh, s, 1e-6, 3)
    h3 = mesh.h ** 3
    assert max(len(v) for v in R.leaves.values()) > 8  # refinement happened near the nucleus
    for e in R.cells.tolist():
        vol = sum(sz ** 3 for (_, sz) in R.leaves[e])
        assert abs(vol - h3) <= 1e-13 * h3
        assert abs(R.weights[e].sum() - h3) <= 1e-13 * h3
        x = R.points[e] - mesh.cell_origin[e][None, :]
        assert x.min() > 0 and x.max() < mesh.h
        # x^(2q-1) y^(2q-2) z: exact under every leaf's Gauss rule
        q = mesh.q1
        f = x[:, 0] ** (2 * q - 1) * x[:, 1] ** (2 * q - 2) * x[:, 2]
        exact = mesh.h ** (2 * q) / (2 * q) * mesh.h ** (2 * q - 1) / (2 * q - 1) * mesh.h ** 2 / 2
        assert abs((R.weights[e] * f).sum() / exact - 1) < 1e-12


def _trial_totals(s, R):
    P, W = R.all_points(), R.all_weights()
    out = []
    for fn in s.enr:
        d = min_image(P - s.pos[fn.atom][None, :], s.L)
        v, g = atomic_function(d, fn.power, fn.zeta, fn.axis, s.r0, s.r1)
        A, B = ad.radial_scales(fn, s.r0, s.r1)
        out.append(((W * v * v).sum() / A - 1, (W * (g * g).sum(-1)).sum() / B - 1))
    return np.abs(np.array(out)).max()


def test_trial_totals_converge_to_whole_space_integrals():
    s = _sharp()
    mesh = Mesh(s.L, s.nc, s.p)
    errs = [_trial_totals(s, ad.AdaptiveRule(mesh, s, tol, depth)) for tol, depth in ((1e-2, 0), (1e-4, 1), (1e-5, 2), (1e-6, 3))]
    assert errs[0] > 0.1  # the plain Gauss rule: tens of percent off for exp(-12 r)
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 2e-3, errs  # depth-limited at the nucleus (the cusp of exp(-6 r)): 1.4e-3 at depth 3


@pytest.mark.parametrize("kvec", [None, K])
def test_depth0_is_the_gauss_operator(kvec):
    s = wl.tiny_system(nc=3, p=2, n_atoms=2, seed=7, L=5.0, r0=0.8, r1=2.0)
    if kvec is not None:
        s = s.with_k(kvec)
    g = OEFEOperator(s)
    a = ad.AdaptiveOEFEOperator(s, 1e-6, 0)
    assert a.rule.n_points == a.rule.cells.size * a.mesh.nq
    for X, Y in ((a.enr.Moo, g.enr.Moo), (a.enr.Hoo, g.enr.Hoo), (a.enr.Hco.toarray(), g.enr.Hco.toarray())):
        assert np.abs(X - Y).max() <= 1e-13 * np.abs(Y).max()
    # N^O at the Gauss points (the fields' enrichment part) equal the Gauss-rule oracle's
    for (I, idx, cells, Phi, gPhi), (J, jdx, cj, Pg, gPg) in zip(a.enr.atom_fn, g.enr.atom_fn):
        assert I == J and np.array_equal(cells, cj)
        assert np.abs(Phi - Pg).max() <= 1e-13 * np.abs(Pg).max()
        assert np.abs(gPhi - gPg).max() <= 1e-13 * np.abs(gPg).max()


@pytest.mark.parametrize("kvec,zero_v,bound", [(None, True, 1e-8), (K, False, 2e-6)])
def test_blocks_approach_uniform_refinement(kvec, zero_v, bound):
    s = _sharp(nc=3, p=2)
    if kvec is not None:
        s = s.with_k(kvec)
    mesh = Mesh(s.L, s.nc, s.p)

    def op(tol):
        if not zero_v:
            return ad.AdaptiveOEFEOperator(s, tol, 2)
        n = ad.AdaptiveRule(mesh, s, tol, 2).n_points
        return ad.AdaptiveOEFEOperator(s, tol, 2, V=np.zeros((mesh.n_cells, mesh.nq)), V_adapt=np.zeros(n))

    ref = op(0.0)  # every box where the functions do not vanish split twice
    errs = []
    for tol in (1e-2, 1e-4, 1e-7):
        a = op(tol)
        assert a.rule.n_points <= ref.rule.n_points
        e = 0.0
        for X, Y in ((a.enr.Moo, ref.enr.Moo), (a.enr.Hoo, ref.enr.Hoo), (a.enr.Hco.toarray(), ref.enr.Hco.toarray())):
            e = max(e, np.abs(X - Y).max() / np.abs(Y).max())
        errs.append(e)
        M = a.enr.Moo
        assert np.abs(M - M.conj().T).max() <= 1e-14 * np.abs(M).max()
        assert np.linalg.eigvalsh(M).min() > 0
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < bound, errs


def test_uform_depth0_is_the_uform_operator():
    from oracle.uform import UFormOperator
    s = wl.tiny_system(nc=3, p=2, n_atoms=2, seed=7, L=5.0, r0=0.8, r1=2.0).with_k(K)
    u = UFormOperator(s, K)
    a = ad.AdaptiveUFormOperator(s, K, 1e-6, 0)
    for X, Y in ((a.Moo, u.Moo), (a.Hoo, u.Hoo), (a.Hco.toarray(), u.Hco.toarray())):
        assert np.abs(X - Y).max() <= 1e-13 * np.abs(Y).max()


def test_uform_adaptive_hermitian_and_k0_is_gamma():
    s = _sharp(nc=3, p=2)
    a = ad.AdaptiveUFormOperator(s.with_k(K), K, 1e-5, 2)
    assert np.abs(a.Hoo - a.Hoo.conj().T).max() <= 1e-13 * np.abs(a.Hoo).max()
    assert np.abs(a.Moo - a.Moo.conj().T).max() <= 1e-14 * np.abs(a.Moo).max()
    z = ad.AdaptiveUFormOperator(s.with_k(np.zeros(3)), np.zeros(3), 1e-5, 2)
    g = ad.AdaptiveOEFEOperator(s, 1e-5, 2)
    for X, Y in ((z.Moo, g.enr.Moo), (z.Hoo, g.enr.Hoo), (z.Hco.toarray(), g.enr.Hco.toarray())):
        assert np.abs(X - Y).max() <= 1e-13 * np.abs(Y).max()


def _pois_sys(nc=3, p=3, Z=14.0):
    s = wl.tiny_system(nc=nc, p=p, n_atoms=2, seed=5, L=8.0, r0=2.0, r1=3.5)
    return dataclasses.replace(s, Z=np.full(2, Z))


def test_poisson_depth0_is_the_gauss_rule_problem():
    from oracle import poisson as po
    s = _pois_sys()
    g = po.PoissonOEFE(s)
    a = ad.AdaptivePoissonOEFE(s, 1e-6, 0)
    assert a.rule.n_points == a.rule.cells.size * a.mesh.nq
    assert np.abs(a.Aco.toarray() - g.Aco.toarray()).max() <= 1e-13 * np.abs(g.Aco.toarray()).max()
    assert np.abs(a.Aoo - g.Aoo).max() <= 1e-13 * np.abs(g.Aoo).max()
    rho = g.model_electron_density()
    c = a.force_vector(rho, a.model_density_at(a.rule.all_points()))
    cg = g.force_vector(g.neutral_charge(rho))
    assert np.abs(c - cg).max() <= 1e-12 * np.abs(cg).max()


def test_poisson_adaptive_converges_and_keeps_the_null_space():
    s = _pois_sys()
    ref = ad.AdaptivePoissonOEFE(s, 0.0, 2)  # every box where the functions do not vanish split twice
    rho = ref.base.model_electron_density()

    def blocks_and_phi(P):
        c = P.force_vector(rho, P.model_density_at(P.rule.all_points()))
        return P.Aco.toarray(), P.Aoo, c[P.N:], P.solve(rho, P.model_density_at(P.rule.all_points()))

    Ar, Or, cr, pr = blocks_and_phi(ref)
    errs, perr = [], []
    for tol in (1e-2, 1e-5, 1e-8):
        P = ad.AdaptivePoissonOEFE(s, tol, 2)
        A, O, c, phi = blocks_and_phi(P)
        errs.append(max(np.abs(A - Ar).max() / np.abs(Ar).max(), np.abs(O - Or).max() / np.abs(Or).max(),
                        np.abs(c - cr).max() / np.abs(cr).max()))
        perr.append(np.abs(phi - pr).max() / np.abs(pr).max())
        M = P.matrix().toarray()
        assert np.abs(M - M.T).max() <= 1e-14 * np.abs(M).max()
        one = np.concatenate([np.ones(P.N), np.zeros(P.n_enr)])
        assert np.abs(M @ one).max() <= 1e-12 * np.abs(M).max()
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6, errs  # the charge in c^O is not a trial integral
    assert perr[0] > perr[2] and perr[2] < 1e-6, perr
