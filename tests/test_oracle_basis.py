"""Pins of the oracle's 1D rules, mesh, mass and cell stiffness.

Each check compares against something other than the oracle's own formula:
textbook node/weight values, exactness on monomials, polynomial integrals
done symbolically with numpy.polynomial, and counting identities.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

from oracle.mesh import Mesh
from oracle.quadrature import gauss_rule, gll_rule, lagrange_basis


def test_gll_textbook_values():
    x, w = gll_rule(2)
    np.testing.assert_allclose(x, [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], rtol=1e-14)
    x, w = gll_rule(4)
    s = np.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(x, [-1, -s, 0, s, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], rtol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_rules_exact_on_monomials(p):
    x, w = gll_rule(p)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(0, 2 * p):  # GLL exact to degree 2p - 1
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(w, x ** k) - exact) < 1e-13
    q = p + 1
    xg, wg = gauss_rule(q)
    for k in range(0, 2 * q):  # Gauss exact to degree 2q - 1
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(wg, xg ** k) - exact) < 1e-13


@pytest.mark.parametrize("p", [2, 3, 4])
def test_lagrange_basis(p):
    xi, _ = gll_rule(p)
    V, D = lagrange_basis(xi, xi)
    np.testing.assert_allclose(V, np.eye(p + 1), atol=1e-14)
    t = np.linspace(-1, 1, 11)
    V, D = lagrange_basis(xi, t)
    # reproduces polynomials of degree <= p and their derivatives
    for k in range(p + 1):
        np.testing.assert_allclose(V @ xi ** k, t ** k, atol=1e-13)
        np.testing.assert_allclose(D @ xi ** k, k * t ** max(k - 1, 0) if k > 0 else 0 * t, atol=1e-12)


def _exact_1d(p, h):
    """1D cell stiffness int l_a' l_b' and consistent mass int l_a l_b by exact polynomial integration."""
    xi, _ = gll_rule(p)
    polys = []
    for a in range(p + 1):
        roots = [xi[j] for j in range(p + 1) if j != a]
        c = P.polyfromroots(roots)
        c = c / P.polyval(xi[a], c)
        polys.append(c)
    K = np.zeros((p + 1, p + 1))
    M = np.zeros((p + 1, p + 1))
    for a in range(p + 1):
        for b in range(p + 1):
            kk = P.polyint(P.polymul(P.polyder(polys[a]), P.polyder(polys[b])))
            mm = P.polyint(P.polymul(polys[a], polys[b]))
            K[a, b] = (P.polyval(1, kk) - P.polyval(-1, kk)) * (2.0 / h)
            M[a, b] = (P.polyval(1, mm) - P.polyval(-1, mm)) * (h / 2.0)
    return K, M


@pytest.mark.parametrize("p", [2, 4])
def test_cell_stiffness_matches_exact_kronecker(p):
    h = 0.7
    mesh = Mesh(L=2 * h, nc=2, p=p)
    K1, M1 = _exact_1d(p, h)
    # local index a = ax + (p+1) ay + (p+1)^2 az -> kron(z, y, x)
    Kx = np.kron(M1, np.kron(M1, K1))
    Ky = np.kron(M1, np.kron(K1, M1))
    Kz = np.kron(K1, np.kron(M1, M1))
    Kexp = 0.5 * (Kx + Ky + Kz)
    Ke = mesh.cell_stiffness()
    np.testing.assert_allclose(Ke, Kexp, atol=1e-12 * np.abs(Kexp).max())
    # consistent mass by the Gauss rule = exact Kronecker mass
    Mg = mesh.B.T @ (mesh.Wcell[:, None] * mesh.B)
    np.testing.assert_allclose(Mg, np.kron(M1, np.kron(M1, M1)), atol=1e-14 * 10)


@pytest.mark.parametrize("nc,p", [(2, 2), (3, 4), (4, 3)])
def test_mesh_counts_and_mass(nc, p):
    L = 3.3
    mesh = Mesh(L, nc, p)
    counts = np.bincount(mesh.cell_dofs.ravel(), minlength=mesh.N)
    # every node belongs to 1, 2, 4 or 8 cells; total incidences = cells * (p+1)^3
    assert set(np.unique(counts)).issubset({1, 2, 4, 8})
    assert counts.sum() == mesh.n_cells * (p + 1) ** 3
    m = mesh.lumped_mass()
    assert abs(m.sum() - L ** 3) < 1e-12 * L ** 3
    assert np.all(m > 0)
    # closed form: m_g = (h/2)^3 prod_d w'_(i_d mod p), w'_0 = 2 w_0
    _, wh = gll_rule(p)
    wp = wh[:p].copy()
    wp[0] *= 2.0
    n = nc * p
    g = np.arange(mesh.N)
    ix, iy, iz = g % n, (g // n) % n, g // (n * n)
    mexp = (mesh.h / 2) ** 3 * wp[ix % p] * wp[iy % p] * wp[iz % p]
    np.testing.assert_allclose(m, mexp, rtol=1e-14)
    assert abs(mesh.quad_weights().sum() - L ** 3) < 1e-12 * L ** 3


def test_node_coordinates_match_cell_geometry():
    mesh = Mesh(5.0, 3, 4)
    X = mesh.node_coords()
    # the quadrature-free check: node coordinates of cell e, local a, equal origin + (xi+1) h/2 modulo L
    xi = mesh.ref.xi
    for e in [0, 5, 26]:
        for a in [0, 7, 124]:
            ax, ay, az = a % 5, (a // 5) % 5, a // 25
            expect = mesh.cell_origin[e] + (np.array([xi[ax], xi[ay], xi[az]]) + 1) * mesh.h / 2
            np.testing.assert_allclose(X[mesh.cell_dofs[e, a]], np.mod(expect, 5.0), atol=1e-12)
