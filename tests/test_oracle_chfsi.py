"""Pins of the oracle's filter, orthonormalization, Rayleigh-Ritz and bounds.

* filter on eigenvectors equals T_m(tau_i) / T_m(tau(a0)) from the closed forms
  cos(m acos t) / cosh(m acosh t) (no recurrence);
* the scaled recurrence equals the plain Chebyshev recurrence divided by one
  scalar;
* Cholesky-Gram-Schmidt against LAPACK QR (sign-fixed R), orthogonality and span;
* Rayleigh-Ritz values against direct eigvalsh, Courant-Fischer bounds;
* Lanczos bound b >= lambda_max (and close to it);
* the paper-literal path (filter p_m(M^-1 H) on u-coefficients, Euclidean QR,
  generalized projected problem Q*HQ, Q*MQ) gives the same Ritz values.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import chfsi as ch
from oracle.operator import OEFEOperator
from paper_2010_09701_amd import workloads as wl


@pytest.fixture(scope="module")
def atom_op():
    op = OEFEOperator(wl.single_atom())
    H = op.dense()
    lam, U = np.linalg.eigh(H)
    return op, H, lam, U


def test_filter_on_eigenvectors_matches_closed_form(atom_op):
    op, H, lam, U = atom_op
    m, a0, a, b = 20, lam[0], lam[30], lam[-1] * 1.01
    Y = ch.chebyshev_filter(op.apply, U, m, a, b, a0)
    e, c = (b - a) / 2, (b + a) / 2
    gain = ch.chebyshev_T(m, (lam - c) / e) / ch.chebyshev_T(m, np.array([(a0 - c) / e]))[0]
    np.testing.assert_allclose(Y, U * gain[None, :], atol=1e-11 * np.abs(gain).max())


def test_filter_on_diagonal_operator():
    rng = np.random.default_rng(0)
    lam = np.sort(rng.uniform(-3, 50, 300))
    X = rng.standard_normal((300, 5))
    m, a0, a, b = 37, lam[0], lam[20], 51.0
    Y = ch.chebyshev_filter(lambda Z: lam[:, None] * Z if Z.ndim == 2 else lam * Z, X, m, a, b, a0)
    e, c = (b - a) / 2, (b + a) / 2
    gain = ch.chebyshev_T(m, (lam - c) / e) / ch.chebyshev_T(m, np.array([(a0 - c) / e]))[0]
    np.testing.assert_allclose(Y, gain[:, None] * X, rtol=1e-11, atol=1e-13)


def test_scaled_equals_unscaled_over_scalar(atom_op):
    op, H, lam, U = atom_op
    rng = np.random.default_rng(1)
    X = rng.standard_normal((op.n_tot, 4))
    m, a0, a, b = 12, lam[0], lam[40], lam[-1] * 1.02
    e, c = (b - a) / 2, (b + a) / 2
    T0, T1 = X, (H @ X - c * X) / e
    for _ in range(1, m):
        T0, T1 = T1, 2 * (H @ T1 - c * T1) / e - T0
    Ys = ch.chebyshev_filter(op.apply, X, m, a, b, a0)
    scal = ch.chebyshev_T(m, np.array([(a0 - c) / e]))[0]
    np.testing.assert_allclose(Ys * scal, T1, rtol=1e-10, atol=1e-10 * np.abs(T1).max())
    # identical orthonormal factor after CholGS (up to column signs)
    Q1, _ = ch.cholgs(Ys)
    Q2, _ = ch.cholgs(T1)
    np.testing.assert_allclose(np.abs(Q1.T @ Q2), np.eye(4), atol=1e-8)


def test_cholgs_against_qr():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((400, 12)) @ np.diag(np.logspace(0, 5, 12))
    Q, rep = ch.cholgs(Y)
    np.testing.assert_allclose(Q.T @ Q, np.eye(12), atol=1e-13)
    Qr, Rr = np.linalg.qr(Y)
    s = np.sign(np.diag(Rr))
    np.testing.assert_allclose(Q, Qr * s[None, :], atol=1e-10)
    _, L = ch.cholgs_once(Y)
    np.testing.assert_allclose(L.T, Rr * s[:, None], rtol=1e-10, atol=1e-10 * np.abs(Rr).max())


def test_cholgs_breakdown_reports_column():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((50, 6))
    Y[:, 4] = Y[:, 1] + Y[:, 2]
    with pytest.raises(ch.CholeskyBreakdown) as ei:
        ch.cholgs(Y)
    assert ei.value.column == 4


def test_rayleigh_ritz_and_courant_fischer(atom_op):
    op, H, lam, U = atom_op
    rng = np.random.default_rng(4)
    Q, _ = ch.cholgs(rng.standard_normal((op.n_tot, 10)))
    th, X = ch.rayleigh_ritz(op.apply, Q)
    np.testing.assert_allclose(th, np.linalg.eigvalsh(Q.T @ H @ Q), atol=1e-11 * abs(lam).max())
    assert np.all(th >= lam[:10] - 1e-10)
    np.testing.assert_allclose(X.T @ X, np.eye(10), atol=1e-12)


def test_lanczos_bounds(atom_op):
    op, H, lam, U = atom_op
    v0 = wl.lanczos_start(op.n_tot, 2)
    a0, b, alpha, beta = ch.lanczos_bounds(op.apply, v0, 10)
    assert b >= lam[-1]
    assert b <= lam[-1] * 1.05
    assert a0 >= lam[0] - 1e-10


def test_chfsi_converges_and_bounds_hold(atom_op):
    op, H, lam, U = atom_op
    cfg = wl.config("single_atom")
    X0 = wl.start_block(op.n_tot, cfg.nv, 0)
    v0 = wl.lanczos_start(op.n_tot, 2)
    r = ch.chfsi(op.apply, X0, v0, cfg.m, cfg.passes, cfg.lanczos_k)
    for p in r["passes"]:
        assert np.all(p["theta"] >= lam[:cfg.nv] - 1e-10)
    # the lowest 5 Ritz values (well separated from the cut) have converged
    np.testing.assert_allclose(r["theta"][:5], lam[:5], atol=1e-7)


def test_paper_literal_u_space_path_gives_same_ritz_values(atom_op):
    """u-space: filter p_m(M^-1 H), Euclidean QR, generalized RR (Q*HQ, Q*MQ)."""
    op, H, lam, U = atom_op
    Hg, Mg = op.dense_generalized()
    Minv = np.linalg.inv(Mg)
    A = Minv @ Hg
    w, Vm = np.linalg.eigh(Mg)
    Mh = (Vm * np.sqrt(w)) @ Vm.T
    Mmh = (Vm / np.sqrt(w)) @ Vm.T
    rng = np.random.default_rng(5)
    Yy = rng.standard_normal((op.n_tot, 8))
    Yu = Mmh @ Yy
    m, a0, a, b = 15, lam[0], lam[20], lam[-1] * 1.01
    Fy = ch.chebyshev_filter(op.apply, Yy, m, a, b, a0)
    Fu = ch.chebyshev_filter(lambda Z: A @ Z, Yu, m, a, b, a0)
    Qy, _ = ch.cholgs(Fy)
    th_y, _ = ch.rayleigh_ritz(op.apply, Qy)
    Qu, _ = np.linalg.qr(Fu)
    th_u = sla.eigh(Qu.T @ Hg @ Qu, Qu.T @ Mg @ Qu, eigvals_only=True)
    np.testing.assert_allclose(th_y, th_u, atol=1e-10 * abs(lam).max())
