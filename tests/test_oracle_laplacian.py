"""V = 0, no enrichment: the operator is the periodic FE Laplacian.

Semi-closed form (Bloch reduction on the uniform periodic mesh): the spectrum
of D^-1/2 H D^-1/2 is the union over Bloch angles theta_d = (2 pi j_d + k_d L)
/ nc of the p^3 x p^3 problems with H(theta) = 1/2 [K1 (x) M1 (x) M1 + ...]
(exact 1D stiffness and consistent mass from polynomial integrals) and the
lumped diagonal mass.  Also the continuum limit 1/2 (2 pi / L)^2 |n|^2 with an
error that decays like h^(2p) (the rate the paper reports for energies in its
convergence study).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.operator import OEFEOperator
from oracle.quadrature import gll_rule
from paper_2010_09701_amd import workloads as wl
from test_oracle_basis import _exact_1d


def _bloch_spectrum(L, nc, p, kvec=None):
    h = L / nc
    K1, M1 = _exact_1d(p, h)
    _, wh = gll_rule(p)
    ML = np.diag(wh) * (h / 2)

    def reduce(A, th):
        R = np.zeros((p, p), dtype=complex)
        ph = np.array([1.0] * p + [np.exp(1j * th)])
        for a in range(p + 1):
            for b in range(p + 1):
                R[a % p, b % p] += np.conj(ph[a]) * A[a, b] * ph[b]
        return R

    k = np.zeros(3) if kvec is None else np.asarray(kvec)
    out = []
    for jz in range(nc):
        for jy in range(nc):
            for jx in range(nc):
                th = [(2 * np.pi * j + k[d] * L) / nc for d, j in enumerate((jx, jy, jz))]
                Kr = [reduce(K1, t) for t in th]
                Mr = [reduce(M1, t) for t in th]
                Lr = [np.real(np.diag(reduce(ML, t))) for t in th]
                H = 0.5 * (np.kron(Mr[2], np.kron(Mr[1], Kr[0])) + np.kron(Mr[2], np.kron(Kr[1], Mr[0]))
                           + np.kron(Kr[2], np.kron(Mr[1], Mr[0])))
                m = np.kron(Lr[2], np.kron(Lr[1], Lr[0]))
                d = 1 / np.sqrt(m)
                out.append(np.linalg.eigvalsh(d[:, None] * H * d[None, :]))
    return np.sort(np.concatenate(out))


@pytest.mark.parametrize("nc,p", [(2, 2), (3, 2), (2, 4)])
def test_free_spectrum_equals_bloch_reduction(nc, p):
    L = 4.0
    op = OEFEOperator(wl.free_system(L, nc, p))
    lam = np.linalg.eigvalsh(op.dense())
    ref = _bloch_spectrum(L, nc, p)
    np.testing.assert_allclose(lam, ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("nc,p", [(3, 2), (2, 3)])
def test_free_spectrum_at_k_equals_bloch_reduction(nc, p):
    L = 4.0
    k = np.array([0.3, -0.2, 0.45])
    op = OEFEOperator(wl.free_system(L, nc, p).with_k(k))
    H = op.dense()
    assert np.abs(H - np.conj(H.T)).max() < 1e-13 * np.abs(H).max()
    lam = np.linalg.eigvalsh(H)
    ref = _bloch_spectrum(L, nc, p, k)
    np.testing.assert_allclose(lam, ref, atol=1e-12 * np.abs(ref).max())


def test_constant_is_null_vector():
    op = OEFEOperator(wl.free_system(5.0, 3, 4))
    x = np.sqrt(op.m)  # M^1/2 * 1 in the symmetric form
    y = op.apply(x)
    assert np.abs(y).max() < 1e-12 * np.abs(op.apply(np.random.default_rng(0).standard_normal(op.n_tot))).max()


def test_continuum_limit_rate():
    L, p = 2 * np.pi, 2
    errs = []
    for nc in (4, 8):
        op = OEFEOperator(wl.free_system(L, nc, p))
        H = op.hcc_csr()
        D = op.dm12
        import scipy.sparse as sp
        Ht = sp.diags(D) @ H @ sp.diags(D)
        vals = np.sort(spla.eigsh(Ht, k=8, sigma=-0.1, which="LM")[0])
        # lowest nonzero continuum eigenvalue 1/2 (2 pi / L)^2 = 0.5, six-fold
        assert abs(vals[0]) < 1e-10
        errs.append(np.abs(vals[1:7] - 0.5).max())
    rate = np.log2(errs[0] / errs[1])
    assert 2 * p - 0.6 < rate < 2 * p + 0.6, (errs, rate)
