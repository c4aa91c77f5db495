"""Pins of the band energy and its gradients.

E is linear in V and quadratic in X, so central differences are exact up to
rounding: the FD error is about u |E| / h, which sets the tolerance.
"""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle.operator import OEFEOperator
from paper_2010_09701_amd import workloads as wl


def _system(kvec=None):
    return wl.tiny_system(nc=2, p=2, n_atoms=2, seed=7, L=5.0, r0=0.8, r1=2.0).with_k(kvec)


@pytest.mark.parametrize("kvec", [None, np.array([0.2, 0.3, -0.1])])
def test_grad_V_by_central_differences(kvec):
    sysm = _system(kvec)
    op = OEFEOperator(sysm)
    nv = 5
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (op.n_tot, nv))
    if kvec is not None:
        X = X + 1j * rng.uniform(-1, 1, (op.n_tot, nv))
    f = wl.occupations(nv, 3)
    g = adj.grad_V(op, X, f)
    hstep = 1e-5
    for seed in range(3):
        dV = wl.potential_perturbation(op.mesh.n_cells, op.mesh.nq, 100 + seed)
        Ep = adj.band_energy(OEFEOperator(sysm, V=op.V + hstep * dV), X, f)
        Em = adj.band_energy(OEFEOperator(sysm, V=op.V - hstep * dV), X, f)
        fd = (Ep - Em) / (2 * hstep)
        E = adj.band_energy(op, X, f)
        tol = 50 * np.finfo(float).eps * abs(E) / hstep
        assert abs(fd - np.sum(g * dV)) < tol, (fd, np.sum(g * dV), tol)


@pytest.mark.parametrize("kvec", [None, np.array([0.2, 0.3, -0.1])])
def test_grad_X_by_central_differences(kvec):
    op = OEFEOperator(_system(kvec))
    nv = 4
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (op.n_tot, nv)).astype(op.dtype)
    f = wl.occupations(nv, 3)
    G = adj.grad_X(op, X, f)
    hstep = 1e-5
    for seed in range(3):
        dX = np.random.default_rng(10 + seed).uniform(-1, 1, X.shape)
        fd = (adj.band_energy(op, X + hstep * dX, f) - adj.band_energy(op, X - hstep * dX, f)) / (2 * hstep)
        # real directional derivative = Re <G, dX> with PyTorch's complex convention
        assert abs(fd - np.real(np.sum(np.conj(G) * dX))) < 1e-6 * max(1, abs(fd))


def test_density_sums_to_gauss_norms():
    op = OEFEOperator(wl.single_atom())
    nv = 6
    X = np.linalg.eigh(op.dense())[1][:, :nv]  # smooth (low-energy) orthonormal states
    f = np.ones(nv)
    g = adj.grad_V(op, X, f)
    # sum_{e,q} dE/dV = sum_i f_i int_Gauss |psi_i|^2 = sum_i z_i^* M_gauss z_i
    Psi = op.basis_values_at_quad()
    W = np.tile(op.mesh.Wcell, op.mesh.n_cells)
    Z = np.concatenate([op.dm12[:, None] * X[:op.N], op.enr.S @ X[op.N:]], axis=0)
    ref = np.sum(W[:, None] * np.abs(Psi @ Z) ** 2)
    assert abs(g.sum() - ref) < 1e-11 * ref
    # and, to quadrature accuracy, the number of states (orthonormal in the lumped/GLL metric)
    assert abs(g.sum() - nv) < 0.05 * nv
