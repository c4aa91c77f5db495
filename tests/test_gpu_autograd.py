"""Band-energy adjoint through torch.autograd (library kernels) against the oracle and
central finite differences of the library's own float64 energy.

E is linear in V and quadratic in X, so central differences are exact up to
rounding: the FD error is ~ u |E| / h, which sets the tolerance.
"""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle.operator import OEFEOperator
from paper_2010_09701_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available()
    from paper_2010_09701_amd import autograd, oefe
    return torch, oefe, autograd


@pytest.mark.parametrize("kvec", [None, np.array([0.2, 0.3, -0.1])])
def test_autograd_matches_oracle(mods, kvec):
    torch, oefe, ag = mods
    sysm = wl.tiny_system(nc=2, p=2, n_atoms=2, seed=7, L=5.0, r0=0.8, r1=2.0).with_k(kvec)
    op = OEFEOperator(sysm)
    gop = oefe.Operator(sysm)
    nv = 4
    X = wl.start_block(op.n_tot, nv, 1, complex_=kvec is not None)
    f = wl.occupations(nv, 3)
    V = op.V.copy()
    Xt = torch.from_numpy(X).cuda().requires_grad_(True)
    Vt = torch.from_numpy(V).requires_grad_(True)
    E = ag.band_energy(Xt, Vt, torch.from_numpy(f), gop)
    E.backward()
    E = float(E.detach())
    assert abs(E - adj.band_energy(op, X, f)) < 1e-10 * abs(E)
    gv = adj.grad_V(op, X, f)
    np.testing.assert_allclose(Vt.grad.numpy(), gv, rtol=1e-9, atol=1e-12 * np.abs(gv).max())
    gx = adj.grad_X(op, X, f)
    np.testing.assert_allclose(Xt.grad.cpu().numpy(), gx, rtol=1e-9, atol=1e-11 * np.abs(gx).max())


def test_potential_gradient_by_central_differences(mods):
    """16 random potential perturbations, h = 1e-5, on the single-atom workload at its Ritz vectors."""
    torch, oefe, ag = mods
    from paper_2010_09701_amd.chfsi import chfsi_run
    cfg = wl.config("single_atom")
    gop = oefe.Operator(cfg.system)
    X0 = torch.from_numpy(wl.start_block(gop.n_tot, cfg.nv, 0)).cuda()
    v0 = torch.from_numpy(wl.lanczos_start(gop.n_tot, 2)).cuda()
    X = chfsi_run(gop, X0, v0, cfg.m, cfg.passes, cfg.lanczos_k)["X"]
    f = torch.full((cfg.nv,), 2.0, dtype=torch.float64)
    V0, _ = gop.get_potential()
    Vt = torch.from_numpy(V0.copy()).requires_grad_(True)
    E = ag.band_energy(X, Vt, f, gop)
    E.backward()
    g = Vt.grad.numpy()
    h = 1e-5
    for j in range(16):
        dV = wl.potential_perturbation(gop.n_cells, gop.nq, 100 + j)
        gop.set_potential(V0 + h * dV)
        Ep = float(oefe.band_energy_grad(gop, X, f, want_dV=False, want_dX=False)[0])
        gop.set_potential(V0 - h * dV)
        Em = float(oefe.band_energy_grad(gop, X, f, want_dV=False, want_dX=False)[0])
        fd = (Ep - Em) / (2 * h)
        tol = 100 * np.finfo(float).eps * abs(float(E)) / h
        assert abs(fd - np.sum(g * dV)) < tol, (j, fd, np.sum(g * dV), tol)
    gop.set_potential(V0)


def test_vector_gradient_by_central_differences(mods):
    torch, oefe, ag = mods
    sysm = wl.diamond8(nc=4, p=4)
    gop = oefe.Operator(sysm)
    nv = 12
    X = torch.from_numpy(wl.start_block(gop.n_tot, nv, 4)).cuda().requires_grad_(True)
    f = torch.from_numpy(wl.occupations(nv, 3))
    V0, _ = gop.get_potential()
    E = ag.band_energy(X, torch.from_numpy(V0), f, gop)
    E.backward()
    G = X.grad.cpu().numpy()
    h = 1e-5
    for j in range(4):
        dX = torch.from_numpy(np.random.default_rng(50 + j).uniform(-1, 1, X.shape)).cuda()
        Ep = float(oefe.band_energy_grad(gop, (X + h * dX).detach(), f, False, False)[0])
        Em = float(oefe.band_energy_grad(gop, (X - h * dX).detach(), f, False, False)[0])
        fd = (Ep - Em) / (2 * h)
        an = float(np.sum(G * dX.cpu().numpy()))
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (fd, an)


def test_gradcheck_tiny_complex(mods):
    torch, oefe, ag = mods
    sysm = wl.tiny_system(nc=2, p=2, n_atoms=1, seed=3, L=4.0, r0=0.7, r1=1.5).with_k(np.array([0.3, 0.1, 0.2]))
    gop = oefe.Operator(sysm)
    V0, _ = gop.get_potential()
    Vt = torch.from_numpy(V0.copy())
    f = torch.tensor([2.0, 0.5], dtype=torch.float64)
    X = torch.from_numpy(wl.start_block(gop.n_tot, 2, 8, complex_=True)).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: ag.band_energy(x, Vt, f, gop), (X,), eps=1e-6, atol=1e-5, rtol=1e-4)
