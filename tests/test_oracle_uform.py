"""Pins of the oracle's periodic-function (u) form of the k-point Hamiltonian (oracle/uform.py).

* k = 0: the u-form operator is the Gamma-point operator of operator.OEFEOperator.
* Hermitian at k != 0 (the first-derivative term's assembled matrix is anti-symmetric).
* A second route: H and M^oo from the values and gradients of every basis function at every
  quadrature point, with eqnHOEFEelelements written out (its first-derivative term in the
  Hermitian form), equal the assembled blocks.
* Free electrons (no atoms, V = 0): the constant function is an exact eigenvector with
  eigenvalue |k|^2/2, and the lowest levels approach the plane waves' |k + G|^2/2 (G on the
  reciprocal lattice 2 pi/L Z^3) with refinement.
* With atoms, the u-form and the Bloch-function (phase-twisted basis) form discretize the same
  operator: their lowest eigenvalues approach each other as the mesh is refined.
"""
import numpy as np

from oracle.operator import OEFEOperator
from oracle.uform import UFormOperator
from paper_2010_09701_amd import workloads as wl

K = np.array([0.21, -0.13, 0.07])


def _sys(nc=2, p=2):
    return wl.tiny_system(nc=nc, p=p, n_atoms=2, seed=7, L=5.0, r0=0.8, r1=2.0)


def test_k0_is_gamma_operator():
    s = _sys()
    a = UFormOperator(s, np.zeros(3)).dense()
    b = OEFEOperator(s).dense()
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_hermitian():
    H = UFormOperator(_sys(), K).dense()
    assert np.abs(H - H.conj().T).max() <= 1e-13 * np.abs(H).max()


def test_second_route():
    s = _sys()
    op = UFormOperator(s, K)
    mesh = op.mesh
    nq, nd = mesh.nq, mesh.nd
    nrow = mesh.n_cells * nq
    val = np.zeros((nrow, op.n_tot), dtype=np.complex128)
    grad = np.zeros((3, nrow, op.n_tot), dtype=np.complex128)
    sc = 2.0 / mesh.h
    for e in range(mesh.n_cells):
        rows = e * nq + np.arange(nq)
        for a in range(nd):
            g = mesh.cell_dofs[e, a]
            val[rows, g] += mesh.B[:, a]
            for d in range(3):
                grad[d, rows, g] += sc * mesh.Gref[d][:, a]
    for (idx, cells, Phi, gPhi) in op.atom_fn:
        for ci, e in enumerate(cells):
            rows = e * nq + np.arange(nq)
            val[np.ix_(rows, op.N + idx)] = Phi[ci]
            for d in range(3):
                grad[d][np.ix_(rows, op.N + idx)] = gPhi[ci, :, :, d]
    Wr = np.tile(mesh.Wcell, mesh.n_cells)
    Vr = op.V.ravel() + 0.5 * K @ K
    H = sum(0.5 * grad[d].conj().T @ (Wr[:, None] * grad[d]) for d in range(3))
    # the first-derivative term in its Hermitian form (the written form on FE-FE pairs, exactly)
    H += sum(-0.5j * K[d] * (val.conj().T @ (Wr[:, None] * grad[d]) - grad[d].conj().T @ (Wr[:, None] * val))
             for d in range(3))
    H += val.conj().T @ ((Wr * Vr)[:, None] * val)
    N = op.N
    scale = np.abs(H).max()
    assert np.abs(H[:N, :N] - op.Hcc.toarray()).max() <= 1e-12 * scale
    assert np.abs(H[:N, N:] - op.Hco.toarray()).max() <= 1e-12 * scale
    assert np.abs(H[N:, N:] - op.Hoo).max() <= 1e-12 * scale
    Moo = val[:, N:].conj().T @ (Wr[:, None] * val[:, N:])
    assert np.abs(Moo - op.Moo).max() <= 1e-13 * np.abs(op.Moo).max()


def test_free_electrons():
    L = 6.0
    errs = []
    for nc in (2, 3, 4):
        s = wl.free_system(L, nc, 3)
        op = UFormOperator(s, K)
        lam, U = np.linalg.eigh(op.dense())
        assert abs(lam[0] - 0.5 * K @ K) <= 1e-12
        u = op.dm12 * U[:, 0]  # the coefficients of u: M^-1/2 y
        assert np.abs(u / u[0] - 1.0).max() <= 1e-10
        G = 2.0 * np.pi / L
        exact = sorted(0.5 * np.sum((K + G * np.array([i, j, l])) ** 2)
                       for i in range(-2, 3) for j in range(-2, 3) for l in range(-2, 3))
        errs.append(np.abs(lam[:10] - np.array(exact[:10])).max())
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-3


def test_u_form_and_bloch_form_converge_together():
    diffs = []
    for nc in (2, 3, 4):
        s = wl.tiny_system(nc=nc, p=3, n_atoms=1, seed=3, L=6.0, r0=1.0, r1=2.0)
        a = np.linalg.eigvalsh(UFormOperator(s, K).dense())[:6]
        b = np.linalg.eigvalsh(OEFEOperator(s.with_k(K)).dense())[:6]
        diffs.append(np.abs(a - b).max())
    assert diffs[2] < diffs[0] / 4, diffs
