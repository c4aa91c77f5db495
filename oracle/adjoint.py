"""Band energy of a block of vectors and its gradients.

E = sum_i f_i x_i^* Ht x_i  (the band energy of the paper's Sec. II with the
occupations f_i supplied by the caller; f includes the factor 2 w_k).

dE/dX = 2 Ht X diag(f)   (for complex X this is PyTorch's convention for a
real loss: twice the conjugate Wirtinger derivative).

dE/dV_{e,q} = W_{e,q} sum_i f_i |psi_i(x_{e,q})|^2, where psi_i is the field
of the generalized-problem coefficients z_i = M^-1/2 x_i at the quadrature
point.  H depends on V only through sum_{e,q} V W n n^* (n = basis values at
x_{e,q}) and M does not depend on V, so this is the electron density of
eqnrho times W when f carries the factor 2 w_k.
"""
from __future__ import annotations

import numpy as np


def band_energy(op, X: np.ndarray, f: np.ndarray) -> float:
    HX = op.apply(X)
    return float(np.real(np.sum(f * np.sum(np.conj(X) * HX, axis=0))))


def grad_X(op, X: np.ndarray, f: np.ndarray) -> np.ndarray:
    return 2.0 * op.apply(X) * f[None, :]


def fields_at_quad(op, X: np.ndarray) -> np.ndarray:
    """psi_i(x_{e,q}) for all cells and quadrature points, [n_cells, nq, nv]."""
    mesh = op.mesh
    N = op.N
    nv = X.shape[1]
    dt = np.result_type(X.dtype, op.dtype)
    Zc = op.dm12[:, None] * X[:N].astype(dt)
    Zo = op.enr.S @ X[N:].astype(dt)
    Xe = (op.P @ Zc).reshape(mesh.n_cells, mesh.nd, nv)
    psi = np.matmul(mesh.B, Xe)
    for (I, idx, cells, Phi, gPhi) in op.enr.atom_fn:
        psi[cells] += np.einsum("eqf,fv->eqv", Phi, Zo[idx])
    return psi


def grad_V(op, X: np.ndarray, f: np.ndarray) -> np.ndarray:
    psi = fields_at_quad(op, X)
    W = op.mesh.Wcell
    return W[None, :] * np.einsum("eqv,v->eq", np.abs(psi) ** 2, f)
