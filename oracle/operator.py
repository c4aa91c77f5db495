"""The OEFE Kohn-Sham operator in symmetric standard form.

Discrete generalized problem H u = eps M u (eqnKSEigGenDiscrete) with the
block-diagonal overlap M = diag(M^cc, M^oo) (eqnMOEFE) whose inverse is
block-diagonal (eqnMOEFEInv).  The paper transforms to the standard problem
M^-1 H u = eps u (eqnKSEignStandDiscrete); the oracle (and the HIP library)
use the similar symmetric form

    Ht = M^-1/2 H M^-1/2,   M^-1/2 = diag(m^-1/2) (+) S,   S = (M^oo)^-1/2,

which has the same eigenvalues; eigenvectors map by y = M^1/2 u.

Blocks: H^cc = sum_e P_e^* (K_e + B^T diag(W_e V_e) B) P_e with the cell
stiffness K_e = 1/2 int grad N . grad N and the potential term int V N N
(eqnHOEFEelelements), both with the q = p + 1 Gauss rule; H^co, H^oo, M^oo
from ``enrichment``.

    Ht X = [ D^-1/2 (H^cc D^-1/2 X^C + H^co S X^O) ;
             S (H^co* D^-1/2 X^C + H^oo S X^O) ]
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .enrichment import EnrichmentBlocks
from .mesh import Mesh
from .potential import nuclear_potential


class OEFEOperator:
    def __init__(self, system, V: np.ndarray | None = None, kvec="system"):
        if isinstance(kvec, str):
            kvec = system.kvec
        self.system = system
        self.kvec = None if kvec is None else np.asarray(kvec, dtype=np.float64)
        self.complex = self.kvec is not None
        self.dtype = np.complex128 if self.complex else np.float64
        mesh = Mesh(system.L, system.nc, system.p)
        self.mesh = mesh
        self.m = mesh.lumped_mass()
        self.dm12 = 1.0 / np.sqrt(self.m)
        if V is None:
            V = nuclear_potential(mesh.quad_points(), system.pos, system.Z, system.sigma, system.L)
        self.V = np.ascontiguousarray(V, dtype=np.float64).reshape(mesh.n_cells, mesh.nq)
        self.Ke = mesh.cell_stiffness()
        self.theta = mesh.bloch_phase(self.kvec)
        nd = mesh.nd
        rows = np.arange(mesh.n_cells * nd)
        self.P = sp.csr_matrix((self.theta.ravel().astype(self.dtype), (rows, mesh.cell_dofs.ravel())),
                               shape=(mesh.n_cells * nd, mesh.N))
        self.PH = self.P.conj().T.tocsr()
        self.enr = EnrichmentBlocks(mesh, system, self.V, self.m, self.kvec)
        self.N = mesh.N
        self.n_enr = system.n_enr
        self.n_tot = self.N + self.n_enr
        self._hcc = None

    # -------------------------------------------------------------- H^cc z
    def hcc_apply_cells(self, Zc: np.ndarray, chunk: int = 512) -> np.ndarray:
        """H^cc Zc by cells: gather, K_e z_e + B^T (W V_e o (B z_e)), scatter (Sigma_e P_e^* A_e P_e)."""
        mesh = self.mesh
        nd, nv = mesh.nd, Zc.shape[1]
        Xe = (self.P @ Zc).reshape(mesh.n_cells, nd, nv)
        WV = mesh.Wcell[None, :] * self.V  # [n_cells, nq]
        Ye = np.empty_like(Xe)
        for s in range(0, mesh.n_cells, chunk):
            xe = Xe[s:s + chunk]
            u = np.matmul(mesh.B, xe)  # [c, nq, nv]
            u *= WV[s:s + chunk, :, None]
            Ye[s:s + chunk] = np.matmul(self.Ke, xe) + np.matmul(mesh.B.T, u)
        return self.PH @ Ye.reshape(mesh.n_cells * nd, nv)

    def hcc_csr(self) -> sp.csr_matrix:
        """Assembled H^cc as CSR (independent summation order from the cell route)."""
        if self._hcc is None:
            mesh = self.mesh
            nd = mesh.nd
            WV = mesh.Wcell[None, :] * self.V
            Ae = self.Ke[None, :, :] + np.einsum("qa,eq,qb->eab", mesh.B, WV, mesh.B)
            th = self.theta
            Ae = np.conj(th)[:, :, None] * Ae * th[:, None, :]
            dofs = mesh.cell_dofs
            r = np.repeat(dofs, nd, axis=1).ravel()
            c = np.tile(dofs, (1, nd)).ravel()
            self._hcc = sp.coo_matrix((Ae.ravel(), (r, c)), shape=(mesh.N, mesh.N)).tocsr()
            self._hcc.sum_duplicates()
        return self._hcc

    # -------------------------------------------------------------- Ht X
    def apply(self, X: np.ndarray, route: str = "cells") -> np.ndarray:
        """Y = Ht X for a block X [n_tot, nv] (or a vector)."""
        vec = X.ndim == 1
        if vec:
            X = X[:, None]
        N = self.N
        dt = np.result_type(X.dtype, self.dtype)
        Xc, Xo = X[:N].astype(dt), X[N:].astype(dt)
        Zc = self.dm12[:, None] * Xc
        S = self.enr.S
        Zo = S @ Xo
        if route == "cells":
            Hz = self.hcc_apply_cells(Zc)
        else:
            Hz = self.hcc_csr() @ Zc
        Hco = self.enr.Hco
        Yc = self.dm12[:, None] * (Hz + Hco @ Zo)
        Yo = S @ (Hco.conj().T @ Zc + self.enr.Hoo @ Zo)
        Y = np.concatenate([Yc, Yo], axis=0)
        return Y[:, 0] if vec else Y

    def dense(self) -> np.ndarray:
        """Dense Ht (tiny meshes only)."""
        N, n = self.N, self.n_tot
        Hcc = self.hcc_csr().toarray()
        D = self.dm12
        S = self.enr.S
        Hco = self.enr.Hco.toarray()
        H = np.zeros((n, n), dtype=self.dtype)
        H[:N, :N] = D[:, None] * Hcc * D[None, :]
        H[:N, N:] = D[:, None] * (Hco @ S)
        H[N:, :N] = S @ (np.conj(Hco.T) * D[None, :])
        H[N:, N:] = S @ self.enr.Hoo @ S
        return H

    def dense_generalized(self):
        """Dense (H, M) of the generalized problem (tiny meshes only)."""
        N, n = self.N, self.n_tot
        H = np.zeros((n, n), dtype=self.dtype)
        M = np.zeros((n, n), dtype=self.dtype)
        H[:N, :N] = self.hcc_csr().toarray()
        Hco = self.enr.Hco.toarray()
        H[:N, N:] = Hco
        H[N:, :N] = np.conj(Hco.T)
        H[N:, N:] = self.enr.Hoo
        M[:N, :N] = np.diag(self.m)
        M[N:, N:] = self.enr.Moo
        return H, M

    def basis_values_at_quad(self):
        """Values of every basis function at every quadrature point, [n_cells * nq, n_tot] (tiny meshes).

        Column g < N: the (Bloch-twisted) FE function; column N + nu: N^O_nu.
        """
        mesh = self.mesh
        Bg = np.zeros((mesh.n_cells, mesh.nq, self.N), dtype=self.dtype)
        for e in range(mesh.n_cells):
            for a in range(mesh.nd):
                Bg[e, :, mesh.cell_dofs[e, a]] += mesh.B[:, a] * self.theta[e, a]
        Phi, _ = self.enr.values_at_quad()
        return np.concatenate([Bg, Phi], axis=2).reshape(mesh.n_cells * mesh.nq, self.n_tot)
