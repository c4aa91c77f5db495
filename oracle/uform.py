"""The k-point Hamiltonian in the periodic-function (u) form (Sec. II eqnksdftu; Sec. III.A
eqnUOEFEAtomic, eqnHOEFEelelements, eqnMoo).  Test infrastructure only.

The Bloch function psi = exp(i k.x) u with u periodic; u in the OEFE basis of periodic FE
functions plus orthogonalized enrichment functions whose atomic part is
N^A = exp(-i k.(x - R^x)) psi~(x - R^x) (eqnUOEFEAtomic, R^x the image of the atom nearest to x).
The Hamiltonian (eqnHOEFEelelements):

    H_mn = 1/2 int grad N_m^* . grad N_n - i k . int N_m^* grad N_n + int (|k|^2/2 + V) N_m^* N_n,

the overlap M = diag(M^cc, M^oo_k) with the lumped GLL M^cc (eqnMcc) and
M^oo_k = int N^O* N^O (eqnMoo).  Reading: in the blocks with an enrichment function the
first-derivative term is taken in its Hermitian form
-i/2 k . int (N_m^* grad N_n - grad N_m^* N_n), equal to the written term when the rule integrates
grad (N_m^* N_n) exactly, which the Gauss rule does for two FE functions (there the written form is
used) but not with an enrichment function, where the written form is not Hermitian.  The
orthogonalization is the one of the Bloch-function form (Gauss-rule numerator, GLL mass) with the
FE functions periodic (no phase).  Symmetric standard
form as for the other operator: Ht_k = M^-1/2 H_k M^-1/2.  At k = 0 this is the Gamma-point
operator of operator.OEFEOperator.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .enrichment import atomic_function, orthogonalize
from .mesh import Mesh
from .potential import nuclear_potential


class UFormOperator:
    def __init__(self, system, kvec, V: np.ndarray | None = None):
        self.system = system
        self.kvec = np.asarray(kvec, dtype=np.float64)
        k = self.kvec
        mesh = Mesh(system.L, system.nc, system.p)
        self.mesh = mesh
        self.m = mesh.lumped_mass()
        self.dm12 = 1.0 / np.sqrt(self.m)
        if V is None:
            V = nuclear_potential(mesh.quad_points(), system.pos, system.Z, system.sigma, system.L)
        self.V = np.ascontiguousarray(V, dtype=np.float64).reshape(mesh.n_cells, mesh.nq)
        self.N = mesh.N
        self.n_enr = system.n_enr
        self.n_tot = self.N + self.n_enr
        W = mesh.Wcell
        s = 2.0 / mesh.h
        nd = mesh.nd
        k2 = 0.5 * float(k @ k)
        # cell matrices: 1/2 stiffness, the first-derivative term -i k . int N_a grad N_b, and the
        # (|k|^2/2 + V) mass term per cell
        Ke = np.zeros((nd, nd))
        Ge = np.zeros((nd, nd))
        for d in range(3):
            Ke += mesh.Gref[d].T @ (W[:, None] * mesh.Gref[d])
            Ge += k[d] * s * (mesh.B.T @ (W[:, None] * mesh.Gref[d]))
        self.Ke = 0.5 * s * s * Ke
        self.Ge = -1j * Ge
        WV = W[None, :] * (self.V + k2)  # [n_cells, nq]
        dofs = mesh.cell_dofs
        r_ = np.repeat(dofs, nd, axis=1).ravel()
        c_ = np.tile(dofs, (1, nd)).ravel()
        Ae = (self.Ke + self.Ge)[None, :, :] + np.einsum("qa,eq,qb->eab", mesh.B, WV, mesh.B, optimize=True)
        self.Hcc = sp.coo_matrix((Ae.ravel(), (r_, c_)), shape=(self.N, self.N)).tocsr()
        self.Hcc.sum_duplicates()
        # enrichment: N^A = exp(-i k.(x - R^x)) psi~(x - R^x), orthogonalized against the periodic FE basis
        theta = np.ones(dofs.shape)
        atom_of = np.array([f.atom for f in system.enr], dtype=np.int64)
        self.atom_fn = []
        for I in range(system.n_atoms):
            idx = np.nonzero(atom_of == I)[0]
            if idx.size == 0:
                continue
            cells = mesh.dilate_cells(mesh.cells_near(system.pos[I], system.r1))
            x = mesh.quad_points(cells)
            draw = x - system.pos[I][None, None, :]
            d = draw - mesh.L * np.round(draw / mesh.L)
            ph = np.exp(-1j * (d @ k))  # exp(-i k.(x - R^x))
            F = idx.size
            NA = np.zeros(x.shape[:2] + (F,), dtype=np.complex128)
            gNA = np.zeros(x.shape[:2] + (F, 3), dtype=np.complex128)
            for j, i in enumerate(idx):
                fn = system.enr[i]
                v, g = atomic_function(d, fn.power, fn.zeta, fn.axis, system.r0, system.r1)
                NA[:, :, j] = ph * v
                gNA[:, :, j, :] = ph[..., None] * (g - 1j * k[None, None, :] * v[..., None])
            _, Phi, gPhi = orthogonalize(mesh, cells, NA, gNA, theta, self.m)
            self.atom_fn.append((idx, cells, Phi, gPhi))
        nO = self.n_enr
        Moo = np.zeros((nO, nO), dtype=np.complex128)
        Hoo = np.zeros((nO, nO), dtype=np.complex128)
        for (iI, cI, PI, gI) in self.atom_fn:
            for (iJ, cJ, PJ, gJ) in self.atom_fn:
                common, a_, b_ = np.intersect1d(cI, cJ, return_indices=True)
                if common.size == 0:
                    continue
                a, b, ga, gb = PI[a_], PJ[b_], gI[a_], gJ[b_]
                Wc = W[None, :]
                Moo[np.ix_(iI, iJ)] += np.einsum("eqf,eqg,eq->fg", np.conj(a), b, np.broadcast_to(Wc, a.shape[:2]))
                Hoo[np.ix_(iI, iJ)] += 0.5 * np.einsum("eqfd,eqgd,eq->fg", np.conj(ga), gb,
                                                       np.broadcast_to(Wc, a.shape[:2]))
                Hoo[np.ix_(iI, iJ)] += -0.5j * np.einsum("eqf,eqgd,d,eq->fg", np.conj(a), gb, k,
                                                         np.broadcast_to(Wc, a.shape[:2]))
                Hoo[np.ix_(iI, iJ)] += 0.5j * np.einsum("eqfd,eqg,d,eq->fg", np.conj(ga), b, k,
                                                        np.broadcast_to(Wc, a.shape[:2]))
                Hoo[np.ix_(iI, iJ)] += np.einsum("eqf,eqg,eq->fg", np.conj(a), b, Wc * (self.V[common] + k2))
        self.Moo, self.Hoo = Moo, Hoo
        rows, cols, vals = [], [], []
        for (idx, cells, Phi, gPhi) in self.atom_fn:
            Wv = W[None, :] * (self.V[cells] + k2)
            he = np.einsum("qa,eqf->eaf", mesh.B, Wv[:, :, None] * Phi, optimize=True)
            for d in range(3):
                he += 0.5 * s * np.einsum("qa,eqf->eaf", mesh.Gref[d], W[None, :, None] * gPhi[..., d], optimize=True)
                he += -0.5j * k[d] * np.einsum("qa,eqf->eaf", mesh.B, W[None, :, None] * gPhi[..., d], optimize=True)
                he += 0.5j * k[d] * s * np.einsum("qa,eqf->eaf", mesh.Gref[d], W[None, :, None] * Phi, optimize=True)
            F = idx.size
            rows.append(np.repeat(dofs[cells].ravel(), F))
            cols.append(np.tile(idx, dofs[cells].size))
            vals.append(he.reshape(-1))
        if rows:
            self.Hco = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                     shape=(self.N, nO)).tocsr()
            self.Hco.sum_duplicates()
        else:
            self.Hco = sp.csr_matrix((self.N, 0), dtype=np.complex128)
        if nO:
            lam, U = np.linalg.eigh(Moo)
            self.Moo_eigs = lam
            self.S = (U / np.sqrt(lam)[None, :]) @ np.conj(U.T)
        else:
            self.Moo_eigs = np.zeros(0)
            self.S = np.zeros((0, 0), dtype=np.complex128)

    def apply(self, X: np.ndarray) -> np.ndarray:
        """Ht_k X for a block X [n_tot, nv] (complex)."""
        vec = X.ndim == 1
        if vec:
            X = X[:, None]
        N = self.N
        Xc, Xo = X[:N].astype(np.complex128), X[N:].astype(np.complex128)
        Zc = self.dm12[:, None] * Xc
        Zo = self.S @ Xo
        Yc = self.dm12[:, None] * (self.Hcc @ Zc + self.Hco @ Zo)
        Yo = self.S @ (self.Hco.conj().T @ Zc + self.Hoo @ Zo)
        Y = np.concatenate([Yc, Yo], axis=0)
        return Y[:, 0] if vec else Y

    def dense(self) -> np.ndarray:
        N, n = self.N, self.n_tot
        D = self.dm12
        H = np.zeros((n, n), dtype=np.complex128)
        H[:N, :N] = D[:, None] * self.Hcc.toarray() * D[None, :]
        Hco = self.Hco.toarray()
        H[:N, N:] = D[:, None] * (Hco @ self.S)
        H[N:, :N] = self.S @ (np.conj(Hco.T) * D[None, :])
        H[N:, N:] = self.S @ self.Hoo @ self.S
        return H
