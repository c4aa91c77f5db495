"""Orthogonalized enrichment functions and the enrichment blocks of H and M.

Follows Sec. III.A of the paper:

* atomic part N^A = phase * psi~(x - R^x) (eqnUOEFEAtomic), psi~ = radial and
  angular factor times a smooth cutoff h(r) (eqnKSAtomicTrunc,
  eqnCutoffProperties); R^x is the periodic image of the atom nearest to x;
* orthogonalizing part N^B = sum_l c_l N^C_l (eqnUOEFEOrtho) with
  c = d / M^cc_ll (eqnorthC, eqnorthCGLL): numerator by the Gauss rule,
  denominator the GLL (lumped) mass;
* N^O = N^A - N^B (eqnUOEFESplit);
* M^oo = int N^O* N^O (eqnMoo);
* H^co, H^oo = 1/2 int grad N* . grad N + int V N* N (eqnHOEFEelelements in
  the Bloch-function form: the basis functions carry the Bloch phase, so the
  k-dependent terms are absent).

Readings where the paper is silent: the cutoff is the C-infinity step
h = 1 / (1 + exp(1/x - 1/(1-x))), x = (r1 - r) / (r1 - r0) on (r0, r1);
the enrichment radial factors are Slater-type proxies r^a exp(-zeta r) with an
optional Cartesian factor d_x, d_y or d_z (atomic solver output is not
available); all H integrals use the q = p + 1 Gauss rule.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh
from .potential import min_image


def cutoff(r: np.ndarray, r0: float, r1: float):
    """Smooth cutoff h(r) and its derivative h'(r)."""
    r = np.asarray(r, dtype=np.float64)
    h = np.zeros_like(r)
    dh = np.zeros_like(r)
    h[r <= r0] = 1.0
    mid = (r > r0) & (r < r1)
    x = (r1 - r[mid]) / (r1 - r0)
    u = 1.0 / x - 1.0 / (1.0 - x)
    # s = 1 / (1 + e^u), written to avoid overflow for large |u|
    s = np.where(u > 0, np.exp(-np.abs(u)) / (1.0 + np.exp(-np.abs(u))), 1.0 / (1.0 + np.exp(-np.abs(u))))
    h[mid] = s
    ds_dx = s * (1.0 - s) * (1.0 / x ** 2 + 1.0 / (1.0 - x) ** 2)
    dh[mid] = -ds_dx / (r1 - r0)
    return h, dh


def atomic_function(d: np.ndarray, power: int, zeta: float, axis: int, r0: float, r1: float):
    """psi~(d) = r^power exp(-zeta r) [d_axis] h(r) and its gradient, for displacements d [..., 3]."""
    r = np.sqrt((d * d).sum(-1))
    f = r ** power * np.exp(-zeta * r)
    if power == 0:
        fp = -zeta * np.exp(-zeta * r)
    else:
        fp = (power * r ** (power - 1) - zeta * r ** power) * np.exp(-zeta * r)
    h, dh = cutoff(r, r0, r1)
    rhat = d / r[..., None]
    if axis < 0:
        val = f * h
        grad = (fp * h + f * dh)[..., None] * rhat
    else:
        P = d[..., axis]
        val = P * f * h
        grad = (P * (fp * h + f * dh))[..., None] * rhat
        grad[..., axis] += f * h
    return val, grad


def atomic_part(mesh: Mesh, R: np.ndarray, fns, cells: np.ndarray, r0: float, r1: float, kvec=None):
    """N^A for the functions `fns` of one atom at the quadrature points of `cells`.

    Returns values [nc, nq, F] and gradients [nc, nq, F, 3] (complex at k != 0).
    """
    x = mesh.quad_points(cells)  # [nc, nq, 3]
    draw = x - R[None, None, :]
    t = np.round(draw / mesh.L)
    d = draw - mesh.L * t  # displacement from the nearest image R^x = R + L t
    F = len(fns)
    dtype = np.float64 if kvec is None else np.complex128
    val = np.zeros(x.shape[:2] + (F,), dtype=dtype)
    grad = np.zeros(x.shape[:2] + (F, 3), dtype=dtype)
    phase = 1.0 if kvec is None else np.exp(1j * mesh.L * (t @ np.asarray(kvec)))
    for j, fn in enumerate(fns):
        v, g = atomic_function(d, fn.power, fn.zeta, fn.axis, r0, r1)
        val[:, :, j] = phase * v
        grad[:, :, j, :] = (phase[..., None] if kvec is not None else 1.0) * g
    return val, grad


def orthogonalize(mesh: Mesh, cells: np.ndarray, NA: np.ndarray, gNA: np.ndarray, theta: np.ndarray, m: np.ndarray):
    """Orthogonalize atomic functions against the FE space (eqnorthC, eqnorthCGLL).

    d_g = sum_{(e,a)->g} conj(theta_ea) sum_q W_q B[q,a] N^A(x_eq);  c_g = d_g / m_g;
    N^O(x_eq) = N^A(x_eq) - sum_a B[q,a] theta_ea c_{g(e,a)}  (and the same for gradients).
    `cells` must contain every cell where N^A is nonzero plus one layer of neighbours.
    Returns (c [N, F], Phi [nc, nq, F], gradPhi [nc, nq, F, 3]).
    """
    F = NA.shape[-1]
    dofs = mesh.cell_dofs[cells]  # [nc, nd]
    th = theta[cells]  # [nc, nd]
    W = mesh.Wcell
    # d_e[a, f] = sum_q W_q B[q,a] NA[q,f]
    de = np.einsum("qa,eqf->eaf", mesh.B, W[None, :, None] * NA, optimize=True)
    de = np.conj(th)[:, :, None] * de
    dtype = NA.dtype
    d = np.zeros((mesh.N, F), dtype=dtype)
    np.add.at(d, dofs.ravel(), de.reshape(-1, F))
    c = d / m[:, None]
    ce = th[:, :, None] * c[dofs]  # [nc, nd, F]
    Phi = NA - np.einsum("qa,eaf->eqf", mesh.B, ce, optimize=True)
    s = 2.0 / mesh.h
    gPhi = gNA.copy()
    for dd in range(3):
        gPhi[..., dd] -= s * np.einsum("qa,eaf->eqf", mesh.Gref[dd], ce, optimize=True)
    return c, Phi, gPhi


class EnrichmentBlocks:
    """All enrichment data of one operator: per-atom N^O at quadrature points and the blocks."""

    def __init__(self, mesh: Mesh, system, V: np.ndarray, m: np.ndarray, kvec=None):
        self.mesh = mesh
        self.kvec = kvec
        self.n_enr = system.n_enr
        complex_ = kvec is not None
        dtype = np.complex128 if complex_ else np.float64
        theta = mesh.bloch_phase(kvec)
        self.theta = theta
        atom_of = np.array([f.atom for f in system.enr], dtype=np.int64)
        self.atom_fn = []  # list of (atom, global fn indices, cells, Phi, gradPhi)
        c_cols = []
        for I in range(system.n_atoms):
            idx = np.nonzero(atom_of == I)[0]
            if idx.size == 0:
                continue
            fns = [system.enr[i] for i in idx]
            core = mesh.cells_near(system.pos[I], system.r1)
            cells = mesh.dilate_cells(core)
            NA, gNA = atomic_part(mesh, system.pos[I], fns, cells, system.r0, system.r1, kvec)
            c, Phi, gPhi = orthogonalize(mesh, cells, NA, gNA, theta, m)
            self.atom_fn.append((I, idx, cells, Phi, gPhi))
            c_cols.append((idx, c))
        n_O = self.n_enr
        C = np.zeros((mesh.N, n_O), dtype=dtype) if mesh.N * max(n_O, 1) <= 4e7 else None
        if C is not None:
            for idx, c in c_cols:
                C[:, idx] = c
        self.C = C
        W = mesh.Wcell
        half = 0.5
        Moo = np.zeros((n_O, n_O), dtype=dtype)
        Hoo = np.zeros((n_O, n_O), dtype=dtype)
        for (I, idxI, cI, PI, gI) in self.atom_fn:
            for (J, idxJ, cJ, PJ, gJ) in self.atom_fn:
                common, iI, iJ = np.intersect1d(cI, cJ, return_indices=True)
                if common.size == 0:
                    continue
                a = PI[iI]
                b = PJ[iJ]
                ga = gI[iI]
                gb = gJ[iJ]
                Vc = V[common]
                Moo[np.ix_(idxI, idxJ)] += np.einsum("eqf,eqg->fg", np.conj(a) * W[None, :, None], b, optimize=True)
                Hoo[np.ix_(idxI, idxJ)] += half * np.einsum("eqfd,eqgd->fg", np.conj(ga) * W[None, :, None, None], gb, optimize=True)
                Hoo[np.ix_(idxI, idxJ)] += np.einsum("eqf,eqg->fg", np.conj(a) * (W[None, :] * Vc)[:, :, None], b, optimize=True)
        self.Moo = Moo
        self.Hoo = Hoo
        # H^co[g, nu] = sum_{(e,a)->g} conj(theta_ea) sum_q W [1/2 (2/h) G_d[q,a] dPhi_d + V B[q,a] Phi]
        s = 2.0 / mesh.h
        rows, cols, vals = [], [], []
        for (I, idx, cells, Phi, gPhi) in self.atom_fn:
            Wv = W[None, :] * V[cells]  # [nc, nq]
            he = np.einsum("qa,eqf->eaf", mesh.B, Wv[:, :, None] * Phi, optimize=True)
            for dd in range(3):
                he += half * s * np.einsum("qa,eqf->eaf", mesh.Gref[dd], W[None, :, None] * gPhi[..., dd], optimize=True)
            he = np.conj(theta[cells])[:, :, None] * he
            dofs = mesh.cell_dofs[cells]
            F = idx.size
            rows.append(np.repeat(dofs.ravel(), F))
            cols.append(np.tile(idx, dofs.size))
            vals.append(he.reshape(-1))
        if rows:
            Hco = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(mesh.N, n_O)).tocsr()
            Hco.sum_duplicates()
        else:
            Hco = sp.csr_matrix((mesh.N, n_O), dtype=dtype)
        self.Hco = Hco
        if n_O > 0:
            lam, U = np.linalg.eigh(Moo)
            self.Moo_eigs = lam
            self.S = (U * (1.0 / np.sqrt(lam))[None, :]) @ np.conj(U.T)
        else:
            self.Moo_eigs = np.zeros(0)
            self.S = np.zeros((0, 0), dtype=dtype)

    def values_at_quad(self, cells=None):
        """Dense N^O at all quadrature points [n_cells, nq, n_O] (small meshes only)."""
        mesh = self.mesh
        dtype = np.complex128 if self.kvec is not None else np.float64
        out = np.zeros((mesh.n_cells, mesh.nq, self.n_enr), dtype=dtype)
        gout = np.zeros((mesh.n_cells, mesh.nq, self.n_enr, 3), dtype=dtype)
        for (I, idx, cells_I, Phi, gPhi) in self.atom_fn:
            out[np.ix_(cells_I, np.arange(mesh.nq), idx)] = Phi
            gout[np.ix_(cells_I, np.arange(mesh.nq), idx, np.arange(3))] = gPhi
        return out, gout
