"""The auxiliary electrostatic potential in the OEFE basis (Sec. II, end of Sec. III.A).

Test infrastructure only (see the package docstring).

* Unit smeared charge g(r, rc) (eqngr) and its potential v_g(r, rc) (eqnvg); smeared nuclear
  charge b(x) = -sum_I Z_I g(|x - R_I^x|, rc_I) (eqnsmeared) with the nearest periodic image R_I^x.
* rc_I: the paper takes the largest radii for which no two smeared charges overlap; here (a
  reading) half the distance from atom I to the nearest other atom or periodic image.
* -(1/4 pi) lap phi_aux = b + rho (eqnpoissonaux) on the periodic cell, with phi_aux in the OEFE
  basis (eqnPhiOEFE): the FE functions plus one orthogonalized enrichment function per atom,
  N^{O,phi}_I = N^{A,phi}_I - N^{B,phi}_I (eqnOrthoEnrichedPhiAux), N^{A,phi}_I = phi_I(r) h(r)
  (eqnPhiAuxAtomic) with the cutoff h of the wavefunction enrichment, and
  phi_I = V_H,I - Z_I v_g(r, rc_I) (eqnEnrichedPhiAux, eqnnucsmear).  N^{B,phi} is the same
  orthogonalization as for the wavefunction enrichment (Gauss numerator, GLL mass).
* V_H,I, the Hartree potential of the isolated atom, comes from an atomic solver in the paper;
  here (a reading) it is the potential of a model neutral-atom electron density
  rho_I(r) = Z_I alpha^3 / (8 pi) exp(-alpha r), alpha = 2 Z_I^(1/3):
  V_H,I(r) = Z_I (1 - (1 + alpha r / 2) exp(-alpha r)) / r.
* A_mn = 1/(4 pi) int grad N_m . grad N_n (eqnDiscLaplace), c_m = int (b + rho) N_m
  (eqnDiscForceVec), A phi = c (eqnpoissX); all integrals with the q = p + 1 Gauss rule.
* On the periodic cell A has the constants (1 on the FE part, 0 on the enrichment part) as its
  null space.  The discrete charge's quadrature integral is removed as a uniform background
  before c is formed, so that A phi = c is consistent, and phi is the solution whose FE part has
  zero GLL-mass-weighted mean (readings).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .enrichment import cutoff, orthogonalize
from .mesh import Mesh

FOUR_PI = 4.0 * np.pi


def g_smeared(r, rc: float) -> np.ndarray:
    """Unit smeared charge g(r, rc) of eqngr (zero beyond rc)."""
    r = np.asarray(r, dtype=np.float64)
    val = -21.0 * (r - rc) ** 3 * (6.0 * r * r + 3.0 * r * rc + rc * rc) / (5.0 * np.pi * rc ** 8)
    return np.where(r <= rc, val, 0.0)


def v_g(r, rc: float):
    """Potential v_g(r, rc) of the unit smeared charge (eqnvg) and its radial derivative."""
    r = np.asarray(r, dtype=np.float64)
    inside = r <= rc
    rs = np.where(inside, r, rc)
    ro = np.where(inside, rc, r)
    vin = (9 * rs ** 7 - 30 * rs ** 6 * rc + 28 * rs ** 5 * rc ** 2 - 14 * rs ** 2 * rc ** 5 + 12 * rc ** 7) / (5 * rc ** 8)
    din = (63 * rs ** 6 - 180 * rs ** 5 * rc + 140 * rs ** 4 * rc ** 2 - 28 * rs * rc ** 5) / (5 * rc ** 8)
    return np.where(inside, vin, 1.0 / ro), np.where(inside, din, -1.0 / ro ** 2)


def smear_radii(pos: np.ndarray, L: float) -> np.ndarray:
    """rc_I = half the distance from atom I to the nearest other atom or periodic image."""
    pos = np.asarray(pos, dtype=np.float64)
    shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)], dtype=np.float64) * L
    rc = np.empty(len(pos))
    for I in range(len(pos)):
        d = pos[None, :, :] + shifts[:, None, :] - pos[I][None, None, :]
        dist = np.sqrt((d * d).sum(-1))
        dist[13, I] = np.inf  # the atom itself (zero shift)
        rc[I] = 0.5 * dist.min()
    return rc


def model_alpha(Z) -> np.ndarray:
    return 2.0 * np.asarray(Z, dtype=np.float64) ** (1.0 / 3.0)


def model_density(r, Z: float, alpha: float) -> np.ndarray:
    """Model isolated-atom electron density Z alpha^3/(8 pi) exp(-alpha r) (integrates to Z)."""
    return Z * alpha ** 3 / (8.0 * np.pi) * np.exp(-alpha * np.asarray(r, dtype=np.float64))


def hartree_model(r, Z: float, alpha: float):
    """V_H of the model density and its radial derivative (series below r alpha = 1e-3)."""
    r = np.asarray(r, dtype=np.float64)
    x = alpha * r
    small = x < 1e-3
    xs = np.where(small, 1.0, x)
    e = np.exp(-xs)
    v = Z * alpha * (1.0 - (1.0 + 0.5 * xs) * e) / xs
    # dV/dr = Z alpha^2 [ (1 + x/2) e / x + (x/2 + ...) ] ; from d/dx [(1 - (1 + x/2) e^-x) / x]
    dvdx = ((0.5 + 0.5 * xs) * e * xs - (1.0 - (1.0 + 0.5 * xs) * e)) / xs ** 2
    xz = np.where(small, x, 0.0)
    v_series = Z * alpha * (0.5 - xz * xz / 12.0 + xz ** 3 / 24.0)
    d_series = -xz / 6.0 + xz * xz / 8.0
    v = np.where(small, v_series, v)
    dv = Z * alpha * alpha * np.where(small, d_series, dvdx)
    return v, dv


def phi_atomic(r, Z: float, alpha: float, rc: float):
    """phi_I(r) = V_H,I(r) - Z v_g(r, rc) and its radial derivative."""
    vh, dvh = hartree_model(r, Z, alpha)
    vg, dvg = v_g(r, rc)
    return vh - Z * vg, dvh - Z * dvg


def _nearest(mesh: Mesh, x: np.ndarray, R: np.ndarray):
    d = x - R
    return d - mesh.L * np.round(d / mesh.L)


class PoissonOEFE:
    """Discrete Poisson problem for phi_aux in the OEFE basis of one system (real, Gamma);
    enrich=False keeps the FE functions only (the classical basis, for comparisons)."""

    def __init__(self, system, enrich: bool = True):
        self.system = system
        mesh = Mesh(system.L, system.nc, system.p)
        self.mesh = mesh
        self.m = mesh.lumped_mass()
        self.Z = np.asarray(system.Z, dtype=np.float64)
        self.pos = np.asarray(system.pos, dtype=np.float64)
        self.rc = smear_radii(self.pos, system.L)
        self.alpha = model_alpha(self.Z)
        self.N = mesh.N
        self.n_atoms = len(self.Z)
        self.n_enr = self.n_atoms if enrich else 0
        self.n_tot = self.N + self.n_enr
        W = mesh.Wcell
        s = 2.0 / mesh.h
        # A^cc = sum_e P_e^T A_e P_e, A_e = 1/(4 pi) int grad N . grad N (Gauss rule)
        Ke = np.zeros((mesh.nd, mesh.nd))
        for d in range(3):
            Ke += mesh.Gref[d].T @ (W[:, None] * mesh.Gref[d])
        self.Ae = s * s * Ke / FOUR_PI
        dofs = mesh.cell_dofs
        nd = mesh.nd
        r_ = np.repeat(dofs, nd, axis=1).ravel()
        c_ = np.tile(dofs, (1, nd)).ravel()
        self.Acc = sp.coo_matrix((np.broadcast_to(self.Ae, (mesh.n_cells, nd, nd)).ravel(), (r_, c_)),
                                 shape=(self.N, self.N)).tocsr()
        self.Acc.sum_duplicates()
        # one orthogonalized enrichment function per atom
        theta = np.ones(dofs.shape)
        self.atoms = []  # (cells, Phi [nc, nq], gradPhi [nc, nq, 3])
        for I in range(self.n_enr):
            cells = mesh.dilate_cells(mesh.cells_near(self.pos[I], system.r1))
            d = _nearest(mesh, mesh.quad_points(cells), self.pos[I])
            r = np.sqrt((d * d).sum(-1))
            f, fp = phi_atomic(r, self.Z[I], self.alpha[I], self.rc[I])
            h, dh = cutoff(r, system.r0, system.r1)
            rhat = d / np.where(r > 0, r, 1.0)[..., None]
            NA = (f * h)[..., None]
            gNA = ((fp * h + f * dh)[..., None] * rhat)[:, :, None, :]
            _, Phi, gPhi = orthogonalize(mesh, cells, NA, gNA, theta, self.m)
            self.atoms.append((cells, Phi[..., 0], gPhi[:, :, 0, :]))
        # A^co [N x n_atoms] and A^oo
        rows, cols, vals = [], [], []
        for I, (cells, Phi, gPhi) in enumerate(self.atoms):
            he = np.zeros((len(cells), nd))
            for d in range(3):
                he += s * np.einsum("qa,eq->ea", mesh.Gref[d], W[None, :] * gPhi[..., d], optimize=True)
            rows.append(dofs[cells].ravel())
            cols.append(np.full(he.size, I))
            vals.append(he.ravel() / FOUR_PI)
        if rows:
            self.Aco = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                     shape=(self.N, self.n_enr)).tocsr()
        else:
            self.Aco = sp.csr_matrix((self.N, 0))
        self.Aco.sum_duplicates()
        Aoo = np.zeros((self.n_enr, self.n_enr))
        for I, (cI, _, gI) in enumerate(self.atoms):
            for J, (cJ, _, gJ) in enumerate(self.atoms):
                common, iI, iJ = np.intersect1d(cI, cJ, return_indices=True)
                if common.size:
                    Aoo[I, J] = np.einsum("eqd,eqd,q->", gI[iI], gJ[iJ], W, optimize=True) / FOUR_PI
        self.Aoo = Aoo

    # ------------------------------------------------------------------ charges
    def smeared_charge(self) -> np.ndarray:
        """b(x) at every quadrature point [n_cells, nq] (eqnsmeared, nearest image)."""
        mesh = self.mesh
        x = mesh.quad_points()
        b = np.zeros(x.shape[:2])
        for I in range(self.n_atoms):
            d = _nearest(mesh, x, self.pos[I])
            b -= self.Z[I] * g_smeared(np.sqrt((d * d).sum(-1)), self.rc[I])
        return b

    def model_electron_density(self) -> np.ndarray:
        """Sum of the model atomic densities at the quadrature points (nearest image)."""
        mesh = self.mesh
        x = mesh.quad_points()
        rho = np.zeros(x.shape[:2])
        for I in range(self.n_atoms):
            d = _nearest(mesh, x, self.pos[I])
            rho += model_density(np.sqrt((d * d).sum(-1)), self.Z[I], self.alpha[I])
        return rho

    def neutral_charge(self, rho_q: np.ndarray) -> np.ndarray:
        """b + rho minus its quadrature mean (the uniform background that makes A phi = c consistent)."""
        f = self.smeared_charge() + np.asarray(rho_q, dtype=np.float64).reshape(self.mesh.n_cells, self.mesh.nq)
        W = self.mesh.Wcell[None, :]
        return f - (W * f).sum() / (W.sum() * self.mesh.n_cells)

    # ------------------------------------------------------------------ system
    def force_vector(self, f_q: np.ndarray) -> np.ndarray:
        """c_m = int f N_m (eqnDiscForceVec) for a charge f at the quadrature points."""
        mesh = self.mesh
        Wf = mesh.Wcell[None, :] * f_q
        ce = Wf @ mesh.B  # [n_cells, nd]
        cC = np.zeros(self.N)
        np.add.at(cC, mesh.cell_dofs.ravel(), ce.ravel())
        cO = np.array([(Wf[cells] * Phi).sum() for (cells, Phi, _) in self.atoms])
        return np.concatenate([cC, cO])

    def matrix(self) -> sp.csr_matrix:
        """A^O = [[A^cc, A^co], [A^oc, A^oo]] (eqnDiscLaplace)."""
        return sp.bmat([[self.Acc, self.Aco], [self.Aco.T, sp.csr_matrix(self.Aoo)]], format="csr")

    def fix_constant(self, phi: np.ndarray) -> np.ndarray:
        """The member of phi + span{(1, 0)} whose FE part has zero GLL-mass-weighted mean."""
        out = np.array(phi, dtype=np.float64, copy=True)
        out[:self.N] -= (self.m * out[:self.N]).sum() / self.m.sum()
        return out

    def solve(self, f_q: np.ndarray, rtol: float = 1e-13) -> np.ndarray:
        """phi with A phi = c(f) (f: a neutral charge at the quadrature points).

        Small systems: dense least squares (the minimum-norm solution, then fix_constant).
        Larger: conjugate gradients with the Jacobi preconditioner (scipy) on the consistent system.
        """
        c = self.force_vector(f_q)
        A = self.matrix()
        if self.n_tot <= 3000:
            phi = np.linalg.lstsq(A.toarray(), c, rcond=None)[0]
        else:
            dinv = 1.0 / A.diagonal()
            M = sp.diags(dinv)
            phi, info = spla.cg(A, c, rtol=rtol, atol=0.0, maxiter=20000, M=M)
            if info != 0:
                raise RuntimeError(f"oracle CG did not converge ({info})")
        return self.fix_constant(phi)

    def field_at_quad(self, phi: np.ndarray) -> np.ndarray:
        """phi_aux^h at the quadrature points [n_cells, nq] (eqnPhiOEFE)."""
        mesh = self.mesh
        out = phi[mesh.cell_dofs] @ mesh.B.T  # [n_cells, nq]
        for I, (cells, Phi, _) in enumerate(self.atoms):
            out[cells] += phi[self.N + I] * Phi
        return out


def exact_potential(points: np.ndarray, system, rc: np.ndarray, alpha: np.ndarray, shells: int = 1) -> np.ndarray:
    """The exact potential of the neutral charge b + sum_I rho_I on the periodic cell, up to a constant:
    each atom's smeared nuclear charge plus model density is neutral and spherical, with the
    potential phi_I(r) = V_H,I(r) - Z_I v_g(r, rc_I), which decays exponentially beyond rc_I, so the
    lattice sum over the periodic images (|shift| <= shells cells) converges absolutely."""
    L = system.L
    pts = points.reshape(-1, 3)
    rng = range(-shells, shells + 1)
    out = np.zeros(pts.shape[0])
    for I in range(len(system.Z)):
        for i in rng:
            for j in rng:
                for k in rng:
                    d = pts - (system.pos[I] + L * np.array([i, j, k], dtype=np.float64))
                    v, _ = phi_atomic(np.sqrt((d * d).sum(-1)), system.Z[I], alpha[I], rc[I])
                    out += v
    return out.reshape(points.shape[:-1])
