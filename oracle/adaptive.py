"""Adaptive quadrature for the integrals of the enrichment functions (Sec. III.B), and the
Kohn-Sham operator whose enrichment blocks use it.  Test infrastructure only.

The enrichment functions vary sharply near the nuclei, so the paper integrates them with a
quadrature built by dividing each finite element recursively until a set of trial integrals
of the enrichment functions converges (divide and conquer; the details are in a cited work).
Readings used here:

* the rule of a box is the tensor Gauss rule with q = p + 1 points per direction mapped to
  the box; a box is split into its 8 half-size children;
* trial integrals of a box, for every atomic function nu (radial part times angular factor
  times cutoff, without Bloch phase) whose atom's support contains the cell: int psi~^2 and
  int |grad psi~|^2 (the enrichment blocks are quadratic in the functions), and for every local
  node a of the cell int psi~ N_a and int grad psi~ . grad^ N_a (grad^ the gradient in the
  cell's reference coordinates): the FE-enrichment integrals of the orthogonalization
  numerator and of H^co;
* a box is accepted when, for every trial integral, its own rule and the sum of its
  children's rules differ by at most tol times the trial integral's scale: the whole-space
  integrals A_nu = int psi~^2 and B_nu = int |grad psi~|^2 (radial integrals) for the quadratic
  ones, and sqrt(A_nu v) and sqrt(B_nu v) for the ones with N_a (v = 4/3 pi r1^3, the volume
  where psi~ is nonzero: Cauchy-Schwarz bounds of int |psi~| and int |grad psi~|); otherwise
  each child is treated the same way, down to max_depth levels, where boxes are accepted;
* a box that meets the ball of radius r1 around one of its atoms (nearest image) while none
  of its Gauss points lies inside that ball is split without the test: its rule cannot see
  the part of the functions it holds;
* the accepted boxes (leaves) of a cell are ordered depth first, children in the order
  cx + 2 cy + 4 cz; the points of a leaf in the order qx + q qy + q^2 qz; the rule covers the
  union of the supports (core cells within r1 of an atom, plus one layer), cells ascending;
* with the adaptive rule: the numerator of the orthogonalization coefficients
  (eqnorthC; the denominator stays the GLL mass), M^oo, H^oo and H^co; H^cc keeps the
  Gauss rule.  V at the adaptive points is an input (by default the nuclear potential
  evaluated there).

With max_depth = 0 every cell is one leaf and the blocks are those of enrichment.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .enrichment import atomic_function, atomic_part
from .mesh import Mesh
from .operator import OEFEOperator
from .potential import min_image, nuclear_potential
from .quadrature import gauss_rule

CHILD_OFFSETS = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.float64)


def radial_scales_of(gfun, axis: int, r1: float, panels: int = 64, order: int = 20):
    """A = int psi~^2 and B = int |grad psi~|^2 over R^3 for psi~ = g(r) (axis < 0) or d_axis g(r),
    g(r), g'(r) = gfun(r) vanishing beyond r1.  Angular integrals: 4 pi g^2 (s) or 4 pi r^2 g^2 / 3
    (p) for the value; 4 pi g'^2 (s) or 4 pi (g^2 + 2/3 r g g' + r^2 g'^2 / 3) (p) for the gradient.
    """
    x, w = gauss_rule(order)
    edges = np.linspace(0.0, r1, panels + 1)
    a, b = edges[:-1, None], edges[1:, None]
    r = (0.5 * (b - a) * (x[None, :] + 1.0) + a).ravel()
    wr = (0.5 * (b - a) * w[None, :]).ravel()
    g, gp = gfun(r)
    if axis < 0:
        A = np.sum(wr * 4.0 * np.pi * r * r * g * g)
        B = np.sum(wr * 4.0 * np.pi * r * r * gp * gp)
    else:
        A = np.sum(wr * 4.0 * np.pi * r ** 4 * g * g / 3.0)
        B = np.sum(wr * 4.0 * np.pi * r * r * (g * g + 2.0 / 3.0 * r * g * gp + r * r * gp * gp / 3.0))
    return A, B


def radial_scales(fn, r0: float, r1: float, panels: int = 64, order: int = 20):
    """radial_scales_of for an atomic function r^power exp(-zeta r) [d_axis] h(r)."""
    def gfun(r):
        d = np.zeros((r.size, 3))
        d[:, 0] = r
        g, gg = atomic_function(d, fn.power, fn.zeta, -1, r0, r1)
        return g, gg[:, 0]
    return radial_scales_of(gfun, fn.axis, r1, panels, order)


class TrialFn:
    """One function of the refinement's trial integrals: its atom, its value and gradient at
    displacements d [..., 3] from the atom's nearest image, and its scales (A, B)."""

    def __init__(self, atom: int, evaluate, scales):
        self.atom = atom
        self.evaluate = evaluate
        self.scales = scales


def kohn_sham_trials(system):
    """The atomic functions of the system's enrichment list (no phase)."""
    out = []
    for fn in system.enr:
        out.append(TrialFn(fn.atom, lambda d, fn=fn: atomic_function(d, fn.power, fn.zeta, fn.axis, system.r0, system.r1),
                           radial_scales(fn, system.r0, system.r1)))
    return out


def lagrange_at(nodes: np.ndarray, t: np.ndarray):
    """ell_a(t) and ell_a'(t) of the Lagrange basis on `nodes` at points t (product formula;
    the derivative as the sum over the dropped factor).  Returns [len(t), len(nodes)] each."""
    n = nodes.size
    V = np.ones((t.size, n))
    D = np.zeros((t.size, n))
    for a in range(n):
        others = [j for j in range(n) if j != a]
        den = np.prod([nodes[a] - nodes[j] for j in others])
        V[:, a] = np.prod([t - nodes[j] for j in others], axis=0) / den
        D[:, a] = sum(np.prod([t - nodes[j] for j in others if j != k], axis=0) for k in others) / den
    return V, D


def box_rule(lo: np.ndarray, size: float, q: int):
    """Tensor Gauss points [q^3, 3] and weights [q^3] of the box [lo, lo + size]^3."""
    eta, w = gauss_rule(q)
    t = lo[None, :] + 0.5 * size * (eta[:, None] + 1.0)  # [q, 3] per direction
    wt = 0.5 * size * w
    iz, iy, ix = np.meshgrid(np.arange(q), np.arange(q), np.arange(q), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()  # qx fastest
    pts = np.stack([t[ix, 0], t[iy, 1], t[iz, 2]], axis=-1)
    return pts, wt[ix] * wt[iy] * wt[iz]


class AdaptiveRule:
    """The adaptive rule on the union of the enrichment supports of `system`."""

    def __init__(self, mesh: Mesh, system, tol: float, max_depth: int, trials=None):
        """trials: the TrialFn list (default: the system's atomic functions, kohn_sham_trials)."""
        self.mesh = mesh
        self.tol = float(tol)
        self.max_depth = int(max_depth)
        q = mesh.q1
        if trials is None:
            trials = kohn_sham_trials(system)
        atom_of = np.array([t.atom for t in trials], dtype=np.int64)
        self.support = {}  # atom -> support cells (ascending)
        fns_of_cell = {}
        for I in range(system.n_atoms):
            idx = np.nonzero(atom_of == I)[0]
            if idx.size == 0:
                continue
            cells = mesh.dilate_cells(mesh.cells_near(system.pos[I], system.r1))
            self.support[I] = cells
            for e in cells.tolist():
                fns_of_cell.setdefault(e, []).extend((I, int(i)) for i in idx)
        scales = {}
        vol = 4.0 / 3.0 * np.pi * system.r1 ** 3
        nd = mesh.nd
        for i, t in enumerate(trials):
            A, B = t.scales
            scales[i] = np.concatenate([[A, B], np.full(nd, np.sqrt(A * vol)), np.full(nd, np.sqrt(B * vol))])
        xi = mesh.ref.xi
        p1 = mesh.p1
        ia = np.arange(nd)
        iax, iay, iaz = ia % p1, (ia // p1) % p1, ia // (p1 * p1)
        self.cells = np.array(sorted(fns_of_cell), dtype=np.int64)
        self.leaves = {}  # cell -> list of (lo [3], size)
        h = mesh.h

        def trial(lo, size, fl, org):
            pts, wq = box_rule(lo, size, q)
            ref = 2.0 * (pts - org[None, :]) / h - 1.0
            Vx, Dx = lagrange_at(xi, ref[:, 0])
            Vy, Dy = lagrange_at(xi, ref[:, 1])
            Vz, Dz = lagrange_at(xi, ref[:, 2])
            Na = Vx[:, iax] * Vy[:, iay] * Vz[:, iaz]  # [q^3, nd]
            Ga = np.stack([Dx[:, iax] * Vy[:, iay] * Vz[:, iaz], Vx[:, iax] * Dy[:, iay] * Vz[:, iaz],
                           Vx[:, iax] * Vy[:, iay] * Dz[:, iaz]], axis=-1)  # [q^3, nd, 3]
            out = np.zeros((len(fl), 2 + 2 * nd))
            for j, (I, i) in enumerate(fl):
                d = min_image(pts - system.pos[I][None, :], mesh.L)
                v, g = trials[i].evaluate(d)
                out[j, 0] = np.sum(wq * v * v)
                out[j, 1] = np.sum(wq * (g * g).sum(-1))
                out[j, 2:2 + nd] = (wq * v) @ Na
                out[j, 2 + nd:] = np.einsum("q,qd,qad->a", wq, g, Ga)
            return out

        for e in self.cells.tolist():
            fl = fns_of_cell[e]
            bound = self.tol * np.array([scales[i] for (_, i) in fl])  # [nfn, 2 + 2 nd]
            leaves = []
            org = mesh.cell_origin[e].astype(np.float64)

            atoms = sorted({I for (I, _) in fl})

            def blind(lo, size):
                # the box meets an atom's ball of radius r1 but none of its Gauss points is inside
                pts, _ = box_rule(lo, size, q)
                for I in atoms:
                    c = min_image(lo + 0.5 * size - system.pos[I], mesh.L)
                    ex = np.maximum(np.abs(c) - 0.5 * size, 0.0)
                    if np.sqrt((ex * ex).sum()) < system.r1:
                        d = min_image(pts - system.pos[I][None, :], mesh.L)
                        if np.sqrt((d * d).sum(-1)).min() >= system.r1:
                            return True
                return False

            def refine(lo, size, depth):
                if depth == self.max_depth:
                    leaves.append((lo, size))
                    return
                kids = [(lo + 0.5 * size * CHILD_OFFSETS[c], 0.5 * size) for c in range(8)]
                if blind(lo, size):
                    for (k_lo, k_s) in kids:
                        refine(k_lo, k_s, depth + 1)
                    return
                own = trial(lo, size, fl, org)
                ksum = sum(trial(k_lo, k_s, fl, org) for (k_lo, k_s) in kids)
                if np.all(np.abs(own - ksum) <= bound):
                    leaves.append((lo, size))
                    return
                for (k_lo, k_s) in kids:
                    refine(k_lo, k_s, depth + 1)

            refine(org, h, 0)
            self.leaves[e] = leaves
        # points, weights and the FE basis at them, per cell
        xi = mesh.ref.xi
        self.points, self.weights, self.B, self.G = {}, {}, {}, {}
        for e in self.cells.tolist():
            P, Wt = [], []
            for (lo, size) in self.leaves[e]:
                pts, wq = box_rule(lo, size, q)
                P.append(pts)
                Wt.append(wq)
            P = np.concatenate(P)
            self.points[e] = P
            self.weights[e] = np.concatenate(Wt)
            ref = 2.0 * (P - mesh.cell_origin[e][None, :]) / h - 1.0  # reference coordinates in [-1, 1]
            Vx, Dx = lagrange_at(xi, ref[:, 0])
            Vy, Dy = lagrange_at(xi, ref[:, 1])
            Vz, Dz = lagrange_at(xi, ref[:, 2])
            p1 = mesh.p1
            a = np.arange(mesh.nd)
            ax, ay, az = a % p1, (a // p1) % p1, a // (p1 * p1)
            self.B[e] = Vx[:, ax] * Vy[:, ay] * Vz[:, az]  # [n_pts, nd]
            self.G[e] = np.stack([Dx[:, ax] * Vy[:, ay] * Vz[:, az], Vx[:, ax] * Dy[:, ay] * Vz[:, az],
                                  Vx[:, ax] * Vy[:, ay] * Dz[:, az]])  # [3, n_pts, nd], reference derivatives
        self.offsets = np.concatenate([[0], np.cumsum([self.points[e].shape[0] for e in self.cells.tolist()])])
        self.n_points = int(self.offsets[-1])

    def all_points(self) -> np.ndarray:
        """Every point of the rule [n_points, 3], cells ascending, leaves and points in rule order."""
        return np.concatenate([self.points[e] for e in self.cells.tolist()])

    def all_weights(self) -> np.ndarray:
        return np.concatenate([self.weights[e] for e in self.cells.tolist()])

    def cell_slice(self, e: int) -> slice:
        k = int(np.searchsorted(self.cells, e))
        return slice(int(self.offsets[k]), int(self.offsets[k + 1]))


class AdaptiveEnrichment:
    """Enrichment blocks (eqnorthC, eqnMoo, eqnHOEFEelelements in the Bloch-function form) with
    the adaptive rule.  V_adapt: V at every point of the rule (rule order).  atom_fn holds N^O
    at the Gauss points (for fields there, with the coefficients c of the adaptive numerator),
    atom_fn_adapt at the rule's points."""

    def __init__(self, mesh: Mesh, system, m: np.ndarray, kvec, rule: AdaptiveRule, V_adapt: np.ndarray):
        self.mesh = mesh
        self.rule = rule
        self.n_enr = system.n_enr
        dtype = np.float64 if kvec is None else np.complex128
        theta = mesh.bloch_phase(kvec)
        s = 2.0 / mesh.h
        atom_of = np.array([f.atom for f in system.enr], dtype=np.int64)
        self.atom_fn_adapt = []  # (atom, fn indices, cells, [Phi per cell], [gradPhi per cell])
        self.atom_fn = []  # (atom, fn indices, cells, Phi [nc, nq, F], gradPhi [nc, nq, F, 3]) at the Gauss points
        for I, cells in rule.support.items():
            idx = np.nonzero(atom_of == I)[0]
            F = idx.size
            NA, gNA = [], []
            for e in cells.tolist():
                x = rule.points[e]
                draw = x - system.pos[I][None, :]
                t = np.round(draw / mesh.L)
                d = draw - mesh.L * t
                ph = np.ones(x.shape[0]) if kvec is None else np.exp(1j * mesh.L * (t @ np.asarray(kvec)))
                v = np.zeros((x.shape[0], F), dtype=dtype)
                g = np.zeros((x.shape[0], F, 3), dtype=dtype)
                for j, i in enumerate(idx):
                    fn = system.enr[i]
                    vv, gg = atomic_function(d, fn.power, fn.zeta, fn.axis, system.r0, system.r1)
                    v[:, j] = ph * vv
                    g[:, j, :] = ph[:, None] * gg
                NA.append(v)
                gNA.append(g)
            # d_g = sum over (e, a) -> g of conj(theta_ea) sum_points w B_a N^A ; c = d / m
            dnum = np.zeros((mesh.N, F), dtype=dtype)
            for ci, e in enumerate(cells.tolist()):
                de = rule.B[e].T @ (rule.weights[e][:, None] * NA[ci])  # [nd, F]
                np.add.at(dnum, mesh.cell_dofs[e], np.conj(theta[e])[:, None] * de)
            c = dnum / m[:, None]
            Phi, gPhi = [], []
            for ci, e in enumerate(cells.tolist()):
                ce = theta[e][:, None] * c[mesh.cell_dofs[e]]  # [nd, F]
                Phi.append(NA[ci] - rule.B[e] @ ce)
                gp = gNA[ci].copy()
                for dd in range(3):
                    gp[:, :, dd] -= s * (rule.G[e][dd] @ ce)
                gPhi.append(gp)
            self.atom_fn_adapt.append((I, idx, cells, Phi, gPhi))
            # the same orthogonalized functions at the Gauss points of the support cells
            NAg, gNAg = atomic_part(mesh, system.pos[I], [system.enr[i] for i in idx], cells, system.r0, system.r1,
                                    kvec)
            ceg = theta[cells][:, :, None] * c[mesh.cell_dofs[cells]]  # [nc, nd, F]
            Phig = NAg - np.einsum("qa,eaf->eqf", mesh.B, ceg)
            gPhig = gNAg.copy()
            for dd in range(3):
                gPhig[..., dd] -= s * np.einsum("qa,eaf->eqf", mesh.Gref[dd], ceg)
            self.atom_fn.append((I, idx, cells, Phig, gPhig))
        nO = self.n_enr
        Moo = np.zeros((nO, nO), dtype=dtype)
        Hoo = np.zeros((nO, nO), dtype=dtype)
        for (I, iI, cI, PI, gI) in self.atom_fn_adapt:
            for (J, iJ, cJ, PJ, gJ) in self.atom_fn_adapt:
                common, aI, aJ = np.intersect1d(cI, cJ, return_indices=True)
                for e, i, j in zip(common.tolist(), aI.tolist(), aJ.tolist()):
                    w = rule.weights[e]
                    Ve = V_adapt[rule.cell_slice(e)]
                    a, b = PI[i], PJ[j]
                    Moo[np.ix_(iI, iJ)] += np.conj(a).T @ (w[:, None] * b)
                    Hoo[np.ix_(iI, iJ)] += 0.5 * np.einsum("pfd,pgd->fg", np.conj(gI[i]) * w[:, None, None], gJ[j])
                    Hoo[np.ix_(iI, iJ)] += np.conj(a).T @ ((w * Ve)[:, None] * b)
        self.Moo, self.Hoo = Moo, Hoo
        rows, cols, vals = [], [], []
        for (I, idx, cells, Phi, gPhi) in self.atom_fn_adapt:
            for ci, e in enumerate(cells.tolist()):
                w = rule.weights[e]
                Ve = V_adapt[rule.cell_slice(e)]
                he = rule.B[e].T @ ((w * Ve)[:, None] * Phi[ci])
                for dd in range(3):
                    he += 0.5 * s * rule.G[e][dd].T @ (w[:, None] * gPhi[ci][:, :, dd])
                he = np.conj(theta[e])[:, None] * he
                rows.append(np.repeat(mesh.cell_dofs[e], idx.size))
                cols.append(np.tile(idx, mesh.nd))
                vals.append(he.reshape(-1))
        if rows:
            self.Hco = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                     shape=(mesh.N, nO)).tocsr()
            self.Hco.sum_duplicates()
        else:
            self.Hco = sp.csr_matrix((mesh.N, nO), dtype=dtype)
        if nO:
            lam, U = np.linalg.eigh(Moo)
            self.Moo_eigs = lam
            self.S = (U / np.sqrt(lam)[None, :]) @ np.conj(U.T)
        else:
            self.Moo_eigs = np.zeros(0)
            self.S = np.zeros((0, 0), dtype=dtype)


class AdaptiveOEFEOperator(OEFEOperator):
    """The Kohn-Sham operator (Gamma or Bloch-function form) with the enrichment blocks on the
    adaptive rule; H^cc and V at the Gauss points as in OEFEOperator."""

    def __init__(self, system, tol: float, max_depth: int, V: np.ndarray | None = None,
                 V_adapt: np.ndarray | None = None, kvec="system"):
        super().__init__(system, V=V, kvec=kvec)
        self.rule = AdaptiveRule(self.mesh, system, tol, max_depth)
        if V_adapt is None:
            V_adapt = nuclear_potential(self.rule.all_points(), system.pos, system.Z, system.sigma, system.L)
        self.V_adapt = np.ascontiguousarray(V_adapt, dtype=np.float64)
        self.enr = AdaptiveEnrichment(self.mesh, system, self.m, self.kvec, self.rule, self.V_adapt)


class AdaptiveUFormOperator:
    """The k-point operator in the periodic-function form (oracle/uform.py: eqnksdftu,
    eqnUOEFEAtomic, eqnHOEFEelelements with its k terms, the enrichment blocks' first-derivative
    term in the Hermitian form) with the enrichment integrals on the adaptive rule: N^A =
    exp(-i k.(x - R^x)) psi~ at the rule's points, the orthogonalization numerator, M^oo, H^oo
    and H^co on the rule; H^cc on the Gauss rule.  V_adapt: V at the rule's points (without the
    |k|^2/2, which is added here as on the Gauss points)."""

    def __init__(self, system, kvec, tol: float, max_depth: int, V: np.ndarray | None = None,
                 V_adapt: np.ndarray | None = None):
        from .uform import UFormOperator
        base = UFormOperator(system, kvec, V=V)
        self.base = base
        self.mesh = mesh = base.mesh
        self.kvec = k = base.kvec
        self.N, self.n_enr, self.n_tot = base.N, base.n_enr, base.n_tot
        self.dm12, self.Hcc, self.V = base.dm12, base.Hcc, base.V
        self.rule = rule = AdaptiveRule(mesh, system, tol, max_depth)
        if V_adapt is None:
            V_adapt = nuclear_potential(rule.all_points(), system.pos, system.Z, system.sigma, system.L)
        self.V_adapt = np.ascontiguousarray(V_adapt, dtype=np.float64)
        k2 = 0.5 * float(k @ k)
        s = 2.0 / mesh.h
        m = base.m
        atom_of = np.array([f.atom for f in system.enr], dtype=np.int64)
        fn = []
        for I, cells in rule.support.items():
            idx = np.nonzero(atom_of == I)[0]
            F = idx.size
            NA, gNA = [], []
            for e in cells.tolist():
                x = rule.points[e]
                d = min_image(x - system.pos[I][None, :], mesh.L)
                ph = np.exp(-1j * (d @ k))
                v = np.zeros((x.shape[0], F), dtype=np.complex128)
                g = np.zeros((x.shape[0], F, 3), dtype=np.complex128)
                for j, i in enumerate(idx):
                    f = system.enr[i]
                    vv, gg = atomic_function(d, f.power, f.zeta, f.axis, system.r0, system.r1)
                    v[:, j] = ph * vv
                    g[:, j, :] = ph[:, None] * (gg - 1j * k[None, :] * vv[:, None])
                NA.append(v)
                gNA.append(g)
            dnum = np.zeros((mesh.N, F), dtype=np.complex128)
            for ci, e in enumerate(cells.tolist()):
                np.add.at(dnum, mesh.cell_dofs[e], rule.B[e].T @ (rule.weights[e][:, None] * NA[ci]))
            c = dnum / m[:, None]
            Phi, gPhi = [], []
            for ci, e in enumerate(cells.tolist()):
                ce = c[mesh.cell_dofs[e]]  # periodic FE functions: no phase
                Phi.append(NA[ci] - rule.B[e] @ ce)
                gp = gNA[ci].copy()
                for dd in range(3):
                    gp[:, :, dd] -= s * (rule.G[e][dd] @ ce)
                gPhi.append(gp)
            fn.append((I, idx, cells, Phi, gPhi))
        self.atom_fn_adapt = fn
        nO = self.n_enr
        Moo = np.zeros((nO, nO), dtype=np.complex128)
        Hoo = np.zeros((nO, nO), dtype=np.complex128)
        for (I, iI, cI, PI, gI) in fn:
            for (J, iJ, cJ, PJ, gJ) in fn:
                common, aI, aJ = np.intersect1d(cI, cJ, return_indices=True)
                for e, i, j in zip(common.tolist(), aI.tolist(), aJ.tolist()):
                    w = rule.weights[e]
                    Ve = self.V_adapt[rule.cell_slice(e)] + k2
                    a, b, ga, gb = PI[i], PJ[j], gI[i], gJ[j]
                    Moo[np.ix_(iI, iJ)] += np.conj(a).T @ (w[:, None] * b)
                    Hoo[np.ix_(iI, iJ)] += 0.5 * np.einsum("pfd,pgd->fg", np.conj(ga) * w[:, None, None], gb)
                    Hoo[np.ix_(iI, iJ)] += -0.5j * np.einsum("pf,pgd,d->fg", np.conj(a) * w[:, None], gb, k)
                    Hoo[np.ix_(iI, iJ)] += 0.5j * np.einsum("pfd,pg,d->fg", np.conj(ga) * w[:, None, None], b, k)
                    Hoo[np.ix_(iI, iJ)] += np.conj(a).T @ ((w * Ve)[:, None] * b)
        self.Moo, self.Hoo = Moo, Hoo
        rows, cols, vals = [], [], []
        for (I, idx, cells, Phi, gPhi) in fn:
            for ci, e in enumerate(cells.tolist()):
                w = rule.weights[e]
                Ve = self.V_adapt[rule.cell_slice(e)] + k2
                he = rule.B[e].T @ ((w * Ve)[:, None] * Phi[ci])
                for dd in range(3):
                    he += 0.5 * s * rule.G[e][dd].T @ (w[:, None] * gPhi[ci][:, :, dd])
                    he += -0.5j * k[dd] * rule.B[e].T @ (w[:, None] * gPhi[ci][:, :, dd])
                    he += 0.5j * k[dd] * s * rule.G[e][dd].T @ (w[:, None] * Phi[ci])
                rows.append(np.repeat(mesh.cell_dofs[e], idx.size))
                cols.append(np.tile(idx, mesh.nd))
                vals.append(he.reshape(-1))
        self.Hco = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                 shape=(mesh.N, nO)).tocsr()
        self.Hco.sum_duplicates()
        lam, U = np.linalg.eigh(Moo)
        self.Moo_eigs = lam
        self.S = (U / np.sqrt(lam)[None, :]) @ np.conj(U.T)

    def apply(self, X: np.ndarray) -> np.ndarray:
        """Ht_k X for a block X [n_tot, nv] (complex)."""
        N = self.N
        Zc = self.dm12[:, None] * X[:N].astype(np.complex128)
        Zo = self.S @ X[N:].astype(np.complex128)
        Yc = self.dm12[:, None] * (self.Hcc @ Zc + self.Hco @ Zo)
        Yo = self.S @ (self.Hco.conj().T @ Zc + self.Hoo @ Zo)
        return np.concatenate([Yc, Yo], axis=0)


def poisson_trials(system, rc: np.ndarray, alpha: np.ndarray):
    """The auxiliary-potential enrichment's atomic functions (V_H - Z v_g) h(r), one per atom
    (oracle/poisson.py), as trial functions of the rule."""
    from .enrichment import cutoff
    from .poisson import phi_atomic
    out = []
    for I in range(system.n_atoms):
        Z, a, r_c = float(system.Z[I]), float(alpha[I]), float(rc[I])

        def gfun(r, Z=Z, a=a, r_c=r_c):
            f, fp = phi_atomic(r, Z, a, r_c)
            h, dh = cutoff(r, system.r0, system.r1)
            return f * h, fp * h + f * dh

        def evaluate(d, gfun=gfun):
            r = np.sqrt((d * d).sum(-1))
            g, gp = gfun(r)
            rhat = d / np.where(r > 0, r, 1.0)[..., None]
            return g, gp[..., None] * rhat

        out.append(TrialFn(I, evaluate, radial_scales_of(gfun, -1, system.r1)))
    return out


class AdaptivePoissonOEFE:
    """The auxiliary-potential Poisson problem (oracle/poisson.py: eqnpoissonaux, eqnPhiOEFE,
    eqnpoissX, eqnDiscLaplace, eqnDiscForceVec) with the integrals of its enrichment functions on
    the adaptive rule built from them: the orthogonalization numerator, A^co, A^oo and the
    enrichment rows of the force vector, for which the charge is taken at the rule's points.
    A^cc and the FE rows of the force vector keep the Gauss rule, and so does the background
    (the Gauss-rule mean of b + rho)."""

    def __init__(self, system, tol: float, max_depth: int):
        from .poisson import FOUR_PI, PoissonOEFE
        base = PoissonOEFE(system)
        self.base = base
        self.mesh = mesh = base.mesh
        self.N, self.n_enr, self.n_tot, self.m = base.N, base.n_enr, base.n_tot, base.m
        self.Acc, self.rc, self.alpha = base.Acc, base.rc, base.alpha
        self.system = system
        trials = poisson_trials(system, base.rc, base.alpha)
        self.rule = rule = AdaptiveRule(mesh, system, tol, max_depth, trials=trials)
        s = 2.0 / mesh.h
        self.atoms = []  # (cells, [Phi per cell], [gradPhi per cell]) at the rule's points
        self.atoms_gauss = []  # (cells, Phi [nc, nq]) at the Gauss points, same coefficients
        for I in range(self.n_enr):
            cells = rule.support[I]
            NA, gNA = [], []
            for e in cells.tolist():
                v, g = trials[I].evaluate(min_image(rule.points[e] - system.pos[I][None, :], mesh.L))
                NA.append(v)
                gNA.append(g)
            dnum = np.zeros(mesh.N)
            for ci, e in enumerate(cells.tolist()):
                np.add.at(dnum, mesh.cell_dofs[e], rule.B[e].T @ (rule.weights[e] * NA[ci]))
            c = dnum / self.m
            Phi, gPhi = [], []
            for ci, e in enumerate(cells.tolist()):
                ce = c[mesh.cell_dofs[e]]
                Phi.append(NA[ci] - rule.B[e] @ ce)
                gPhi.append(gNA[ci] - s * np.stack([rule.G[e][dd] @ ce for dd in range(3)], axis=-1))
            self.atoms.append((cells, Phi, gPhi))
            vg, _ = trials[I].evaluate(min_image(mesh.quad_points(cells) - system.pos[I], mesh.L))
            self.atoms_gauss.append((cells, vg - c[mesh.cell_dofs[cells]] @ mesh.B.T))
        rows, cols, vals = [], [], []
        for I, (cells, Phi, gPhi) in enumerate(self.atoms):
            for ci, e in enumerate(cells.tolist()):
                w = rule.weights[e]
                he = sum(s * rule.G[e][dd].T @ (w * gPhi[ci][:, dd]) for dd in range(3)) / FOUR_PI
                rows.append(mesh.cell_dofs[e])
                cols.append(np.full(mesh.nd, I))
                vals.append(he)
        self.Aco = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                 shape=(self.N, self.n_enr)).tocsr()
        self.Aco.sum_duplicates()
        Aoo = np.zeros((self.n_enr, self.n_enr))
        for I, (cI, _, gI) in enumerate(self.atoms):
            for J, (cJ, _, gJ) in enumerate(self.atoms):
                common, iI, iJ = np.intersect1d(cI, cJ, return_indices=True)
                for e, i, j in zip(common.tolist(), iI.tolist(), iJ.tolist()):
                    Aoo[I, J] += np.sum(rule.weights[e][:, None] * gI[i] * gJ[j]) / FOUR_PI
        self.Aoo = Aoo

    def smeared_charge_at(self, x: np.ndarray) -> np.ndarray:
        """b at points x [..., 3] (eqnsmeared, nearest image)."""
        from .poisson import g_smeared
        b = np.zeros(x.shape[:-1])
        for I in range(self.n_enr):
            d = min_image(x - self.system.pos[I], self.mesh.L)
            b -= self.system.Z[I] * g_smeared(np.sqrt((d * d).sum(-1)), self.rc[I])
        return b

    def model_density_at(self, x: np.ndarray) -> np.ndarray:
        """The model atomic densities at points x [..., 3] (nearest image)."""
        from .poisson import model_density
        rho = np.zeros(x.shape[:-1])
        for I in range(self.n_enr):
            d = min_image(x - self.system.pos[I], self.mesh.L)
            rho += model_density(np.sqrt((d * d).sum(-1)), self.system.Z[I], self.alpha[I])
        return rho

    def force_vector(self, rho_q: np.ndarray, rho_adapt: np.ndarray) -> np.ndarray:
        """c: FE rows int f N_m on the Gauss rule with f = b + rho - background (the Gauss-rule
        mean of b + rho), enrichment rows int f N^O on the rule with f at its points."""
        f_q = self.base.neutral_charge(rho_q)
        tot = self.base.smeared_charge() + rho_q.reshape(f_q.shape)
        W = self.mesh.Wcell[None, :]
        mean = (W * tot).sum() / (W.sum() * self.mesh.n_cells)
        cC = self.base.force_vector(f_q)[:self.N]
        f_a = self.smeared_charge_at(self.rule.all_points()) + rho_adapt - mean
        cO = np.zeros(self.n_enr)
        for I, (cells, Phi, _) in enumerate(self.atoms):
            for ci, e in enumerate(cells.tolist()):
                cO[I] += np.sum(self.rule.weights[e] * f_a[self.rule.cell_slice(e)] * Phi[ci])
        return np.concatenate([cC, cO])

    def matrix(self) -> sp.csr_matrix:
        return sp.bmat([[self.Acc, self.Aco], [self.Aco.T, sp.csr_matrix(self.Aoo)]], format="csr")

    def solve(self, rho_q: np.ndarray, rho_adapt: np.ndarray) -> np.ndarray:
        """phi with A phi = c (dense least squares on small systems, Jacobi CG otherwise), the FE part
        with zero GLL-mass-weighted mean."""
        import scipy.sparse.linalg as spla
        c = self.force_vector(rho_q, rho_adapt)
        A = self.matrix()
        if self.n_tot <= 3000:
            phi = np.linalg.lstsq(A.toarray(), c, rcond=None)[0]
        else:
            phi, info = spla.cg(A, c, rtol=1e-13, atol=0.0, maxiter=20000, M=sp.diags(1.0 / A.diagonal()))
            if info != 0:
                raise RuntimeError(f"oracle CG did not converge ({info})")
        return self.base.fix_constant(phi)

    def field_at_quad(self, phi: np.ndarray) -> np.ndarray:
        """phi_aux^h at the Gauss points [n_cells, nq] (eqnPhiOEFE)."""
        mesh = self.mesh
        out = phi[mesh.cell_dofs] @ mesh.B.T
        for I, (cells, Phi) in enumerate(self.atoms_gauss):
            out[cells] += phi[self.N + I] * Phi
        return out
