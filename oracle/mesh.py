"""Structured periodic hex mesh with spectral (GLL) Lagrange elements.

Conventions (the paper is silent on ordering; these are the readings used on
both sides of the parity tests):

* n = nc * p nodes per direction; global FE index g = i + n j + n^2 k.
* cell e = cx + nc cy + nc^2 cz; local node a = ax + (p+1) ay + (p+1)^2 az
  (x fastest); local quadrature point q = qx + (p+1) qy + (p+1)^2 qz.
* node i = c p + a sits at x = c h + (xi_a + 1) h / 2 (periodic mod n).
* The lumped FE overlap is the GLL-quadrature mass (Sec. III.A: spectral
  elements with GLL quadrature make M^cc diagonal, eqnMcc, eqnorthCGLL).
"""
from __future__ import annotations

import numpy as np

from .quadrature import Reference1D


class Mesh:
    def __init__(self, L: float, nc: int, p: int):
        self.L = float(L)
        self.nc = int(nc)
        self.p = int(p)
        self.h = self.L / self.nc
        self.n = self.nc * self.p
        self.N = self.n ** 3
        self.ref = Reference1D(self.p)
        self.p1 = self.p + 1
        self.nd = self.p1 ** 3
        self.q1 = self.ref.q
        self.nq = self.q1 ** 3
        self.n_cells = self.nc ** 3
        self._build_maps()
        self._build_reference_3d()

    # -- DoF map -------------------------------------------------------------
    def _build_maps(self):
        nc, p, n, p1 = self.nc, self.p, self.n, self.p1
        cells = np.arange(self.n_cells)
        cx, cy, cz = cells % nc, (cells // nc) % nc, cells // (nc * nc)
        a = np.arange(self.nd)
        ax, ay, az = a % p1, (a // p1) % p1, a // (p1 * p1)
        ix = cx[:, None] * p + ax[None, :]
        iy = cy[:, None] * p + ay[None, :]
        iz = cz[:, None] * p + az[None, :]
        self.cell_dofs = (ix % n) + n * (iy % n) + n * n * (iz % n)  # [n_cells, nd]
        # wrap counts (0 or 1 per direction): how many periods the local node
        # lies beyond the primary cell range; used for Bloch phases.
        self.wrap = np.stack([ix // n, iy // n, iz // n], axis=-1)  # [n_cells, nd, 3]
        self.cell_origin = np.stack([cx, cy, cz], axis=-1) * self.h  # [n_cells, 3]

    def _build_reference_3d(self):
        r = self.ref
        p1, q1 = self.p1, self.q1
        # 3D interpolation B[q, a] and reference gradients G[d][q, a]
        B = np.zeros((self.nq, self.nd))
        G = np.zeros((3, self.nq, self.nd))
        for qz in range(q1):
            for qy in range(q1):
                for qx in range(q1):
                    q = qx + q1 * qy + q1 * q1 * qz
                    for az in range(p1):
                        for ay in range(p1):
                            for ax in range(p1):
                                a = ax + p1 * ay + p1 * p1 * az
                                bx, by, bz = r.B1[qx, ax], r.B1[qy, ay], r.B1[qz, az]
                                dx, dy, dz = r.D1[qx, ax], r.D1[qy, ay], r.D1[qz, az]
                                B[q, a] = bx * by * bz
                                G[0, q, a] = dx * by * bz
                                G[1, q, a] = bx * dy * bz
                                G[2, q, a] = bx * by * dz
        self.B = B
        self.Gref = G
        # quadrature weights of one cell (all cells are identical cubes)
        w = r.w
        wq = np.zeros(self.nq)
        for qz in range(q1):
            for qy in range(q1):
                for qx in range(q1):
                    wq[qx + q1 * qy + q1 * q1 * qz] = w[qx] * w[qy] * w[qz]
        self.Wcell = wq * (self.h / 2.0) ** 3  # [nq]
        # reference quadrature coordinates (in [0, h)^3 relative to the cell origin)
        eta = (r.eta + 1.0) * self.h / 2.0
        qc = np.zeros((self.nq, 3))
        for qz in range(q1):
            for qy in range(q1):
                for qx in range(q1):
                    qc[qx + q1 * qy + q1 * q1 * qz] = (eta[qx], eta[qy], eta[qz])
        self.qoffset = qc

    # -- geometry ------------------------------------------------------------
    def quad_points(self, cells=None) -> np.ndarray:
        """Physical quadrature points x_{e,q}, shape [len(cells), nq, 3]."""
        if cells is None:
            cells = np.arange(self.n_cells)
        return self.cell_origin[cells][:, None, :] + self.qoffset[None, :, :]

    def quad_weights(self) -> np.ndarray:
        """W_{e,q} for all cells, shape [n_cells, nq]."""
        return np.broadcast_to(self.Wcell, (self.n_cells, self.nq)).copy()

    def node_coords(self) -> np.ndarray:
        """Coordinates of all global nodes, shape [N, 3]."""
        n, p, h = self.n, self.p, self.h
        i = np.arange(n)
        c, a = i // p, i % p
        x1 = c * h + (self.ref.xi[a] + 1.0) * h / 2.0
        g = np.arange(self.N)
        return np.stack([x1[g % n], x1[(g // n) % n], x1[g // (n * n)]], axis=-1)

    def lumped_mass(self) -> np.ndarray:
        """m_g = sum over cells containing g of (h/2)^3 what_ax what_ay what_az."""
        p1 = self.p1
        wh = self.ref.what
        wa = np.zeros(self.nd)
        for az in range(p1):
            for ay in range(p1):
                for ax in range(p1):
                    wa[ax + p1 * ay + p1 * p1 * az] = wh[ax] * wh[ay] * wh[az]
        wa *= (self.h / 2.0) ** 3
        m = np.zeros(self.N)
        np.add.at(m, self.cell_dofs.ravel(), np.broadcast_to(wa, self.cell_dofs.shape).ravel())
        return m

    def cell_stiffness(self) -> np.ndarray:
        """K_e[a, a'] = 1/2 sum_q W_q (2/h)^2 sum_d G_d[q,a] G_d[q,a'] (identical for all cells)."""
        s = (2.0 / self.h) ** 2
        K = np.zeros((self.nd, self.nd))
        for d in range(3):
            K += self.Gref[d].T @ (self.Wcell[:, None] * self.Gref[d])
        return 0.5 * s * K

    def bloch_phase(self, kvec) -> np.ndarray:
        """theta(e, a) = exp(i k . L w(e, a)); all ones at Gamma."""
        if kvec is None:
            return np.ones(self.cell_dofs.shape)
        kvec = np.asarray(kvec, dtype=np.float64)
        return np.exp(1j * self.L * (self.wrap @ kvec))

    def cells_near(self, center, radius: float) -> np.ndarray:
        """Cells whose box comes within `radius` of `center` (minimum image)."""
        lo = self.cell_origin  # [n_cells, 3]
        d = np.asarray(center)[None, :] - (lo + self.h / 2.0)
        d -= self.L * np.round(d / self.L)
        # distance from point to axis-aligned box of half-width h/2 centred at 0
        ex = np.maximum(np.abs(d) - self.h / 2.0, 0.0)
        dist = np.sqrt((ex ** 2).sum(-1))
        return np.nonzero(dist < radius)[0]

    def dilate_cells(self, cells: np.ndarray) -> np.ndarray:
        """The given cells plus every cell that shares a node with one of them."""
        nc = self.nc
        c = np.asarray(cells)
        cx, cy, cz = c % nc, (c // nc) % nc, c // (nc * nc)
        out = set()
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    e = ((cx + dx) % nc) + nc * ((cy + dy) % nc) + nc * nc * ((cz + dz) % nc)
                    out.update(e.tolist())
        return np.array(sorted(out), dtype=np.int64)
