"""Seeded synthetic workloads for the ChFSI filter on the OEFE operator.

This module only describes *inputs*: periodic cell geometry, atom positions and
charges, the enrichment-function list, and seeded random blocks (starting
vectors, Lanczos start vector, occupations, potential perturbations).  It holds
none of the method's arithmetic (no quadrature, no basis, no potential, no
enrichment evaluation); both the CPU oracle and the HIP library build their
operators from these descriptions independently.

All random numbers come from ``numpy.random.default_rng(seed)`` in C order.

Workloads (stand-ins for the paper's solids; the paper's own systems need
atomic data and full SCF that are not part of the hot path):

* ``single_atom``: L = 10 bohr cube, 4^3 cells, degree-2 GLL, one Z = 3 atom at
  the centre, two s-type enrichment functions r^(n-1) exp(-Z r / n), n = 1, 2.
* ``diamond8``: 8-atom diamond cell (L = 10.26 bohr, Z = 14), atoms jittered by
  U[-0.1, 0.1] bohr (seed 1), 12^3 cells, degree 4, 5 enrichment functions per
  atom (1s, 2s, 2p_x, 2p_y, 2p_z Slater-type proxies).
* ``diamond64``: 2x2x2 supercell of ``diamond8`` (64 atoms, L = 20.52 bohr,
  24^3 cells, degree 4, 320 enrichment functions).

The enrichment functions follow the structure of the truncated atomic orbitals
of the paper (Sec. III.A, eqnKSAtomicTrunc): a radial factor r^a exp(-zeta r),
optionally times one Cartesian component of the displacement (a p-type
angular factor), times a smooth cutoff that is 1 inside r0 and 0 beyond r1.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

# Diamond-lattice fractional positions (conventional cubic cell, 8 atoms).
_DIAMOND_FRAC = np.array(
    [
        [0.0, 0.0, 0.0],
        [0.0, 0.5, 0.5],
        [0.5, 0.0, 0.5],
        [0.5, 0.5, 0.0],
        [0.25, 0.25, 0.25],
        [0.25, 0.75, 0.75],
        [0.75, 0.25, 0.75],
        [0.75, 0.75, 0.25],
    ]
)


@dataclasses.dataclass(frozen=True)
class EnrichmentFn:
    """One enrichment function: r^power * exp(-zeta r) * (d_axis if axis >= 0)."""

    atom: int
    power: int
    zeta: float
    axis: int  # -1: no angular factor; 0/1/2: multiply by d_x / d_y / d_z


@dataclasses.dataclass
class System:
    """Periodic cubic cell with a uniform hex mesh and atoms."""

    name: str
    L: float
    nc: int  # cells per dimension
    p: int  # FE degree (GLL nodes per cell edge = p + 1)
    pos: np.ndarray  # [n_atoms, 3] bohr, inside [0, L)
    Z: np.ndarray  # [n_atoms]
    sigma: float  # erf smoothing length of the nuclear potential
    r0: float  # cutoff: h = 1 for r <= r0
    r1: float  # cutoff: h = 0 for r >= r1
    enr: List[EnrichmentFn]
    kvec: Optional[np.ndarray] = None  # [3] Bloch wavevector (1/bohr); None = Gamma

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_fe(self) -> int:
        return (self.nc * self.p) ** 3

    @property
    def n_enr(self) -> int:
        return len(self.enr)

    @property
    def n_tot(self) -> int:
        return self.n_fe + self.n_enr

    @property
    def n_cells(self) -> int:
        return self.nc ** 3

    @property
    def nq(self) -> int:
        return (self.p + 1) ** 3

    def with_k(self, kvec) -> "System":
        s = dataclasses.replace(self)
        s.kvec = None if kvec is None else np.asarray(kvec, dtype=np.float64)
        return s

    def enr_arrays(self):
        """Flat arrays (atom, power, zeta, axis) of the enrichment list."""
        atom = np.array([f.atom for f in self.enr], dtype=np.int32)
        power = np.array([f.power for f in self.enr], dtype=np.int32)
        zeta = np.array([f.zeta for f in self.enr], dtype=np.float64)
        axis = np.array([f.axis for f in self.enr], dtype=np.int32)
        return atom, power, zeta, axis


def _s_type_pair(atom: int, Z: float) -> List[EnrichmentFn]:
    # r^(n-1) exp(-Z r / n) for n = 1, 2
    return [EnrichmentFn(atom, 0, Z, -1), EnrichmentFn(atom, 1, Z / 2.0, -1)]


def _sp_shell(atom: int, Z: float) -> List[EnrichmentFn]:
    # 1s, 2s, 2p_x, 2p_y, 2p_z Slater-type proxies
    return [
        EnrichmentFn(atom, 0, Z, -1),
        EnrichmentFn(atom, 1, Z / 2.0, -1),
        EnrichmentFn(atom, 0, Z / 2.0, 0),
        EnrichmentFn(atom, 0, Z / 2.0, 1),
        EnrichmentFn(atom, 0, Z / 2.0, 2),
    ]


def single_atom(nc: int = 4, p: int = 2) -> System:
    L = 10.0
    pos = np.array([[5.0, 5.0, 5.0]])
    Z = np.array([3.0])
    return System("single_atom", L, nc, p, pos, Z, 0.5, 2.0, 4.0, _s_type_pair(0, 3.0))


def diamond8(nc: int = 12, p: int = 4, jitter_seed: int = 1) -> System:
    a = 10.26
    rng = np.random.default_rng(jitter_seed)
    jit = rng.uniform(-0.1, 0.1, size=(8, 3))
    pos = np.mod(_DIAMOND_FRAC * a + jit, a)
    Z = np.full(8, 14.0)
    enr = []
    for i in range(8):
        enr += _sp_shell(i, 14.0)
    return System("diamond8", a, nc, p, pos, Z, 0.5, 2.0, 4.0, enr)


def diamond64(nc: int = 24, p: int = 4, jitter_seed: int = 1) -> System:
    a = 10.26
    frac = []
    for sz in range(2):
        for sy in range(2):
            for sx in range(2):
                frac.append(_DIAMOND_FRAC + np.array([sx, sy, sz], dtype=np.float64))
    frac = np.concatenate(frac, axis=0)  # [64, 3] in units of a
    rng = np.random.default_rng(jitter_seed)
    jit = rng.uniform(-0.1, 0.1, size=(64, 3))
    L = 2 * a
    pos = np.mod(frac * a + jit, L)
    Z = np.full(64, 14.0)
    enr = []
    for i in range(64):
        enr += _sp_shell(i, 14.0)
    return System("diamond64", L, nc, p, pos, Z, 0.5, 2.0, 4.0, enr)


def tiny_system(nc: int = 2, p: int = 2, n_atoms: int = 1, seed: int = 5, L: float = 6.0,
                r0: float = 1.0, r1: float = 2.0) -> System:
    """Very small system for brute-force checks (dense eigensolves)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, L, size=(n_atoms, 3))
    Z = np.full(n_atoms, 2.0)
    enr = []
    for i in range(n_atoms):
        enr += [EnrichmentFn(i, 0, 2.0, -1), EnrichmentFn(i, 0, 1.0, 0)]
    return System("tiny", L, nc, p, pos, Z, 0.5, r0, r1, enr)


def free_system(L: float, nc: int, p: int) -> System:
    """No atoms, no enrichment: the operator reduces to the periodic Laplacian."""
    return System("free", L, nc, p, np.zeros((0, 3)), np.zeros(0), 0.5, 2.0, 4.0, [])


def monkhorst_pack_2(L: float) -> np.ndarray:
    """The 8 k-points {+-1/4}^3 * 2 pi / L of a 2x2x2 Monkhorst-Pack grid."""
    ks = []
    for sz in (-1, 1):
        for sy in (-1, 1):
            for sx in (-1, 1):
                ks.append(np.array([sx, sy, sz], dtype=np.float64) * 0.25 * 2.0 * np.pi / L)
    return np.array(ks)


KPOINT_NV = [48, 54, 61, 68, 75, 82, 89, 96]


# ---------------------------------------------------------------- random blocks

def start_block(n_tot: int, nv: int, seed: int = 0, complex_: bool = False) -> np.ndarray:
    """Starting vectors U[-1, 1], shape [n_tot, nv] (row-major, vectors contiguous per DoF)."""
    rng = np.random.default_rng(seed)
    if complex_:
        re = rng.uniform(-1.0, 1.0, size=(n_tot, nv))
        im = rng.uniform(-1.0, 1.0, size=(n_tot, nv))
        return re + 1j * im
    return rng.uniform(-1.0, 1.0, size=(n_tot, nv))


def lanczos_start(n_tot: int, seed: int = 2) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=n_tot)


def occupations(nv: int, seed: int = 3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0, size=nv)


def potential_perturbation(n_cells: int, nq: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(n_cells, nq))


@dataclasses.dataclass
class RunConfig:
    system: System
    nv: int
    m: int  # Chebyshev degree
    passes: int = 5
    lanczos_k: int = 10
    x0_seed: int = 0
    v0_seed: int = 2


def config(name: str) -> RunConfig:
    """Named run configurations (filter degree, block width, passes)."""
    if name == "single_atom":
        return RunConfig(single_atom(), nv=8, m=20)
    if name == "diamond8":
        return RunConfig(diamond8(), nv=72, m=50)
    if name == "diamond64":
        return RunConfig(diamond64(), nv=320, m=60)
    raise KeyError(name)
