"""The operator with the adaptive quadrature of the enrichment integrals on the GPU
(oefe_op_create_adaptive, oefe_op_set_potential_adaptive) against the oracle (oracle/adaptive.py).

* The rule: the library's points and weights equal the oracle's (same leaves in the same order,
  coordinates to rounding).
* ham_apply column by column against the oracle's Ht X to 1e-10 relative (float64, complex128 at
  a Bloch k), on sharp-function systems at p = 2, 3, 4 (the rule refined near the nuclei).
* max_depth = 0 reproduces the Gauss-rule operator of oefe_op_create (1e-12).
* The potential on the device: after oefe_op_set_potential_adaptive with new V at the Gauss
  points and at the rule's points, ham_apply against the oracle built with the same values
  (1e-10); the plain oefe_op_set_potential and dE/dV of band_energy_grad are refused.
* Five ChFSI passes against the oracle's passes (Ritz values to 1e-9 relative), and the density
  at the Gauss points from the filtered block against the oracle's fields (1e-12).
* The periodic-function k-point form on the rule (oefe_op_create_uform_adaptive): ham_apply
  against the oracle to 1e-10, after oefe_op_set_potential_adaptive too (potentials without the
  |k|^2/2), and two k-points filtered in one batched call equal the per-operator filters.
* diamond8 (tol 1e-6, depth 2; 601,000 rule points) against the oracle's stored values
  (tests/golden/make_golden.py adaptive_diamond8): the rule's point count in every cell, sampled
  rows of Ht X column by column and the column norms to 1e-10, the eigenvalues of M^oo to 1e-12.
"""
import dataclasses
import os

import numpy as np
import pytest

from oracle import adaptive as ad
from oracle import chfsi as och
from oracle import occupations as oocc
from paper_2010_09701_amd import workloads as wl

pytestmark = pytest.mark.gpu
K = np.array([0.21, -0.13, 0.07])
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2010_09701_amd import oefe
    return oefe


def _sharp(nc, p, n_atoms=1, seed=3, L=6.0):
    s = wl.tiny_system(nc=nc, p=p, n_atoms=n_atoms, seed=seed, L=L, r0=1.0, r1=2.0)
    enr = []
    for i in range(n_atoms):
        enr += [wl.EnrichmentFn(i, 0, 6.0, -1), wl.EnrichmentFn(i, 1, 3.0, 0), wl.EnrichmentFn(i, 1, 3.0, 2)]
    return dataclasses.replace(s, enr=enr)


CASES = {
    "p2_two_atoms": (lambda: _sharp(3, 2, n_atoms=2, seed=7), 1e-7, 3, None),
    "p3": (lambda: _sharp(3, 3), 1e-6, 2, None),
    "p4": (lambda: _sharp(2, 4, L=5.0), 1e-6, 2, None),
    "p3_bloch": (lambda: _sharp(3, 3), 1e-6, 2, K),
}


def _block(n, nv, seed, cx):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(n, nv))
    return X + 1j * rng.uniform(-1, 1, size=(n, nv)) if cx else X


def _ops(lib, name):
    make, tol, depth, kv = CASES[name]
    s = make()
    if kv is not None:
        s = s.with_k(kv)
    return s, ad.AdaptiveOEFEOperator(s, tol, depth), lib.Operator(s, adaptive=(tol, depth))


@pytest.mark.parametrize("name", list(CASES))
def test_adaptive_rule_and_ham_apply_vs_oracle(lib, name):
    import torch
    s, o, g = _ops(lib, name)
    n, xyz, w = g.adaptive_points()
    assert n == o.rule.n_points and n > o.rule.cells.size * o.mesh.nq  # refined somewhere
    assert np.abs(xyz - o.rule.all_points()).max() <= 1e-13 * s.L
    assert np.abs(w - o.rule.all_weights()).max() <= 1e-14 * o.mesh.h ** 3
    X = _block(o.n_tot, 5, 1, o.complex)
    Yo = o.apply(X)
    Y = lib.ham_apply(g, torch.from_numpy(X).cuda()).cpu().numpy()
    err = np.abs(Y - Yo).max(axis=0) / np.abs(Yo).max(axis=0)
    assert err.max() <= 1e-10, err


def test_adaptive_depth0_is_the_gauss_operator(lib):
    import torch
    s = _sharp(3, 3)
    g0 = lib.Operator(s, adaptive=(1e-6, 0))
    gg = lib.Operator(s)
    X = torch.from_numpy(_block(gg.n_tot, 4, 2, False)).cuda()
    Y0 = lib.ham_apply(g0, X).cpu().numpy()
    Yg = lib.ham_apply(gg, X).cpu().numpy()
    assert np.abs(Y0 - Yg).max() <= 1e-12 * np.abs(Yg).max()


def test_adaptive_set_potential_vs_oracle_and_refusals(lib):
    import torch
    s, o, g = _ops(lib, "p3")
    rng = np.random.default_rng(5)
    V2 = o.V + rng.uniform(-1, 1, size=o.V.shape)
    Va2 = o.V_adapt + rng.uniform(-1, 1, size=o.V_adapt.shape)
    g.set_potential(V2, Va2)
    o2 = ad.AdaptiveOEFEOperator(s, 1e-6, 2, V=V2, V_adapt=Va2)
    X = _block(o.n_tot, 4, 3, False)
    Y = lib.ham_apply(g, torch.from_numpy(X).cuda()).cpu().numpy()
    Yo = o2.apply(X)
    err = np.abs(Y - Yo).max(axis=0) / np.abs(Yo).max(axis=0)
    assert err.max() <= 1e-10, err
    with pytest.raises(lib.OefeError):
        g.set_potential(V2)
    with pytest.raises(lib.OefeError):
        lib.band_energy_grad(g, torch.from_numpy(X).cuda(), torch.ones(4, dtype=torch.float64, device="cuda"))
    with pytest.raises(lib.OefeError):
        lib.Operator(s, adaptive=(0.0, 2))
    with pytest.raises(lib.OefeError):
        lib.Operator(s, adaptive=(1e-6, 6))


def test_adaptive_chfsi_passes_and_density_vs_oracle(lib):
    import torch
    from paper_2010_09701_amd.chfsi import chfsi_run
    s, o, g = _ops(lib, "p3")
    nv, m, passes = 12, 12, 5
    X0 = wl.start_block(o.n_tot, nv, 0)
    v0 = wl.lanczos_start(o.n_tot, 2)
    r = och.chfsi(o.apply, X0, v0, m, passes, 10)
    res = chfsi_run(g, torch.from_numpy(X0).cuda(), torch.from_numpy(v0).cuda(), m, passes, 10)
    for pg, po in zip(res["passes"], r["passes"]):
        scale = np.abs(po["theta"]).max()
        assert np.abs(pg["theta"] - po["theta"]).max() <= 1e-9 * scale
    X = torch.from_numpy(X0).cuda()
    wts = np.linspace(2.0, 0.5, nv)
    rho = lib.density(g, X, torch.from_numpy(wts)).cpu().numpy()
    rho_o = oocc.density(o, X0, wts)
    assert np.abs(rho - rho_o).max() <= 1e-12 * np.abs(rho_o).max()


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "adaptive_diamond8_oracle.npz")), reason="golden file missing")
def test_adaptive_diamond8_vs_stored_oracle(lib):
    import torch
    g = np.load(os.path.join(GOLD, "adaptive_diamond8_oracle.npz"))
    cfg = wl.config("diamond8")
    s = cfg.system
    op = lib.Operator(s, adaptive=(float(g["tol"]), int(g["max_depth"])))
    n, xyz, _ = op.adaptive_points()
    assert n == int(g["counts"].sum())
    h = s.L / s.nc
    c = np.floor(xyz / h).astype(np.int64)
    cell = c[:, 0] + s.nc * (c[:, 1] + s.nc * c[:, 2])
    per_cell = np.bincount(cell, minlength=s.nc ** 3)
    assert np.array_equal(per_cell[g["cells"]], g["counts"])
    X0 = wl.start_block(op.n_tot, 16, cfg.x0_seed)
    Y = lib.ham_apply(op, torch.from_numpy(X0).cuda()).cpu().numpy()
    rows, ref = g["rows"], g["hx_rows"]
    err = np.abs(Y[rows] - ref).max(axis=0) / np.abs(ref).max(axis=0)
    assert err.max() <= 1e-10, err.max()
    cn = np.linalg.norm(Y, axis=0)
    assert np.abs(cn - g["hx_colnorm"]).max() <= 1e-10 * cn.max()
    _, eig = op.get_enrichment()
    assert np.abs(eig - g["Moo_eigs"]).max() <= 1e-12 * np.abs(g["Moo_eigs"]).max()


def test_adaptive_uform_vs_oracle(lib):
    import torch
    s = _sharp(3, 3)
    o = ad.AdaptiveUFormOperator(s.with_k(K), K, 1e-6, 2)
    g = lib.Operator(s.with_k(K), uform=True, adaptive=(1e-6, 2))
    n, xyz, _ = g.adaptive_points()
    assert n == o.rule.n_points and np.abs(xyz - o.rule.all_points()).max() <= 1e-13 * s.L
    X = _block(o.n_tot, 5, 7, True)
    Y = lib.ham_apply(g, torch.from_numpy(X).cuda()).cpu().numpy()
    Yo = o.apply(X)
    err = np.abs(Y - Yo).max(axis=0) / np.abs(Yo).max(axis=0)
    assert err.max() <= 1e-10, err
    rng = np.random.default_rng(8)
    V2 = o.V + rng.uniform(-1, 1, size=o.V.shape)
    Va2 = o.V_adapt + rng.uniform(-1, 1, size=o.V_adapt.shape)
    g.set_potential(V2, Va2)
    o2 = ad.AdaptiveUFormOperator(s.with_k(K), K, 1e-6, 2, V=V2, V_adapt=Va2)
    Y = lib.ham_apply(g, torch.from_numpy(X).cuda()).cpu().numpy()
    Yo = o2.apply(X)
    err = np.abs(Y - Yo).max(axis=0) / np.abs(Yo).max(axis=0)
    assert err.max() <= 1e-10, err


def test_adaptive_uform_batched_equals_single(lib):
    import torch
    s = _sharp(3, 3)
    ks = [K, -0.5 * K]
    ops = [lib.Operator(s.with_k(k), uform=True, adaptive=(1e-6, 2)) for k in ks]
    X = [torch.from_numpy(_block(ops[0].n_tot, 4 + i, 11 + i, True)).cuda() for i in range(2)]
    abc = []
    for o in ops:
        v0 = torch.from_numpy(wl.lanczos_start(o.n_tot, 2).astype(np.complex128)).cuda()
        a0, b, a = lib.lanczos_bounds(o, v0, 8, with_cut=True)
        abc.append((a, b, a0))
    Xb = [x.clone() for x in X]
    lib.chebyshev_filter_batched(ops, Xb, 6, abc)
    for o, x, xb, (a, b, a0) in zip(ops, X, Xb, abc):
        xs = x.clone()
        lib.chebyshev_filter(o, xs, 6, a, b, a0)
        assert torch.equal(xs, xb)
