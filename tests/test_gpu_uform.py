"""The k-point operator in the periodic-function form on the GPU (oefe_op_create_uform) against the
oracle (oracle/uform.py).

* ham_apply (complex128) column by column against the oracle's Ht_k X to 1e-10 relative, on small
  systems at p = 2, 3, 4 and on single_atom; complex64 to 1e-5.
* k = 0: the form's operator equals the real Gamma-point operator (applied to real and imaginary
  parts) to 1e-12.
* Five ChFSI passes (complex128) on single_atom at a k-point: Ritz values against the oracle's passes
  to 1e-9 relative.
* Batches: two k-points of the form filtered in one batched call equal the per-operator filters
  bit for bit; a batch mixing the two forms is refused.
* set_potential / get_potential take and return V without the form's |k|^2/2.
* diamond8 at the Monkhorst-Pack k-points with the fewest and the most vectors (48, 96):
  sampled rows of Ht_k X column by column to 1e-10 and the column norms of the whole product to
  1e-10 against the oracle's stored values (tests/golden/make_golden.py uform_kpoints).
"""
import os

import numpy as np
import pytest

from oracle import chfsi as och
from oracle.uform import UFormOperator
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


def _systems():
    return {
        "tiny_p2": wl.tiny_system(nc=3, p=2, n_atoms=2, seed=7, L=5.0, r0=0.8, r1=2.0),
        "tiny_p3": wl.tiny_system(nc=3, p=3, n_atoms=2, seed=5, L=6.0, r0=1.0, r1=2.0),
        "tiny_p4": wl.tiny_system(nc=2, p=4, n_atoms=1, seed=3, L=6.0, r0=1.0, r1=2.0),
        "single_atom": wl.single_atom(),
    }


def _block(n, nv, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, size=(n, nv)) + 1j * rng.uniform(-1, 1, size=(n, nv))


@pytest.mark.parametrize("name", list(_systems()))
def test_uform_ham_apply_vs_oracle(lib, name):
    import torch
    sysm = _systems()[name].with_k(K)
    op = UFormOperator(sysm, K)
    gop = lib.Operator(sysm, uform=True)
    assert gop.is_complex and gop.n_tot == op.n_tot
    X = _block(op.n_tot, 6, 1)
    Yo = op.apply(X)
    Y = lib.ham_apply(gop, torch.from_numpy(X).cuda()).cpu().numpy()
    err = np.abs(Y - Yo).max(axis=0) / np.abs(Yo).max(axis=0)
    assert err.max() <= 1e-10, err
    Y32 = lib.ham_apply(gop, torch.from_numpy(X.astype(np.complex64)).cuda()).cpu().numpy()
    err32 = np.abs(Y32 - Yo).max(axis=0) / np.abs(Yo).max(axis=0)
    assert err32.max() <= 1e-5, err32


def test_uform_k0_is_gamma(lib):
    import torch
    sysm = _systems()["tiny_p3"]
    g0 = lib.Operator(sysm.with_k(np.zeros(3)), uform=True)
    gr = lib.Operator(sysm)
    X = _block(g0.n_tot, 4, 2)
    Y = lib.ham_apply(g0, torch.from_numpy(X).cuda()).cpu().numpy()
    Yr = lib.ham_apply(gr, torch.from_numpy(X.real.copy()).cuda()).cpu().numpy()
    Yi = lib.ham_apply(gr, torch.from_numpy(X.imag.copy()).cuda()).cpu().numpy()
    assert np.abs(Y - (Yr + 1j * Yi)).max() <= 1e-12 * np.abs(Y).max()


def test_uform_chfsi_passes_vs_oracle(lib):
    import torch
    from paper_2010_09701_amd.chfsi import chfsi_run
    cfg = wl.config("single_atom")
    sysm = cfg.system.with_k(K)
    op = UFormOperator(sysm, K)
    gop = lib.Operator(sysm, uform=True)
    X0 = wl.start_block(op.n_tot, cfg.nv, 0, complex_=True)
    v0 = wl.lanczos_start(op.n_tot, 2)
    r = och.chfsi(op.apply, X0, v0, cfg.m, cfg.passes, cfg.lanczos_k)
    g = chfsi_run(gop, torch.from_numpy(X0).cuda(), torch.from_numpy(v0).cuda(), cfg.m, cfg.passes, cfg.lanczos_k)
    for pg, po in zip(g["passes"], r["passes"]):
        scale = np.abs(po["theta"]).max()
        assert np.abs(pg["theta"] - po["theta"]).max() <= 1e-9 * scale


def test_uform_batched_equals_single_and_mixed_refused(lib):
    import torch
    sysm = _systems()["tiny_p4"]
    ks = [K, -0.5 * K]
    ops = [lib.Operator(sysm.with_k(k), uform=True) for k in ks]
    X = [torch.from_numpy(_block(ops[0].n_tot, 5 + i, 3 + i)).cuda() for i in range(2)]
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
    psi = lib.Operator(sysm.with_k(K))
    with pytest.raises(lib.OefeError):
        lib.chebyshev_filter_batched([ops[0], psi], [X[0].clone(), X[0].clone()], 2, [abc[0], abc[0]])


def test_uform_potential_round_trip(lib):
    sysm = _systems()["tiny_p2"].with_k(K)
    gop = lib.Operator(sysm, uform=True)
    op = UFormOperator(sysm, K)
    V, _ = gop.get_potential()
    assert np.abs(V - op.V).max() <= 1e-12 * np.abs(op.V).max()
    rng = np.random.default_rng(4)
    V2 = op.V + rng.uniform(-1, 1, size=op.V.shape)
    gop.set_potential(V2)
    V3, _ = gop.get_potential()
    assert np.abs(V3 - V2).max() <= 1e-13 * np.abs(V2).max()


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "uform_kpoints_oracle.npz")), reason="golden file missing")
def test_uform_diamond8_kpoint_rows(lib):
    import torch
    g = np.load(os.path.join(GOLD, "uform_kpoints_oracle.npz"))
    base = wl.config("diamond8").system
    for q in (0, 7):
        kv = g[f"k{q}"]
        op = lib.Operator(base.with_k(kv), uform=True)
        X0 = wl.start_block(op.n_tot, wl.KPOINT_NV[q], 10 + q, complex_=True)
        Y = lib.ham_apply(op, torch.from_numpy(X0).cuda()).cpu().numpy()
        rows, ref = g[f"rows{q}"], g[f"hx_rows{q}"]
        err = np.abs(Y[rows] - ref).max(axis=0) / np.abs(ref).max(axis=0)
        assert err.max() <= 1e-10, (q, err.max())
        cn = np.linalg.norm(Y, axis=0)
        assert np.abs(cn - g[f"hx_colnorm{q}"]).max() <= 1e-10 * cn.max(), q
