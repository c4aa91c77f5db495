"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Tolerances (float64): element/column-wise relative 1e-10 for one operator
application and for a filter from random vectors; Ritz values to
1e-10 max(1, |theta|); subspaces per gap-separated multiplet (sine of the
largest principal angle) to 1e-8.  Sizes span several cell tiles and ragged
vector blocks.
"""
import os

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import chfsi as och
from oracle.operator import OEFEOperator
from paper_2010_09701_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2010_09701_amd import oefe
    return oefe


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _colrel(A, B):
    num = np.linalg.norm(A - B, axis=0)
    den = np.maximum(np.linalg.norm(B, axis=0), 1e-300)
    return float((num / den).max())


SYSTEMS = {
    "single_atom": lambda: wl.single_atom(),
    "tiny2": lambda: wl.tiny_system(nc=2, p=2, n_atoms=2, seed=7, L=5.0, r0=0.8, r1=2.0),
    "p3": lambda: wl.tiny_system(nc=3, p=3, n_atoms=2, seed=11, L=7.0, r0=1.0, r1=2.5),
    "diamond_nc4": lambda: wl.diamond8(nc=4, p=4),
}


@pytest.mark.parametrize("name,nv", [("single_atom", 8), ("single_atom", 13), ("tiny2", 5), ("p3", 24),
                                     ("diamond_nc4", 72), ("diamond_nc4", 17),
                                     ("single_atom", 1), ("tiny2", 1), ("p3", 1), ("diamond_nc4", 1)])
def test_ham_apply_f64(lib, name, nv):
    sysm = SYSTEMS[name]()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    assert gop.n_tot == op.n_tot
    X = wl.start_block(op.n_tot, nv, 0)
    Y = lib.ham_apply(gop, _dev(X)).cpu().numpy()
    assert _colrel(Y, op.apply(X)) < 1e-10


@pytest.mark.parametrize("name", ["single_atom", "tiny2", "p3", "diamond_nc4"])
def test_ham_apply_one_column_matches_block(lib, name):
    """One column (cells in the lanes of the cell stage; at few coupled functions per tile, one wave
    per tile in the node stage) against the same column inside a block of 9 (columns in the lanes,
    matrix-core coupling): equal up to the order of the coupling sums."""
    sysm = SYSTEMS[name]()
    gop = lib.Operator(sysm)
    X = wl.start_block(gop.n_tot, 9, 4)
    Yb = lib.ham_apply(gop, _dev(X)).cpu().numpy()
    for j in (0, 5):
        y1 = lib.ham_apply(gop, _dev(np.ascontiguousarray(X[:, j:j + 1]))).cpu().numpy()[:, 0]
        assert np.abs(y1 - Yb[:, j]).max() <= 1e-13 * np.abs(Yb[:, j]).max(), (name, j)


def test_ham_apply_leading_dimension(lib):
    import torch
    sysm = SYSTEMS["single_atom"]()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    X = wl.start_block(op.n_tot, 20, 0)
    Xd = _dev(X)[:, 3:14]  # ld = 20, nv = 11
    Yd = torch.zeros(op.n_tot, 20, dtype=torch.float64, device="cuda")[:, 3:14]
    lib.ham_apply(gop, Xd, Yd)
    assert _colrel(Yd.cpu().numpy(), op.apply(X[:, 3:14])) < 1e-10


@pytest.mark.parametrize("name,nv", [("single_atom", 8), ("tiny2", 6), ("p3", 16)])
def test_ham_apply_bloch_c128(lib, name, nv):
    k = np.array([0.21, -0.37, 0.13])
    sysm = SYSTEMS[name]().with_k(k)
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    X = wl.start_block(op.n_tot, nv, 3, complex_=True)
    Y = lib.ham_apply(gop, _dev(X)).cpu().numpy()
    assert _colrel(Y, op.apply(X)) < 1e-10


@pytest.mark.parametrize("nv", [40, 1])
def test_ham_apply_f32(lib, nv):
    import torch
    sysm = SYSTEMS["diamond_nc4"]()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    X = wl.start_block(op.n_tot, nv, 0)
    Y = lib.ham_apply(gop, _dev(X, torch.float32)).cpu().numpy().astype(np.float64)
    # float32 arithmetic: relative error a few 1e-7 times the operator's spread
    assert _colrel(Y, op.apply(X.astype(np.float32).astype(np.float64))) < 5e-5


@pytest.mark.parametrize("name,nv,m", [("single_atom", 8, 20), ("diamond_nc4", 24, 30)])
def test_filter_f64(lib, name, nv, m):
    sysm = SYSTEMS[name]()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    X = wl.start_block(op.n_tot, nv, 0)
    H = None
    a0, b, _, _ = och.lanczos_bounds(op.apply, wl.lanczos_start(op.n_tot, 2), 10)
    a = 0.5 * (a0 + b)
    Xd = _dev(X)
    lib.chebyshev_filter(gop, Xd, m, a, b, a0)
    Y = och.chebyshev_filter(op.apply, X, m, a, b, a0)
    assert _colrel(Xd.cpu().numpy(), Y) < 1e-10


def test_filter_on_diagonal_operator_matches_closed_form(lib):
    rng = np.random.default_rng(0)
    lam = np.sort(rng.uniform(-3, 50, 777))
    gop = lib.Operator.diagonal(lam)
    X = rng.standard_normal((777, 9))
    m, a0, a, b = 33, lam[0], lam[40], 51.0
    Xd = _dev(X)
    lib.chebyshev_filter(gop, Xd, m, a, b, a0)
    e, c = (b - a) / 2, (b + a) / 2
    gain = och.chebyshev_T(m, (lam - c) / e) / och.chebyshev_T(m, np.array([(a0 - c) / e]))[0]
    np.testing.assert_allclose(Xd.cpu().numpy(), gain[:, None] * X, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("name,kvec,nv,m,dt", [("single_atom", None, 8, 20, "f64"), ("diamond_nc4", None, 24, 30, "f64"),
                                                ("single_atom", None, 13, 7, "f32"), ("single_atom", None, 5, 1, "f64"),
                                                ("tiny2", np.array([0.2, 0.3, -0.1]), 6, 9, "c128")])
def test_filter_dev_matches_filter(lib, name, kvec, nv, m, dt):
    """Bounds read from device memory give the same block, bit for bit, as the same bounds passed by value."""
    import torch
    sysm = SYSTEMS[name]() if kvec is None else SYSTEMS[name]().with_k(kvec)
    gop = lib.Operator(sysm)
    X = wl.start_block(gop.n_tot, nv, 3)
    if dt == "c128":
        X = X + 1j * wl.start_block(gop.n_tot, nv, 4)
    Xd = _dev(X)
    if dt == "f32":
        Xd = Xd.float()
    a0, b = lib.lanczos_bounds(gop, _dev(wl.lanczos_start(gop.n_tot, 2)), 10)
    a = 0.37 * a0 + 0.63 * b
    Y1, Y2 = Xd.clone(), Xd.clone()
    lib.chebyshev_filter(gop, Y1, m, a, b, a0)
    bounds = torch.tensor([a, b, a0], dtype=torch.float64, device="cuda")
    st = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    lib.chebyshev_filter_dev(gop, Y2, m, bounds, st)
    torch.cuda.synchronize()
    assert st.tolist() == [0, -1]
    assert torch.equal(Y1, Y2)


def test_filter_dev_invalid_bounds_in_status(lib):
    import torch
    gop = lib.Operator(SYSTEMS["single_atom"]())
    Xd = _dev(wl.start_block(gop.n_tot, 4, 1))
    st = torch.zeros(2, dtype=torch.int32, device="cuda")
    for bad in ([5.0, 1.0, 0.0], [1.0, 5.0, 2.0], [float("nan"), 5.0, 0.0]):
        bounds = torch.tensor(bad, dtype=torch.float64, device="cuda")
        lib.chebyshev_filter_dev(gop, Xd, 6, bounds, st)  # no exception: the status carries it
        torch.cuda.synchronize()
        assert st.tolist() == [-1, 0]
        assert not Xd.abs().max().item()  # zero scalars: the filter writes zeros
    with pytest.raises(lib.OefeError):
        lib.chebyshev_filter_dev(gop, Xd, 161, bounds, st)


def test_chfsi_device_bounds_match_host_bounds(lib):
    """The device-resident pass sequence (float64, no callback) against the per-pass host path
    (forced by a callback): same Ritz values and block, bit for bit."""
    from paper_2010_09701_amd.chfsi import chfsi_run
    sysm = SYSTEMS["single_atom"]()
    gop = lib.Operator(sysm)
    X0 = _dev(wl.start_block(gop.n_tot, 10, 1))
    v0 = _dev(wl.lanczos_start(gop.n_tot, 2))
    rd = chfsi_run(gop, X0, v0, 12, 4, 10)
    rh = chfsi_run(gop, X0, v0, 12, 4, 10, callback=lambda it, X, th: None)
    for pd, ph in zip(rd["passes"], rh["passes"]):
        assert (pd["a"], pd["b"], pd["a0"]) == (ph["a"], ph["b"], ph["a0"])
        assert np.array_equal(pd["theta"], ph["theta"])
    assert np.array_equal(rd["X"].cpu().numpy(), rh["X"].cpu().numpy())


def test_lanczos_bounds(lib):
    """Both bounds to 1e-10 relative each, the first pass's cut (a0 + b) / 2 from the library, and
    the device copy {a, b, a0} the device-bounds filter reads."""
    import torch
    sysm = SYSTEMS["single_atom"]()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    v0 = wl.lanczos_start(op.n_tot, 2)
    a0, b, _, _ = och.lanczos_bounds(op.apply, v0, 10)
    dev = torch.zeros(3, dtype=torch.float64, device="cuda")
    ga0, gb, ga = lib.lanczos_bounds(gop, _dev(v0), 10, dev_bounds=dev, with_cut=True)
    assert abs(ga0 - a0) <= 1e-10 * abs(a0) and abs(gb - b) <= 1e-10 * abs(b)
    assert ga == 0.5 * (ga0 + gb)
    assert dev.cpu().tolist() == [ga, gb, ga0]


def test_rayleigh_ritz_status_and_next_bounds(lib):
    """The eigensolver status {0, sweeps} and the next pass's bounds a = theta_nv, a0 = theta_1
    written into device memory (b left as it was)."""
    import torch
    sysm = SYSTEMS["single_atom"]()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    lam, U = np.linalg.eigh(op.dense())
    rng = np.random.default_rng(3)
    Q, _ = och.cholgs(U[:, :12] + 1e-3 * rng.standard_normal((op.n_tot, 12)))
    st = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    nb = torch.tensor([0.0, 123.5, 0.0], dtype=torch.float64, device="cuda")
    th = lib.rayleigh_ritz(gop, _dev(Q), st, nb)
    sth, nbh, thh = st.cpu().tolist(), nb.cpu().tolist(), th.cpu().numpy()
    assert sth[0] == 0 and 1 <= sth[1] <= 40
    assert nbh == [thh[-1], 123.5, thh[0]]


def test_rayleigh_ritz_sweep_limit_reports_enoconv(lib):
    """A sweep limit below what the projected matrix needs: the eigensolver stops there, the call
    returns normally and the status carries OEFE_ENOCONV with the sweep count; chfsi_run raises.
    The limit also reaches the Lanczos bounds' eigensolver.  Restored afterwards."""
    import torch
    from paper_2010_09701_amd.chfsi import chfsi_run
    sysm = SYSTEMS["p3"]()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    rng = np.random.default_rng(5)
    Q, _ = och.cholgs(rng.standard_normal((op.n_tot, 40)))
    st = torch.zeros(2, dtype=torch.int32, device="cuda")
    try:
        lib.set_eig_sweep_limit(gop, 1)
        lib.rayleigh_ritz(gop, _dev(Q), st)
        assert st.cpu().tolist() == [-5, 1]
        with pytest.raises(lib.OefeError) as ei:
            lib.lanczos_bounds(gop, _dev(wl.lanczos_start(op.n_tot, 2)), 10)
        assert ei.value.code == -5
        with pytest.raises(lib.OefeError) as ei:
            chfsi_run(gop, _dev(Q), _dev(wl.lanczos_start(op.n_tot, 2)), 4, 1, 10,
                      bounds=(-1.0, 50.0, 10.0))
        assert ei.value.code == -5
    finally:
        lib.set_eig_sweep_limit(gop, 0)
    lib.rayleigh_ritz(gop, _dev(Q), st)
    assert st.cpu().tolist()[0] == 0


@pytest.mark.parametrize("nv", [1, 2, 15, 16, 37, 80, 81])
def test_cholgs_matches_oracle(lib, nv):
    """Block widths on both sides of the matrix-core Gram path (16..80 columns) and of its
    3-row-block groups; 1 and 2 columns for the degenerate schedules."""
    sysm = SYSTEMS["diamond_nc4"]()
    gop = lib.Operator(sysm)
    rng = np.random.default_rng(5)
    Y = rng.standard_normal((gop.n_tot, nv)) @ np.diag(np.logspace(0, 4, nv))
    Q, _ = och.cholgs(Y)
    Yd = _dev(Y)
    lib.cholgs(gop, Yd)
    Qg = Yd.cpu().numpy()
    np.testing.assert_allclose(Qg, Q, atol=1e-10)
    np.testing.assert_allclose(Qg.T @ Qg, np.eye(nv), atol=1e-12)


def test_cholgs_breakdown_is_reported(lib):
    import torch
    sysm = SYSTEMS["single_atom"]()
    gop = lib.Operator(sysm)
    rng = np.random.default_rng(6)
    Y = rng.standard_normal((gop.n_tot, 6))
    Y[:, 4] = Y[:, 1] + Y[:, 2]
    st = torch.zeros(2, dtype=torch.int32, device="cuda")
    Yd = _dev(Y)
    with pytest.raises(lib.OefeError) as ei:
        lib.cholgs(gop, Yd, st)
    assert ei.value.code == -4
    assert int(st[1]) == 4
    # the failed factorization leaves the block as it was
    assert np.array_equal(Yd.cpu().numpy(), Y)


@pytest.mark.parametrize("nv", [6, 72, 81])
def test_cholgs_async_matches_cholgs(lib, nv):
    """The queued CholGS gives the synchronous one's block bit for bit (6 and 72 columns on the
    device-gated path, 81 through the synchronous fallback) and status {0, -1}."""
    import torch
    sysm = SYSTEMS["diamond_nc4"]()
    gop = lib.Operator(sysm)
    rng = np.random.default_rng(8)
    Y = rng.standard_normal((gop.n_tot, nv)) @ np.diag(np.logspace(0, 4, nv))
    A, B = _dev(Y), _dev(Y)
    lib.cholgs(gop, A)
    st = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    lib.cholgs_async(gop, B, st)
    torch.cuda.synchronize()
    assert st.tolist() == [0, -1]
    assert torch.equal(A, B)


def test_cholgs_async_breakdown_in_status(lib):
    import torch
    sysm = SYSTEMS["single_atom"]()
    gop = lib.Operator(sysm)
    rng = np.random.default_rng(6)
    Y = rng.standard_normal((gop.n_tot, 6))
    Y[:, 4] = Y[:, 1] + Y[:, 2]
    st = torch.zeros(2, dtype=torch.int32, device="cuda")
    Yd = _dev(Y)
    lib.cholgs_async(gop, Yd, st)  # no exception: the status carries the breakdown
    torch.cuda.synchronize()
    assert st.tolist() == [-4, 4]
    assert np.array_equal(Yd.cpu().numpy(), Y)


def _multiplet_angles(th, Xa, Xb, tol=1e-6):
    """Largest sine of principal angles between Xa and Xb restricted to each gap-separated multiplet."""
    groups = np.split(np.arange(len(th)), np.nonzero(np.diff(th) > tol * max(1, np.abs(th).max()))[0] + 1)
    worst = 0.0
    for g in groups[:-1]:  # the last group may straddle the block edge
        A, B = Xa[:, g], Xb[:, g]
        s = np.linalg.norm(B - A @ (np.conj(A.T) @ B), 2)
        worst = max(worst, s)
    return worst


def test_rayleigh_ritz_matches_oracle(lib):
    sysm = SYSTEMS["single_atom"]()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    H = op.dense()
    lam, U = np.linalg.eigh(H)
    rng = np.random.default_rng(7)
    Q, _ = och.cholgs(U[:, :10] + 1e-3 * rng.standard_normal((op.n_tot, 10)))
    th, Xr = och.rayleigh_ritz(op.apply, Q)
    Qd = _dev(Q)
    thg = lib.rayleigh_ritz(gop, Qd).cpu().numpy()
    assert np.abs(thg - th).max() < 1e-10 * max(1, np.abs(th).max())
    assert _multiplet_angles(th, Xr, Qd.cpu().numpy()) < 1e-8


@pytest.mark.parametrize("name,kvec,nv", [("single_atom", None, 1), ("single_atom", None, 2), ("single_atom", None, 11),
                                          ("p3", None, 40), ("p3", None, 80), ("p3", None, 91), ("p3", None, 100),
                                          ("p3", None, 130),
                                          ("single_atom", (0.3, -0.2, 0.1), 21), ("p3", (-0.4, 0.25, 0.1), 33),
                                          ("p3", (-0.4, 0.25, 0.1), 80)])
def test_rayleigh_ritz_odd_sizes_and_bloch(lib, name, kvec, nv):
    """Odd block widths (a padded round-robin schedule) and Hermitian (Bloch) projected
    matrices: Ritz values and multiplet subspaces against the oracle's eigh.  Real widths up
    to 86 and complex widths up to 68 take the one-barrier Jacobi (double-buffered matrix);
    91 and 100 (two blocks per thread), 130 (three) and complex 80 take the two-barrier
    kernel; 130 also takes the LDS eigenvector kernel (more than 64 pairs) and the vector-ALU
    Gram and Ritz products (more than 80 columns)."""
    base = SYSTEMS[name]()
    sysm = base if kvec is None else base.with_k(np.array(kvec))
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    lam, U = np.linalg.eigh(op.dense())
    rng = np.random.default_rng(11)
    noise = rng.standard_normal((op.n_tot, nv))
    if kvec is not None:
        noise = noise + 1j * rng.standard_normal((op.n_tot, nv))
    Q, _ = och.cholgs(U[:, :nv] + 1e-3 * noise)
    th, Xr = och.rayleigh_ritz(op.apply, Q)
    Qd = _dev(Q)
    thg = lib.rayleigh_ritz(gop, Qd).cpu().numpy()
    assert np.abs(thg - th).max() < 1e-10 * max(1, np.abs(th).max())
    assert _multiplet_angles(th, Xr, Qd.cpu().numpy()) < 1e-8


def test_chfsi_single_atom_passes(lib):
    from paper_2010_09701_amd.chfsi import chfsi_run
    cfg = wl.config("single_atom")
    op = OEFEOperator(cfg.system)
    gop = lib.Operator(cfg.system)
    X0 = wl.start_block(op.n_tot, cfg.nv, 0)
    v0 = wl.lanczos_start(op.n_tot, 2)
    r = och.chfsi(op.apply, X0, v0, cfg.m, cfg.passes, cfg.lanczos_k)
    g = chfsi_run(gop, _dev(X0), _dev(v0), cfg.m, cfg.passes, cfg.lanczos_k)
    assert abs(g["b"] - r["b"]) < 1e-9 * abs(r["b"])
    for pg, po in zip(g["passes"], r["passes"]):
        assert np.abs(pg["theta"] - po["theta"]).max() < 1e-10 * max(1.0, np.abs(po["theta"]).max())


@pytest.mark.parametrize("kvec", [None, np.array([0.2, 0.3, -0.1])])
def test_band_energy_grad(lib, kvec):
    sysm = SYSTEMS["tiny2"]().with_k(kvec)
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    nv = 5
    X = wl.start_block(op.n_tot, nv, 1, complex_=kvec is not None)
    f = wl.occupations(nv, 3)
    import torch
    E, dV, dX = lib.band_energy_grad(gop, _dev(X), torch.from_numpy(f))
    Eo = adj.band_energy(op, X, f)
    assert abs(float(E) - Eo) < 1e-10 * abs(Eo)
    gv = adj.grad_V(op, X, f)
    np.testing.assert_allclose(dV.cpu().numpy(), gv, rtol=1e-10, atol=1e-12 * np.abs(gv).max())
    assert _colrel(dX.cpu().numpy(), adj.grad_X(op, X, f)) < 1e-10


def test_band_energy_grad_p4(lib):
    import torch
    sysm = SYSTEMS["diamond_nc4"]()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    nv = 70
    X = wl.start_block(op.n_tot, nv, 1)
    f = wl.occupations(nv, 3)
    E, dV, dX = lib.band_energy_grad(gop, _dev(X), torch.from_numpy(f))
    gv = adj.grad_V(op, X, f)
    np.testing.assert_allclose(dV.cpu().numpy(), gv, rtol=1e-10, atol=1e-12 * np.abs(gv).max())
    assert abs(float(E) - adj.band_energy(op, X, f)) < 1e-10 * abs(float(E))


@pytest.mark.parametrize("name,kvec", [("tiny2", None), ("diamond_nc4", None), ("p3", (-0.4, 0.25, 0.1)),
                                       ("single_atom", (0.3, -0.2, 0.1))])
def test_set_potential(lib, name, kvec):
    """The potential-dependent operator data rebuilt on the device (W V, H^co in every layout, H^oo):
    re-setting the creation potential reproduces the operator built on the host, and a perturbed
    potential gives the oracle's operator for that potential, in float64 and float32."""
    import torch
    base = SYSTEMS[name]()
    sysm = base if kvec is None else base.with_k(np.array(kvec))
    gop = lib.Operator(sysm)
    V0, W = gop.get_potential()
    op0 = OEFEOperator(sysm)
    np.testing.assert_allclose(V0, op0.V, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(W, np.broadcast_to(op0.mesh.Wcell, W.shape), rtol=1e-13)
    X = wl.start_block(op0.n_tot, 7, 2, complex_=kvec is not None)
    Y0 = lib.ham_apply(gop, _dev(X)).cpu().numpy()
    gop.set_potential(V0)
    Y1 = lib.ham_apply(gop, _dev(X)).cpu().numpy()
    assert _colrel(Y1, Y0) < 1e-13
    dV = wl.potential_perturbation(op0.mesh.n_cells, op0.mesh.nq, 101)
    gop.set_potential(torch.from_numpy(V0 + 0.3 * dV).cuda())
    Vg, _ = gop.get_potential()
    assert np.array_equal(Vg, V0 + 0.3 * dV)
    op = OEFEOperator(sysm, V=op0.V + 0.3 * dV)
    Y = lib.ham_apply(gop, _dev(X)).cpu().numpy()
    ref = op.apply(X)
    assert _colrel(Y, ref) < 1e-10
    dt = torch.complex64 if kvec is not None else torch.float32
    Yf = lib.ham_apply(gop, _dev(X, dt)).cpu().numpy().astype(ref.dtype)
    assert _colrel(Yf, ref) < 1e-5


def test_enrichment_overlap_and_S(lib):
    sysm = SYSTEMS["diamond_nc4"]()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    S, ev = gop.get_enrichment()
    np.testing.assert_allclose(ev, op.enr.Moo_eigs, rtol=1e-9)
    np.testing.assert_allclose(S, op.enr.S, atol=1e-9 * np.abs(op.enr.S).max())


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "diamond8_oracle.npz")), reason="golden file missing")
def test_diamond8_full_size(lib):
    """Workload diamond8 (12^3 cells, p = 4, 72 vectors): sampled rows of Ht X0, the bounds, and
    pass-1 filter rows against stored oracle values."""
    cfg = wl.config("diamond8")
    g = np.load(os.path.join(GOLD, "diamond8_oracle.npz"))
    gop = lib.Operator(cfg.system)
    X0 = wl.start_block(gop.n_tot, cfg.nv, 0)
    Y = lib.ham_apply(gop, _dev(X0)).cpu().numpy()
    rows = g["rows"]
    scale = g["hx_colnorm"][None, :] / np.sqrt(gop.n_tot)
    assert np.abs(Y[rows] - g["hx_rows"]).max() / np.abs(g["hx_rows"]).max() < 1e-10
    a0, b = lib.lanczos_bounds(gop, _dev(wl.lanczos_start(gop.n_tot, 2)), 10)
    assert abs(a0 - float(g["a0L"])) <= 1e-10 * abs(a0) and abs(b - float(g["b"])) <= 1e-10 * abs(b)
    Xd = _dev(X0)
    a0o, bo = float(g["a0L"]), float(g["b"])
    lib.chebyshev_filter(gop, Xd, cfg.m, 0.5 * (a0o + bo), bo, a0o)
    Yf = Xd.cpu().numpy()
    assert np.abs(Yf[rows] - g["filt1_rows"]).max() / np.abs(g["filt1_rows"]).max() < 1e-9
    np.testing.assert_allclose(np.linalg.norm(Yf, axis=0), g["filt1_colnorm"], rtol=1e-9)
    del scale


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "diamond8_oracle.npz")), reason="golden file missing")
def test_diamond8_chfsi_ritz_values(lib):
    from paper_2010_09701_amd.chfsi import chfsi_run
    cfg = wl.config("diamond8")
    g = np.load(os.path.join(GOLD, "diamond8_oracle.npz"))
    gop = lib.Operator(cfg.system)
    X0 = wl.start_block(gop.n_tot, cfg.nv, 0)
    v0 = wl.lanczos_start(gop.n_tot, 2)
    r = chfsi_run(gop, _dev(X0), _dev(v0), cfg.m, cfg.passes, cfg.lanczos_k)
    th = np.stack([p["theta"] for p in r["passes"]])
    assert np.abs(th - g["thetas"]).max() < 1e-10 * np.abs(g["thetas"]).max()


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "diamond64_oracle.npz")), reason="golden file missing")
def test_diamond64_full_size_rows(lib):
    """Workload diamond64 (24^3 cells, 320 enrichment functions, 320 vectors): sampled rows of Ht X0."""
    cfg = wl.config("diamond64")
    g = np.load(os.path.join(GOLD, "diamond64_oracle.npz"))
    gop = lib.Operator(cfg.system)
    X0 = wl.start_block(gop.n_tot, cfg.nv, 0)
    Y = lib.ham_apply(gop, _dev(X0)).cpu().numpy()
    rows = g["rows"]
    assert np.abs(Y[rows] - g["hx_rows"]).max() / np.abs(g["hx_rows"]).max() < 1e-10


@pytest.mark.parametrize("dt", ["float64", "float32"])
def test_filter_bitwise_across_launch_shapes_and_runs(lib, dt):
    """Fixed-order sums everywhere (no atomics): the same filter on a real operator gives the same
    bits from run to run and for every launch shape of the cell and node stages."""
    import torch
    dtype = getattr(torch, dt)
    sysm = SYSTEMS["diamond_nc4"]()
    gop = lib.Operator(sysm)
    X0 = _dev(wl.start_block(gop.n_tot, 72, 0), dtype)
    a0, b, a = lib.lanczos_bounds(gop, _dev(wl.lanczos_start(gop.n_tot, 2)), 10, with_cut=True)
    ref = X0.clone()
    lib.chebyshev_filter(gop, ref, 7, a, b, a0)
    again = X0.clone()
    lib.chebyshev_filter(gop, again, 7, a, b, a0)
    assert torch.equal(ref, again)
    try:
        for cw, cb in ((8, 32), (16, 64), (32, 128), (64, 16)):
            lib.set_launch_shape(gop, cw, cb)
            X = X0.clone()
            lib.chebyshev_filter(gop, X, 7, a, b, a0)
            assert torch.equal(ref, X), (cw, cb)
    finally:
        lib.set_launch_shape(gop, 0, 0)


@pytest.mark.parametrize("name,kvec,nv", [("diamond_nc4", None, 150), ("diamond_nc4", None, 161),
                                          ("diamond_nc4", None, 320), ("p3", (-0.4, 0.25, 0.1), 110)])
def test_rayleigh_ritz_large_blocks(lib, name, kvec, nv):
    """Projected matrices above the LDS size (real from 141 columns, complex from 100): the Jacobi
    with one launch per round in global memory, the column-group-tiled matrix-core Gram and the
    eliminated Cholesky of CholGS; Ritz values and multiplet subspaces against the oracle."""
    import torch
    base = SYSTEMS[name]()
    sysm = base if kvec is None else base.with_k(np.array(kvec))
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    rng = np.random.default_rng(nv)
    X = rng.uniform(-1, 1, (op.n_tot, nv))
    if kvec is not None:
        X = X + 1j * rng.uniform(-1, 1, (op.n_tot, nv))
    # two filter degrees so that the projected matrix has a spread spectrum, as in a pass
    lam = och.lanczos_bounds(op.apply, wl.lanczos_start(op.n_tot, 2), 10)
    Y = och.chebyshev_filter(op.apply, X, 2, 0.5 * (lam[0] + lam[1]), lam[1], lam[0])
    Q, _ = och.cholgs(Y)
    th, Xr = och.rayleigh_ritz(op.apply, Q)
    Qd = _dev(Q)
    st = torch.zeros(2, dtype=torch.int32, device="cuda")
    thg = lib.rayleigh_ritz(gop, Qd, st).cpu().numpy()
    sth = st.cpu().tolist()
    assert sth[0] == 0 and 1 <= sth[1] <= 60, sth
    assert np.abs(thg - th).max() < 1e-10 * max(1, np.abs(th).max())
    assert _multiplet_angles(th, Xr, Qd.cpu().numpy()) < 1e-8
    # CholGS of the filtered block on the same path: orthonormal, same span as the oracle's Q
    Yd = _dev(Y)
    lib.cholgs(gop, Yd)
    Qg = Yd.cpu().numpy()
    assert np.abs(np.conj(Qg.T) @ Qg - np.eye(nv)).max() < 1e-12
    assert np.abs(Qg - Q @ (np.conj(Q.T) @ Qg)).max() < 1e-9
    # the eigensolver's sweep limit on this path
    try:
        lib.set_eig_sweep_limit(gop, 1)
        lib.rayleigh_ritz(gop, _dev(Q), st)
        assert st.cpu().tolist() == [-5, 1]
    finally:
        lib.set_eig_sweep_limit(gop, 0)


def test_cholgs_large_block_breakdown(lib):
    """A repeated column in a 150-column block: the eliminated Cholesky reports its index."""
    sysm = SYSTEMS["diamond_nc4"]()
    gop = lib.Operator(sysm)
    rng = np.random.default_rng(9)
    X = rng.uniform(-1, 1, (gop.n_tot, 150))
    X[:, 97] = X[:, 12]
    with pytest.raises(lib.OefeError) as ei:
        lib.cholgs(gop, _dev(X))
    assert ei.value.code == -4
    Xo = X.copy()
    with pytest.raises(och.CholeskyBreakdown) as eo:
        och.cholgs(Xo)
    assert f"column {eo.value.column}" in str(ei.value)
