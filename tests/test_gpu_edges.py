"""Edge cases of the HIP path against the oracle: an operator without enrichment (the periodic
Laplacian: no coupling blocks, no enrichment rows), a single vector, leading dimensions with
padding columns that must stay untouched, degree-1 filters, and argument errors."""
import numpy as np
import pytest

from oracle import chfsi as och
from oracle.operator import OEFEOperator
from paper_2010_09701_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_2010_09701_amd import oefe
    return oefe


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _colrel(A, B):
    return float((np.linalg.norm(A - B, axis=0) / np.maximum(np.linalg.norm(B, axis=0), 1e-300)).max())


def test_free_laplacian_operator_and_spectrum(lib):
    """No atoms: H = -1/2 Laplacian.  ham_apply against the oracle; 6 ChFSI passes reach the
    lowest eigenvalues of the oracle's dense operator (0 and the first plane-wave shell)."""
    from paper_2010_09701_amd.chfsi import chfsi_run
    sysm = wl.free_system(L=5.0, nc=3, p=3)
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    assert gop.n_enr == 0 and gop.n_tot == op.n_tot
    X = wl.start_block(op.n_tot, 9, 1)
    assert _colrel(lib.ham_apply(gop, _dev(X)).cpu().numpy(), op.apply(X)) < 1e-10
    lam = np.linalg.eigvalsh(op.dense())
    nv = 12
    r = chfsi_run(gop, _dev(wl.start_block(op.n_tot, nv, 2)), _dev(wl.lanczos_start(op.n_tot, 2)), 12, 6, 10)
    assert abs(lam[0]) < 1e-10  # the constant vector
    np.testing.assert_allclose(r["theta"][:7], lam[:7], atol=1e-8)


def test_single_vector(lib):
    sysm = wl.single_atom()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    X = wl.start_block(op.n_tot, 1, 5)
    assert _colrel(lib.ham_apply(gop, _dev(X)).cpu().numpy(), op.apply(X)) < 1e-10
    a0, b = -20.0, 60.0
    Y = _dev(X)
    lib.chebyshev_filter(gop, Y, 7, 5.0, b, a0)
    assert _colrel(Y.cpu().numpy(), och.chebyshev_filter(op.apply, X, 7, 5.0, b, a0)) < 1e-10


def test_degree_one_filter(lib):
    sysm = wl.single_atom()
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    X = wl.start_block(op.n_tot, 6, 6)
    Y = _dev(X)
    lib.chebyshev_filter(gop, Y, 1, 5.0, 60.0, -20.0)
    assert _colrel(Y.cpu().numpy(), och.chebyshev_filter(op.apply, X, 1, 5.0, 60.0, -20.0)) < 1e-10


def test_padding_columns_untouched(lib):
    """ld > nv: the filter and the operator write only the first nv columns of each row."""
    import torch
    sysm = wl.diamond8(nc=3, p=4)
    op = OEFEOperator(sysm)
    gop = lib.Operator(sysm)
    nv, ld = 11, 16
    X = wl.start_block(op.n_tot, nv, 8)
    full = np.full((op.n_tot, ld), 7.25)
    full[:, :nv] = X
    Fd = _dev(full)
    lib.chebyshev_filter(gop, Fd[:, :nv], 4, 500.0, 2000.0, -20.0)
    got = Fd.cpu().numpy()
    assert np.all(got[:, nv:] == 7.25)
    assert _colrel(got[:, :nv], och.chebyshev_filter(op.apply, X, 4, 500.0, 2000.0, -20.0)) < 1e-10
    Y = torch.full((op.n_tot, ld), -3.5, dtype=torch.float64, device="cuda")
    lib.ham_apply(gop, _dev(full)[:, :nv], Y[:, :nv])
    assert np.all(Y.cpu().numpy()[:, nv:] == -3.5)


def test_argument_errors(lib):
    import torch
    gop = lib.Operator(wl.single_atom())
    X = torch.zeros((gop.n_tot, 4), dtype=torch.float64, device="cuda")
    w = gop.work(lib.F64, 4)
    L = lib._lib
    # nv = 0, ld < nv, degree 0, bounds out of order
    assert L.ham_apply(gop.handle, lib.F64, X.data_ptr(), X.data_ptr(), 4, 0, w.data_ptr(), None) != 0
    assert L.ham_apply(gop.handle, lib.F64, X.data_ptr(), X.data_ptr(), 3, 4, w.data_ptr(), None) != 0
    assert L.chebyshev_filter(gop.handle, lib.F64, X.data_ptr(), 4, 4, 0, 1.0, 2.0, 0.0, w.data_ptr(), None) != 0
    assert L.chebyshev_filter(gop.handle, lib.F64, X.data_ptr(), 4, 4, 5, 1.0, 2.0, 1.5, w.data_ptr(), None) != 0
    # a complex precision for a Gamma-point operator, a null block
    assert L.ham_apply(gop.handle, lib.C128, X.data_ptr(), X.data_ptr(), 4, 4, w.data_ptr(), None) != 0
    assert L.ham_apply(gop.handle, lib.F64, None, X.data_ptr(), 4, 4, w.data_ptr(), None) != 0
    assert L.oefe_strerror(-1)
    # the device is still healthy afterwards
    Y = lib.ham_apply(gop, X + 1.0)
    assert torch.isfinite(Y).all()


def test_copy_rate_copies_exactly(lib):
    """The stream-copy kernel behind the bench's achievable-bandwidth figure: an exact copy
    (ragged element count, not a multiple of the grid), a positive rate, and argument checks."""
    import torch
    src = torch.arange(1_000_003 * 2, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    g = lib.copy_rate(src, dst, 2)
    torch.cuda.synchronize()
    assert g > 0 and torch.equal(src, dst)
    with pytest.raises(lib.OefeError):
        lib.copy_rate(src[1:], dst[1:], 1)  # 8-byte aligned, odd size
