"""Python binding of liboefe.so (the C ABI in include/oefe.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  Vector blocks are torch tensors on the HIP device (row-major
[n_tot, nv] with unit column stride; complex dtypes for a Bloch operator);
calls are ordered on torch's current stream.  There is no CPU fallback: if
the library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch

from . import workloads

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboefe.so")

F64, F32, BF16, C128, C64 = 0, 1, 2, 3, 4
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOTSPD", -5: "ENOCONV", -6: "EUNSUPPORTED"}


class OefeError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {_STATUS.get(code, code)} ({msg})")
        self.code = code


class _Desc(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_double),
        ("nc", ctypes.c_int32),
        ("p", ctypes.c_int32),
        ("n_atoms", ctypes.c_int32),
        ("pos", ctypes.POINTER(ctypes.c_double)),
        ("Z", ctypes.POINTER(ctypes.c_double)),
        ("sigma", ctypes.c_double),
        ("r0", ctypes.c_double),
        ("r1", ctypes.c_double),
        ("n_enr", ctypes.c_int32),
        ("enr_atom", ctypes.POINTER(ctypes.c_int32)),
        ("enr_power", ctypes.POINTER(ctypes.c_int32)),
        ("enr_zeta", ctypes.POINTER(ctypes.c_double)),
        ("enr_axis", ctypes.POINTER(ctypes.c_int32)),
        ("kvec", ctypes.POINTER(ctypes.c_double)),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2010_09701_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "oefe_op_create": ([ctypes.POINTER(_Desc), ctypes.POINTER(vp)], i32),
        "oefe_op_create_diagonal": ([vp, i64, ctypes.POINTER(vp)], i32),
        "oefe_op_create_uform": ([vp, ctypes.POINTER(vp)], i32),
        "oefe_op_create_adaptive": ([vp, dbl, i32, ctypes.POINTER(vp)], i32),
        "oefe_op_create_uform_adaptive": ([vp, dbl, i32, ctypes.POINTER(vp)], i32),
        "oefe_op_adaptive_points": ([vp, vp, vp, vp], i32),
        "oefe_op_set_potential_adaptive": ([vp, vp, vp, vp], i32),
        "oefe_op_destroy": ([vp], i32),
        "oefe_op_dims": ([vp, vp], i32),
        "oefe_op_set_potential": ([vp, vp, vp], i32),
        "oefe_op_get_potential": ([vp, vp, vp], i32),
        "oefe_op_get_enrichment": ([vp, vp, vp], i32),
        "oefe_work_size": ([vp, i32, i32], ctypes.c_size_t),
        "ham_apply": ([vp, i32, vp, vp, i64, i32, vp, vp], i32),
        "chebyshev_filter": ([vp, i32, vp, i64, i32, i32, dbl, dbl, dbl, vp, vp], i32),
        "chebyshev_filter_mixed": ([vp, i32, vp, i64, i32, i32, dbl, dbl, dbl, vp, vp], i32),
        "chebyshev_filter_batched": ([i32, vp, i32, vp, vp, vp, i32, vp, vp, vp], i32),
        "oefe_batched_work_size": ([i32, vp, i32, vp], ctypes.c_size_t),
        "oefe_set_launch_shape": ([vp, i32, i32], i32),
        "oefe_autotune": ([i32, vp, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp], i32),
        "lanczos_bounds": ([vp, i32, vp, vp, vp, vp, vp], i32),
        "cholgs": ([vp, i32, vp, i64, i32, vp, vp, vp], i32),
        "cholgs_async": ([vp, i32, vp, i64, i32, vp, vp, vp], i32),
        "cholgs_noalloc": ([vp, i32, vp, i64, i32, vp, vp], i32),
        "chebyshev_filter_dev": ([vp, i32, vp, i64, i32, i32, vp, vp, vp, vp], i32),
        "rayleigh_ritz": ([vp, i32, vp, i64, i32, vp, vp, vp, vp, vp], i32),
        "oefe_set_eig_sweep_limit": ([vp, i32], i32),
        "band_energy_grad": ([vp, i32, vp, i64, i32, vp, vp, vp, vp, vp, vp], i32),
        "oefe_fermi_occupations": ([i32, vp, vp, vp, dbl, dbl, vp, vp, vp, vp], i32),
        "oefe_density": ([vp, i32, vp, i64, i32, vp, vp, i32, vp, vp], i32),
        "oefe_poisson_create": ([vp, ctypes.POINTER(vp)], i32),
        "oefe_poisson_create_adaptive": ([vp, dbl, i32, ctypes.POINTER(vp)], i32),
        "oefe_poisson_solve_adaptive": ([vp, vp, vp, vp, dbl, i32, vp, vp, vp], i32),
        "oefe_poisson_work_size": ([vp], ctypes.c_size_t),
        "oefe_poisson_solve": ([vp, vp, vp, dbl, i32, vp, vp, vp], i32),
        "oefe_kernel_timer": ([vp, i32], i32),
        "oefe_kernel_timer_read": ([vp, vp, vp], i32),
        "oefe_copy_rate": ([vp, vp, ctypes.c_size_t, i32, vp, vp], i32),
        "oefe_strerror": ([i32], ctypes.c_char_p),
        "oefe_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()

EXPORTED = [
    "oefe_op_create", "oefe_op_create_diagonal", "oefe_op_create_uform", "oefe_op_create_adaptive",
    "oefe_op_create_uform_adaptive",
    "oefe_op_adaptive_points", "oefe_op_set_potential_adaptive", "oefe_op_destroy", "oefe_op_dims", "oefe_op_set_potential",
    "oefe_op_get_potential", "oefe_op_get_enrichment", "oefe_work_size", "ham_apply", "chebyshev_filter",
    "chebyshev_filter_mixed", "chebyshev_filter_dev", "chebyshev_filter_batched", "oefe_batched_work_size", "oefe_set_launch_shape",
    "oefe_autotune",
    "lanczos_bounds", "cholgs", "cholgs_async", "cholgs_noalloc", "rayleigh_ritz", "oefe_set_eig_sweep_limit", "band_energy_grad",
    "oefe_fermi_occupations", "oefe_density", "oefe_poisson_create", "oefe_poisson_work_size", "oefe_poisson_solve",
    "oefe_poisson_create_adaptive", "oefe_poisson_solve_adaptive",
    "oefe_kernel_timer",
    "oefe_kernel_timer_read", "oefe_copy_rate", "oefe_strerror", "oefe_last_error",
]


def _check(rc: int, where: str):
    if rc != 0:
        raise OefeError(rc, where, _lib.oefe_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _prec(t: torch.Tensor, bf16: bool = False) -> int:
    if bf16 and t.dtype != torch.float32:
        raise TypeError("bf16 operands apply to float32 blocks of real operators")
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return BF16 if bf16 else F32
    if t.dtype == torch.complex128:
        return C128
    if t.dtype == torch.complex64:
        return C64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _block(X: torch.Tensor, n_tot: int) -> Tuple[int, int]:
    if not X.is_cuda:
        raise ValueError("vector blocks must live on the HIP device")
    if X.dim() != 2 or X.shape[0] != n_tot or X.stride(1) != 1:
        raise ValueError(f"expected a [n_tot={n_tot}, nv] block with unit column stride, got {tuple(X.shape)}")
    return X.stride(0), X.shape[1]


class Operator:
    """Device-resident OEFE operator (or a diagonal test operator)."""

    def __init__(self, system: Optional[workloads.System] = None, _handle=None, poisson: bool = False,
                 uform: bool = False, adaptive=None):
        """poisson: the operator of the auxiliary-potential Poisson problem on the system's mesh and
        atoms (oefe_poisson_create) instead of the Kohn-Sham operator; uform: the k-point operator
        in the periodic-function form (oefe_op_create_uform; the system needs a wavevector);
        adaptive = (tol, max_depth): the Kohn-Sham operator with the enrichment integrals on the
        adaptive rule (oefe_op_create_adaptive)."""
        self._h = ctypes.c_void_p(0)
        self.is_poisson = poisson
        self.is_adaptive = adaptive is not None
        if _handle is not None:
            self._h = _handle
        else:
            s = system
            atom, power, zeta, axis = s.enr_arrays()
            self._keep = [np.ascontiguousarray(s.pos, dtype=np.float64).ravel(),
                          np.ascontiguousarray(s.Z, dtype=np.float64), atom, power, zeta, axis]
            kv = None if s.kvec is None else np.ascontiguousarray(s.kvec, dtype=np.float64)
            self._keep.append(kv)
            P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t)) if a is not None and a.size else None
            d = _Desc(
                s.L, s.nc, s.p, s.n_atoms, P(self._keep[0], ctypes.c_double), P(self._keep[1], ctypes.c_double),
                s.sigma, s.r0, s.r1, s.n_enr, P(atom, ctypes.c_int32), P(power, ctypes.c_int32),
                P(zeta, ctypes.c_double), P(axis, ctypes.c_int32), P(kv, ctypes.c_double) if kv is not None else None)
            if not torch.cuda.is_available():
                raise RuntimeError("no HIP device")
            torch.cuda.current_device()
            if poisson and adaptive is not None:
                tol, depth = adaptive
                _check(_lib.oefe_poisson_create_adaptive(ctypes.byref(d), float(tol), int(depth), ctypes.byref(self._h)),
                       "oefe_poisson_create_adaptive")
            elif poisson:
                _check(_lib.oefe_poisson_create(ctypes.byref(d), ctypes.byref(self._h)), "oefe_poisson_create")
            elif uform and adaptive is not None:
                tol, depth = adaptive
                _check(_lib.oefe_op_create_uform_adaptive(ctypes.byref(d), float(tol), int(depth),
                                                          ctypes.byref(self._h)), "oefe_op_create_uform_adaptive")
            elif uform:
                _check(_lib.oefe_op_create_uform(ctypes.byref(d), ctypes.byref(self._h)), "oefe_op_create_uform")
            elif adaptive is not None:
                tol, depth = adaptive
                _check(_lib.oefe_op_create_adaptive(ctypes.byref(d), float(tol), int(depth), ctypes.byref(self._h)),
                       "oefe_op_create_adaptive")
            else:
                _check(_lib.oefe_op_create(ctypes.byref(d), ctypes.byref(self._h)), "oefe_op_create")
        dims = (ctypes.c_int64 * 11)()
        _check(_lib.oefe_op_dims(self._h, dims), "oefe_op_dims")
        (self.n_fe, self.n_enr, self.n_tot, self.n_cells, self.nq, self.nc, self.p, cx, self.tile_slots,
         self.tile_rows, self.hco_nnz) = [int(x) for x in dims]
        self.is_complex = bool(cx)
        self.is_diagonal = False
        self._work = {}

    @classmethod
    def diagonal(cls, lam: np.ndarray) -> "Operator":
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        torch.cuda.current_device()
        h = ctypes.c_void_p(0)
        _check(_lib.oefe_op_create_diagonal(lam.ctypes.data_as(ctypes.c_void_p), lam.size, ctypes.byref(h)),
               "oefe_op_create_diagonal")
        op = cls(_handle=h)
        op.is_diagonal = True
        return op

    def close(self):
        if self._h:
            _lib.oefe_op_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def work_size(self, prec: int, nv: int) -> int:
        return int(_lib.oefe_work_size(self._h, prec, nv))

    def work(self, prec: int, nv: int) -> torch.Tensor:
        """A cached device work buffer of at least work_size(prec, nv) bytes."""
        need = self.work_size(prec, nv)
        w = self._work.get("buf")
        if w is None or w.numel() < need:
            w = torch.empty(need, dtype=torch.uint8, device="cuda")
            self._work["buf"] = w
        return w

    TIMER_KINDS = {"off": 0, "cell": 1, "node": 2, "coupling": 3}

    def kernel_timer(self, which="cell"):
        """Bracket the launches of one stage ("cell", "node", "coupling"; "off"/None/False stops) with HIP events."""
        if which is True:
            which = "cell"
        if which in (None, False):
            which = "off"
        _check(_lib.oefe_kernel_timer(self._h, self.TIMER_KINDS[which]), "oefe_kernel_timer")

    def kernel_timer_read(self):
        """(launches, total milliseconds) of the bracketed launches since the last read."""
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        _check(_lib.oefe_kernel_timer_read(self._h, ctypes.byref(n), ctypes.byref(ms)), "oefe_kernel_timer_read")
        return int(n.value), float(ms.value)

    def set_potential(self, V, V_adapt=None):
        """Replace V at the quadrature points ([n_cells, nq] numpy array or torch tensor) and, for an
        operator with the adaptive rule, V_adapt at the rule's points ([n_points]); the operator
        data that depend on V are rebuilt on the device, on torch's current stream."""
        def dev(a):
            if isinstance(a, torch.Tensor):
                return a.detach().to(device="cuda", dtype=torch.float64).contiguous().reshape(-1)
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()
        Vd = dev(V)
        if Vd.numel() != self.n_cells * self.nq:
            raise ValueError("V must have n_cells * nq entries")
        if V_adapt is None:
            _check(_lib.oefe_op_set_potential(self._h, _ptr(Vd), _stream()), "oefe_op_set_potential")
            self._keep_V = Vd  # held until the queued rebuild has read it (the next call replaces it)
            return
        Va = dev(V_adapt)
        n, _, _ = self.adaptive_points(coords=False)
        if Va.numel() != n:
            raise ValueError("V_adapt must have one entry per point of the adaptive rule")
        _check(_lib.oefe_op_set_potential_adaptive(self._h, _ptr(Vd), _ptr(Va), _stream()),
               "oefe_op_set_potential_adaptive")
        self._keep_V = (Vd, Va)

    def adaptive_points(self, coords: bool = True):
        """(n_points, xyz [n, 3], weights [n]) of the adaptive rule (host arrays; None without coords)."""
        n = ctypes.c_int64(0)
        _check(_lib.oefe_op_adaptive_points(self._h, ctypes.byref(n), None, None), "oefe_op_adaptive_points")
        if not coords:
            return int(n.value), None, None
        xyz = np.empty((n.value, 3))
        w = np.empty(n.value)
        _check(_lib.oefe_op_adaptive_points(self._h, ctypes.byref(n), xyz.ctypes.data_as(ctypes.c_void_p),
                                            w.ctypes.data_as(ctypes.c_void_p)), "oefe_op_adaptive_points")
        return int(n.value), xyz, w

    def get_potential(self):
        V = np.empty(self.n_cells * self.nq)
        W = np.empty(self.n_cells * self.nq)
        _check(_lib.oefe_op_get_potential(self._h, V.ctypes.data_as(ctypes.c_void_p),
                                          W.ctypes.data_as(ctypes.c_void_p)), "oefe_op_get_potential")
        return V.reshape(self.n_cells, self.nq), W.reshape(self.n_cells, self.nq)

    def get_enrichment(self):
        n = self.n_enr
        S = np.empty(n * n * (2 if self.is_complex else 1))
        ev = np.empty(n)
        _check(_lib.oefe_op_get_enrichment(self._h, S.ctypes.data_as(ctypes.c_void_p),
                                           ev.ctypes.data_as(ctypes.c_void_p)), "oefe_op_get_enrichment")
        if self.is_complex:
            S = S.reshape(n, n, 2)
            S = S[..., 0] + 1j * S[..., 1]
        return S.reshape(n, n), ev


def ham_apply(op: Operator, X: torch.Tensor, Y: Optional[torch.Tensor] = None, bf16: bool = False) -> torch.Tensor:
    ld, nv = _block(X, op.n_tot)
    if Y is None:
        Y = torch.empty_like(X)
    ldy, _ = _block(Y, op.n_tot)
    if ldy != ld:
        raise ValueError("X and Y must share the leading dimension")
    prec = _prec(X, bf16)
    w = op.work(prec, nv)
    _check(_lib.ham_apply(op.handle, prec, _ptr(X), _ptr(Y), ld, nv, _ptr(w), _stream()), "ham_apply")
    return Y


def chebyshev_filter(op: Operator, X: torch.Tensor, m: int, a: float, b: float, a0: float,
                     bf16: bool = False) -> torch.Tensor:
    ld, nv = _block(X, op.n_tot)
    prec = _prec(X, bf16)
    w = op.work(prec, nv)
    _check(_lib.chebyshev_filter(op.handle, prec, _ptr(X), ld, nv, int(m), float(a), float(b), float(a0),
                                 _ptr(w), _stream()), "chebyshev_filter")
    return X


def chebyshev_filter_dev(op: Operator, X: torch.Tensor, m: int, bounds: torch.Tensor,
                         status: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The filter with bounds = (a, b, a0) in a device float64 tensor (no host wait)."""
    ld, nv = _block(X, op.n_tot)
    prec = _prec(X)
    if bounds.dtype != torch.float64 or bounds.device != X.device or bounds.numel() < 3 or not bounds.is_contiguous():
        raise ValueError("bounds: a contiguous device float64 tensor (a, b, a0)")
    if status is not None and (status.device != X.device or status.dtype != torch.int32 or status.numel() < 2
                               or not status.is_contiguous()):
        raise ValueError("status: a contiguous device int32 tensor of 2 elements")
    w = op.work(prec, nv)
    _check(_lib.chebyshev_filter_dev(op.handle, prec, _ptr(X), ld, nv, int(m), _ptr(bounds), _ptr(w), _ptr(status),
                                     _stream()), "chebyshev_filter_dev")
    return X


def copy_rate(src: torch.Tensor, dst: torch.Tensor, reps: int = 5) -> float:
    """Device-memory rate (GB/s, read + write) of the library's stream-copy kernel from src to dst."""
    if src.device.type != "cuda" or dst.device != src.device or not src.is_contiguous() or not dst.is_contiguous():
        raise ValueError("copy_rate takes two contiguous tensors on one device")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    g = ctypes.c_double(0.0)
    _check(_lib.oefe_copy_rate(_ptr(src), _ptr(dst), nbytes, int(reps), ctypes.byref(g), _stream()), "oefe_copy_rate")
    return float(g.value)


def chebyshev_filter_mixed(op: Operator, X: torch.Tensor, m: int, a: float, b: float, a0: float,
                           bf16: bool = False) -> torch.Tensor:
    """Filter a float64 (complex128) block with float32 (or bf16-operand) arithmetic, in place."""
    ld, nv = _block(X, op.n_tot)
    if X.dtype == torch.float64:
        prec = BF16 if bf16 else F32
    elif X.dtype == torch.complex128:
        prec = C64
    else:
        raise TypeError("chebyshev_filter_mixed takes a float64 or complex128 block")
    w = op.work(prec, nv)
    _check(_lib.chebyshev_filter_mixed(op.handle, prec, _ptr(X), ld, nv, int(m), float(a), float(b), float(a0),
                                       _ptr(w), _stream()), "chebyshev_filter_mixed")
    return X


def chebyshev_filter_batched(ops, Xs, m: int, abc, bf16: bool = False):
    """Filter several blocks (one per operator of the same mesh, e.g. k-points) in lockstep, in place.

    abc: sequence of (a, b, a0) per operator.  All blocks share one dtype.
    """
    nk = len(ops)
    if nk != len(Xs) or nk != len(abc):
        raise ValueError("ops, Xs and abc must have the same length")
    prec = _prec(Xs[0], bf16)
    lds, nvs = [], []
    for op, X in zip(ops, Xs):
        if X.dtype != Xs[0].dtype:
            raise TypeError("all blocks must share one dtype")
        ld, nv = _block(X, op.n_tot)
        lds.append(ld)
        nvs.append(nv)
    H = (ctypes.c_void_p * nk)(*[o.handle.value if isinstance(o.handle, ctypes.c_void_p) else o.handle for o in ops])
    P = (ctypes.c_void_p * nk)(*[X.data_ptr() for X in Xs])
    LD = (ctypes.c_int64 * nk)(*lds)
    NV = (ctypes.c_int32 * nk)(*nvs)
    ABC = (ctypes.c_double * (3 * nk))(*[float(v) for t in abc for v in t])
    need = int(_lib.oefe_batched_work_size(nk, H, prec, NV))
    w = ops[0]._work.get("batched")
    if w is None or w.numel() < need:
        w = torch.empty(need, dtype=torch.uint8, device="cuda")
        ops[0]._work["batched"] = w
    _check(_lib.chebyshev_filter_batched(nk, H, prec, P, LD, NV, int(m), ABC, _ptr(w), _stream()),
           "chebyshev_filter_batched")
    return Xs


def set_launch_shape(op: Operator, cw: int = 0, cb: int = 0):
    _check(_lib.oefe_set_launch_shape(op.handle, int(cw), int(cb)), "oefe_set_launch_shape")


def _tune_key(ops, Xs, prec) -> str:
    o = ops[0]
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    nvs = ",".join(str(_block(X, op.n_tot)[1]) for op, X in zip(ops, Xs))
    return (f"{dev}|nc={o.nc}|p={o.p}|n_enr={o.n_enr}|slots={o.tile_slots}|cplx={int(o.is_complex)}|prec={prec}"
            f"|nv={nvs}")


def autotune(ops, Xs, reps: int = 3, cache: Optional[str] = None, bf16: bool = False):
    """Choose the launch shape (cell-tile width cw, node vector-block width cb) for a batch.

    The library times each candidate on copies of the blocks (oefe_autotune) and sets the
    fastest on every operator.  With `cache` (a JSON file), a shape measured before for the
    same device, mesh, enrichment layout, precision and block widths is reused without timing.
    Returns {"cw", "cb", "ms_per_step", "cached"}.
    """
    import json
    nk = len(ops)
    if nk == 0 or nk != len(Xs):
        raise ValueError("ops and Xs must be non-empty and of equal length")
    prec = _prec(Xs[0], bf16)
    key = _tune_key(ops, Xs, prec)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            r = table[key]
            for op in ops:
                set_launch_shape(op, r["cw"], r["cb"])
            return dict(r, cached=True)
    lds, nvs = [], []
    for op, X in zip(ops, Xs):
        ld, nv = _block(X, op.n_tot)
        lds.append(ld)
        nvs.append(nv)
    H = (ctypes.c_void_p * nk)(*[o.handle.value if isinstance(o.handle, ctypes.c_void_p) else o.handle for o in ops])
    P = (ctypes.c_void_p * nk)(*[X.data_ptr() for X in Xs])
    LD = (ctypes.c_int64 * nk)(*lds)
    NV = (ctypes.c_int32 * nk)(*nvs)
    need = int(_lib.oefe_batched_work_size(nk, H, prec, NV))
    w = torch.empty(need, dtype=torch.uint8, device="cuda")
    cw, cb, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(_lib.oefe_autotune(nk, H, prec, P, LD, NV, int(reps), _ptr(w), ctypes.byref(cw), ctypes.byref(cb),
                              ctypes.byref(ms), _stream()), "oefe_autotune")
    r = {"cw": int(cw.value), "cb": int(cb.value), "ms_per_step": float(ms.value)}
    if cache:
        table[key] = r
        d = os.path.dirname(os.path.abspath(cache))
        os.makedirs(d, exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(r, cached=False)


def lanczos_bounds(op: Operator, v0: torch.Tensor, k: int = 10, dev_bounds: Optional[torch.Tensor] = None,
                   with_cut: bool = False):
    """(a0, b), or (a0, b, a) with the first pass's cut a when with_cut; dev_bounds (device float64[3],
    optional) receives (a, b, a0) for chebyshev_filter_dev."""
    if v0.dim() != 1 or v0.shape[0] != op.n_tot:
        raise ValueError("v0 must be a vector of length n_tot")
    if dev_bounds is not None and (dev_bounds.dtype != torch.float64 or not dev_bounds.is_cuda
                                   or dev_bounds.numel() < 3 or not dev_bounds.is_contiguous()):
        raise ValueError("dev_bounds: a contiguous device float64 tensor of 3 elements")
    dt = torch.complex128 if op.is_complex else torch.float64
    v0 = v0.to(dtype=dt).contiguous()
    prec = C128 if op.is_complex else F64
    w = op.work(prec, k + 2)
    out = (ctypes.c_double * 3)()
    _check(_lib.lanczos_bounds(op.handle, int(k), _ptr(v0), out, _ptr(w), _ptr(dev_bounds), _stream()),
           "lanczos_bounds")
    if with_cut:
        return float(out[0]), float(out[1]), float(out[2])
    return float(out[0]), float(out[1])


def set_eig_sweep_limit(op: Operator, sweeps: int = 0):
    _check(_lib.oefe_set_eig_sweep_limit(op.handle, int(sweeps)), "oefe_set_eig_sweep_limit")


def cholgs(op: Operator, X: torch.Tensor, status: Optional[torch.Tensor] = None) -> torch.Tensor:
    ld, nv = _block(X, op.n_tot)
    prec = _prec(X)
    w = op.work(prec, nv)
    _check(_lib.cholgs(op.handle, prec, _ptr(X), ld, nv, _ptr(w), _ptr(status), _stream()), "cholgs")
    return X


def cholgs_async(op: Operator, X: torch.Tensor, status: torch.Tensor) -> torch.Tensor:
    """CholGS queued without waiting; status (device int32[2]) receives {code, column}."""
    ld, nv = _block(X, op.n_tot)
    prec = _prec(X)
    w = op.work(prec, nv)
    if (status is None or status.device != X.device or status.dtype != torch.int32 or status.numel() < 2
            or not status.is_contiguous()):
        raise ValueError("cholgs_async needs a device int32 status tensor of 2 elements")
    _check(_lib.cholgs_async(op.handle, prec, _ptr(X), ld, nv, _ptr(w), _ptr(status), _stream()), "cholgs_async")
    return X


def cholgs_noalloc(op: Operator, X: torch.Tensor, status: torch.Tensor) -> torch.Tensor:
    """cholgs_async with the library's own device scratch (no work buffer); float64 blocks of <= 80 columns."""
    ld, nv = _block(X, op.n_tot)
    prec = _prec(X)
    if (status is None or status.device != X.device or status.dtype != torch.int32 or status.numel() < 2
            or not status.is_contiguous()):
        raise ValueError("cholgs_noalloc needs a device int32 status tensor of 2 elements")
    _check(_lib.cholgs_noalloc(op.handle, prec, _ptr(X), ld, nv, _ptr(status), _stream()), "cholgs_noalloc")
    return X


def rayleigh_ritz(op: Operator, Q: torch.Tensor, status: Optional[torch.Tensor] = None,
                  next_bounds: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Ritz values (device float64, ascending); Q becomes the Ritz vectors.

    status (device int32[2], optional) receives {code, sweeps} of the eigensolver; next_bounds
    (device float64[3], optional) receives a = theta_nv at [0] and a0 = theta_1 at [2].
    """
    ld, nv = _block(Q, op.n_tot)
    prec = _prec(Q)
    for t, dt, n in ((status, torch.int32, 2), (next_bounds, torch.float64, 3)):
        if t is not None and (t.device != Q.device or t.dtype != dt or t.numel() < n or not t.is_contiguous()):
            raise ValueError("status / next_bounds: contiguous device tensors (int32[2], float64[3])")
    w = op.work(prec, nv)
    ev = torch.empty(nv, dtype=torch.float64, device=Q.device)
    _check(_lib.rayleigh_ritz(op.handle, prec, _ptr(Q), ld, nv, _ptr(ev), _ptr(w), _ptr(status), _ptr(next_bounds),
                              _stream()), "rayleigh_ritz")
    return ev


def band_energy_grad(op: Operator, X: torch.Tensor, f: torch.Tensor, want_dV: bool = True, want_dX: bool = True,
                     bf16: bool = False):
    """(E, dE/dV [n_cells, nq] or None, dE/dX or None)."""
    ld, nv = _block(X, op.n_tot)
    prec = _prec(X, bf16)
    f = f.to(device=X.device, dtype=torch.float64).contiguous()
    E = torch.empty((), dtype=torch.float64, device=X.device)
    dV = torch.empty(op.n_cells, op.nq, dtype=torch.float64, device=X.device) if want_dV else None
    dX = torch.empty_like(X) if want_dX else None
    w = op.work(prec, nv)
    _check(_lib.band_energy_grad(op.handle, prec, _ptr(X), ld, nv, _ptr(f), _ptr(E), _ptr(dV), _ptr(dX), _ptr(w),
                                 _stream()), "band_energy_grad")
    return E, dV, dX


def fermi_occupations(thetas, wk, n_elec: float, kT: float):
    """Occupations of the Ritz values of nk k-points (list of device float64 tensors), weights wk:
    (list of occupation tensors, mu, E_band, electron count at mu).  Raises when n_elec cannot
    be reached with these states."""
    nk = len(thetas)
    if nk == 0 or nk != len(wk):
        raise ValueError("one weight per k-point")
    th = torch.cat([t.to(torch.float64).reshape(-1) for t in thetas]).contiguous()
    if not th.is_cuda:
        raise ValueError("Ritz values must be device tensors")
    NV = (ctypes.c_int32 * nk)(*[int(t.numel()) for t in thetas])
    WK = (ctypes.c_double * nk)(*[float(w) for w in wk])
    f = torch.empty_like(th)
    out = torch.empty(3, dtype=torch.float64, device=th.device)
    st = torch.zeros(2, dtype=torch.int32, device=th.device)
    _check(_lib.oefe_fermi_occupations(nk, NV, WK, _ptr(th), float(n_elec), float(kT), _ptr(f), _ptr(out), _ptr(st),
                                       _stream()), "oefe_fermi_occupations")
    sth = st.cpu().tolist()
    if sth[0] != 0:
        raise OefeError(sth[0], "oefe_fermi_occupations", "the electron count cannot be reached with these states")
    o = out.cpu().tolist()
    return list(torch.split(f, [int(t.numel()) for t in thetas])), o[0], o[1], o[2]


def density(op: Operator, X: torch.Tensor, weights: torch.Tensor, rho: Optional[torch.Tensor] = None,
            accumulate: bool = False) -> torch.Tensor:
    """sum_i weights_i |psi_i|^2 at the quadrature points ([n_cells, nq], float64), added to rho when
    accumulate (k-point sums)."""
    ld, nv = _block(X, op.n_tot)
    prec = _prec(X)
    weights = weights.to(device=X.device, dtype=torch.float64).contiguous()
    if weights.numel() != nv:
        raise ValueError("one weight per vector")
    if rho is None:
        rho = torch.zeros(op.n_cells, op.nq, dtype=torch.float64, device=X.device)
    elif rho.dtype != torch.float64 or rho.numel() != op.n_cells * op.nq or not rho.is_contiguous():
        raise ValueError("rho: contiguous float64 [n_cells, nq]")
    w = op.work(prec, nv)
    _check(_lib.oefe_density(op.handle, prec, _ptr(X), ld, nv, _ptr(weights), _ptr(rho), 1 if accumulate else 0,
                             _ptr(w), _stream()), "oefe_density")
    return rho


def poisson_solve(pop: Operator, rho: torch.Tensor, tol: float = 1e-10, max_iter: int = 2000,
                  rho_adapt: Optional[torch.Tensor] = None):
    """phi_aux coefficients (device float64 [n_tot]: FE part with zero mass-weighted mean, then one
    per atom) for the electron density rho at the quadrature points ([n_cells, nq] float64, device)
    and the smeared nuclear charges; returns (phi, iterations, relative residual).  An operator with
    the adaptive rule also takes rho_adapt at the rule's points (oefe_poisson_solve_adaptive)."""
    if not pop.is_poisson:
        raise ValueError("not a Poisson operator (Operator(system, poisson=True))")
    if not rho.is_cuda or rho.dtype != torch.float64 or rho.numel() != pop.n_cells * pop.nq:
        raise ValueError("rho: device float64 [n_cells, nq]")
    rho = rho.contiguous()
    phi = torch.empty(pop.n_tot, dtype=torch.float64, device=rho.device)
    w = pop._work.get("poisson")
    if w is None:
        w = torch.empty(int(_lib.oefe_poisson_work_size(pop.handle)), dtype=torch.uint8, device=rho.device)
        pop._work["poisson"] = w
    info = (ctypes.c_double * 2)()
    if rho_adapt is not None:
        ra = rho_adapt.to(device=rho.device, dtype=torch.float64).contiguous()
        _check(_lib.oefe_poisson_solve_adaptive(pop.handle, _ptr(rho), _ptr(ra), _ptr(phi), float(tol), int(max_iter),
                                                info, _ptr(w), _stream()), "oefe_poisson_solve_adaptive")
        return phi, int(info[0]), float(info[1])
    _check(_lib.oefe_poisson_solve(pop.handle, _ptr(rho), _ptr(phi), float(tol), int(max_iter), info, _ptr(w),
                                   _stream()), "oefe_poisson_solve")
    return phi, int(info[0]), float(info[1])
