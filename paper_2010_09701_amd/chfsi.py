"""ChFSI driver over the C ABI (Sec. IV of the paper).

A pass is: Chebyshev filter (float64, or float32 / bf16-operand arithmetic on
a float64 block), Cholesky-Gram-Schmidt (float64), Rayleigh-Ritz (float64).
Bounds: k-step Lanczos once per operator (the library also returns the first
pass's cut a); later passes use a0 = theta_1 and a = theta_nv of the previous
pass, which the library's Rayleigh-Ritz writes into device memory.  A float64
run without a callback keeps those bounds on the device (the filter reads them
from there) and reads the Ritz values and statuses once, after the last pass;
otherwise they cross to the host once per pass.  Every CholGS and eigensolver
status is checked.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import oefe


def chfsi_run(op: "oefe.Operator", X0: torch.Tensor, v0: torch.Tensor, m: int, passes: int, lanczos_k: int = 10,
              filter_prec="f64", bounds: Optional[tuple] = None, callback=None) -> dict:
    """Run `passes` ChFSI passes from X0 (float64 / complex128, on device); returns bounds and Ritz values.

    filter_prec: "f64", "f32" / "c64" or "bf16" for every pass, or a sequence with one entry per
    pass (a precision schedule, e.g. bf16 for the first passes and f32 for the last).
    bounds: (a0, b, a) of an earlier oefe.lanczos_bounds(..., with_cut=True) on the same operator.
    """
    sched = [filter_prec] * passes if isinstance(filter_prec, str) else list(filter_prec)
    if len(sched) != passes:
        raise ValueError("one filter precision per pass")
    dev_bounds = torch.zeros(3, dtype=torch.float64, device=X0.device)
    if bounds is None:
        a0L, b, a = oefe.lanczos_bounds(op, v0, lanczos_k, dev_bounds=dev_bounds, with_cut=True)
    else:
        a0L, b, a = bounds
        dev_bounds.copy_(torch.tensor([a, b, a0L], dtype=torch.float64))
    a0 = a0L
    X = X0.clone()
    if callback is None and all(fp == "f64" for fp in sched) and not op.is_diagonal and m <= 160:
        return _run_device_bounds(op, X, m, passes, a0L, a, b, dev_bounds)
    hist = []
    # CholGS is queued without waiting; its status and the eigensolver's are read with the Ritz values
    st_dev = torch.zeros(2, 2, dtype=torch.int32, device=X.device)
    st_host = torch.zeros(2, 2, dtype=torch.int32).pin_memory()
    for it in range(passes):
        fp = sched[it]
        if fp == "f64":
            oefe.chebyshev_filter(op, X, m, a, b, a0)
        elif fp in ("f32", "c64"):
            oefe.chebyshev_filter_mixed(op, X, m, a, b, a0)
        elif fp == "bf16":
            oefe.chebyshev_filter_mixed(op, X, m, a, b, a0, bf16=True)
        else:
            raise ValueError(fp)
        oefe.cholgs_async(op, X, st_dev[0])
        ev = oefe.rayleigh_ritz(op, X, st_dev[1], dev_bounds)
        st_host.copy_(st_dev, non_blocking=True)
        th = ev.cpu().numpy()
        if int(st_host[0, 0]) != 0:
            raise oefe.OefeError(int(st_host[0, 0]), "cholgs",
                                 f"Gram matrix not positive definite at column {int(st_host[0, 1])}")
        if int(st_host[1, 0]) != 0:
            raise oefe.OefeError(int(st_host[1, 0]), "rayleigh_ritz",
                                 f"eigensolver stopped after {int(st_host[1, 1])} sweeps")
        hist.append(dict(a=a, b=b, a0=a0, theta=th))
        if callback is not None:
            callback(it, X, th)
        nb = dev_bounds.cpu().numpy()  # the next pass's bounds, written by rayleigh_ritz
        a, a0 = float(nb[0]), float(nb[2])
    return dict(a0_lanczos=a0L, b=b, passes=hist, X=X, theta=hist[-1]["theta"])


def _run_device_bounds(op: "oefe.Operator", X: torch.Tensor, m: int, passes: int, a0L: float, a1: float, b: float,
                       bounds: torch.Tensor) -> dict:
    """Float64 passes queued back to back: each Rayleigh-Ritz writes the next filter's bounds
    (a = theta_nv, a0 = theta_1) into device memory; one host wait at the end."""
    dev = X.device
    # [pass][filter, cholgs, rayleigh-ritz][code, column or sweeps]
    st = torch.zeros(passes, 3, 2, dtype=torch.int32, device=dev)
    thetas = []
    for it in range(passes):
        oefe.chebyshev_filter_dev(op, X, m, bounds, st[it, 0])
        oefe.cholgs_async(op, X, st[it, 1])
        thetas.append(oefe.rayleigh_ritz(op, X, st[it, 2], bounds))
    st_h = st.cpu().numpy()
    th_h = [t.cpu().numpy() for t in thetas]
    hist = []
    a0, a = a0L, a1
    for it in range(passes):
        if st_h[it, 0, 0] != 0:
            raise oefe.OefeError(int(st_h[it, 0, 0]), "chebyshev_filter_dev",
                                 f"pass {it}: need a0 < a < b, got a={a}, a0={a0}")
        if st_h[it, 1, 0] != 0:
            raise oefe.OefeError(int(st_h[it, 1, 0]), "cholgs",
                                 f"pass {it}: Gram matrix not positive definite at column {int(st_h[it, 1, 1])}")
        if st_h[it, 2, 0] != 0:
            raise oefe.OefeError(int(st_h[it, 2, 0]), "rayleigh_ritz",
                                 f"pass {it}: eigensolver stopped after {int(st_h[it, 2, 1])} sweeps")
        hist.append(dict(a=a, b=b, a0=a0, theta=th_h[it]))
        a0, a = float(th_h[it][0]), float(th_h[it][-1])
    return dict(a0_lanczos=a0L, b=b, passes=hist, X=X, theta=hist[-1]["theta"])
