"""Throughput of the ChFSI hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload diamond8] [--no-cpu-baseline]

Workload "diamond8": 8-atom diamond cell (Z = 14, L = 10.26 bohr, jittered),
12^3 degree-4 spectral cells (110,592 FE DoF) + 40 orthogonalized enrichment
functions, 72 vectors, Chebyshev degree 50.  Synthetic, seeded inputs.

A step is one ChFSI pass in float64: Chebyshev filter (50 applications of
M^-1/2 H M^-1/2), Cholesky-Gram-Schmidt, Rayleigh-Ritz.  The spectrum bounds
(Lanczos, once per operator) and the operator setup are outside the timed
region.  value = N_tot * nv * m / (seconds per step), in DoF*vec*deg/s.

Also reported: the filter-only rate, the float32-arithmetic filter's speedup
and its Ritz-value error against the float64 path after 5 passes, the cell
kernel's roofline figures (HIP events bracketing each launch on the stream it
runs on), and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks used for the roofline fraction
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_VECTOR_TFLOPS = 157.3

# Algorithmic flops of the sum-factorized cell kernel per cell and real column
# (p = 4): 11 one-dimensional 5x5 passes over 25 lines (6875 FMA) + the
# quadrature-point terms (3 x 125 FMA + 2 x 5 x 125 FMA for the y/z collocation
# Laplacian) = 7250 FMA = 14500 flops.
CELL_FLOPS_P4 = 14500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diamond8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(cfg, degrees=3):
    """The oracle's float64 filter on the same workload, a few Chebyshev degrees on the host."""
    from oracle import chfsi as och
    from oracle.operator import OEFEOperator
    from paper_2010_09701_amd import workloads as wl
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = 1
    op = OEFEOperator(cfg.system)
    X0 = wl.start_block(op.n_tot, cfg.nv, cfg.x0_seed)
    b = 1500.0
    a0 = -15.0
    a = 0.5 * (a0 + b)
    och.chebyshev_filter(op.apply, X0[:, :4], 1, a, b, a0)  # warm-up
    t = time.perf_counter()
    och.chebyshev_filter(op.apply, X0, degrees, a, b, a0)
    dt = time.perf_counter() - t
    rate = op.n_tot * cfg.nv * degrees / dt
    cores = len(os.sched_getaffinity(0))
    return {"value": rate, "unit": "DoF*vec*deg/s", "cores": int(max(cores, blas_threads)), "kind": "oracle",
            "sample": f"{cfg.system.name}: {degrees} Chebyshev degrees of the float64 oracle filter on all "
                      f"{cfg.nv} vectors ({dt:.1f} s), numpy/scipy, {cores} host cores available, "
                      f"{blas_threads} BLAS threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_2010_09701_amd import oefe
    from paper_2010_09701_amd import workloads as wl

    cfg = wl.config(args.workload)
    sysm = cfg.system
    torch.cuda.set_device(0)
    t = time.time()
    gop = oefe.Operator(sysm)
    log(f"operator setup {time.time() - t:.1f} s, n_tot={gop.n_tot}, nv={cfg.nv}, m={cfg.m}")
    X0 = torch.from_numpy(wl.start_block(gop.n_tot, cfg.nv, cfg.x0_seed)).cuda()
    v0 = torch.from_numpy(wl.lanczos_start(gop.n_tot, cfg.v0_seed)).cuda()
    a0L, b = oefe.lanczos_bounds(gop, v0, cfg.lanczos_k)
    log(f"bounds a0={a0L:.6f} b={b:.6f}")
    state = {"a0": a0L, "a": 0.5 * (a0L + b)}
    X = X0.clone()

    def step():
        oefe.chebyshev_filter(gop, X, cfg.m, state["a"], b, state["a0"])
        oefe.cholgs(gop, X)
        th = oefe.rayleigh_ritz(gop, X)
        th_h = th.cpu().numpy()
        state["a0"], state["a"] = float(th_h[0]), float(th_h[-1])
        return th_h

    for i in range(args.warmup):
        step()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    work = gop.n_tot * cfg.nv * cfg.m
    value = work / (ms / 1e3)
    log(f"pass: {ms:.3f} ms, {value:.3e} DoF*vec*deg/s")

    # filter-only rate and cell-kernel timing (events bracketing each launch)
    Xf = X0.clone()
    reps = max(2, args.steps)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(reps):
        oefe.chebyshev_filter(gop, Xf, cfg.m, 0.5 * (a0L + b), b, a0L)
        Xf.copy_(X0)
    e1.record(stream)
    torch.cuda.synchronize()
    filt_ms = e0.elapsed_time(e1) / reps
    gop.kernel_timer(True)
    oefe.chebyshev_filter(gop, Xf, cfg.m, 0.5 * (a0L + b), b, a0L)
    n_launch, tot_ms = gop.kernel_timer_read()
    gop.kernel_timer(False)
    cell_ms = tot_ms / max(n_launch, 1)
    cell_flops = CELL_FLOPS_P4 * (sysm.p + 1) ** 3 / 125.0 * gop.n_cells * cfg.nv
    achieved = cell_flops / (cell_ms / 1e3) / 1e12
    log(f"filter: {filt_ms:.3f} ms; cell kernel avg {cell_ms * 1e3:.1f} us over {n_launch} launches, "
        f"{achieved:.2f} TFLOP/s")

    extra = {"filter_ms": filt_ms, "filter_rate": work / (filt_ms / 1e3), "pass_ms": ms,
             "lanczos_bounds": [a0L, b], "n_tot": gop.n_tot, "n_fe": gop.n_fe, "n_enr": gop.n_enr}

    if not args.no_fp32:
        from paper_2010_09701_amd.chfsi import chfsi_run
        Xm = X0.clone()
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(reps):
            oefe.chebyshev_filter_mixed(gop, Xm, cfg.m, 0.5 * (a0L + b), b, a0L)
            Xm.copy_(X0)
        e1.record(stream)
        torch.cuda.synchronize()
        f32_ms = e0.elapsed_time(e1) / reps
        r64 = chfsi_run(gop, X0, v0, cfg.m, cfg.passes, cfg.lanczos_k, "f64", bounds=(a0L, b))
        r32 = chfsi_run(gop, X0, v0, cfg.m, cfg.passes, cfg.lanczos_k, "f32", bounds=(a0L, b))
        n_occ = cfg.nv - 16
        err = [float(np.abs(p32["theta"][:n_occ] - p64["theta"][:n_occ]).max())
               for p32, p64 in zip(r32["passes"], r64["passes"])]
        extra.update({"fp32_filter_ms": f32_ms, "fp32_filter_speedup": filt_ms / f32_ms,
                      "fp32_ritz_err_vs_fp64_per_pass_Ha": err, "fp32_occupied_states": n_occ})
        log(f"fp32 filter {f32_ms:.3f} ms (x{filt_ms / f32_ms:.2f}); Ritz err per pass {err}")

    out = {
        "metric": "ChFSI filter DoF*vec*deg/s (one float64 ChFSI pass: filter + CholGS + Rayleigh-Ritz)",
        "value": value,
        "unit": "DoF*vec*deg/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{sysm.name}: {sysm.nc}^3 cells p={sysm.p}, {gop.n_fe} FE + {gop.n_enr} "
                               f"enrichment DoF, {cfg.nv} vectors, Chebyshev degree {cfg.m}",
                   "global_batch": cfg.nv, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "fe_cell_kernel<double,5>", "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": None, "avg_launch_us": cell_ms * 1e3},
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(cfg)
        log(f"cpu baseline {out['cpu_baseline']['value']:.3e}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
