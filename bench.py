"""Throughput of the ChFSI hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload diamond8] [--no-cpu-baseline]

Workload "diamond8": 8-atom diamond cell (Z = 14, L = 10.26 bohr, jittered),
12^3 degree-4 spectral cells (110,592 FE DoF) + 40 orthogonalized enrichment
functions, 72 vectors, Chebyshev degree 50.  Synthetic, seeded inputs.

A step is one ChFSI pass in float64: Chebyshev filter (50 applications of
M^-1/2 H M^-1/2), Cholesky-Gram-Schmidt, Rayleigh-Ritz.  The spectrum bounds
(Lanczos, once per operator) and the operator setup are outside the timed
region; inputs are resident in device memory.  Each pass's filter bounds come
from the previous pass's Ritz values through device memory (no host wait
between passes); statuses and Ritz values are checked after the timed passes.
value = N_tot * nv * m / (seconds per step), in DoF*vec*deg/s.

Also reported: the filter-only rate, the float32-arithmetic filter's speedup
and its Ritz-value error against the float64 path after 5 passes, the node
kernel's memory roofline and the cell kernel's arithmetic roofline (HIP events
bracketing each launch on the stream it runs on), the rate of the library's
stream-copy kernel over 4 GiB (the node kernel's rate is also given as a
fraction of it), and the CPU oracle on a bounded sample.

Helpers for the committed profile summaries (they read rocprofv3 output):
    python bench.py --summarize-trace DIR           kernel-trace statistics table
    python bench.py --summarize-traffic FETCH_DIR WRITE_DIR
                                                    HBM bytes per node-kernel launch from
                                                    FETCH_SIZE / WRITE_SIZE, calibrated on
                                                    the device-to-device copy of --calib-copy
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks used for the roofline fractions
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_VECTOR_TFLOPS = 157.3

# Algorithmic flops of the sum-factorized cell kernel per cell and real column
# (p = 4): 11 one-dimensional 5x5 passes over 25 lines (6875 FMA) + the
# quadrature-point terms (3 x 125 FMA + 2 x 5 x 125 FMA for the y/z collocation
# Laplacian) = 7250 FMA = 14500 flops.
CELL_FLOPS_P4 = 14500.0

OPS_SOURCE = os.path.join(ROOT, "paper_2010_09701_amd", "csrc", "oefe_ops.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "fe_node_fused_kernel_diamond8_traffic.md")
CALIB_BYTES = 512 * 2**20
COPY_BW_BYTES = 4 * 2**30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diamond8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the float32 / bf16 filter measurements")
    ap.add_argument("--no-kpoints", action="store_true", help="skip the batched k-point filter measurement")
    ap.add_argument("--no-d64", action="store_true", help="skip the diamond64 filter measurement")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with one 512 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--no-copy-bw", action="store_true", help="skip the 4 GiB copy-bandwidth measurement (also skipped with --calib-copy)")
    ap.add_argument("--summarize-trace", metavar="DIR")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def ops_source_hash() -> str:
    with open(OPS_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def node_kernel_bytes(gop, ncr: int, m: int) -> float:
    """Algorithmic HBM bytes of one node-kernel launch inside the filter, averaged over its m steps.

    Per launch: the cell results of every node slot ((nc (p+1))^3 rows), X and the
    output (N rows each), the previous iterate (N rows, read in m-1 of the m steps),
    the dense coupling blocks (tile_slots x tile_rows, once per column block) and
    the tile partials written (tile_slots rows), all x ncr real columns of 8 bytes.
    """
    slots = (gop.nc * (gop.p + 1)) ** 3
    nb_all = -(-ncr // 16)
    ncb = -(-nb_all // 5)  # column blocks of at most 5 x 16 real columns per workgroup
    rows = slots + 2 * gop.n_fe + gop.n_fe * (m - 1) / m + gop.tile_slots
    return 8.0 * (rows * ncr + gop.tile_slots * gop.tile_rows * ncb)


def load_traffic():
    """HBM bytes per node-kernel launch from the committed counter summary, if the kernel source is unchanged."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    vals = {}
    for line in open(TRAFFIC_SUMMARY):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().split()[0]
    if vals.get("source_sha256_16") != ops_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_bandwidth(oefe, torch, reps=5):
    """Achievable HBM rate: the library's hand-written stream-copy kernel over 4 GiB (read + write
    bytes per second, median of `reps` copies after one warm-up, HIP events on the stream)."""
    a = torch.empty(COPY_BW_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    c = torch.empty_like(a)
    gbs = oefe.copy_rate(a, c, reps)
    del a, c
    torch.cuda.empty_cache()
    return gbs


def cpu_baseline(cfg):
    """One whole float64 pass of the oracle on the same workload (filter of degree m on all
    vectors, CholGS, Rayleigh-Ritz), timed on the host; the same unit as the GPU value."""
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
    a0, b, _, _ = och.lanczos_bounds(op.apply, wl.lanczos_start(op.n_tot, cfg.v0_seed), cfg.lanczos_k)
    a = 0.5 * (a0 + b)
    och.chebyshev_filter(op.apply, X0[:, :4], 1, a, b, a0)  # warm-up
    t = time.perf_counter()
    Y = och.chebyshev_filter(op.apply, X0, cfg.m, a, b, a0)
    Q, _ = och.cholgs(Y)
    och.rayleigh_ritz(op.apply, Q)
    dt = time.perf_counter() - t
    rate = op.n_tot * cfg.nv * cfg.m / dt
    cores = len(os.sched_getaffinity(0))
    return {"value": rate, "unit": "DoF*vec*deg/s", "cores": int(min(cores, max(blas_threads, 1))), "kind": "oracle",
            "sample": f"{cfg.system.name}: one float64 oracle pass (degree-{cfg.m} filter on all {cfg.nv} vectors, "
                      f"CholGS, Rayleigh-Ritz; {dt:.1f} s; numpy/scipy with {blas_threads} BLAS threads, "
                      f"{cores} host cores available)"}


def kpoint_bench(oefe, wl, torch, base, m, reps):
    """The 8 k-points of the 2x2x2 Monkhorst-Pack grid, 48..96 vectors each, in one batched
    filter per precision (complex128, complex64), after the launch-shape autotuner."""
    ks = wl.monkhorst_pack_2(base.L)
    ops = [oefe.Operator(base.with_k(k)) for k in ks]
    blocks = [torch.from_numpy(wl.start_block(op.n_tot, wl.KPOINT_NV[q], 10 + q, complex_=True)).cuda()
              for q, op in enumerate(ops)]
    abc = []
    for op in ops:
        v0 = torch.from_numpy(wl.lanczos_start(op.n_tot, 2)).cuda()
        a0, bb = oefe.lanczos_bounds(op, v0, 10)
        abc.append((0.5 * (a0 + bb), bb, a0))
    work = sum(op.n_tot * nv for op, nv in zip(ops, wl.KPOINT_NV)) * m
    res = {"k_points": len(ops), "nv": wl.KPOINT_NV, "m": m}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for name, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        Xs = [X.to(dt) for X in blocks]
        tune = oefe.autotune(ops, Xs, reps=3)
        oefe.chebyshev_filter_batched(ops, Xs, m, abc)  # warm-up (the filter is scaled: values stay bounded)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            oefe.chebyshev_filter_batched(ops, Xs, m, abc)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        # per-launch stage durations (HIP events on the stream each stage runs on; the
        # coupling kernel runs on the side stream beside the cell stage)
        stages = {}
        for which in ("cell", "node", "coupling"):
            ops[0].kernel_timer(which)
            oefe.chebyshev_filter_batched(ops, Xs, m, abc)
            n_launch, tot_ms = ops[0].kernel_timer_read()
            ops[0].kernel_timer("off")
            stages[which + "_us"] = tot_ms / max(n_launch, 1) * 1e3
        res[name] = {"filter_ms": ms, "rate": work / (ms / 1e3), "shape": {"cw": tune["cw"], "cb": tune["cb"]},
                     "stage_avg_us": stages}
        log(f"k-points {name}: batched filter {ms:.3f} ms, {work / (ms / 1e3):.3e} DoF*vec*deg/s, shape {tune}, "
            + ", ".join(f"{k} {v:.1f}" for k, v in stages.items()))
    res["unit"] = "DoF*vec*deg/s (complex vectors)"
    return res


def d64_bench(oefe, wl, torch):
    """diamond64 (885,056 DoF x 320 vectors, degree 60): one float64 and one float32 filter,
    and the per-launch node / cell kernel durations, at a shape whose working set (several
    GB) is far above the 256 MB Infinity Cache."""
    cfg = wl.config("diamond64")
    t = time.time()
    gop = oefe.Operator(cfg.system)
    setup_s = time.time() - t
    X0 = torch.from_numpy(wl.start_block(gop.n_tot, cfg.nv, cfg.x0_seed)).cuda()
    v0 = torch.from_numpy(wl.lanczos_start(gop.n_tot, cfg.v0_seed)).cuda()
    a0L, b = oefe.lanczos_bounds(gop, v0, cfg.lanczos_k)
    a = 0.5 * (a0L + b)
    work = gop.n_tot * cfg.nv * cfg.m
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    res = {"workload": "diamond64: 24^3 cells p=4, 884736 FE + 320 enrichment DoF, 320 vectors, degree 60",
           "setup_s": setup_s}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        X = X0.to(dt)
        oefe.chebyshev_filter(gop, X, 2, a, b, a0L)  # warm-up
        X.copy_(X0)
        torch.cuda.synchronize()
        e0.record()
        oefe.chebyshev_filter(gop, X, cfg.m, a, b, a0L)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        r = {"filter_ms": ms, "rate": work / (ms / 1e3)}
        for which in ("node", "cell"):
            X.copy_(X0)
            gop.kernel_timer(which)
            oefe.chebyshev_filter(gop, X, 10, a, b, a0L)
            n_launch, tot_ms = gop.kernel_timer_read()
            gop.kernel_timer("off")
            r[which + "_avg_us"] = tot_ms / max(n_launch, 1) * 1e3
        if name == "f64":
            nbytes = node_kernel_bytes(gop, cfg.nv, 10)
            r["node_gbs"] = nbytes / (r["node_avg_us"] / 1e6) / 1e9
            r["node_frac_of_8TBs"] = r["node_gbs"] / PEAK_HBM_GBS
        res[name] = r
        log(f"diamond64 {name}: filter {ms:.1f} ms, {work / (ms / 1e3):.3e} DoF*vec*deg/s; node {r['node_avg_us']:.0f} us, "
            f"cell {r['cell_avg_us']:.0f} us" + (f", node {r['node_gbs']:.0f} GB/s" if name == "f64" else ""))
        del X
    res["unit"] = "DoF*vec*deg/s"
    return res


def summarize_trace(d):
    f = sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True))
    if not f:
        sys.exit(f"no kernel_stats.csv under {d}")
    print("| kernel | calls | avg us | min us | max us | share % |")
    print("|---|---:|---:|---:|---:|---:|")
    for r in list(csv.DictReader(open(f[0])))[:24]:
        print(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
              f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")


def _short(name):
    n = name.replace("void ", "").replace("oefe::(anonymous namespace)::", "").replace("oefe::", "")
    out, depth = "", 0
    for ch in n:
        if ch == "(" and depth == 0:
            break
        depth += (ch == "<") - (ch == ">")
        out += ch
    return out


def _counter_rows(d):
    f = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
    if not f:
        sys.exit(f"no counter_collection.csv under {d}")
    return list(csv.DictReader(open(f[0])))


def _per_kernel(rows, counter):
    """kernel short name -> list of per-dispatch values (KiB) of one counter."""
    acc = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        key = (_short(r["Kernel_Name"]), r["Dispatch_Id"])
        acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (k, _), v in acc.items():
        out.setdefault(k, []).append(v)
    return out


def summarize_traffic(fetch_dir, write_dir):
    fe = _per_kernel(_counter_rows(fetch_dir), "FETCH_SIZE")
    wr = _per_kernel(_counter_rows(write_dir), "WRITE_SIZE")
    # the filter's node-kernel instance is the float64 one launched most often
    node = sorted((k for k in fe if k.startswith("fe_node_fused_kernel<double")), key=lambda k: -len(fe[k]))
    copy = [k for k in fe if "copyBuffer" in k or "copy_kernel" in k]
    if not node or not copy:
        sys.exit(f"kernels not found: {sorted(fe)}")
    k, c = node[0], copy[0]
    cf = max(fe[c]) * 1024.0 / CALIB_BYTES  # the largest dispatch is the 512 MiB calibration copy
    cw = max(wr[c]) * 1024.0 / CALIB_BYTES
    f_kib, w_kib = float(np.median(fe[k])), float(np.median(wr[k]))
    hbm = f_kib * 1024.0 / cf + w_kib * 1024.0 / cw
    print(f"- kernel: {k}")
    print(f"- dispatches: {len(fe[k])}")
    print(f"- fetch_kib_median: {f_kib:.0f}")
    print(f"- write_kib_median: {w_kib:.0f}")
    print(f"- calib_kernel: {c}")
    print(f"- calib_fetch_factor: {cf:.4f} (FETCH_SIZE bytes / bytes copied, 512 MiB copy)")
    print(f"- calib_write_factor: {cw:.4f} (WRITE_SIZE bytes / bytes copied)")
    print(f"- hbm_bytes_per_launch: {hbm:.0f}")
    print(f"- source_sha256_16: {ops_source_hash()}")


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; runs on several GPUs are not supported",
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
    a0L, b, a1 = oefe.lanczos_bounds(gop, v0, cfg.lanczos_k, with_cut=True)
    log(f"bounds a0={a0L:.6f} b={b:.6f}")
    X = X0.clone()

    # The bounds of each pass's filter stay on the device: (a, b, a0), pass 1 cut at
    # (a0 + b) / 2, later passes a = theta_nv and a0 = theta_1 written there by the previous
    # Rayleigh-Ritz.  Filter and CholGS statuses and the Ritz values are checked after the
    # timed passes, so the host never waits inside a pass.
    n_pass = args.warmup + args.steps
    bounds = torch.tensor([0.5 * (a0L + b), b, a0L], dtype=torch.float64, device=X.device)
    st_dev = torch.zeros(n_pass, 2, 2, dtype=torch.int32, device=X.device)  # [pass][filter, cholgs][code, col]
    thetas = []

    def step(i):
        oefe.chebyshev_filter_dev(gop, X, cfg.m, bounds, st_dev[i, 0])
        oefe.cholgs_async(gop, X, st_dev[i, 1])
        th = oefe.rayleigh_ritz(gop, X)
        bounds[0:1].copy_(th[-1:])
        bounds[2:3].copy_(th[:1])
        thetas.append(th)

    for i in range(args.warmup):
        step(i)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        step(args.warmup + i)
    e1.record(stream)
    torch.cuda.synchronize()
    st_h = st_dev.cpu().numpy()
    if (st_h[:, :, 0] != 0).any():
        raise RuntimeError(f"pass failed: statuses [pass][filter, cholgs][code, column] {st_h.tolist()}")
    th_all = np.stack([t.cpu().numpy() for t in thetas])
    if not np.isfinite(th_all).all() or (np.diff(th_all, axis=1) < 0).any():
        raise RuntimeError("Ritz values not finite and ascending")
    ms = e0.elapsed_time(e1) / args.steps
    work = gop.n_tot * cfg.nv * cfg.m
    value = work / (ms / 1e3)
    log(f"pass: {ms:.3f} ms, {value:.3e} DoF*vec*deg/s")

    # filter-only rate
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

    # per-launch durations of the node and cell kernels: HIP events recorded by the
    # library around each launch, on the stream the kernel runs on
    def stage_ms(which):
        gop.kernel_timer(which)
        oefe.chebyshev_filter(gop, Xf, cfg.m, 0.5 * (a0L + b), b, a0L)
        n_launch, tot_ms = gop.kernel_timer_read()
        gop.kernel_timer("off")
        Xf.copy_(X0)
        return tot_ms / max(n_launch, 1), n_launch

    node_ms, node_n = stage_ms("node")
    cell_ms, cell_n = stage_ms("cell")
    node_bytes = node_kernel_bytes(gop, cfg.nv, cfg.m)
    node_gbs = node_bytes / (node_ms / 1e3) / 1e9
    cell_flops = CELL_FLOPS_P4 * (sysm.p + 1) ** 3 / 125.0 * gop.n_cells * cfg.nv
    cell_tfs = cell_flops / (cell_ms / 1e3) / 1e12
    traffic = load_traffic()
    log(f"filter: {filt_ms:.3f} ms; node kernel avg {node_ms * 1e3:.1f} us ({node_n} launches), "
        f"{node_gbs:.0f} GB/s algorithmic; cell kernel avg {cell_ms * 1e3:.1f} us, {cell_tfs:.2f} TFLOP/s")

    extra = {"filter_ms": filt_ms, "filter_rate": work / (filt_ms / 1e3), "pass_ms": ms,
             "lanczos_bounds": [a0L, b], "n_tot": gop.n_tot, "n_fe": gop.n_fe, "n_enr": gop.n_enr,
             "cell_kernel": {"bound": "alu", "kernel": "fe_cell_kernel<double,5>", "achieved": cell_tfs,
                             "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": cell_tfs / PEAK_FP64_TFLOPS,
                             "avg_launch_us": cell_ms * 1e3, "flops_per_launch": cell_flops}}

    if not args.no_fp32:
        from paper_2010_09701_amd.chfsi import chfsi_run
        r64 = chfsi_run(gop, X0, v0, cfg.m, cfg.passes, cfg.lanczos_k, "f64", bounds=(a0L, b, a1))
        n_occ = cfg.nv - 16
        Q64 = r64["X"][:, :n_occ]
        for name, bf in (("fp32", False), ("bf16", True)):
            Xm = X0.clone()
            torch.cuda.synchronize()
            e0.record(stream)
            for i in range(reps):
                oefe.chebyshev_filter_mixed(gop, Xm, cfg.m, 0.5 * (a0L + b), b, a0L, bf16=bf)
                Xm.copy_(X0)
            e1.record(stream)
            torch.cuda.synchronize()
            mixed_ms = e0.elapsed_time(e1) / reps
            rm = chfsi_run(gop, X0, v0, cfg.m, cfg.passes, cfg.lanczos_k, "bf16" if bf else "f32", bounds=(a0L, b, a1))
            err = [float(np.abs(pm["theta"][:n_occ] - p64["theta"][:n_occ]).max())
                   for pm, p64 in zip(rm["passes"], r64["passes"])]
            Q = rm["X"][:, :n_occ]
            sin_angle = float(torch.linalg.matrix_norm(Q - Q64 @ (Q64.T @ Q), ord=2))
            extra.update({f"{name}_filter_ms": mixed_ms, f"{name}_filter_speedup": filt_ms / mixed_ms,
                          f"{name}_ritz_err_vs_fp64_per_pass_Ha": err,
                          f"{name}_subspace_sin_angle_vs_fp64": sin_angle})
            log(f"{name} filter {mixed_ms:.3f} ms (x{filt_ms / mixed_ms:.2f}); Ritz err per pass "
                f"{['%.1e' % x for x in err]}; sin(max angle) {sin_angle:.1e}")
        extra["mixed_occupied_states"] = n_occ

    if not args.no_kpoints and sysm.name == "diamond8":
        extra["kpoints"] = kpoint_bench(oefe, wl, torch, sysm, cfg.m, reps)
    if not args.no_d64 and sysm.name == "diamond8":
        extra["diamond64"] = d64_bench(oefe, wl, torch)
    copy_gbs = None
    if not args.no_copy_bw and not args.calib_copy:  # (the counter calibration takes the largest copy)
        copy_gbs = copy_bandwidth(oefe, torch)
        extra["hbm_copy_gbs"] = copy_gbs
        log(f"stream copy of {COPY_BW_BYTES >> 30} GiB: {copy_gbs:.0f} GB/s (read + write); node kernel "
            f"{node_gbs / copy_gbs:.2f} of it")

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
        "roofline": {"bound": "hbm", "kernel": "fe_node_fused_kernel<double>", "achieved": node_gbs,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": node_gbs / PEAK_HBM_GBS,
                     "traffic": traffic, "avg_launch_us": node_ms * 1e3, "bytes_per_launch": node_bytes,
                     "frac_of_copy": (node_gbs / copy_gbs) if copy_gbs else None},
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(cfg)
        log(f"cpu baseline {out['cpu_baseline']['value']:.3e}")
    if args.calib_copy:
        a = torch.empty(CALIB_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        c = torch.empty_like(a)
        torch.cuda.synchronize()
        c.copy_(a)
        torch.cuda.synchronize()
        del a, c
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
