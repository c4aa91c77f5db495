"""Write the stored oracle values used by the full-size GPU parity tests.

Every value here comes from the CPU oracle (oracle/) on the seeded synthetic
workloads of paper_2010_09701_amd/workloads.py; nothing is read from the HIP
library.  The paper prints no values that apply to these synthetic operators.

    python tests/golden/make_golden.py diamond8     (about 10 min on 8 cores)
    python tests/golden/make_golden.py diamond64    (about 20 min)
    python tests/golden/make_golden.py kpoints      (about 5 min)
    python tests/golden/make_golden.py kpoint_passes   (about 20 min)
    python tests/golden/make_golden.py diamond64_pass1 (about 40 min, ~20 GB of host memory)
    python tests/golden/make_golden.py poisson_diamond8 (about 2 min)
    python tests/golden/make_golden.py uform_kpoints    (about 5 min)
    python tests/golden/make_golden.py adaptive_diamond8 (about 10 min)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import chfsi as ch  # noqa: E402
from oracle.operator import OEFEOperator  # noqa: E402
from paper_2010_09701_amd import workloads as wl  # noqa: E402


def sample_rows(n_fe: int, n_enr: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    fe = np.sort(rng.choice(n_fe, size=count, replace=False))
    return np.concatenate([fe, n_fe + np.arange(n_enr)]).astype(np.int64)


def diamond8():
    cfg = wl.config("diamond8")
    t = time.time()
    op = OEFEOperator(cfg.system)
    print("operator", time.time() - t, flush=True)
    X0 = wl.start_block(op.n_tot, cfg.nv, cfg.x0_seed)
    v0 = wl.lanczos_start(op.n_tot, cfg.v0_seed)
    rows = sample_rows(op.N, op.n_enr, 200, 17)
    HX = op.apply(X0)
    a0L, b, _, _ = ch.lanczos_bounds(op.apply, v0, cfg.lanczos_k)
    print("bounds", a0L, b, flush=True)
    a = 0.5 * (a0L + b)
    Y1 = ch.chebyshev_filter(op.apply, X0, cfg.m, a, b, a0L)
    r = ch.chfsi(op.apply, X0, v0, cfg.m, cfg.passes, cfg.lanczos_k)
    thetas = np.stack([p["theta"] for p in r["passes"]])
    print("passes", thetas[:, :4], flush=True)
    np.savez_compressed(os.path.join(HERE, "diamond8_oracle.npz"), rows=rows, hx_rows=HX[rows], a0L=a0L, b=b,
                        filt1_rows=Y1[rows], filt1_colnorm=np.linalg.norm(Y1, axis=0), thetas=thetas,
                        hx_colnorm=np.linalg.norm(HX, axis=0))


def diamond64():
    cfg = wl.config("diamond64")
    t = time.time()
    op = OEFEOperator(cfg.system)
    print("operator", time.time() - t, flush=True)
    X0 = wl.start_block(op.n_tot, cfg.nv, cfg.x0_seed)
    rows = sample_rows(op.N, op.n_enr, 400, 19)
    # column chunks keep the oracle's intermediates within host memory
    hx_rows = np.empty((rows.size, cfg.nv))
    hx_colnorm = np.empty(cfg.nv)
    for j0 in range(0, cfg.nv, 32):
        HX = op.apply(X0[:, j0:j0 + 32])
        hx_rows[:, j0:j0 + 32] = HX[rows]
        hx_colnorm[j0:j0 + 32] = np.linalg.norm(HX, axis=0)
        print("columns", j0 + HX.shape[1], time.time() - t, flush=True)
    np.savez_compressed(os.path.join(HERE, "diamond64_oracle.npz"), rows=rows, hx_rows=hx_rows,
                        hx_colnorm=hx_colnorm, Moo_eigs=op.enr.Moo_eigs)


def kpoints():
    """diamond8 at the 8 k-points of the 2x2x2 Monkhorst-Pack grid, uneven complex blocks."""
    base = wl.config("diamond8").system
    ks = wl.monkhorst_pack_2(base.L)
    out = {}
    t = time.time()
    for q, kv in enumerate(ks):
        op = OEFEOperator(base.with_k(kv))
        nv = wl.KPOINT_NV[q]
        X0 = wl.start_block(op.n_tot, nv, 10 + q, complex_=True)
        rows = sample_rows(op.N, op.n_enr, 100, 30 + q)
        hx_rows = np.empty((rows.size, nv), dtype=np.complex128)
        for j0 in range(0, nv, 32):
            hx_rows[:, j0:j0 + 32] = op.apply(X0[:, j0:j0 + 32])[rows]
        out[f"k{q}"] = kv
        out[f"rows{q}"] = rows
        out[f"hx_rows{q}"] = hx_rows
        print("k-point", q, nv, time.time() - t, flush=True)
    np.savez_compressed(os.path.join(HERE, "kpoints_oracle.npz"), **out)


def _passes(op, X0, v0, m, passes, k, rows):
    """The oracle's ChFSI step by step: bounds, pass-1 filtered rows / column norms, Ritz values per pass."""
    a0L, b, _, _ = ch.lanczos_bounds(op.apply, v0, k)
    a0, a = a0L, 0.5 * (a0L + b)
    X = X0
    thetas = []
    out = dict(a0L=a0L, b=b)
    for it in range(passes):
        Y = ch.chebyshev_filter(op.apply, X, m, a, b, a0)
        if it == 0:
            out["filt1_rows"] = Y[rows]
            out["filt1_colnorm"] = np.linalg.norm(Y, axis=0)
        Q, _ = ch.cholgs(Y)
        th, X = ch.rayleigh_ritz(op.apply, Q)
        thetas.append(th)
        a0, a = float(th[0]), float(th[-1])
    out["thetas"] = np.stack(thetas)
    return out


def kpoint_passes():
    """Five float64 (complex128) ChFSI passes at the k-points with the fewest (48) and the most (96)
    vectors of the 2x2x2 Monkhorst-Pack grid on diamond8."""
    base = wl.config("diamond8").system
    cfg = wl.config("diamond8")
    ks = wl.monkhorst_pack_2(base.L)
    out = {}
    t = time.time()
    for q in (0, 7):
        op = OEFEOperator(base.with_k(ks[q]))
        nv = wl.KPOINT_NV[q]
        X0 = wl.start_block(op.n_tot, nv, 10 + q, complex_=True)
        v0 = wl.lanczos_start(op.n_tot, cfg.v0_seed)
        rows = sample_rows(op.N, op.n_enr, 200, 50 + q)
        r = _passes(op, X0, v0, cfg.m, cfg.passes, cfg.lanczos_k, rows)
        out[f"rows{q}"] = rows
        for key, val in r.items():
            out[f"{key}{q}"] = val
        print("k-point", q, nv, r["thetas"][:, :3], time.time() - t, flush=True)
    np.savez_compressed(os.path.join(HERE, "kpoint_passes_oracle.npz"), **out)


def diamond64_pass1():
    """diamond64: bounds and the first float64 ChFSI pass (degree-60 filter on all 320 vectors in
    column chunks, which the filter treats independently; CholGS and Rayleigh-Ritz on the block)."""
    cfg = wl.config("diamond64")
    t = time.time()
    op = OEFEOperator(cfg.system)
    print("operator", time.time() - t, flush=True)
    X0 = wl.start_block(op.n_tot, cfg.nv, cfg.x0_seed)
    v0 = wl.lanczos_start(op.n_tot, cfg.v0_seed)
    a0L, b, _, _ = ch.lanczos_bounds(op.apply, v0, cfg.lanczos_k)
    print("bounds", a0L, b, time.time() - t, flush=True)
    a = 0.5 * (a0L + b)
    Y = np.empty_like(X0)
    for j0 in range(0, cfg.nv, 64):
        Y[:, j0:j0 + 64] = ch.chebyshev_filter(op.apply, X0[:, j0:j0 + 64], cfg.m, a, b, a0L)
        print("filtered columns", j0 + 64, time.time() - t, flush=True)
    del X0
    rows = sample_rows(op.N, op.n_enr, 400, 23)
    filt1_rows = Y[rows]
    filt1_colnorm = np.linalg.norm(Y, axis=0)
    Q, _ = ch.cholgs(Y)
    del Y
    th, _ = ch.rayleigh_ritz(op.apply, Q)
    print("pass 1 Ritz values", th[:4], th[-2:], time.time() - t, flush=True)
    np.savez_compressed(os.path.join(HERE, "diamond64_pass1_oracle.npz"), a0L=a0L, b=b, rows=rows,
                        filt1_rows=filt1_rows, filt1_colnorm=filt1_colnorm, theta1=th)


def poisson_diamond8():
    """The auxiliary potential of diamond8 for the model atomic densities (oracle/poisson.py)."""
    from oracle import poisson as po
    t = time.time()
    P = po.PoissonOEFE(wl.diamond8())
    rho = P.model_electron_density()
    phi = P.solve(P.neutral_charge(rho), rtol=1e-13)
    print("poisson diamond8", P.n_tot, time.time() - t, flush=True)
    np.savez_compressed(os.path.join(HERE, "poisson_diamond8_oracle.npz"), rho=rho, phi=phi)


def uform_kpoints():
    """diamond8 in the periodic-function k-point form (oracle/uform.py) at the Monkhorst-Pack
    k-points with the fewest and the most vectors: sampled rows of Ht_k X and column norms."""
    from oracle.uform import UFormOperator
    base = wl.config("diamond8").system
    ks = wl.monkhorst_pack_2(base.L)
    out = {}
    t = time.time()
    for q in (0, 7):
        kv = ks[q]
        op = UFormOperator(base.with_k(kv), kv)
        nv = wl.KPOINT_NV[q]
        X0 = wl.start_block(op.n_tot, nv, 10 + q, complex_=True)
        rows = sample_rows(op.N, op.n_enr, 100, 50 + q)
        hx_rows = np.empty((rows.size, nv), dtype=np.complex128)
        colnorm = np.empty(nv)
        for j0 in range(0, nv, 32):
            HX = op.apply(X0[:, j0:j0 + 32])
            hx_rows[:, j0:j0 + 32] = HX[rows]
            colnorm[j0:j0 + 32] = np.linalg.norm(HX, axis=0)
        out[f"k{q}"] = kv
        out[f"rows{q}"] = rows
        out[f"hx_rows{q}"] = hx_rows
        out[f"hx_colnorm{q}"] = colnorm
        print("u-form k-point", q, nv, time.time() - t, flush=True)
    np.savez_compressed(os.path.join(HERE, "uform_kpoints_oracle.npz"), **out)


def adaptive_diamond8():
    """diamond8 with the enrichment integrals on the adaptive rule (oracle/adaptive.py, tol 1e-6,
    depth 2): the rule's point count per cell, sampled rows of Ht X for 16 vectors, column norms,
    and the eigenvalues of M^oo."""
    from oracle.adaptive import AdaptiveOEFEOperator
    cfg = wl.config("diamond8")
    t = time.time()
    op = AdaptiveOEFEOperator(cfg.system, 1e-6, 2)
    print("adaptive operator", op.rule.n_points, time.time() - t, flush=True)
    X0 = wl.start_block(op.n_tot, 16, cfg.x0_seed)
    rows = sample_rows(op.N, op.n_enr, 200, 23)
    HX = op.apply(X0)
    counts = np.array([op.rule.points[e].shape[0] for e in op.rule.cells.tolist()], dtype=np.int64)
    np.savez_compressed(os.path.join(HERE, "adaptive_diamond8_oracle.npz"), tol=1e-6, max_depth=2,
                        cells=op.rule.cells, counts=counts, rows=rows, hx_rows=HX[rows],
                        hx_colnorm=np.linalg.norm(HX, axis=0), Moo_eigs=op.enr.Moo_eigs)


if __name__ == "__main__":
    which = sys.argv[1:] or ["diamond8"]
    for w in which:
        {"diamond8": diamond8, "diamond64": diamond64, "kpoints": kpoints, "kpoint_passes": kpoint_passes,
         "diamond64_pass1": diamond64_pass1, "poisson_diamond8": poisson_diamond8, "uform_kpoints": uform_kpoints,
         "adaptive_diamond8": adaptive_diamond8}[w]()
