#!/usr/bin/env python3
"""Benchmark of the GKB / HKT hot path on one MI355X.

Workload: unit ball, N = 100000 nodes (80000 uniform interior nodes by
rejection, 20000 Fibonacci-lattice boundary nodes), kappa = 30, eps = 6,
manufactured u = sin(kappa (x+y+z)/sqrt(3)) (so f = 0 inside, g = u on the
sphere), Golub-Kahan with ell = 300 steps and full reorthogonalisation,
projected SVD, GCV and the HKT solution (Algorithm 4).

One step = one whole HKT solve from device-resident data (f, g) to the
coefficients on the device.  The headline variant evaluates matrix entries
in FP32 inside every product and accumulates in FP64 (reorthogonalisation,
Krylov scalars, projected SVD and GCV in FP64).  The stored-FP64 and
matrix-free-FP64 variants are timed beside it for the time-to-solution
comparison.

value = equivalent GKB product throughput of the whole solve,
2 ell 8 N^2 bytes (the FP64 matrix traffic the ell steps would need) divided
by the time to solution.  The roofline object describes the dominant kernel
of the headline variant (the matrix-free product, bound by VALU issue).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X peaks (vendor figures) and issue model
HBM_PEAK_GBS = 8000.0
CUS, SIMDS, LANES, CLOCK = 256, 4, 16, 2.4e9
VALU_SLOTS_PER_S = CUS * SIMDS * LANES * CLOCK  # 39.3e12 lane-operations per second (non-packed)
TRANS_SLOTS = 4  # a transcendental (rsq) occupies four issue slots (quarter rate)
# VALU lane-operations per entry in the FP32-evaluated product (per the entry formula):
#   interior: 3 sub + 3 fma (t) + rsq + 2 fma (polynomial) + 3 mul (s^3, product) + cvt + fma64
#   boundary: 3 sub + 3 fma (t) + rsq + 1 mul (t s) + cvt + fma64
SLOTS_INT_F32 = 13 + TRANS_SLOTS
SLOTS_BND_F32 = 9 + TRANS_SLOTS
#   FP64 evaluation: rsq + 2 Newton steps (8) instead of the FP32 rsq, no cvt
SLOTS_INT_F64 = 3 + 3 + TRANS_SLOTS + 8 + 2 + 3 + 1
SLOTS_BND_F64 = 3 + 3 + TRANS_SLOTS + 8 + 1 + 1


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def rel_l2(a, b):
    import numpy as np

    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_linf(a, b):
    import numpy as np

    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def run_variant(mq, torch, p, mode, steps, warmup, dev, want_kernel_times=True):
    """Create the problem, run warmup + timed solves; returns a dict of figures."""
    import numpy as np

    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pr = mq.Problem(p.x_int, p.x_bnd, p.kappa, p.eps, mode, stream=stream)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    f_int = torch.from_numpy(p.f_int).to(dev)
    g_bnd = torch.from_numpy(p.g_bnd).to(dev)
    coef = torch.empty(p.n, dtype=torch.float64, device=dev)
    for w in range(warmup):
        log(mode, "warmup", w)
        pr.solve(f_int, g_bnd, p.ell, coef=coef)
    torch.cuda.synchronize()
    times, outs = [], []
    for k in range(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = pr.solve(f_int, g_bnd, p.ell, coef=coef, time_products=want_kernel_times)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        outs.append(out)
        log(mode, "step", k, f"{times[-1]:.3f} s", "ell_done", out.ell_done, "lambda", f"{out.lam:.3e}")
    x_eval = torch.from_numpy(p.x_eval).to(dev)
    u = pr.eval(coef, x_eval).cpu().numpy()
    out = outs[-1]
    res = dict(mode=mode, setup_s=setup_s, step_s=times, solve_s=float(np.mean(times)), ell_done=out.ell_done,
               lam=out.lam, flags=out.flags, rel_l2=rel_l2(u, p.u_eval), rel_linf=rel_linf(u, p.u_eval),
               phase_ms=dict(upload=out.t_ms[0], gkb=out.t_ms[1], proj_svd=out.t_ms[2], param=out.t_ms[3],
                             lift=out.t_ms[4], total=out.t_ms[5]))
    if want_kernel_times:
        res["kernel_ms_AT"] = float(np.mean([o.t_ms[6] for o in outs])) / max(1, p.ell)
        res["kernel_ms_A"] = float(np.mean([o.t_ms[7] for o in outs])) / max(1, p.ell)
    pr.close()
    torch.cuda.synchronize()
    return res


def cpu_baseline(p, rows):
    """The oracle's entry-by-entry FP64 products on a row / column sample."""
    import numpy as np

    from oracle import oracle as O
    from paper_2511_09798_amd import inputs as I

    O.lib()
    x = I.random_vector(p.n, 1)
    idx = np.linspace(0, p.n - 1, rows).astype(np.int64)
    X = p.nodes
    t = time.perf_counter()
    O.apply_sampled(X, p.n_int, p.kappa, p.eps, x, idx, trans=True)
    O.apply_sampled(X, p.n_int, p.kappa, p.eps, x, idx, trans=False)
    dt = time.perf_counter() - t
    entries = 2.0 * rows * p.n
    per_product_s = dt / entries * p.n * p.n
    return dict(value=8.0 * p.n * p.n / per_product_s / 1e9, unit="GB/s (FP64-A-equivalent per product)",
                cores=O.num_threads(), kind="oracle",
                sample=f"{rows} rows of A x and {rows} columns of A^T x (entry-by-entry FP64, "
                       f"{entries:.2e} entries, {dt:.1f} s), scaled to whole products",
                seconds=dt, hkt_solve_s_extrapolated=2 * p.ell * per_product_s)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere_n100000")
    ap.add_argument("--ell", type=int, default=0, help="override the Golub-Kahan steps (0: workload's)")
    ap.add_argument("--variants", default="matfree_fp32,stored_fp64,matfree_fp64",
                    help="first one is the headline")
    ap.add_argument("--context-steps", type=int, default=1, help="timed solves of the non-headline variants")
    ap.add_argument("--cpu-rows", type=int, default=6000, help="row/column sample of the CPU baseline (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2511_09798_amd import inputs as I
    from paper_2511_09798_amd import mqhelm as mq

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = I.WORKLOADS[args.workload]()
    if args.ell:
        p.ell = args.ell
    log("workload", p.name, "n", p.n, "n_int", p.n_int, "ell", p.ell)
    variants = [v.strip() for v in args.variants.split(",") if v.strip()]
    results = {}
    for i, v in enumerate(variants):
        steps = args.steps if i == 0 else args.context_steps
        warm = args.warmup if i == 0 else min(args.warmup, 1)
        results[v] = run_variant(mq, torch, p, v, steps, warm, dev)
        log(v, json.dumps({k: results[v][k] for k in ("setup_s", "solve_s", "rel_l2", "lam")}))
    head = results[variants[0]]
    n = p.n
    ms = head["solve_s"] * 1000.0
    equiv_bytes = 2.0 * p.ell * 8.0 * n * n
    value = equiv_bytes / head["solve_s"] / 1e9

    # roofline of the dominant kernel of the headline variant
    k_at, k_a = head.get("kernel_ms_AT", float("nan")), head.get("kernel_ms_A", float("nan"))
    dom_ms, dom_name = (k_at, "A^T x") if k_at >= k_a else (k_a, "A x")
    mode = variants[0]
    if mode.startswith("matfree"):
        si, sb = (SLOTS_INT_F32, SLOTS_BND_F32) if mode == "matfree_fp32" else (SLOTS_INT_F64, SLOTS_BND_F64)
        work = (p.n_int * n * si + p.n_bnd * n * sb)  # VALU lane-operation slots per product
        achieved = work / (dom_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=VALU_SLOTS_PER_S / 1e12, unit="TOP/s",
                    frac=achieved / (VALU_SLOTS_PER_S / 1e12), traffic=None, kernel=f"{mode} {dom_name}",
                    kernel_ms=dom_ms, other_kernel_ms=min(k_at, k_a))
    else:
        achieved = 8.0 * n * n / (dom_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=None, kernel=f"{mode} {dom_name}", kernel_ms=dom_ms, other_kernel_ms=min(k_at, k_a))

    ctx = {}
    for v, r in results.items():
        tts = r["solve_s"] + (r["setup_s"] if v == "stored_fp64" else 0.0)
        ctx[v] = dict(time_to_solution_s=tts, solve_s=r["solve_s"], setup_s=r["setup_s"], rel_l2=r["rel_l2"],
                      rel_linf=r["rel_linf"], lam=r["lam"], ell_done=r["ell_done"],
                      product_ms_AT=r.get("kernel_ms_AT"), product_ms_A=r.get("kernel_ms_A"),
                      product_equiv_GBs=(8.0 * n * n / (0.5e-3 * (r["kernel_ms_AT"] + r["kernel_ms_A"])) / 1e9)
                      if "kernel_ms_AT" in r else None,
                      phase_ms=r["phase_ms"])
    line = dict(metric="HKT time-to-solution & GKB matvec GB/s at N=100k sphere, equal rel-L2 err",
                value=value, unit="GB/s (FP64-A-equivalent product traffic over the whole HKT solve)",
                n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f32-entries/f64-accumulate", data="synthetic",
                config=dict(workload=p.name, n=n, n_int=p.n_int, n_bnd=p.n_bnd, kappa=p.kappa, eps=p.eps,
                            ell=p.ell, method="HKT", rule="GCV", operator=variants[0]),
                hkt_time_to_solution_s=head["solve_s"], roofline=roof, variants=ctx)
    if args.cpu_rows > 0:
        log("cpu baseline", args.cpu_rows, "rows")
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_rows)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
