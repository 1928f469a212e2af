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

# MI355X peaks (vendor unit counts and clock) and the VALU issue model.
HBM_PEAK_GBS = 8000.0
CUS, SIMDS, LANES, CLOCK = 256, 4, 16, 2.4e9
# A SIMD issues one wave64 VALU instruction per 4 cycles; gfx950 can issue two
# FP32 instructions together when neither reads a scalar register (measured
# with SQ_ACTIVE_INST_VALU2).  FP64 and transcendental instructions issue
# alone; v_rsq_f32 / v_sqrt_f32 occupy two issue slots, v_rsq_f64 four.
VALU_PEAK_DUAL = CUS * SIMDS * 2 * LANES * CLOCK  # 78.6e12 lane-operations/s (= FP32 vector peak / 2 flops)
VALU_PEAK_SINGLE = CUS * SIMDS * LANES * CLOCK  # 39.3e12 lane-operations/s (FP64 rate)
MFMA_F32_PEAK = 157.3e12  # dense FP32 matrix-core flop/s
# Algorithmic operations per matrix entry (the entry formula evaluated
# directly, a transcendental counted once):
#   FP32: interior 3 sub + 3 fma (t) + rsq + mul (s^2) + 2 fma + fma (accumulate) = 11
#         boundary 3 sub + 3 fma (t) + sqrt + fma (accumulate)                    = 8
#   FP64: interior 3 sub + 3 fma + rsq + 8 (two Newton steps) + mul + 2 fma + mul + fma = 20
#         boundary 3 sub + 3 fma + rsq + 8 + mul + fma                                  = 17
# The FP32 product computes t (the first 6 operations) on the matrix cores;
# the achieved rate still counts all 11 / 8 against the FP32 vector peak.
OPS = {"matfree_fp32": (11, 8), "matfree_fp64": (20, 17)}
# Issue quad-cycles per 64 entries of the instructions the FP32 product runs,
# if every pairable VALU instruction were paired: one 16x16x32 bf16 MFMA per
# 256 entries (16 cycles, no co-execution with the VALU measured: 1 quad per 64),
# interior rsq (2) + 4 pairable (2), boundary sqrt (2) + 1 pairable (0.5).
QUADS_IDEAL_F32 = (5.0, 3.5)
PROFILES = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def measured_traffic(kernel_key: str):
    """HBM bytes per launch from the committed counter runs, or None when the
    kernel source changed since they were taken."""
    import hashlib

    try:
        with open(PROFILES) as fh:
            rec = json.load(fh).get(kernel_key)
        with open(os.path.join(ROOT, rec["source"]), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, KeyError, TypeError, ValueError):
        return None
    if sha != rec.get("source_sha256"):
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def measure_peaks(mq):
    """The reference kernels of mqh_peak_probe on this GPU: HBM copy and read
    (GB/s, bytes moved), FP32 / FP64 FMA chains and FP64 matrix-core chains
    (TFLOP/s)."""
    copy = mq.mqh_peak_probe(mq.MQH_PEAK_COPY, 1 << 31, reps=5)
    read = mq.mqh_peak_probe(mq.MQH_PEAK_READ, 1 << 32, reps=5)
    f32 = mq.mqh_peak_probe(mq.MQH_PEAK_FMA_F32, 1 << 14, reps=5)
    f64 = mq.mqh_peak_probe(mq.MQH_PEAK_FMA_F64, 1 << 14, reps=5)
    m64 = mq.mqh_peak_probe(mq.MQH_PEAK_MFMA_F64, 1 << 14, reps=5)
    return dict(hbm_copy_GBs=copy / 1e9, hbm_read_GBs=read / 1e9, fp32_fma_TFLOPs=f32 / 1e12, fp64_fma_TFLOPs=f64 / 1e12,
                fp64_mfma_TFLOPs=m64 / 1e12,
                spec=dict(hbm_GBs=HBM_PEAK_GBS, fp32_vector_TFLOPs=157.3, fp64_vector_TFLOPs=78.6,
                          fp64_matrix_TFLOPs=78.6))


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def rel_l2(a, b):
    import numpy as np

    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_linf(a, b):
    import numpy as np

    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def parse_variant(mq, spec):
    """'mode[:method[:rule[:weight]]]' -> (operator mode, solve keyword arguments).

    method: hkt (Algorithm 4, default), tsvd (Algorithm 2), lsqr (Section 3.4);
    rule: gcv (default), lcurve, wgcv (weighted GCV, weight default 0.5)."""
    parts = spec.split(":")
    mode = parts[0]
    method = {"hkt": mq.MQH_METHOD_HKT, "tsvd": mq.MQH_METHOD_INE_TSVD,
              "lsqr": mq.MQH_METHOD_LSQR}[parts[1] if len(parts) > 1 else "hkt"]
    rule = {"gcv": mq.MQH_RULE_GCV, "lcurve": mq.MQH_RULE_LCURVE,
            "wgcv": mq.MQH_RULE_WGCV}[parts[2] if len(parts) > 2 else "gcv"]
    kw = dict(method=method, rule=rule)
    if rule == mq.MQH_RULE_WGCV:
        kw["gcv_weight"] = float(parts[3]) if len(parts) > 3 else 0.5
    if method == mq.MQH_METHOD_LSQR:
        kw["want_sv"] = False  # the LSQR stop needs no projected SVD
    return mode, kw


def run_variant(mq, torch, p, spec, steps, warmup, dev, want_kernel_times=True):
    """Create the problem, run warmup + timed solves; returns a dict of figures."""
    import numpy as np

    mode, kw = parse_variant(mq, spec)
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
        log(spec, "warmup", w)
        pr.solve(f_int, g_bnd, p.ell, coef=coef, **kw)
    torch.cuda.synchronize()
    times, outs = [], []
    for k in range(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = pr.solve(f_int, g_bnd, p.ell, coef=coef, time_products=want_kernel_times, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        outs.append(out)
        log(spec, "step", k, f"{times[-1]:.3f} s", "ell_done", out.ell_done, "lambda", f"{out.lam:.3e}",
            "k", out.k)
    x_eval = torch.from_numpy(p.x_eval).to(dev)
    u = pr.eval(coef, x_eval).cpu().numpy()
    out = outs[-1]
    res = dict(mode=mode, setup_s=setup_s, step_s=times, solve_s=float(np.mean(times)), ell_done=out.ell_done,
               lam=out.lam, k=out.k, flags=out.flags, rel_l2=rel_l2(u, p.u_eval), rel_linf=rel_linf(u, p.u_eval),
               phase_ms=dict(upload=out.t_ms[0], gkb=out.t_ms[1], proj_svd=out.t_ms[2], param=out.t_ms[3],
                             lift=out.t_ms[4], total=out.t_ms[5]))
    if want_kernel_times:
        res["kernel_ms_AT"] = float(np.mean([o.t_ms[6] for o in outs])) / max(1, p.ell)
        res["kernel_ms_A"] = float(np.mean([o.t_ms[7] for o in outs])) / max(1, p.ell)
    pr.close()
    torch.cuda.synchronize()
    return res


def learned_context(mq, torch, dev, count: int, n: int = 60000, ell: int = 60, seed: int = 5):
    """Pump-casing-like solid, n nodes (80% interior), kappa in [5, 35], eps in [2, 8]: the plain
    method (ell steps, GCV) against the learned solve (predicted steps and lambda, GCV as judge)."""
    import numpy as np

    from paper_2511_09798_amd import learned as L

    model = L.load_predictor()
    rng = np.random.default_rng(seed)
    rows = []
    for k in range(count):
        prob = L.sample_problem(rng, kind="casing", n=n, kappa=float(rng.uniform(5, 35)),
                                eps=float(rng.uniform(2, 8)), n_eval=2000)
        pred, keep = L.make_device_predictor(mq, torch, model, prob["h"], dev)
        with mq.Problem(prob["x_int"], prob["x_bnd"], prob["kappa"], prob["eps"], "matfree_fp32") as pr:
            fi = torch.from_numpy(prob["f_int"]).to(dev)
            gb = torch.from_numpy(prob["g_bnd"]).to(dev)
            xe = torch.from_numpy(prob["x_eval"]).to(dev)
            pr.solve(fi, gb, ell)  # warm
            torch.cuda.synchronize()
            t = time.perf_counter()
            base = pr.solve(fi, gb, ell)
            torch.cuda.synchronize()
            t_base = time.perf_counter() - t
            t = time.perf_counter()
            out = pr.solve_learned(fi, gb, ell, pred)
            torch.cuda.synchronize()
            t_net = time.perf_counter() - t
            ub = pr.eval(base.coef, xe).cpu().numpy()
            un = pr.eval(out.coef, xe).cpu().numpy()
        rows.append(dict(kappa=prob["kappa"], eps=prob["eps"], steps=out.ell_pred, used_net=out.used_net_lambda,
                         t_gcv=t_base, t_learned=t_net, err_gcv=rel_l2(ub, prob["u_eval"]),
                         err_learned=rel_l2(un, prob["u_eval"]), lam_gcv=base.lam, lam_learned=out.lam))
        log("learned casing", k, json.dumps(rows[-1]))
    eg = np.array([r["err_gcv"] for r in rows])
    en = np.array([r["err_learned"] for r in rows])
    return dict(workload=f"casing_n{n}", problems=count, ell=ell, mean_steps_learned=float(np.mean([r["steps"] for r in rows])),
                steps_gcv=ell, mean_time_gcv_s=float(np.mean([r["t_gcv"] for r in rows])),
                mean_time_learned_s=float(np.mean([r["t_learned"] for r in rows])),
                median_rel_l2_gcv=float(np.median(eg)), median_rel_l2_learned=float(np.median(en)),
                net_lambda_used=int(sum(r["used_net"] for r in rows)), cases=rows)


def sweep_context(mq, torch, dev, count: int, compare: int, oracle_check: bool, workers: int,
                  fixed_shapes: bool = False):
    """Frequency sweep over cubes: count problems (N uniform on [2000, 30000], kappa evenly spaced
    on [2, 40], eps = 0.2 kappa + 1), 16 Gaussian-blob sources each, ell = 100, HKT with GCV for
    every source through the lockstep runs with block products (FP32 entries).  All problems and
    sources are resident on the device; the sweep runs once one problem at a time (kernel timing)
    and once with `workers` problems side by side, each on its own stream (the sweep time)."""
    import numpy as np

    from paper_2511_09798_amd import inputs as I

    ns = I.sweep_sizes()[:count]
    probs, handles, Fs, coefs = [], [], [], []
    t = time.perf_counter()
    for k in range(count):
        p = I.sweep_member(k)
        probs.append(p)
        handles.append(mq.Problem(p.x_int, p.x_bnd, p.kappa, p.eps, "matfree_fp32", fixed_shapes=fixed_shapes))
        Fs.append(torch.from_numpy(p.F).to(dev))
        coefs.append(torch.empty_like(Fs[-1]))
    torch.cuda.synchronize()
    log("sweep setup", f"{time.perf_counter() - t:.1f} s")
    ell = probs[0].ell
    mq.mqh_solve_sweep(handles, Fs, ell, workers=workers, coefs=coefs)  # warmup (workspaces)
    torch.cuda.synchronize()
    # one problem at a time, product kernels timed
    t = time.perf_counter()
    outs = mq.mqh_solve_sweep(handles, Fs, ell, workers=1, coefs=coefs, time_products=True)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t
    kern_ms = gkb_ms = svd_ms = par_ms = lift_ms = flops = 0.0
    solves = 0
    for p, o in zip(probs, outs):
        tm = o.t_ms[0]
        kern_ms += tm[6] + tm[7]
        gkb_ms += tm[1]
        svd_ms += tm[2]
        par_ms += tm[3]
        lift_ms += tm[4]
        flops += 2.0 * 2.0 * p.ell * p.n * p.n * p.nrhs * (int(o.ell_done.min()) / p.ell)
        solves += p.nrhs
    log("sweep one problem at a time", f"{seq_s:.3f} s", "block kernels", f"{kern_ms / 1e3:.3f} s")
    # side by side, with and without the captured Golub-Kahan loops (the first
    # graph run captures)
    reps, greps = [], []
    for r in range(2):
        torch.cuda.synchronize()
        t = time.perf_counter()
        outs_p = mq.mqh_solve_sweep(handles, Fs, ell, workers=workers, coefs=coefs)
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - t)
        log("sweep", workers, "workers", f"{reps[-1]:.3f} s")
    for r in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        outs_g = mq.mqh_solve_sweep(handles, Fs, ell, workers=workers, coefs=coefs, graph=True)
        torch.cuda.synchronize()
        greps.append(time.perf_counter() - t)
        log("sweep", workers, "workers, graphs", f"{greps[-1]:.3f} s")
    graph_s = min(greps[1:])
    graph_same = all(np.array_equal(a.lam, b.lam) for a, b in zip(outs_p, outs_g))
    par_s = min(min(reps), graph_s)
    same = all(np.array_equal(a.lam, b.lam) for a, b in zip(outs, outs_p))
    res = dict(workload=f"cube frequency sweep: {count} problems, N uniform on [2000, 30000], kappa evenly "
                        "spaced on [2, 40], eps = 0.2 kappa + 1, 16 Gaussian-blob sources (width 0.1), g = 0, "
                        "ell = 100, HKT + GCV per source, FP32 entries, block products",
               problems=count, sources=solves, sum_n2=float((ns.astype(np.float64) ** 2).sum()),
               time_s=par_s, workers=workers, source_solves_per_s=solves / par_s,
               block_shapes="fixed (size heuristic)" if fixed_shapes else "autotuned",
               time_one_at_a_time_s=seq_s, same_choices_side_by_side=bool(same),
               time_no_graph_s=min(reps), time_graph_s=graph_s, graph_capture_run_s=greps[0],
               same_choices_graph=bool(graph_same),
               phase_ms_one_at_a_time=dict(gkb=gkb_ms, proj_svd=svd_ms, param=par_ms, lift=lift_ms),
               block_product_ms=kern_ms,
               roofline=dict(bound="mfma", achieved=flops / (kern_ms * 1e-3) / 1e12, peak=MFMA_F32_PEAK / 1e12,
                             unit="TFLOP/s", frac=flops / (kern_ms * 1e-3) / MFMA_F32_PEAK,
                             kernel="k_mfm_block", flops=flops,
                             note="2 n^2 s flops per block product (the dense n x n by n x s contraction); "
                                  "entries and squared distances are extra issue on the same SIMDs"))
    seq = []
    for k in range(min(compare, count)):
        p, h, F = probs[k], handles[k], Fs[k]
        torch.cuda.synchronize()
        t = time.perf_counter()
        h.solve_multi(F, p.ell, coef=coefs[k])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        for r in range(p.nrhs):  # warmup of the single-source path
            h.solve(F[r, :p.n_int].contiguous(), F[r, p.n_int:].contiguous(), p.ell)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for r in range(p.nrhs):
            h.solve(F[r, :p.n_int].contiguous(), F[r, p.n_int:].contiguous(), p.ell)
        torch.cuda.synchronize()
        seq.append((p.n, dt, time.perf_counter() - t))
        log("sweep", k, "lockstep", f"{dt * 1e3:.1f} ms", "one source at a time", f"{seq[-1][2] * 1e3:.1f} ms")
    if seq:
        res["vs_sequential_single"] = dict(problems=len(seq), n=[q[0] for q in seq],
                                           lockstep_s=sum(q[1] for q in seq), sequential_s=sum(q[2] for q in seq),
                                           speedup=sum(q[2] for q in seq) / sum(q[1] for q in seq))
    if oracle_check:
        from oracle import oracle as O

        k = int(np.argmin(ns))
        p = probs[k]
        x_eval = I.cube_interior_uniform(1000, 77)
        cg = coefs[k].cpu().numpy()
        e = []
        for r in range(p.nrhs):
            ro = O.solve(p.nodes, p.n_int, p.kappa, p.eps, p.F[r], p.ell, stored=True)
            u = O.eval_u(p.nodes, p.eps, cg[r], x_eval)
            uo = O.eval_u(p.nodes, p.eps, ro.coef, x_eval)
            e.append(rel_l2(u, uo))
        res["oracle_check"] = dict(problem=k, n=p.n, kappa=p.kappa, max_rel_l2_vs_oracle=float(max(e)),
                                   median_rel_l2_vs_oracle=float(np.median(e)))
        log("sweep oracle check", json.dumps(res["oracle_check"]))
    for h in handles:
        h.close()
    del Fs, coefs
    torch.cuda.synchronize()
    return res


def block_context(mq, torch, dev, members=(0, 1), steps=(7, 25), ell_lockstep: int = 100):
    """Block Golub-Kahan (one Krylov space for a problem's 16 sources) beside the lockstep runs (one
    space per source, ell = 100) on the largest sweep problems: solve times, and how far the block
    solutions' u at 1000 interior points lies from the lockstep ones; then the block solve against
    the block oracle on the smallest sweep problem (FP32 block products and stored FP64)."""
    import numpy as np

    from oracle import block as B
    from oracle import oracle as O
    from paper_2511_09798_amd import inputs as I

    res = dict(workload="frequency-sweep cubes, 16 Gaussian-blob sources, HKT + GCV per source, FP32-evaluated "
                        "block products", lockstep_ell=ell_lockstep, block_steps=list(steps), problems=[])
    xe = np.random.default_rng(3).random((1000, 3))
    xe_t = torch.from_numpy(xe).to(dev)

    def timed(fn):
        fn()  # warm-up (shapes, workspaces)
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t

    for k in members:
        m = I.sweep_member(k)
        with mq.Problem(m.x_int, m.x_bnd, m.kappa, m.eps, "matfree_fp32") as pr:
            F = torch.from_numpy(m.F).to(dev)
            lk, tl = timed(lambda: pr.solve_multi(F, ell_lockstep))
            ul = torch.stack([pr.eval(lk.coef[q], xe_t) for q in range(F.shape[0])])
            row = dict(n=int(m.F.shape[1]), kappa=m.kappa, lockstep_s=tl)
            for lb in steps:
                bk, tb = timed(lambda: pr.solve_block(F, lb))
                ub = torch.stack([pr.eval(bk.coef[q], xe_t) for q in range(F.shape[0])])
                d = ((ub - ul).norm(dim=1) / ul.norm(dim=1)).cpu().numpy()
                row[f"block{lb}_s"] = tb
                row[f"block{lb}_phases_ms"] = dict(recurrence=float(bk.t_ms[0][1]), projected=float(bk.t_ms[0][2]))
                row[f"block{lb}_u_vs_lockstep_median"] = float(np.median(d))
                row[f"block{lb}_resid_over_lockstep_median"] = float(np.median(bk.resid_norm / lk.resid_norm))
        res["problems"].append(row)
        log("block", json.dumps(row))
    k = int(np.argmin(I.sweep_sizes()))
    m = I.sweep_member(k)
    X = np.vstack([m.x_int, m.x_bnd])
    A = O.assemble(X, m.x_int.shape[0], m.kappa, m.eps)
    lb = steps[-1]
    r = B.block_solve(A, m.F.T, lb)
    chk = dict(problem=k, n=int(X.shape[0]), block_steps=lb)
    for mode in ("matfree_fp32", "stored_fp64"):
        with mq.Problem(m.x_int, m.x_bnd, m.kappa, m.eps, mode) as pr:
            b = pr.solve_block(m.F, lb)
            errs = []
            for q in range(m.F.shape[0]):
                u = pr.eval(b.coef[q], xe)
                uo = O.eval_u(X, m.eps, r.coef[:, q], xe)
                errs.append(float(np.linalg.norm(u - uo) / np.linalg.norm(uo)))
        chk[mode] = dict(max_rel_l2_vs_oracle=max(errs), lambda_max_rel=float(np.max(np.abs(b.lam / r.lam - 1.0))))
    res["oracle_check"] = chk
    log("block oracle check", json.dumps(chk))
    return res


def full_context(mq, torch, dev, level: int):
    """Classical Tikhonov with GCV on the full SVD (Algorithm 3) on the 20 000-node cube, stored FP64 A,
    against HKT (ell = 200, GCV) on the same problem: time to solution and error against the manufactured u."""
    import numpy as np

    from paper_2511_09798_amd import inputs as I

    p = I.cube_medium()
    res = dict(workload=f"{p.name}: kappa {p.kappa}, eps {p.eps}, stored FP64 A")
    with mq.Problem(p.x_int, p.x_bnd, p.kappa, p.eps, "stored_fp64") as pr:
        f_int = torch.from_numpy(p.f_int).to(dev)
        g_bnd = torch.from_numpy(p.g_bnd).to(dev)
        x_eval = torch.from_numpy(p.x_eval).to(dev)
        runs = [("tikh_reg_full_svd", dict(method=mq.MQH_METHOD_HKT))]
        if level >= 2:
            runs.append(("tsvd_full_svd", dict(method=mq.MQH_METHOD_INE_TSVD)))
        for name, kw in runs:
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = pr.full_solve(f_int, g_bnd, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            u = pr.eval(out.coef, x_eval).cpu().numpy()
            res[name] = dict(time_s=dt, sweeps=out.ell_done, off=out.t_ms[6], lam=out.lam, k=out.k,
                             rel_l2=rel_l2(u, p.u_eval), rel_linf=rel_linf(u, p.u_eval),
                             phase_ms=dict(assembly=out.t_ms[0], jacobi=out.t_ms[1], order=out.t_ms[2],
                                           param=out.t_ms[3], solution=out.t_ms[4]),
                             cg_iterations=int(out.t_ms[7]), status=int(out.status),
                             solution_converged=not (out.flags & mq.MQH_INFO_SOLVE_NOCONV))
            log("full", name, json.dumps(res[name]))
        pr.solve(f_int, g_bnd, p.ell)  # warmup
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = pr.solve(f_int, g_bnd, p.ell)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        u = pr.eval(out.coef, x_eval).cpu().numpy()
        res["hkt"] = dict(time_s=dt, ell=p.ell, lam=out.lam, rel_l2=rel_l2(u, p.u_eval), rel_linf=rel_linf(u, p.u_eval))
        log("full hkt", json.dumps(res["hkt"]))
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
    ap.add_argument("--variants",
                    default="matfree_fp32,stored_fp64,matfree_fp64,matfree_fp32:lsqr:gcv,matfree_fp32:lsqr:lcurve,"
                            "matfree_fp32:hkt:wgcv:0.5",
                    help="first one is the headline; each is mode[:method[:rule[:weight]]]")
    ap.add_argument("--context-steps", type=int, default=1, help="timed solves of the non-headline variants")
    ap.add_argument("--cpu-rows", type=int, default=150000, help="row/column sample of the CPU baseline (0: skip)")
    ap.add_argument("--learned", type=int, default=8,
                    help="pump-casing problems for the learned-solve comparison (0: skip)")
    ap.add_argument("--sweep", type=int, default=64, help="problems of the multi-source frequency sweep (0: skip)")
    ap.add_argument("--sweep-compare", type=int, default=2,
                    help="sweep problems also solved one source at a time for comparison")
    ap.add_argument("--sweep-oracle", type=int, default=1, help="check the smallest sweep problem against the oracle")
    ap.add_argument("--sweep-workers", type=int, default=4, help="sweep problems run side by side")
    ap.add_argument("--sweep-fixed-shapes", type=int, default=0, help="block-product shapes from the size heuristic")
    ap.add_argument("--block", type=int, default=1,
                    help="block Golub-Kahan beside the lockstep runs on the largest sweep problems (0: skip)")
    ap.add_argument("--full", type=int, default=1,
                    help="full-SVD reference on the 20 000-node cube beside HKT: 1 Tikh-Reg (about a minute), "
                         "2 also TSVD (0: skip)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (reference for HBM counters)")
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
    if args.copy_ref_mib > 0:
        nel = args.copy_ref_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy reference", args.copy_ref_mib, "MiB read +", args.copy_ref_mib, "MiB written")
        del src, dst
    peaks = measure_peaks(mq)
    log("measured peaks", json.dumps(peaks))
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
    mode = head["mode"]
    kern = {"matfree_fp32": ("k_mfm<false>", "k_mfm<true>"), "matfree_fp64": ("k_mf_cols", "k_mf_rows"),
            "stored_fp64": ("k_stored_cols", "k_stored_rows")}[mode][0 if dom_name == "A^T x" else 1]
    if mode.startswith("matfree"):
        oi, ob = OPS[mode]
        work = p.n_int * n * oi + p.n_bnd * n * ob  # lane-operations per product
        peak = VALU_PEAK_DUAL if mode == "matfree_fp32" else VALU_PEAK_SINGLE
        achieved = work / (dom_ms * 1e-3) / 1e12
        # measured: FMA lane-operations per second of the probe (flop/s / 2)
        mpeak = (peaks["fp32_fma_TFLOPs"] if mode == "matfree_fp32" else peaks["fp64_fma_TFLOPs"]) / 2.0
        roof = dict(bound="alu", achieved=achieved, peak=peak / 1e12, unit="TOP/s", frac=achieved / (peak / 1e12),
                    traffic=measured_traffic(kern), kernel=kern, kernel_ms=dom_ms,
                    other_kernel_ms=min(k_at, k_a), ops_per_product=work,
                    measured_peak=mpeak, frac_of_measured=achieved / mpeak,
                    measured_peak_note=("FMA lane-operations/s of the FMA probe; achieved counts all of the formula's "
                                        "operations, some of which run on the matrix cores, so this fraction is not "
                                        "a VALU efficiency (issue_model_frac is)") if mode == "matfree_fp32" else
                    "FMA lane-operations/s of the FMA probe")
        if mode == "matfree_fp32":
            quads = (p.n_int * n * QUADS_IDEAL_F32[0] + p.n_bnd * n * QUADS_IDEAL_F32[1]) / 64.0
            t_ideal = quads / (CUS * SIMDS * CLOCK / 4.0)
            roof["issue_model_ms"] = t_ideal * 1e3
            roof["issue_model_frac"] = t_ideal / (dom_ms * 1e-3)
            roof["note"] = ("t = 1 + eps^2 r^2 on the matrix cores (bf16x3-split K=32 MFMA), entries on the VALU; "
                            "achieved counts the direct formula's lane-operations")
    else:
        achieved = 8.0 * n * n / (dom_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=measured_traffic(kern), kernel=kern, kernel_ms=dom_ms,
                    other_kernel_ms=min(k_at, k_a), measured_peak=peaks["hbm_read_GBs"],
                    frac_of_measured=achieved / peaks["hbm_read_GBs"])

    ctx = {}
    for v, r in results.items():
        tts = r["solve_s"] + (r["setup_s"] if r["mode"] == "stored_fp64" else 0.0)
        ctx[v] = dict(time_to_solution_s=tts, solve_s=r["solve_s"], setup_s=r["setup_s"], rel_l2=r["rel_l2"],
                      rel_linf=r["rel_linf"], lam=r["lam"], k=r["k"], ell_done=r["ell_done"],
                      product_ms_AT=r.get("kernel_ms_AT"), product_ms_A=r.get("kernel_ms_A"),
                      product_equiv_GBs=(8.0 * n * n / (0.5e-3 * (r["kernel_ms_AT"] + r["kernel_ms_A"])) / 1e9)
                      if "kernel_ms_AT" in r else None,
                      phase_ms=r["phase_ms"])
    line = dict(metric="HKT time-to-solution & GKB matvec GB/s at N=100k sphere, equal rel-L2 err",
                value=value, unit="GB/s (FP64-A-equivalent product traffic over the whole HKT solve)",
                n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f32" if mode == "matfree_fp32" else "f64", data="synthetic",
                config=dict(workload=p.name, n=n, n_int=p.n_int, n_bnd=p.n_bnd, kappa=p.kappa, eps=p.eps,
                            ell=p.ell, method="HKT", rule="GCV", operator=mode),
                hkt_time_to_solution_s=head["solve_s"], roofline=roof, peaks_measured=peaks, variants=ctx)
    if args.learned > 0:
        from paper_2511_09798_amd import learned as L

        if os.path.exists(L.MODEL_PATH):
            line["learned"] = learned_context(mq, torch, dev, args.learned)
        else:
            log("no trained predictor at", L.MODEL_PATH, "- learned comparison skipped")
    if args.sweep > 0:
        line["sweep"] = sweep_context(mq, torch, dev, args.sweep, args.sweep_compare, bool(args.sweep_oracle),
                                      args.sweep_workers, bool(args.sweep_fixed_shapes))
    if args.block > 0:
        line["block_gkb"] = block_context(mq, torch, dev)
    if args.full > 0:
        line["full_svd_reference"] = full_context(mq, torch, dev, args.full)
    if args.cpu_rows > 0:
        log("cpu baseline", args.cpu_rows, "rows")
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_rows)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
