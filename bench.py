#!/usr/bin/env python3
"""Benchmark of the GKB / HKT hot path on one MI355X.

Workload: unit ball, N = 100000 nodes (80000 uniform interior nodes by
rejection, 20000 Fibonacci-lattice boundary nodes), kappa = 30, eps = 6,
manufactured u = sin(kappa (x+y+z)/sqrt(3)) (so f = 0 inside, g = u on the
sphere), Golub-Kahan with ell = 300 steps and full reorthogonalisation,
projected SVD, GCV and the HKT solution (Algorithm 4).

One step = one HKT time to solution on the plain FP64 path: problem
creation from nodes already in HBM (assembly of the stored FP64 matrix),
the solve from f, g in HBM to the coefficients in HBM, and the release of
the problem.  value = GKB matvec throughput of that step: the 2 ell products
stream the stored matrix (53.0 GB of tiles, its symmetric blocks stored
once), so value = 2 ell x 53.0 GB / time to solution.  The roofline object
describes the dominant product kernel, timed with HIP events on the
problem's stream around every product launch of the timed steps.

Beside it, outside the timed steps: the FP32-evaluated matrix-free HKT (the
precision form) and the matrix-free FP64 HKT with their errors against the
FP64 result, the equal-error comparison (the smallest ell whose FP32 HKT
error is within 5% of the FP64 reference) on this workload and on the
20 000-node cube, the row scaling option, other projected-side rules, the
learned stop, the multi-source sweep, the block Golub-Kahan process, the
full-SVD reference and the oracle timed on the host's cores.
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

# MI355X published peaks.
HBM_PEAK_GBS = 8000.0
FP32_PEAK = 157.3e12  # FP32 vector (and FP32 matrix) flop/s
FP64_PEAK = 78.6e12
MFMA_F32_PEAK = 157.3e12  # dense FP32 matrix-core flop/s
CUS, SIMDS, CLOCK = 256, 4, 2.4e9
# Operations per matrix entry of the FP32-evaluated product as the design
# counts them (distances, t, one rsqrt, the interior formula, the conversion
# and the FP64 accumulation): interior 15 FP32 + rsqrt + cvt + FP64 FMA = 18,
# boundary 9 + rsqrt + cvt + FMA = 12.  Rated against the FP32 vector peak.
OPS_F32 = (18, 12)
# FP64 matrix-free product: interior 3 sub + 3 fma + rsq + 5 (its refinement to
# FP64, one third-order step) + mul + 2 fma + mul + fma = 17, boundary 14;
# rated against the FP64 peak.
OPS_F64 = (17, 14)
# The FP32-evaluated product evaluates every unordered pair of nodes once
# (t, the rsqrt and the formula serve A_ij and A_ji).  Issue quad-cycles per
# 64 pairs if every pairable VALU instruction were paired: one bf16 MFMA per
# 256 pairs (1), rsq or sqrt (2), and half the pairable FP32 instructions:
# interior-interior 6 (s^2, 2 for the formula, the product by s, the row and
# the column sums), interior-boundary 7 (also t s), boundary-boundary 2.
QUADS_IDEAL_PAIR = dict(ii=1.0 + 2.0 + 3.0, ib=1.0 + 2.0 + 3.5, bb=1.0 + 2.0 + 1.0)
TILE = 128
PROFILES = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def stored_bytes(n: int, n_int: int) -> int:
    """Bytes of the stored matrix as the library keeps it: 128 x 128 FP64 tiles per class
    (interior, boundary), the symmetric interior-interior and boundary-boundary blocks by
    their upper tiles only."""
    nti = -(-n_int // TILE)
    nt = nti + (-(-(n - n_int) // TILE))
    tiles = sum((nt - r) if r < nti else (nti + nt - r) for r in range(nt))
    return tiles * TILE * TILE * 8


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


def measure_peaks():
    """The reference kernels of the measurement library (libmqhpeak) on this GPU: HBM copy
    and read (GB/s, bytes moved), FP32 / FP64 FMA chains and FP64 matrix-core chains
    (TFLOP/s), v_rsq_f32 alone and followed by four FMAs (lane operations or groups per
    second, in units of 1e12) and the bf16 matrix-core instruction of the FP32 product (TFLOP/s)."""
    from paper_2511_09798_amd import peak as pk

    copy = pk.mqh_peak_probe(pk.MQH_PEAK_COPY, 1 << 31, reps=5)
    read = pk.mqh_peak_probe(pk.MQH_PEAK_READ, 1 << 32, reps=5)
    f32 = pk.mqh_peak_probe(pk.MQH_PEAK_FMA_F32, 1 << 14, reps=5)
    f64 = pk.mqh_peak_probe(pk.MQH_PEAK_FMA_F64, 1 << 14, reps=5)
    m64 = pk.mqh_peak_probe(pk.MQH_PEAK_MFMA_F64, 1 << 14, reps=5)
    rsq = pk.mqh_peak_probe(pk.MQH_PEAK_RSQ_F32, 1 << 12, reps=5)
    mix = pk.mqh_peak_probe(pk.MQH_PEAK_RSQ_FMA_F32, 1 << 12, reps=5)
    mbf = pk.mqh_peak_probe(pk.MQH_PEAK_MFMA_BF16, 1 << 13, reps=5)
    return dict(hbm_copy_GBs=copy / 1e9, hbm_read_GBs=read / 1e9, fp32_fma_TFLOPs=f32 / 1e12, fp64_fma_TFLOPs=f64 / 1e12,
                fp64_mfma_TFLOPs=m64 / 1e12, fp32_rsq_Tps=rsq / 1e12, fp32_rsq_plus_4fma_Tps=mix / 1e12,
                bf16_mfma_TFLOPs=mbf / 1e12,
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
    """'mode[:method[:rule[:weight]]][+rs]' -> (operator mode, solve keyword arguments).

    method: hkt (Algorithm 4, default), tsvd (Algorithm 2), lsqr (Section 3.4);
    rule: gcv (default), lcurve, wgcv (weighted GCV, weight default 0.5);
    +rs: the row scaling D = diag(A)^-1."""
    rs = spec.endswith("+rs")
    parts = spec[:-3].split(":") if rs else spec.split(":")
    mode = parts[0]
    method = {"hkt": mq.MQH_METHOD_HKT, "tsvd": mq.MQH_METHOD_INE_TSVD,
              "lsqr": mq.MQH_METHOD_LSQR}[parts[1] if len(parts) > 1 else "hkt"]
    rule = {"gcv": mq.MQH_RULE_GCV, "lcurve": mq.MQH_RULE_LCURVE,
            "wgcv": mq.MQH_RULE_WGCV}[parts[2] if len(parts) > 2 else "gcv"]
    kw = dict(method=method, rule=rule, row_scale=int(rs))
    if rule == mq.MQH_RULE_WGCV:
        kw["gcv_weight"] = float(parts[3]) if len(parts) > 3 else 0.5
    if method == mq.MQH_METHOD_LSQR:
        kw["want_sv"] = False  # the LSQR stop needs no projected SVD
    return mode, kw


class DeviceInputs:
    """A workload's nodes, data and evaluation points resident in HBM."""

    def __init__(self, torch, p, dev):
        self.x_int = torch.from_numpy(p.x_int).to(dev)
        self.x_bnd = torch.from_numpy(p.x_bnd).to(dev)
        self.f_int = torch.from_numpy(p.f_int).to(dev)
        self.g_bnd = torch.from_numpy(p.g_bnd).to(dev)
        self.rhs = torch.from_numpy(p.rhs).to(dev)
        self.x_eval = torch.from_numpy(p.x_eval).to(dev)


def solve_step(mq, torch, p, d, mode, ell, kw, time_products=False, keep=False):
    """One time to solution from inputs in HBM: create (assembly in the stored mode), solve,
    release.  Returns (seconds, create seconds, solve output, u at the evaluation points as a
    numpy array, the problem when keep)."""
    stream = torch.cuda.current_stream(d.x_int.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pr = mq.Problem(d.x_int, d.x_bnd, p.kappa, p.eps, mode, stream=stream)
    t1 = time.perf_counter()  # create synchronises its stream
    out = pr.solve(d.f_int, d.g_bnd, ell, time_products=time_products, **kw)
    if not keep:
        pr.close()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if keep:
        u = pr.eval(out.coef, d.x_eval).cpu().numpy()
        return t2 - t0, t1 - t0, out, u, pr
    return t2 - t0, t1 - t0, out, None, None


def evaluate(mq, torch, p, d, coef):
    """u at the evaluation points from coefficients on the device (matrix-free FP64, eq. (18))."""
    with mq.Problem(d.x_int, d.x_bnd, p.kappa, p.eps, "matfree_fp64",
                    stream=torch.cuda.current_stream(d.x_int.device)) as pr:
        return pr.eval(coef, d.x_eval).cpu().numpy()


def run_timed(mq, torch, p, d, mode, kw, steps, warmup, tag):
    """warmup untimed steps, then `steps` timed ones bracketed by synchronisations; returns the
    figures of the last step and the per-product kernel times of all timed steps."""
    import numpy as np

    ell = p.ell
    for w in range(warmup):
        dt, _, _, _, _ = solve_step(mq, torch, p, d, mode, ell, kw)
        log(tag, "warmup", w, f"{dt:.3f} s")
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    times, creates, outs = [], [], []
    for k in range(steps):
        dt, dc, out, _, _ = solve_step(mq, torch, p, d, mode, ell, kw, time_products=True)
        times.append(dt)
        creates.append(dc)
        outs.append(out)
        log(tag, "step", k, f"{dt:.3f} s (create {dc * 1e3:.1f} ms)", "ell_done", out.ell_done,
            "lambda", f"{out.lam:.4e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_all
    out = outs[-1]
    u = evaluate(mq, torch, p, d, out.coef)
    ld = max(1, out.ell_done)
    return dict(mode=mode, row_scale=kw.get("row_scale", 0), steps=steps, wall_s=wall, step_s=times,
                time_to_solution_s=float(np.mean(times)), create_s=float(np.mean(creates)),
                ell_done=out.ell_done, lam=out.lam, k=out.k, flags=out.flags,
                rel_l2=rel_l2(u, p.u_eval), rel_linf=rel_linf(u, p.u_eval),
                sv=None if out.sv is None else np.asarray(out.sv.cpu().numpy() if hasattr(out.sv, "cpu") else out.sv),
                u=u,
                kernel_ms_AT=float(np.mean([o.t_ms[6] for o in outs])) / ld,
                kernel_ms_A=float(np.mean([o.t_ms[7] for o in outs])) / ld,
                phase_ms=dict(upload=out.t_ms[0], gkb=out.t_ms[1], proj_svd=out.t_ms[2], param=out.t_ms[3],
                              lift=out.t_ms[4], solve_total=out.t_ms[5]))


def host_input_time(mq, torch, p, mode, kw):
    """Time to solution with every input in host memory (nodes, f, g) and the coefficients
    returned to host memory: the figure that includes the PCIe transfers."""
    torch.cuda.synchronize()
    t = time.perf_counter()
    with mq.Problem(p.x_int, p.x_bnd, p.kappa, p.eps, mode) as pr:
        out = pr.solve(p.f_int, p.g_bnd, p.ell, **kw)
    return time.perf_counter() - t, out


def ell_scan(mq, torch, p, d, mode, ells, row_scale=0):
    """Error against the manufactured u of the HKT-GCV solution at every ell in `ells`, from one
    Golub-Kahan run to max(ells) (the first l steps of a run are those of an l-step run), the
    projected SVD, GCV, projected solution and lift of each prefix through the C ABI."""
    lmax = max(ells)
    res = []
    with mq.Problem(d.x_int, d.x_bnd, p.kappa, p.eps, mode,
                    stream=torch.cuda.current_stream(d.x_int.device)) as pr:
        f = d.rhs
        r = pr.gkb(f, lmax, row_scale=row_scale)
        if r["ell_done"] < lmax:
            ells = [l for l in ells if l <= r["ell_done"]]
        al, be, Z = r["alpha"], r["beta"], r["Z"]
        for l in ells:
            sv, ft, V = mq.mqh_proj_svd(al[:l].contiguous(), be[: l + 1].contiguous())
            ch = mq.mqh_param_choice(sv, ft, mq.MQH_METHOD_HKT, mq.MQH_RULE_GCV)
            y = mq.mqh_proj_solution(sv, ft, V, mq.MQH_METHOD_HKT, ch["lambda_"])
            coef = mq.mqh_lift(Z[:l].contiguous(), y)
            u = pr.eval(coef, d.x_eval).cpu().numpy()
            res.append((l, rel_l2(u, p.u_eval), ch["lambda_"]))
    return res


def equal_error(mq, torch, p, d, ref, ells, tag):
    """The equal-error rule: E_ref is the FP64 (stored) HKT-GCV error at the workload's ell; the
    FP32-evaluated HKT is timed at the smallest ell whose error is at most
    max(1.05 E_ref, E_ref + 1e-12).  Times are times to solution from inputs in HBM
    (create + solve + release)."""
    e_ref = ref["rel_l2"]
    bound = max(1.05 * e_ref, e_ref + 1e-12)
    scan = ell_scan(mq, torch, p, d, "matfree_fp32", ells)
    hit = [s for s in scan if s[1] <= bound]
    res = dict(workload=p.name, reference=dict(operator=ref["mode"], ell=p.ell, rel_l2=e_ref,
                                              time_to_solution_s=ref["time_to_solution_s"]),
               bound=bound, scan=[dict(ell=l, rel_l2=e, lam=lam) for (l, e, lam) in scan])
    if not hit:
        best = min(scan, key=lambda s: s[1])
        res.update(reached=False, best_ell=best[0], best_rel_l2=best[1])
        log(tag, "equal error not reached; best", best)
        return res
    l_star = hit[0][0]
    solve_step(mq, torch, p, d, "matfree_fp32", l_star, dict(method=mq.MQH_METHOD_HKT))  # warm
    dt, dc, out, u, pr = solve_step(mq, torch, p, d, "matfree_fp32", l_star, dict(method=mq.MQH_METHOD_HKT),
                                    keep=True)
    pr.close()
    e = rel_l2(u, p.u_eval)
    res.update(reached=True, fp32_ell=l_star, fp32_rel_l2=e, fp32_time_to_solution_s=dt,
               speedup=ref["time_to_solution_s"] / dt,
               note=("E_ref is about 1: GCV puts lambda at the top of its grid and u is about 0 at this "
                     "workload, so the comparison at equal error is only about speed") if e_ref > 0.9 else "")
    log(tag, json.dumps({k: v for k, v in res.items() if k != "scan"}))
    return res


def c2_context(mq, torch, dev, steps):
    """The 20 000-node cube (stored FP64 A, ell = 200, HKT-GCV), where the method resolves the
    manufactured solution: FP64 time to solution, and the FP32-evaluated HKT at equal error."""
    from paper_2511_09798_amd import inputs as I

    p = I.cube_medium()
    d = DeviceInputs(torch, p, dev)
    ref = run_timed(mq, torch, p, d, "stored_fp64", dict(method=mq.MQH_METHOD_HKT), steps, 1, "c2 fp64")
    ee = equal_error(mq, torch, p, d, ref, list(range(20, p.ell + 1, 10)), "c2 equal error")
    fp32 = run_timed(mq, torch, p, d, "matfree_fp32", dict(method=mq.MQH_METHOD_HKT), steps, 1, "c2 fp32")
    return dict(workload=p.name, n=p.n, ell=p.ell, kappa=p.kappa, eps=p.eps,
                fp64_stored=dict(time_to_solution_s=ref["time_to_solution_s"], rel_l2=ref["rel_l2"],
                                 lam=ref["lam"], product_ms_AT=ref["kernel_ms_AT"], product_ms_A=ref["kernel_ms_A"],
                                 stored_GB=stored_bytes(p.n, p.n_int) / 1e9),
                fp32_matfree_same_ell=dict(time_to_solution_s=fp32["time_to_solution_s"], rel_l2=fp32["rel_l2"],
                                           lam=fp32["lam"],
                                           u_vs_fp64=rel_l2(fp32["u"], ref["u"])),
                equal_error=ee)


def row_scale_context(mq, torch, dev, p_big, d_big):
    """The row scaling D = diag(A)^-1 (opt-in; not in the paper) against the paper's system:
    HKT-GCV errors on the 1 800-node cube at ell = 60 and 300, and on the benchmark workload
    (stored FP64 and FP32-evaluated)."""
    from paper_2511_09798_amd import inputs as I

    res = dict(cube_n1800={})
    p = I.cube_small()
    d = DeviceInputs(torch, p, dev)
    for ell in (60, 300):
        for rs in (0, 1):
            _, _, out, u, pr = solve_step(mq, torch, p, d, "stored_fp64", ell,
                                          dict(method=mq.MQH_METHOD_HKT, row_scale=rs), keep=True)
            pr.close()
            res["cube_n1800"][f"ell{ell}_rs{rs}"] = dict(rel_l2=rel_l2(u, p.u_eval), lam=out.lam,
                                                          gcv_at_edge=bool(out.flags & mq.MQH_INFO_GCV_AT_EDGE))
    res[p_big.name] = {}
    for mode in ("stored_fp64", "matfree_fp32"):
        dt, _, out, u, pr = solve_step(mq, torch, p_big, d_big, mode, p_big.ell,
                                       dict(method=mq.MQH_METHOD_HKT, row_scale=1), keep=True)
        pr.close()
        res[p_big.name][mode + "_rs1"] = dict(rel_l2=rel_l2(u, p_big.u_eval), lam=out.lam, time_to_solution_s=dt,
                                              gcv_at_edge=bool(out.flags & mq.MQH_INFO_GCV_AT_EDGE))
    log("row scale", json.dumps(res))
    return res


def learned_context(mq, torch, dev, count: int, n: int = 60000, ell: int = 60, seed: int = 5):
    """Pump-casing-like solid, n nodes (80% interior), kappa in [5, 35], eps in [2, 8]: the plain
    method (ell steps, GCV) against the learned solve (predicted steps and lambda, GCV as judge),
    on A and, with the predictor trained on row-scaled runs, on the row-scaled problem (D A, D f);
    beside each, the smallest error over a 13-point lambda grid at ell (what any choice of lambda
    on that Krylov space reaches)."""
    import os

    import numpy as np

    from paper_2511_09798_amd import learned as L

    models = {0: L.load_predictor()}
    if os.path.exists(L.MODEL_PATH_RS):
        models[1] = L.load_predictor(L.MODEL_PATH_RS)
    rng = np.random.default_rng(seed)
    rows = []
    for k in range(count):
        prob = L.sample_problem(rng, kind="casing", n=n, kappa=float(rng.uniform(5, 35)),
                                eps=float(rng.uniform(2, 8)), n_eval=2000)
        row = dict(kappa=prob["kappa"], eps=prob["eps"])
        with mq.Problem(prob["x_int"], prob["x_bnd"], prob["kappa"], prob["eps"], "matfree_fp32") as pr:
            fi = torch.from_numpy(prob["f_int"]).to(dev)
            gb = torch.from_numpy(prob["g_bnd"]).to(dev)
            xe = torch.from_numpy(prob["x_eval"]).to(dev)
            for rs, model in models.items():
                sfx = "" if rs == 0 else "_rs"
                pred, keep = L.make_device_predictor(mq, torch, model, prob["h"], dev)
                pr.solve(fi, gb, ell, row_scale=rs)  # warm
                torch.cuda.synchronize()
                t = time.perf_counter()
                base = pr.solve(fi, gb, ell, row_scale=rs)
                torch.cuda.synchronize()
                t_base = time.perf_counter() - t
                t = time.perf_counter()
                out = pr.solve_learned(fi, gb, ell, pred, row_scale=rs)
                torch.cuda.synchronize()
                t_net = time.perf_counter() - t
                ub = pr.eval(base.coef, xe).cpu().numpy()
                un = pr.eval(out.coef, xe).cpu().numpy()
                sv0 = float(base.sv[0])
                best = min(rel_l2(pr.eval(pr.solve(fi, gb, ell, rule=mq.MQH_RULE_FIXED, lambda_fixed=float(lam),
                                                   row_scale=rs).coef, xe).cpu().numpy(), prob["u_eval"])
                           for lam in np.geomspace(sv0 * 1e-12, sv0, 13))
                row.update({"steps" + sfx: out.ell_pred, "used_net" + sfx: out.used_net_lambda,
                            "t_gcv" + sfx: t_base, "t_learned" + sfx: t_net,
                            "err_gcv" + sfx: rel_l2(ub, prob["u_eval"]), "err_learned" + sfx: rel_l2(un, prob["u_eval"]),
                            "err_best_grid" + sfx: best, "lam_gcv" + sfx: base.lam, "lam_learned" + sfx: out.lam})
        rows.append(row)
        log("learned casing", k, json.dumps(rows[-1]))
    res = dict(workload=f"casing_n{n}", problems=count, ell=ell, steps_gcv=ell)
    for rs in models:
        sfx = "" if rs == 0 else "_rs"
        eg = np.array([r["err_gcv" + sfx] for r in rows])
        en = np.array([r["err_learned" + sfx] for r in rows])
        eb = np.array([r["err_best_grid" + sfx] for r in rows])
        res.update({"mean_steps_learned" + sfx: float(np.mean([r["steps" + sfx] for r in rows])),
                    "mean_time_gcv_s" + sfx: float(np.mean([r["t_gcv" + sfx] for r in rows])),
                    "mean_time_learned_s" + sfx: float(np.mean([r["t_learned" + sfx] for r in rows])),
                    "median_rel_l2_gcv" + sfx: float(np.median(eg)), "median_rel_l2_learned" + sfx: float(np.median(en)),
                    "median_rel_l2_best_grid" + sfx: float(np.median(eb)),
                    "learned_better" + sfx: int(np.sum(en < eg)),
                    "net_lambda_used" + sfx: int(sum(r["used_net" + sfx] for r in rows))})
    res["row_scaled"] = ("the same problems with the row scaling D = diag(A)^-1 and the predictor trained on "
                         "row-scaled runs (fields ending _rs)") if 1 in models else "no row-scaled predictor"
    res["cases"] = rows
    return res


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
               roofline=dict(bound="alu", achieved=flops / (kern_ms * 1e-3) / 1e12, peak=MFMA_F32_PEAK / 1e12,
                             unit="TFLOP/s", frac=flops / (kern_ms * 1e-3) / MFMA_F32_PEAK,
                             kernel="k_mfh_block", flops=flops,
                             note="2 n^2 s flops per block product (the dense n x n by n x s contraction) priced "
                                  "against the FP32 peak (vector and matrix alike); the kernel is VALU-issue bound "
                                  "(the FP32 entries: one rsq and about six FP32 instructions each), the contraction "
                                  "runs as FP16 products of split operands on the matrix cores beside it"))
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
                row[f"block{lb}_projected_path"] = ("jacobi" if np.any(bk.flags & mq.MQH_INFO_BLOCK_JACOBI)
                                                    else "band")
                # the same solve with the projected problem on the Jacobi full SVD, for comparison
                bj, tj = timed(lambda: pr.solve_block(F, lb, jacobi=True))
                row[f"block{lb}_jacobi_s"] = tj
                row[f"block{lb}_jacobi_projected_ms"] = float(bj.t_ms[0][2])
                row[f"block{lb}_lambda_max_rel_vs_jacobi"] = float(np.max(np.abs(bk.lam / bj.lam - 1.0)))
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


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def cpu_baseline(p, target_s: float):
    """The oracle (plain FP64, OpenMP, entry by entry) on a row / column sample of the products, sized
    to about target_s seconds, scaled to the whole HKT solve (2 ell products dominate it)."""
    import numpy as np

    from oracle import oracle as O
    from paper_2511_09798_amd import inputs as I

    O.lib()
    x = I.random_vector(p.n, 1)
    X = p.nodes

    def sample(rows):
        idx = np.linspace(0, p.n - 1, rows).astype(np.int64)
        t = time.perf_counter()
        O.apply_sampled(X, p.n_int, p.kappa, p.eps, x, idx, trans=True)
        O.apply_sampled(X, p.n_int, p.kappa, p.eps, x, idx, trans=False)
        return time.perf_counter() - t

    probe_rows = 2000
    dt = sample(probe_rows)
    rows = int(min(p.n, max(probe_rows, probe_rows * target_s / max(dt, 1e-3))))
    dt = sample(rows)
    entries = 2.0 * rows * p.n
    per_product_s = dt / entries * p.n * p.n
    hkt_s = 2 * p.ell * per_product_s
    sb = stored_bytes(p.n, p.n_int)
    return dict(value=2 * p.ell * sb / hkt_s / 1e9, unit="GB/s", cores=O.num_threads(), kind="oracle",
                sample=f"{rows} rows of A x and {rows} columns of A^T x at the benchmark workload (entry-by-entry "
                       f"FP64, {entries:.2e} entries, {dt:.1f} s), scaled to the 2 ell products of the HKT solve; "
                       "value = 2 ell x stored-matrix bytes / extrapolated solve time (the headline's unit)",
                seconds=dt, hkt_solve_s_extrapolated=hkt_s, cpu_model=cpu_info(),
                omp_num_threads=os.environ.get("OMP_NUM_THREADS", "unset"), nproc=os.cpu_count())


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere_n100000")
    ap.add_argument("--ell", type=int, default=0, help="override the Golub-Kahan steps (0: workload's)")
    ap.add_argument("--variants",
                    default="matfree_fp32,matfree_fp64,matfree_fp32:lsqr:gcv,matfree_fp32:lsqr:lcurve,"
                            "matfree_fp32:hkt:wgcv:0.5",
                    help="context variants beside the stored-FP64 headline: mode[:method[:rule[:weight]]][+rs]")
    ap.add_argument("--context-steps", type=int, default=1, help="timed steps of each context variant")
    ap.add_argument("--equal-error", type=int, default=1, help="the equal-error FP32 comparison (0: skip)")
    ap.add_argument("--c2", type=int, default=1, help="the 20 000-node cube context (0: skip)")
    ap.add_argument("--row-scale", type=int, default=1, help="the row-scaling context (0: skip)")
    ap.add_argument("--host-inputs", type=int, default=1, help="time to solution from host inputs (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample size in seconds (0: skip)")
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
                    help="full-SVD reference on the 20 000-node cube beside HKT: 1 Tikh-Reg (about half a minute), "
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
    n = p.n
    log("workload", p.name, "n", n, "n_int", p.n_int, "ell", p.ell)
    if args.copy_ref_mib > 0:
        nel = args.copy_ref_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy reference", args.copy_ref_mib, "MiB read +", args.copy_ref_mib, "MiB written")
        del src, dst
    peaks = measure_peaks()
    log("measured peaks", json.dumps(peaks))
    d = DeviceInputs(torch, p, dev)

    # headline: the plain FP64 path (stored matrix), K timed steps
    hkw = dict(method=mq.MQH_METHOD_HKT, rule=mq.MQH_RULE_GCV)
    head = run_timed(mq, torch, p, d, "stored_fp64", hkw, args.steps, args.warmup, "headline stored_fp64")
    sb = stored_bytes(n, p.n_int)
    ms = head["time_to_solution_s"] * 1000.0
    value = 2.0 * head["ell_done"] * sb / head["time_to_solution_s"] / 1e9
    k_at, k_a = head["kernel_ms_AT"], head["kernel_ms_A"]
    dom_at = k_at >= k_a
    dom_ms = k_at if dom_at else k_a
    kern = "k_packed_product<1>" if dom_at else "k_packed_product<0>"
    achieved = sb / (dom_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=measured_traffic(kern), kernel=kern, kernel_ms=dom_ms,
                other_kernel=("k_packed_product<0>" if dom_at else "k_packed_product<1>"),
                other_kernel_ms=min(k_at, k_a), other_frac=sb / (min(k_at, k_a) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                bytes_per_launch=sb, bytes_note="the stored tiles (128 x 128 FP64; symmetric blocks once) one "
                                                "product streams; per-launch partial sums (< 1%) not counted",
                measured_read_peak=peaks["hbm_read_GBs"], frac_of_measured_read=achieved / peaks["hbm_read_GBs"])

    # context variants at the same workload: errors against the FP64 result
    ctx = {}
    for v in [v.strip() for v in args.variants.split(",") if v.strip()]:
        mode, kw = parse_variant(mq, v)
        r = run_timed(mq, torch, p, d, mode, kw, args.context_steps, 1, v)
        e = dict(time_to_solution_s=r["time_to_solution_s"], create_s=r["create_s"], rel_l2=r["rel_l2"],
                 rel_linf=r["rel_linf"], lam=r["lam"], k=r["k"], ell_done=r["ell_done"],
                 product_ms_AT=r["kernel_ms_AT"], product_ms_A=r["kernel_ms_A"], phase_ms=r["phase_ms"])
        if r["sv"] is not None and len(r["sv"]) >= 10:
            e["ritz_top10_max_rel_diff_vs_fp64"] = float(np.max(np.abs(r["sv"][:10] - head["sv"][:10]) /
                                                                head["sv"][:10]))
        if kw == hkw or kw == dict(hkw, row_scale=0):
            # the same method and rule as the headline: the precision form's error per result
            e["u_rel_diff_vs_fp64"] = rel_l2(r["u"], head["u"])
            e["lam_rel_diff_vs_fp64"] = abs(r["lam"] - head["lam"]) / head["lam"] if head["lam"] else None
        if mode.startswith("matfree") and ":" not in v:
            oi, ob = OPS_F32 if mode == "matfree_fp32" else OPS_F64
            pk = FP32_PEAK if mode == "matfree_fp32" else FP64_PEAK
            kms = max(r["kernel_ms_AT"], r["kernel_ms_A"])
            ops = p.n_int * n * oi + p.n_bnd * n * ob
            kname = (("k_mfs<true>" if r["kernel_ms_AT"] >= r["kernel_ms_A"] else "k_mfs<false>")
                     if mode == "matfree_fp32" else
                     ("k_mfs64<true>" if r["kernel_ms_AT"] >= r["kernel_ms_A"] else "k_mfs64<false>"))
            e["roofline"] = dict(bound="alu", achieved=ops / (kms * 1e-3) / 1e12, peak=pk / 1e12, unit="TOP/s",
                                 frac=ops / (kms * 1e-3) / pk, ops_per_launch=ops, kernel=kname,
                                 traffic=measured_traffic(kname), kernel_ms=kms,
                                 note=f"{oi} / {ob} operations per interior / boundary entry against the published "
                                      f"{'FP32' if mode == 'matfree_fp32' else 'FP64'} vector peak")
            if mode == "matfree_fp64":
                e["roofline"]["note"] += ("; the kernel evaluates each unordered pair of nodes once (one t and "
                                          "one rsqrt for A_ij and A_ji), about half of these operations")
            if mode == "matfree_fp32":
                e["arithmetic"] = ("entries in FP32 from FP32 node coordinates, each unordered pair of nodes "
                                   "evaluated once for A_ij and A_ji; the Krylov vector entering each product "
                                   "rounded to FP32; row sums in FP32 over chunks of 256 loop nodes and column "
                                   "sums in FP32 over 32 fixed nodes, both accumulated in FP64; "
                                   "reorthogonalisation, alpha/beta, the projected SVD and GCV in FP64")
                e["roofline"]["note"] += ("; the kernel evaluates each unordered pair of nodes once, about half "
                                          "of these operations")
                pii = p.n_int * p.n_int / 2.0
                pib = float(p.n_int) * p.n_bnd
                pbb = p.n_bnd * p.n_bnd / 2.0
                quads = (pii * QUADS_IDEAL_PAIR["ii"] + pib * QUADS_IDEAL_PAIR["ib"] + pbb * QUADS_IDEAL_PAIR["bb"]) / 64.0
                t_ideal = quads / (CUS * SIMDS * CLOCK / 4.0)
                e["roofline"]["issue_model_ms"] = t_ideal * 1e3
                e["roofline"]["issue_model_frac"] = t_ideal / (kms * 1e-3)
                if peaks and peaks.get("fp32_rsq_plus_4fma_Tps"):
                    # the pairs' instruction mix at the rates the probes measure on this GPU (the
                    # transcendental unit's work does not overlap the FMAs, nor the matrix cores the
                    # VALU of the same wave): an interior-interior pair = one rsq + 4 FMA group and 2
                    # FMAs more, interior-boundary 3 more, boundary-boundary one sqrt and 2 FMAs; every
                    # pair 64 bf16 matrix-core flops
                    grp = peaks["fp32_rsq_plus_4fma_Tps"] * 1e12
                    fma = peaks["fp32_fma_TFLOPs"] * 1e12 / 2.0
                    rsq = peaks["fp32_rsq_Tps"] * 1e12
                    t_mix = (pii * (1.0 / grp + 2.0 / fma) + pib * (1.0 / grp + 3.0 / fma)
                             + pbb * (1.0 / rsq + 2.0 / fma)
                             + (pii + pib + pbb) * 64.0 / (peaks["bf16_mfma_TFLOPs"] * 1e12))
                    e["roofline"]["measured_mix_model_ms"] = t_mix * 1e3
                    e["roofline"]["measured_mix_model_frac"] = t_mix / (kms * 1e-3)
                e["product_equiv_GBs"] = 8.0 * n * n / (kms * 1e-3) / 1e9
        ctx[v] = e
        log(v, json.dumps({k: e.get(k) for k in ("time_to_solution_s", "rel_l2", "lam", "u_rel_diff_vs_fp64")}))

    line = dict(metric="HKT time-to-solution & GKB matvec GB/s at N=100k sphere, equal rel-L2 err",
                value=value, unit="GB/s", n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=ms,
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
                config=dict(workload=p.name, n=n, n_int=p.n_int, n_bnd=p.n_bnd, kappa=p.kappa, eps=p.eps,
                            ell=p.ell, method="HKT", rule="GCV", operator="stored_fp64",
                            step="create from nodes in HBM (tile assembly) + solve from f, g in HBM to coefficients "
                                 "in HBM + release",
                            value_def="2 ell x stored-matrix bytes (53.0 GB) / time to solution"),
                hkt_time_to_solution_s=head["time_to_solution_s"], create_s=head["create_s"],
                ell_done=head["ell_done"], lam=head["lam"], rel_l2=head["rel_l2"], rel_linf=head["rel_linf"],
                phase_ms=head["phase_ms"], product_ms=dict(AT=k_at, A=k_a), roofline=roof, peaks_measured=peaks,
                variants=ctx)
    if args.equal_error:
        line["equal_error"] = equal_error(mq, torch, p, d, head, list(range(10, p.ell + 1, 10)), "equal error")
    if args.host_inputs:
        dt, out = host_input_time(mq, torch, p, "stored_fp64", hkw)
        line["time_to_solution_host_inputs_s"] = dt
        log("host inputs", f"{dt:.3f} s")
    if args.row_scale:
        line["row_scale"] = row_scale_context(mq, torch, dev, p, d)
    if args.c2:
        line["c2"] = c2_context(mq, torch, dev, args.context_steps)
    del d
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
    if args.cpu_seconds > 0:
        log("cpu baseline, about", args.cpu_seconds, "s")
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
