"""Learned predictor of the Golub-Kahan stopping index and the HKT parameter.

A small network (24-128-128-128-2, tanh; FP32; kernels in csrc/mlp_kernels.hip)
reads the first Golub-Kahan scalars of a problem (alpha_1..alpha_10,
beta_2..beta_11) together with (kappa, eps, n, h) and predicts
    t0 = log(lambda* / alpha_1)      t1 = ell_stop / ell_max
so that mqh_solve_learned can stop the bidiagonalisation early; GCV on the
projected problem (eq. (30)) stays the judge of the predicted lambda and the
fallback.

Everything here runs through the library (libmqhelm.so):
* training data are solves the method itself generates: for each sampled
  problem the Golub-Kahan run to ell_max, the projected SVD, GCV choice and
  projected solution at ell = 10, 15, ..., ell_max (mqh_proj_svd,
  mqh_param_choice, mqh_proj_solution) and the lifted solutions at a few
  evaluation points (mqh_eval on the basis vectors);
* labels: lambda* = the parameter on a 41-point log grid over GCV's range
  [max(s_l, 16 eps_mach s_1), s_1] whose HKT solution at ell_max has the
  smallest error against the manufactured solution at the evaluation points
  (on these problems GCV mostly over-regularises: the error-optimal lambda
  is what a predictor can add); ell_stop = the smallest ell of that list
  whose HKT solution at lambda* is within 1% (relative L2 at the evaluation
  points) of the ell_max one;
* training: forward, weighted MSE, back-propagation and Adam are the
  library's kernels (mqh_mlp_*), driven from here.

Problem distribution: unit cube (Halton interior from a random start, uniform
face nodes) or unit ball (uniform interior, Fibonacci boundary under a random
rotation), n log-uniform in [1000, 8000] with 80% interior nodes, kappa
log-uniform in [1, 35], eps log-uniform in [0.3, 8] (resolved and
unresolved regimes alike), manufactured plane wave
u = sin(kappa d.x + phase) (direction d uniform on the sphere), so f = 0 and
g = u.  h = (domain volume / n)^(1/3).  The pump-casing-like solid (cylinder
of radius 1 and height 0.6 minus a coaxial hub of radius 0.3, united with a
tangential outlet pipe of radius 0.25 and length 1.2) is sampled by rejection
for the out-of-distribution evaluation.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, Optional

import numpy as np

from . import inputs as I

ELL_MAX = 60
ELL_STEP = 5
N_EVAL = 64
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor.npz")
# the same network trained on row-scaled runs (D A c = D f, D = diag(A)^-1): its features are those
# of the scaled process, so it serves the learned solve with row_scale = 1 only
MODEL_PATH_RS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor_rs.npz")


# --------------------------------------------------------------------------
# Domains
# --------------------------------------------------------------------------

def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


class Casing:
    """Cylinder (axis z, radius 1, height 0.6, centred at 0) minus a coaxial hub of radius 0.3,
    united with an outlet pipe of radius 0.25 along +x, tangent to the casing wall (axis at
    y = 0.75, z = 0), from x = 0 to x = 1.2."""

    R, HH, R_HUB, R_PIPE, Y_PIPE, L_PIPE = 1.0, 0.3, 0.3, 0.25, 0.75, 1.2
    LO = np.array([-1.0, -1.0, -0.3])
    HI = np.array([1.2, 1.0, 0.3])

    @classmethod
    def _in_ring(cls, p, tol=0.0):
        r = np.hypot(p[:, 0], p[:, 1])
        return (r < cls.R - tol) & (r > cls.R_HUB + tol) & (np.abs(p[:, 2]) < cls.HH - tol)

    @classmethod
    def _in_pipe(cls, p, tol=0.0):
        d = np.hypot(p[:, 1] - cls.Y_PIPE, p[:, 2])
        return (d < cls.R_PIPE - tol) & (p[:, 0] > tol) & (p[:, 0] < cls.L_PIPE - tol)

    @classmethod
    def inside(cls, p):
        return cls._in_ring(p) | cls._in_pipe(p)

    @classmethod
    def interior(cls, n: int, rng: np.random.Generator) -> np.ndarray:
        out = np.empty((0, 3))
        while out.shape[0] < n:
            c = cls.LO + (cls.HI - cls.LO) * rng.random((4 * (n - out.shape[0]) + 64, 3))
            out = np.concatenate([out, c[cls.inside(c)]])
        return out[:n]

    @classmethod
    def volume(cls, rng: np.random.Generator, samples: int = 2_000_000) -> float:
        c = cls.LO + (cls.HI - cls.LO) * rng.random((samples, 3))
        return float(np.prod(cls.HI - cls.LO) * np.mean(cls.inside(c)))

    @classmethod
    def boundary(cls, n: int, rng: np.random.Generator) -> np.ndarray:
        """Uniform points on the surface of the solid: points of each part's surface, kept where
        they are not inside the other part (area-weighted proposal over the parts)."""
        tol = 1e-9
        parts = [  # (area, sampler)
            (2 * math.pi * cls.R * 2 * cls.HH, "outer"), (2 * math.pi * cls.R_HUB * 2 * cls.HH, "hub"),
            (2 * math.pi * (cls.R ** 2 - cls.R_HUB ** 2), "caps"), (2 * math.pi * cls.R_PIPE * cls.L_PIPE, "pipe"),
            (math.pi * cls.R_PIPE ** 2, "end")]
        area = np.array([a for a, _ in parts])
        out = np.empty((0, 3))
        while out.shape[0] < n:
            m = 4 * (n - out.shape[0]) + 64
            which = rng.choice(len(parts), size=m, p=area / area.sum())
            pts = np.empty((m, 3))
            u, v = rng.random(m), rng.random(m)
            th = 2 * math.pi * u
            for k, (_, name) in enumerate(parts):
                s = which == k
                if name == "outer":
                    pts[s] = np.stack([cls.R * np.cos(th[s]), cls.R * np.sin(th[s]), cls.HH * (2 * v[s] - 1)], 1)
                elif name == "hub":
                    pts[s] = np.stack([cls.R_HUB * np.cos(th[s]), cls.R_HUB * np.sin(th[s]),
                                       cls.HH * (2 * v[s] - 1)], 1)
                elif name == "caps":
                    r = np.sqrt(cls.R_HUB ** 2 + (cls.R ** 2 - cls.R_HUB ** 2) * v[s])
                    z = np.where(rng.random(s.sum()) < 0.5, -cls.HH, cls.HH)
                    pts[s] = np.stack([r * np.cos(th[s]), r * np.sin(th[s]), z], 1)
                elif name == "pipe":
                    pts[s] = np.stack([cls.L_PIPE * v[s], cls.Y_PIPE + cls.R_PIPE * np.cos(th[s]),
                                       cls.R_PIPE * np.sin(th[s])], 1)
                else:
                    r = cls.R_PIPE * np.sqrt(v[s])
                    pts[s] = np.stack([np.full(s.sum(), cls.L_PIPE), cls.Y_PIPE + r * np.cos(th[s]),
                                       r * np.sin(th[s])], 1)
            on_ring = (which <= 2)
            keep = np.where(on_ring, ~cls._in_pipe(pts, tol), ~cls._in_ring(pts, tol))
            out = np.concatenate([out, pts[keep]])
        return out[:n]


def plane_wave(kappa: float, d: np.ndarray, phase: float):
    return lambda x: np.sin(kappa * (x @ d) + phase)


def sample_problem(rng: np.random.Generator, kind: Optional[str] = None, n: Optional[int] = None,
                   kappa: Optional[float] = None, eps: Optional[float] = None, n_eval: int = N_EVAL) -> Dict:
    """One problem of the training distribution (or with the given overrides)."""
    kind = kind or ("cube" if rng.random() < 0.5 else "sphere")
    n = int(n if n is not None else round(math.exp(rng.uniform(math.log(1000), math.log(8000)))))
    kappa = float(kappa if kappa is not None else math.exp(rng.uniform(math.log(1.0), math.log(35.0))))
    eps = float(eps if eps is not None else math.exp(rng.uniform(math.log(0.3), math.log(8.0))))
    n_int = int(round(0.8 * n))
    n_bnd = n - n_int
    if kind == "cube":
        x_int = I.halton_cube(n_int, start=int(rng.integers(1, 1_000_000)))
        x_bnd = I.cube_faces_uniform(I.split_counts(n_bnd, 6), int(rng.integers(1 << 31)))
        x_eval = I.cube_interior_uniform(n_eval, int(rng.integers(1 << 31)))
        vol = 1.0
    elif kind == "sphere":
        x_int = I.ball_interior_uniform(n_int, int(rng.integers(1 << 31)))
        x_bnd = I.sphere_fibonacci(n_bnd) @ _random_rotation(rng).T
        x_eval = I.ball_interior_uniform(n_eval, int(rng.integers(1 << 31)))
        vol = 4.0 * math.pi / 3.0
    elif kind == "casing":
        x_int = Casing.interior(n_int, rng)
        x_bnd = Casing.boundary(n_bnd, rng)
        x_eval = Casing.interior(n_eval, rng)
        vol = CASING_VOLUME
    else:
        raise ValueError(kind)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    u = plane_wave(kappa, d, float(rng.uniform(0, 2 * math.pi)))
    return dict(kind=kind, x_int=np.ascontiguousarray(x_int), x_bnd=np.ascontiguousarray(x_bnd), kappa=kappa,
                eps=eps, n=n, h=(vol / n) ** (1.0 / 3.0), f_int=np.zeros(n_int), g_bnd=u(x_bnd),
                x_eval=np.ascontiguousarray(x_eval), u_eval=u(x_eval))


CASING_VOLUME = Casing.volume(np.random.default_rng(0), 400_000)


# --------------------------------------------------------------------------
# Labels from the method's own solves
# --------------------------------------------------------------------------

def raw_features(alpha: np.ndarray, beta: np.ndarray, kappa: float, eps: float, n: int, h: float) -> np.ndarray:
    p = 10
    return np.concatenate([np.log(alpha[:p]), np.log(beta[1:p + 1]),
                           [math.log(kappa), math.log(eps), math.log(n), math.log(h)]])


def lambda_grid(sv: np.ndarray, n: int = 41) -> np.ndarray:
    """Log grid over GCV's search range [max(s_l, 16 eps_mach s_1), s_1]."""
    hi = float(sv[0])
    lo = max(float(sv[-1]), 16.0 * np.finfo(np.float64).eps * hi)
    if not lo < hi:
        lo = 16.0 * np.finfo(np.float64).eps * hi
    return np.exp(np.linspace(math.log(lo), math.log(hi), n))


def method_labels(mq, torch, prob: Dict, dev, ell_max: int = ELL_MAX, step: int = ELL_STEP,
                  mode: str = "matfree_fp32", row_scale: int = 0) -> Optional[Dict]:
    """Golub-Kahan run to ell_max, HKT solutions over a lambda grid at ell_max and at
    lambda* for ell = 10, 15, ..., ell_max (all projected steps by the library).  row_scale 1:
    the run on D A and D f (the coefficients, hence u, are those of the same unknowns)."""
    with mq.Problem(prob["x_int"], prob["x_bnd"], prob["kappa"], prob["eps"], mode) as pr:
        f = torch.from_numpy(np.concatenate([prob["f_int"], prob["g_bnd"]])).to(dev)
        r = pr.gkb(f, ell_max, row_scale=row_scale)
        le = int(r["ell_done"])
        if le < ell_max:
            return None  # broke down: not a training sample
        xe = torch.from_numpy(prob["x_eval"]).to(dev)
        BZ = np.stack([pr.eval(r["Z"][k], xe).cpu().numpy() for k in range(le)], axis=1)
    alpha = r["alpha"].cpu().numpy()
    beta = r["beta"].cpu().numpy()
    ue = prob["u_eval"]
    nue = float(np.linalg.norm(ue))

    def err(u):
        return float(np.linalg.norm(u - ue) / nue)

    sv, ft, V = mq.mqh_proj_svd(alpha.copy(), beta.copy())
    pc = mq.mqh_param_choice(sv, ft, mq.MQH_METHOD_HKT, mq.MQH_RULE_GCV)
    lam_gcv = pc["lambda_"]
    e_gcv = err(BZ @ mq.mqh_proj_solution(sv, ft, V, mq.MQH_METHOD_HKT, lam=lam_gcv))
    grid = lambda_grid(sv)
    errs = [err(BZ @ mq.mqh_proj_solution(sv, ft, V, mq.MQH_METHOD_HKT, lam=float(lam))) for lam in grid]
    j = int(np.argmin(errs))
    lam_opt, e_opt = float(grid[j]), float(errs[j])
    cands = list(range(10, le + 1, step))
    if cands[-1] != le:
        cands.append(le)
    us = {}
    for l in cands:
        s_l, f_l, V_l = mq.mqh_proj_svd(alpha[:l].copy(), beta[: l + 1].copy())
        us[l] = BZ[:, :l] @ mq.mqh_proj_solution(s_l, f_l, V_l, mq.MQH_METHOD_HKT, lam=lam_opt)
    ref = us[le]
    nref = max(float(np.linalg.norm(ref)), 1e-300)
    stop = next(l for l in cands if np.linalg.norm(us[l] - ref) <= 0.01 * nref)
    return dict(x=raw_features(alpha, beta, prob["kappa"], prob["eps"], prob["n"], prob["h"]),
                t=np.array([math.log(lam_opt / alpha[0]), stop / ell_max]), stop=stop, lam=lam_opt,
                lam_gcv=lam_gcv, err_gcv=e_gcv, err_opt=e_opt, err_stop=err(us[stop]), kind=prob["kind"],
                n=prob["n"], kappa=prob["kappa"], eps=prob["eps"])


def generate(n_samples: int, seed: int, log_every: int = 500, row_scale: int = 0) -> Dict[str, np.ndarray]:
    import torch

    from . import mqhelm as mq

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    rows = []
    t0 = time.time()
    tries = 0
    while len(rows) < n_samples:
        tries += 1
        lab = method_labels(mq, torch, sample_problem(rng), dev, row_scale=row_scale)
        if lab is not None:
            rows.append(lab)
        if len(rows) % log_every == 0 and lab is not None:
            print(f"[learned] {len(rows)}/{n_samples} samples, {time.time() - t0:.0f} s", flush=True)
    return dict(X=np.stack([r["x"] for r in rows]), T=np.stack([r["t"] for r in rows]),
                stop=np.array([r["stop"] for r in rows]), lam=np.array([r["lam"] for r in rows]),
                lam_gcv=np.array([r["lam_gcv"] for r in rows]), err_gcv=np.array([r["err_gcv"] for r in rows]),
                err_opt=np.array([r["err_opt"] for r in rows]), err_stop=np.array([r["err_stop"] for r in rows]),
                kind=np.array([r["kind"] for r in rows]), n=np.array([r["n"] for r in rows]),
                kappa=np.array([r["kappa"] for r in rows]), eps=np.array([r["eps"] for r in rows]),
                tries=np.array(tries))


# --------------------------------------------------------------------------
# Training with the library's network kernels
# --------------------------------------------------------------------------

SIZES = (24, 128, 128, 128, 2)


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases, flat in the library's layout."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(len(SIZES) - 1):
        fan_in, fan_out = SIZES[l], SIZES[l + 1]
        a = math.sqrt(6.0 / (fan_in + fan_out))
        out.append(rng.uniform(-a, a, size=fan_out * fan_in))
        out.append(np.zeros(fan_out))
    return np.concatenate(out).astype(np.float32)


class Trainer:
    """Buffers and one optimisation step on the GPU (all arithmetic in the library's kernels)."""

    def __init__(self, mq, torch, params: np.ndarray, batch: int, dev, weights=(1.0, 1.0)):
        self.mq, self.torch, self.dev, self.B = mq, torch, dev, batch
        f32 = dict(dtype=torch.float32, device=dev)
        self.p = torch.from_numpy(params).to(dev)
        self.g = torch.zeros_like(self.p)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.w = torch.tensor(weights, **f32)
        self.hidden = torch.empty(3 * batch * 128, **f32)
        self.work = torch.empty(2 * batch * 128, **f32)
        self.y = torch.empty((batch, 2), **f32)
        self.dy = torch.empty((batch, 2), **f32)
        self.loss = torch.empty(1, **f32)
        self.step_no = 0

    def step(self, xb, tb, lr: float):
        mq = self.mq
        mq.mqh_mlp_forward(self.p, xb, self.y, self.hidden)
        mq.mqh_mlp_loss(self.y, tb, self.w, self.loss, self.dy)
        mq.mqh_mlp_backward(self.p, xb, self.hidden, self.dy, self.g, self.work)
        self.step_no += 1
        mq.mqh_mlp_adam(self.p, self.g, self.m, self.v, self.step_no, lr)

    def predict(self, x):
        torch = self.torch
        B = x.shape[0]
        y = torch.empty((B, 2), dtype=torch.float32, device=self.dev)
        hid = torch.empty(3 * B * 128, dtype=torch.float32, device=self.dev)
        self.mq.mqh_mlp_forward(self.p, x, y, hid)
        return y


def train(data: Dict[str, np.ndarray], epochs: int = 400, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          val_frac: float = 0.2, log_every: int = 50, check_every: int = 5) -> Dict:
    """Adam with cosine decay; keeps the parameters of the best validation loss (checked every
    check_every epochs)."""
    import torch

    from . import mqhelm as mq

    dev = torch.device("cuda:0")
    X, T = data["X"].astype(np.float64), data["T"].astype(np.float64)
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    nv = int(round(val_frac * n))
    iv, it = perm[:nv], perm[nv:]
    in_mean, in_std = X[it].mean(0), np.maximum(X[it].std(0), 1e-6)
    out_mean, out_std = T[it].mean(0), np.maximum(T[it].std(0), 1e-6)
    Xs = ((X - in_mean) / in_std).astype(np.float32)
    Ts = ((T - out_mean) / out_std).astype(np.float32)
    xt = torch.from_numpy(Xs[it]).to(dev)
    tt = torch.from_numpy(Ts[it]).to(dev)
    xv = torch.from_numpy(Xs[iv]).to(dev)
    tr = Trainer(mq, torch, init_params(seed), batch, dev)
    nb = xt.shape[0] // batch
    hist = []
    best = (math.inf, 0, tr.p.clone())
    t0 = time.time()
    for ep in range(epochs):
        lr_ep = lr * 0.5 * (1.0 + math.cos(math.pi * ep / epochs))  # cosine decay
        order = torch.from_numpy(rng.permutation(xt.shape[0])).to(dev)
        for b in range(nb):
            idx = order[b * batch:(b + 1) * batch]
            tr.step(xt.index_select(0, idx).contiguous(), tt.index_select(0, idx).contiguous(), lr_ep)
        if (ep + 1) % check_every == 0 or ep == epochs - 1:
            pv = tr.predict(xv).cpu().numpy().astype(np.float64)
            vloss = float(np.mean(np.sum((pv - Ts[iv]) ** 2, axis=1)))
            hist.append((ep + 1, vloss))
            if vloss < best[0]:
                best = (vloss, ep + 1, tr.p.clone())
            if (ep + 1) % log_every == 0 or ep == epochs - 1:
                print(f"[learned] epoch {ep + 1}: validation MSE (standardised) {vloss:.4f}, best {best[0]:.4f} "
                      f"at {best[1]}, {time.time() - t0:.0f} s", flush=True)
    tr.p.copy_(best[2])
    pv = tr.predict(xv).cpu().numpy().astype(np.float64) * out_std + out_mean
    params = tr.p.cpu().numpy()
    return dict(params=params, in_mean=in_mean, in_std=in_std, out_mean=out_mean, out_std=out_std,
                val_idx=iv, val_pred=pv, history=np.array(hist), best_epoch=best[1], best_val=best[0])


def save_predictor(path: str, model: Dict, meta: Dict) -> None:
    np.savez(path, params=model["params"].astype(np.float32), in_mean=model["in_mean"].astype(np.float32),
             in_std=model["in_std"].astype(np.float32), out_mean=model["out_mean"].astype(np.float32),
             out_std=model["out_std"].astype(np.float32), meta=np.array(json.dumps(meta)))


def load_predictor(path: str = MODEL_PATH) -> Dict:
    with np.load(path, allow_pickle=False) as z:
        out = {k: z[k] for k in ("params", "in_mean", "in_std", "out_mean", "out_std")}
        out["meta"] = json.loads(str(z["meta"]))
    return out


def make_device_predictor(mq, torch, model: Dict, h: float, dev, ell_step: int = ELL_STEP,
                          judge_ratio: float = 0.0):
    """(predictor struct, device parameter tensor); keep the tensor alive while the struct is used."""
    p = torch.from_numpy(np.ascontiguousarray(model["params"], dtype=np.float32)).to(dev)
    return mq.make_predictor(p, model["in_mean"], model["in_std"], model["out_mean"], model["out_std"], h,
                             ell_step, judge_ratio), p


# --------------------------------------------------------------------------
# Evaluation: the learned solve against the method without it
# --------------------------------------------------------------------------

def compare(problems, model: Dict, ell: int = ELL_MAX, mode: str = "matfree_fp32", log=None,
            row_scale: int = 0) -> Dict:
    """Per problem: HKT with GCV after ell steps (the method) and the learned solve (predicted
    steps and lambda, GCV as judge and fallback); errors at the problems' evaluation points.
    row_scale 1: both on the row-scaled problem (with a predictor trained on such runs)."""
    import torch

    from . import mqhelm as mq

    dev = torch.device("cuda:0")
    rows = []
    for k, prob in enumerate(problems):
        pred, keep = make_device_predictor(mq, torch, model, prob["h"], dev)
        with mq.Problem(prob["x_int"], prob["x_bnd"], prob["kappa"], prob["eps"], mode) as pr:
            base = pr.solve(prob["f_int"], prob["g_bnd"], ell, row_scale=row_scale)
            ub = pr.eval(base.coef, prob["x_eval"])
            out = pr.solve_learned(prob["f_int"], prob["g_bnd"], ell, pred, row_scale=row_scale)
            un = pr.eval(out.coef, prob["x_eval"])
        nu = float(np.linalg.norm(prob["u_eval"]))
        rows.append(dict(kind=prob["kind"], n=prob["n"], kappa=prob["kappa"], eps=prob["eps"], steps=out.ell_pred,
                         used_net=bool(out.used_net_lambda), err_gcv=float(np.linalg.norm(ub - prob["u_eval"]) / nu),
                         err_learned=float(np.linalg.norm(un - prob["u_eval"]) / nu),
                         t_gcv_ms=base.t_ms[5], t_learned_ms=out.t_ms[5]))
        if log:
            log(k, rows[-1])
    eg = np.array([r["err_gcv"] for r in rows])
    en = np.array([r["err_learned"] for r in rows])
    st = np.array([r["steps"] for r in rows])
    return dict(problems=len(rows), ell=ell, mean_steps_learned=float(st.mean()),
                median_err_gcv=float(np.median(eg)), median_err_learned=float(np.median(en)),
                frac_err_below_0_1=dict(gcv=float(np.mean(eg < 0.1)), learned=float(np.mean(en < 0.1))),
                frac_err_below_0_5=dict(gcv=float(np.mean(eg < 0.5)), learned=float(np.mean(en < 0.5))),
                frac_learned_better=float(np.mean(en < eg)),
                mean_time_gcv_ms=float(np.mean([r["t_gcv_ms"] for r in rows])),
                mean_time_learned_ms=float(np.mean([r["t_learned_ms"] for r in rows])),
                net_lambda_used=int(sum(r["used_net"] for r in rows)), cases=rows)


# --------------------------------------------------------------------------
# Command line: generate / train / evaluate
# --------------------------------------------------------------------------

def main(argv=None):
    ap = argparse.ArgumentParser(description="learned predictor: data generation and training")
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--samples", type=int, default=20000)
    g.add_argument("--seed", type=int, default=1)
    g.add_argument("--out", required=True)
    g.add_argument("--row-scale", type=int, default=0)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True, nargs="+")
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--out", default=MODEL_PATH)
    t.add_argument("--report", default=None)
    t.add_argument("--row-scale", type=int, default=0, help="recorded in the model's meta")
    e = sub.add_parser("evaluate")
    e.add_argument("--problems", type=int, default=200)
    e.add_argument("--seed", type=int, default=909)
    e.add_argument("--kind", default=None, help="cube / sphere / casing (default: the training mix)")
    e.add_argument("--n", type=int, default=None)
    e.add_argument("--out", default=None)
    e.add_argument("--row-scale", type=int, default=0)
    a = ap.parse_args(argv)
    if a.cmd == "evaluate":
        rng = np.random.default_rng(a.seed)
        probs = [sample_problem(rng, kind=a.kind, n=a.n) for _ in range(a.problems)]
        rep = compare(probs, load_predictor(MODEL_PATH_RS if a.row_scale else MODEL_PATH), row_scale=a.row_scale)
        print(json.dumps({k: v for k, v in rep.items() if k != "cases"}), flush=True)
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(rep, fh, indent=1)
        return 0
    if a.cmd == "generate":
        d = generate(a.samples, a.seed, row_scale=a.row_scale)
        np.savez(a.out, **d)
        print(f"[learned] wrote {a.out}: {d['X'].shape[0]} samples ({int(d['tries'])} problems drawn)", flush=True)
        return 0
    parts = [np.load(f, allow_pickle=False) for f in a.data]
    data = {k: np.concatenate([p[k] for p in parts]) for k in ("X", "T", "stop", "lam", "err_gcv", "err_opt")}
    model = train(data, a.epochs, a.batch, a.lr)
    meta = dict(samples=int(data["X"].shape[0]), epochs=a.epochs, batch=a.batch, lr=a.lr, ell_max=ELL_MAX,
                ell_step=ELL_STEP, row_scale=a.row_scale, best_epoch=int(model["best_epoch"]),
                best_val_mse=float(model["best_val"]),
                history=model["history"].tolist())
    save_predictor(a.out, model, meta)
    T = data["T"][model["val_idx"]]
    pv = model["val_pred"]
    rep = dict(val_samples=int(T.shape[0]), mae_log_lambda=float(np.mean(np.abs(pv[:, 0] - T[:, 0]))),
               mae_stop_fraction=float(np.mean(np.abs(pv[:, 1] - T[:, 1]))),
               baseline_mae_log_lambda=float(np.mean(np.abs(T[:, 0] - np.median(T[:, 0])))),
               baseline_mae_stop_fraction=float(np.mean(np.abs(T[:, 1] - np.median(T[:, 1])))), **meta)
    print(json.dumps(rep), flush=True)
    if a.report:
        with open(a.report, "w") as fh:
            json.dump(rep, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
