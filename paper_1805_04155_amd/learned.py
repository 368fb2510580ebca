"""Learned warm start around the C ABI: pool of converged point states from
a training load path, training samples from the exact return map
(ep_mlp_datagen), training with the library's Adam kernels, and load paths
whose Newton iterations start from ep_warm_start.  Orchestration only: every
step of the method runs in the library's kernels; torch supplies device
buffers and seeded random numbers (sample indices and strain increments are
inputs of the sample generator)."""
from __future__ import annotations

import math
import time

import numpy as np

from . import _ep, solver


def _embed6(a, dim):
    """[n_comp][n] per-point arrays -> 3D Voigt [6][n] (plane strain: strain
    11, 22, 12 or state 11, 22, 33, 12 embedded, other components 0)."""
    import torch
    if dim == 3:
        return a
    out = torch.zeros((6, a.shape[1]), dtype=a.dtype, device=a.device)
    if a.shape[0] == 3:
        out[0], out[1], out[3] = a[0], a[1], a[2]
    else:
        out[:4] = a
    return out


class Pool:
    """Converged point states (strain, plastic strain, back stress, kappa)
    of every step of a load path, [6][n_total] on the device."""

    def __init__(self):
        self.parts = []

    def add(self, ctx, u):
        import torch
        s = ctx.sizes
        eps = ctx.strain(u)
        ep, beta, kappa = ctx.get_state()
        self.parts.append((_embed6(eps, s["dim"]), _embed6(ep, s["dim"]),
                           _embed6(beta, s["dim"]), kappa.clone()))
        torch.cuda.synchronize()

    def arrays(self):
        import torch
        cat = [torch.cat([p[i] for p in self.parts], dim=-1).contiguous() for i in range(4)]
        return cat

    @property
    def size(self):
        return sum(p[3].shape[0] for p in self.parts)


def training_path(ctx, wl, u, pool, steps=None):
    """Plain Newton load path that records the committed states."""
    recs = []

    def cb(k, rec):
        pool.add(ctx, u)
        recs.append(rec)

    solver.solve_load_path(ctx, wl, u, steps=steps, callback=cb)
    return recs


def make_samples(material, pool, n, seed, deps_std):
    """n samples (X [n][16], T [n][8] float32): pooled states drawn with
    replacement plus strain increments N(0, s^2) per component, with s =
    deps_std, or, for deps_std = (lo, hi), s log-uniform in [lo, hi] per
    sample (a mixture of step sizes)."""
    import torch
    eps_p, ep_p, beta_p, kap_p = pool.arrays()
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    idx = torch.randint(0, pool.size, (n,), generator=g, device="cuda", dtype=torch.int64)
    deps = torch.randn((6, n), generator=g, device="cuda", dtype=torch.float64)
    if isinstance(deps_std, (tuple, list)):
        lo, hi = math.log(deps_std[0]), math.log(deps_std[1])
        s = torch.exp(lo + (hi - lo) * torch.rand(n, generator=g, device="cuda",
                                                  dtype=torch.float64))
        deps = deps * s
    else:
        deps = deps * deps_std
    X = torch.empty((n, _ep.MLP_XS), dtype=torch.float32, device="cuda")
    T = torch.empty((n, _ep.MLP_YS), dtype=torch.float32, device="cuda")
    _ep.ep_mlp_datagen(material, n, idx, pool.size, eps_p, ep_p,
                       beta_p if material.model == "VM" else None,
                       kap_p if material.model == "DP" else None, deps, X, T)
    torch.cuda.synchronize()
    return X, T


def train(mlp, X, T, epochs=3, batch=8192, lr_max=1e-3, lr_min=1e-5, seed=0, log_every=0):
    """Adam over the batches of (X, T), learning rate cosine from lr_max to
    lr_min over all steps; batch order permuted per epoch.  Returns
    (seconds, list of (step, loss))."""
    import torch
    n = X.shape[0]
    nb = n // batch
    total = epochs * nb
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step = 0
    for _ in range(epochs):
        for b in rng.permutation(nb):
            lr = lr_min + 0.5 * (lr_max - lr_min) * (1.0 + math.cos(math.pi * step / max(1, total)))
            sl = slice(int(b) * batch, (int(b) + 1) * batch)
            mlp.adam_step(X[sl], T[sl], lr, loss)
            step += 1
            if log_every and (step % log_every == 0 or step == total):
                hist.append((step, float(loss.item())))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, hist


def evaluate(mlp, X, T):
    """Held-out metrics: flag accuracy, precision, recall; stress RMSE
    (scaled units)."""
    import torch
    Y = mlp.forward(X)
    pred = Y[:, 6] > 0
    true = T[:, 6] > 0.5
    tp = (pred & true).sum().item()
    out = {"accuracy": (pred == true).float().mean().item(),
           "precision": tp / max(1, pred.sum().item()),
           "recall": tp / max(1, true.sum().item()),
           "stress_rmse": torch.sqrt(((Y[:, :6] - T[:, :6]) ** 2).mean()).item()}
    return out


def solve_path_warm(ctx, wl, u, mlp=None, steps=None, max_newton=50, pcg_rtol=1e-2,
                    extrapolate=True, callback=None, plastic_set=False):
    """Load path where each step's Newton iterations start from
    ep_warm_start (mlp given; u_pred is the secant extrapolation of the last
    two converged steps when extrapolate is on), from that extrapolation
    alone (mlp None, extrapolate on: ep_predictor) or from u_{k-1} (mlp None,
    extrapolate off: the paper's start).  The warm-start solve counts as one
    Newton iteration in the records.  plastic_set: each record also holds
    the plastic set the step starts from against the step's converged set,
    as (both, start, converged) point counts: the network's set at u_pred
    (logit > 0) with mlp, else the exact return map's set at the start
    displacement; that bookkeeping is excluded from the step's seconds."""
    import torch
    steps = range(len(wl.load_factors)) if steps is None else steps
    f_unit = ctx.tensor(wl.f_unit)
    lam = [0.0] + [float(x) for x in wl.load_factors]
    u_prev2 = None
    records = []
    for k in steps:
        f = f_unit * lam[k + 1]
        extrap = 0.0
        if u_prev2 is not None and extrapolate:
            d = lam[k] - lam[k - 1] if k >= 1 else 0.0
            extrap = (lam[k + 1] - lam[k]) / d if d != 0.0 else 0.0
        pred = None
        if plastic_set:
            u_pred = torch.empty_like(u)
            _ep.ep_predictor(ctx.h, u, u_prev2 if extrap else None, extrap, u_pred)
            if mlp is not None:
                pred = mlp.forward(ctx.mlp_features(u_pred))[:, 6] > 0
            else:
                pred = ctx.constitutive(u_pred, sig=False, D=False, flag=True)[2] != 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        warm = None
        u_old = u.clone()
        if mlp is not None:
            st, warm = _ep.ep_warm_start(ctx.h, mlp.h, f, u, u_prev2 if extrap else None, extrap,
                                         pcg_rtol, u)
        elif extrap != 0.0:
            _ep.ep_predictor(ctx.h, u, u_prev2, extrap, u)
        hist = solver.solve_load_step(ctx, f, u, max_newton)
        t_set, counts = 0.0, None
        if pred is not None:
            torch.cuda.synchronize()
            ts = time.perf_counter()
            true = ctx.constitutive(u, sig=False, D=False, flag=True)[2] != 0
            counts = ((pred & true).sum().item(), pred.sum().item(), true.sum().item())
            t_set = time.perf_counter() - ts
        ctx.commit_step(u)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0 - t_set
        u_prev2 = u_old
        rec = {"step": k, "load": lam[k + 1], "newton_its": len(hist) - 1 + (warm is not None),
               "pcg_its": sum(h["pcg_its"] for h in hist) + (warm["pcg_its"] if warm else 0),
               "res_rel": hist[-1]["res_rel"], "n_plastic_ip": hist[-1]["n_plastic_ip"],
               "seconds": t, "warm": warm, "res_history": [h["res_rel"] for h in hist],
               "plastic_set": counts}
        records.append(rec)
        if callback is not None:
            callback(k, rec)
    return records
