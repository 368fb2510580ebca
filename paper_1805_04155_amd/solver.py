"""Load-step driver around the C ABI: repeats ep_newton_step until the
residual test passes (ALG-NEWTON, Section 4), then ep_commit_step.
Orchestration only; every step of the path runs in the library."""
from __future__ import annotations

import time

from . import _ep


class NewtonError(RuntimeError):
    pass


def solve_load_step(ctx, f, u, max_newton=50):
    """Newton iterations on u (device tensor, updated in place) for the load
    vector f (device tensor).  Returns the list of per-iteration info dicts;
    the last one has converged = 1."""
    hist = []
    for _ in range(max_newton + 1):
        st, info = _ep.ep_newton_step(ctx.h, f, u)
        info["status"] = st
        hist.append(info)
        if info["converged"]:
            return hist
        if st == _ep.EP_ENOTCONV:
            raise NewtonError(f"PCG did not converge: {info}")
    raise NewtonError(f"Newton did not converge in {max_newton} iterations: "
                      f"{[h['res_rel'] for h in hist[-4:]]}")


def solve_load_path(ctx, wl, u, steps=None, max_newton=50, callback=None, sync=None):
    """Solves the load steps of workload wl in order (u holds the initial
    displacement and is updated in place), committing the state after each.
    Returns per-step records (Newton iterations, PCG iterations, plastic
    points, wall time)."""
    import torch
    steps = range(len(wl.load_factors)) if steps is None else steps
    f_unit = ctx.tensor(wl.f_unit)
    records = []
    for k in steps:
        f = f_unit * float(wl.load_factors[k])
        t0 = time.perf_counter()
        hist = solve_load_step(ctx, f, u, max_newton)
        ctx.commit_step(u)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rec = {"step": k, "load": float(wl.load_factors[k]), "newton_its": len(hist) - 1,
               "pcg_its": sum(h["pcg_its"] for h in hist), "res_rel": hist[-1]["res_rel"],
               "n_plastic_ip": hist[-1]["n_plastic_ip"], "seconds": t,
               "res_history": [h["res_rel"] for h in hist],
               "energy_incr": [h["energy_incr"] for h in hist[:-1]]}
        records.append(rec)
        if callback is not None:
            callback(k, rec)
    return records


def displacement_path(ctx, wl, u, ud_max, du0=1e-3, du_max=None, dp_rel=0.01, max_steps=100,
                      max_newton=50, callback=None):
    """Displacement-controlled load path of the strip-footing example
    (Section 8.3): the prescribed displacement u_D * wl.u_dir_unit grows
    from 0 to ud_max with no forces applied.  The increment starts at du0
    and is doubled (up to du_max) when the footing pressure grew by less than
    dp_rel times itself over the last step; a step whose Newton iteration
    fails is retried from the last converged state with a quarter of the
    increment (at most three times), after which the path stops.  The
    footing has unit length, so its average pressure is the reaction
    F(u) . u_dir_unit.  Returns per-step records."""
    import torch
    dirn = ctx.tensor(wl.u_dir_unit)
    mask = dirn != 0
    f0 = torch.zeros_like(dirn)
    ud, du, p_prev = 0.0, du0, 0.0
    records = []
    for k in range(max_steps):
        if ud >= ud_max - 1e-15:
            break
        hist = None
        for _ in range(4):
            ud_new = min(ud + du, ud_max)
            u_save = u.clone()
            u[mask] = dirn[mask] * ud_new
            t0 = time.perf_counter()
            try:
                hist = solve_load_step(ctx, f0, u, max_newton)
                break
            except NewtonError:
                u.copy_(u_save)
                du *= 0.25
        if hist is None:
            break
        F = ctx.internal_force()
        p = float((F * dirn).sum().item())
        ctx.commit_step(u)
        torch.cuda.synchronize()
        rec = {"step": k, "u_D": ud_new, "pressure": p, "newton_its": len(hist) - 1,
               "pcg_its": sum(h["pcg_its"] for h in hist), "res_rel": hist[-1]["res_rel"],
               "n_plastic_ip": hist[-1]["n_plastic_ip"],
               "ls_evals": sum(h["ls_evals"] for h in hist),
               "steps": [h["step"] for h in hist[:-1]],
               "seconds": time.perf_counter() - t0}
        records.append(rec)
        if callback is not None:
            callback(k, rec)
        if p - p_prev < dp_rel * p:
            du = 2.0 * du if du_max is None else min(2.0 * du, du_max)
        p_prev, ud = p, ud_new
    return records
