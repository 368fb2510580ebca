#!/usr/bin/env python3
"""Throughput of the elastoplastic Newton hot path on one MI355X.

A step is one pass of the hot path over the whole workload: strain and return
map at every integration point with the fused constitutive kernel, plastic-
element compaction, the incremental tangent K_elast + B^T (D - D_elast) B
(colour rounds over the plastic work list) and the internal force / residual.
The metric is millions of integration points per second.  Inputs are
resident in HBM when the timed region starts.  A per-kernel breakdown (every
kernel timed with HIP events) runs first; in the timed region only the
dominant kernel's dispatches carry HIP events, which give its mean launch
duration for the roofline.

Workload (default): unit cube, 64^3 Q1 hexahedra (262144 elements, 2097152
integration points, 823875 dofs), von Mises with linear kinematic hardening
(E = 206900, nu = 0.29, sigma_y = 450, H = 10000), half of the elements
seeded plastic, FP64 throughout.

Also measured (unless switched off), as extra objects of the same line:
  q2_slope: the same pass on the plane-strain slope (512 x 256 nine-node
    quadrilaterals, 1179648 points, Drucker-Prager perfect, half seeded),
    with FP64 and with FP32 tangent values;
  p1_square_newton: time to |Q(f - F)| <= 1e-10 |Q f| over the ten load
    steps of the P1 square (2048 triangles, von Mises), FP64;
  newton: time to 1e-10 summed over a load path, for the plain FP64 solver
    and its variants: FP32 tangent values; the secant predictor; the learned
    warm start (network trained on the GPU by the library's kernels from a
    separate training path, FP32 and BF16 products) on the 64^3 Q1 cube under
    the cyclic traction history; and matrix-core local products (FP32, BF16)
    on the Q2 / P2 blocks' 20-step paths;
  local_precision: incremental tangent error of the FP32 / BF16 local
    products against the FP64 path, and the assembly kernel's matrix-core
    rate, on the Q2 / P2 blocks with half of the elements seeded plastic;
  plastic_sweep: the headline pass on the 64^3 cube with 0/25/50/100 % of
    the elements seeded plastic, FP64 and FP32 tangent values, at u = 0 and
    at the first Newton iterate of the load step t = 324;
  lshape_vm, strip_footing: the paper's two examples (Sections 8.2, 8.3).

Prints one JSON line (rank 0, one GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}
# useful flops of the element-local product per plastic point, exploiting the
# three nonzeros per column of B: 2 (3 (d n_p)^2 + 54 n_p)
LOCAL_FLOPS_PER_IP = {"Q2_3D": 2 * (3 * 81 ** 2 + 54 * 27), "P2_3D": 2 * (3 * 30 ** 2 + 54 * 10)}
KERNEL_SRC = os.path.join(ROOT, "paper_1805_04155_amd", "csrc", "ep_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

WORKLOADS = {
    "q2_slope": "workload_q2_slope",
    "q1_cube": "workload_q1_cube",
    "p1_square": "workload_p1_square",
    "q2_block": "workload_q2_block",
    "p2_block": "workload_p2_block",
}


def kernel_bytes(mesh, mat, counts, tangent_bytes):
    """Algorithmic HBM bytes per step of each kernel in this design (every
    array read or written once at the granularity the design moves it).
    counts: plastic elements, plastic integration points, elements listed."""
    D, NP, NQ = mesh.dim, mesh.n_p, mesh.n_q
    n_e, n_int, n_n = mesh.n_elems, mesh.n_int, mesh.n_nodes
    n_dof = D * n_n
    nsc = 6 if D == 3 else 4
    ndesc = 10 if D == 3 else 7
    pe, pi, listed = counts["plastic_elems"], counts["plastic_ips"], counts["listed"]
    state = (2 * nsc if mat.model == "VM" else nsc + 1) * 8
    s = tangent_bytes
    blk = NP * NP
    return {
        # coords + displacement once per node, connectivity, state per point,
        # flag, descriptor of plastic points, element force vectors and
        # their node-order slots, mask
        "constitutive": 2 * 8 * n_dof + 4 * NP * n_e + state * n_int + n_int
        + 8 * ndesc * pi + (8 * D + 4) * NP * n_e + 4 * n_e,
        # per listed element: position map, one-byte stamp read + write, base
        # value read, tangent write, mask; per plastic element its
        # connectivity and coordinates; per plastic point its tangent
        # descriptor
        "assembly": listed * (blk * (4 + 2 + 2 * D * D * s) + 4) + pe * NP * (4 + 8 * D)
        + 8 * ndesc * pi,
        # colour-major order and two masks read, list written
        "compaction": counts["n_perm"] * 4 + 8 * n_e + 4 * listed,
        # node offsets, element force vectors (node order), free mask, F
        "force": 4 * (n_n + 1) + 8 * D * NP * n_e + n_dof * (8 + 1),
    }


def assembly_bytes_scalar_model(mesh, counts, tangent_bytes):
    """Algorithmic bytes of the incremental assembly in the scalar-CSR
    model: per plastic point its B values and weight plus an 8 x 8 B tangent
    (8 (d n_p + 1) + 64 B); per plastic element a scalar position map entry
    and a read-modify-write of each of its (d n_p)^2 values, counted twice
    (restore of the previous values, then the addition)."""
    nl = mesh.dim * mesh.n_p
    s = tangent_bytes
    return counts["plastic_ips"] * (8 * (nl + 1) + 64) + \
        counts["plastic_elems"] * nl * nl * (4 + 2 * s) * 2


def src_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()


def _host_cpu():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, ep, beta, kappa, u, fraction=16):
    """The FP64 oracle timed on the host for passes over a bounded sample of
    the same workload: the first n_e / fraction elements (lexicographic
    order: the bottom layers of the cube) with their seeded state (strain,
    return map, plain sum w B^T D B assembled by COO sort, internal force;
    geometry and sparsity pattern of the sample precomputed), on one thread
    and on all threads the host offers (OMP_NUM_THREADS, else the CPU
    count).  One untimed pass, then the median of three timed ones per
    thread count; the rate in points per second carries over to the whole
    workload."""
    from oracle import oracle as O
    from paper_1805_04155_amd import workloads as W
    mesh, mat = wl.mesh, wl.material
    k = max(1, mesh.n_elems // fraction)
    sub = W.Mesh(mesh.etype, mesh.coord, mesh.elem[:k])
    nq, dim = mesh.n_q, mesh.dim
    dphi, w = O.geometry(sub)
    pat = O.pattern(sub)
    ep6 = O.state_to_ip6(ep[:, :k * nq], dim)
    beta6 = O.state_to_ip6(beta[:, :k * nq], dim)
    kap = kappa[:k * nq]

    def one_pass():
        t0 = time.perf_counter()
        eps = O.strain(sub, dphi, u)
        out = O.constitutive(mat, eps, ep6, beta6, kap)
        O.assemble(sub, dphi, w, out["D"], *pat)
        O.internal_force(sub, dphi, w, out["sig"])
        return time.perf_counter() - t0

    def leg(threads):
        used = O.set_threads(threads)
        one_pass()
        t = sorted(one_pass() for _ in range(3))[1]
        return {"value": round(sub.n_int / t / 1e6, 4), "seconds_per_pass": round(t, 3),
                "cores": used}

    prev = O.set_threads(0)
    try:
        one = leg(1)
        n_all = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        allc = leg(n_all)
    finally:
        O.set_threads(prev)
    log(f"cpu oracle: 1 thread {one}, all threads {allc}")
    return {"value": allc["value"], "unit": "M integration pts/s", "cores": allc["cores"],
            "kind": "oracle", "seconds_per_pass": allc["seconds_per_pass"],
            "one_thread": one, "host_cpu": _host_cpu(), "host_cpu_count": os.cpu_count(),
            "sample": f"the first {k} of {mesh.n_elems} elements ({sub.n_int} of {mesh.n_int} "
                      "points) with their seeded state: strain, return map, COO-sorted K "
                      "assembly, internal force per pass (geometry and sparsity pattern "
                      "precomputed); median of 3 timed passes after 1 untimed, per thread "
                      "count; the oracle's threads cover its per-point and per-element "
                      "loops, the COO sort and the node sums stay serial"}


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _state_args(mat, ep, beta, kappa):
    return (ep, beta if mat.model == "VM" else None, kappa if mat.model == "DP" else None)


def run_path(wl, state, options, mlp=None, extrapolate=False, keep_u=False, steps=None):
    """One load path solved to |Q(f - F)| <= 1e-10 |Q f| per step; wall time
    summed over the steps, each from its first Newton evaluation (or warm
    start) to its commit (setup excluded); and the precision and recall of the
    plastic set each step starts from (the network's, or the exact map's at
    the start displacement) against the converged set (bookkeeping outside
    the step times)."""
    import torch
    from paper_1805_04155_amd import _ep, learned
    opts = {"newton_rtol": 1e-10}
    opts.update(options)
    ctx = _ep.Context(wl.mesh, wl.free, wl.material, options=opts)
    ctx.set_state(*state)
    u = torch.zeros(wl.mesh.n_dof, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    recs = learned.solve_path_warm(ctx, wl, u, mlp, steps=steps, extrapolate=extrapolate,
                                   plastic_set=True)
    torch.cuda.synchronize()
    t = sum(r["seconds"] for r in recs)
    ctx.close()
    out = {"seconds": round(t, 3), "newton_its": sum(r["newton_its"] for r in recs),
           "pcg_its": sum(r["pcg_its"] for r in recs),
           "max_final_res_rel": max(r["res_rel"] for r in recs),
           "final_plastic_points": recs[-1]["n_plastic_ip"]}
    if mlp is not None:
        out["warm_starts_accepted"] = sum(r["warm"]["accepted"] for r in recs)
    both, npred, ntrue = (sum(r["plastic_set"][i] for r in recs) for i in range(3))
    out["start_plastic_set_precision"] = round(both / npred, 4) if npred else None
    out["start_plastic_set_recall"] = round(both / ntrue, 4) if ntrue else None
    return out, (u if keep_u else None)


def _du(u, ref):
    return float(((u - ref).abs().max() / ref.abs().max()).item())


def newton_report(cube_n, n_samples, block):
    """Metric 2: time-to-1e-10 summed over load paths, plain FP64 against
    the mixed-precision and learned variants."""
    import numpy as np
    import torch
    from paper_1805_04155_amd import _ep, learned
    from paper_1805_04155_amd import workloads as W
    rep = {}
    # warm-up of every kernel on a small path (not reported)
    small = W.workload_q1_cube_cyclic(6, 30)
    st = _state_args(small.material, *W.seeded_state(small, 0.5, seed=0)[:3])
    run_path(small, st, {}, steps=range(3))
    # learned warm start on the cyclic cube
    wl = W.workload_q1_cube_cyclic(cube_n, 30)
    mat = wl.material
    sy = math.sqrt(1.5) * mat.Y
    t0 = time.perf_counter()
    ctx = _ep.Context(wl.mesh, wl.free, mat, options={"newton_rtol": 1e-10})
    ctx.set_state(*_state_args(mat, *W.seeded_state(wl, 0.5, seed=1)[:3]))
    pool = learned.Pool()
    u = torch.zeros(wl.mesh.n_dof, dtype=torch.float64, device="cuda")
    learned.training_path(ctx, wl, u, pool)
    ctx.close()
    del u
    t_path = time.perf_counter() - t0
    log(f"training path {t_path:.1f} s")
    t0 = time.perf_counter()
    ds = (0.01 * sy / mat.E, 2.0 * sy / mat.E)
    X, T = learned.make_samples(mat, pool, n_samples, seed=2, deps_std=ds)
    Xh, Th = learned.make_samples(mat, pool, 1_000_000, seed=4, deps_std=ds)
    t_gen = time.perf_counter() - t0
    del pool
    nets, training = {}, {"training_path_s": round(t_path, 3), "samples": n_samples,
                          "datagen_s": round(t_gen, 3), "epochs": 3, "batch": 8192,
                          "sample_increments": "N(0, s^2), s log-uniform in "
                                               "[0.01, 2] sigma_y/E per sample"}
    init = W.mlp_he_uniform(3).astype(np.float32)
    for prec in ("fp32", "bf16"):
        m = _ep.Mlp(_ep.EP_FP32 if prec == "fp32" else _ep.EP_BF16, 8192)
        m.set_params(init)
        sec, hist = learned.train(m, X, T, epochs=3, batch=8192, lr_max=1e-3, lr_min=1e-5,
                                  log_every=2000)
        ev = learned.evaluate(m, Xh, Th)
        training[prec] = {"train_s": round(sec, 3), "final_loss": hist[-1][1] if hist else None,
                          "held_out": {k: round(v, 5) for k, v in ev.items()}}
        log(f"trained {prec}: {training[prec]}")
        nets[prec] = m
    untrained = _ep.Mlp(_ep.EP_FP32, 8192)
    untrained.set_params(init)
    del X, T, Xh, Th
    torch.cuda.empty_cache()
    st0 = _state_args(mat, *W.seeded_state(wl, 0.5, seed=0)[:3])
    variants = {}
    variants["plain_fp64"], u_ref = run_path(wl, st0, {}, keep_u=True)
    log(f"cube plain_fp64: {variants['plain_fp64']}")
    runs = [("fp32_tangent", {"tangent_prec": _ep.EP_FP32}, None, False),
            ("split_operator", {"operator_form": _ep.EP_OPERATOR_SPLIT}, None, False),
            ("secant_predictor", {}, None, True),
            ("learned_fp32", {}, nets["fp32"], True),
            ("learned_bf16", {}, nets["bf16"], True),
            ("learned_untrained", {}, untrained, True)]
    for name, opts, m, ex in runs:
        r, uu = run_path(wl, st0, opts, mlp=m, extrapolate=ex, keep_u=True)
        r["du_rel_vs_plain"] = _du(uu, u_ref)
        variants[name] = r
        log(f"cube {name}: {r}")
        del uu
    for m in list(nets.values()) + [untrained]:
        m.close()
    base = variants["plain_fp64"]["seconds"]
    for v in variants.values():
        v["speedup_vs_plain"] = round(base / v["seconds"], 3)
    rep["q1_cube_cyclic"] = {
        "workload": f"unit cube, {cube_n}^3 Q1 hexahedra ({wl.mesh.n_int} points), von Mises "
                    "kinematic, half of the elements seeded plastic (seed 0; training path "
                    "seed 1), 30 steps of the cyclic traction history x 540",
        "variants": variants, "training": training}
    # matrix-core local products on the blocks
    for name, fn in (("q2_block", W.workload_q2_block), ("p2_block", W.workload_p2_block)):
        wl = fn(*block)
        st0 = _state_args(wl.material, *W.seeded_state(wl, 0.0, seed=0)[:3])
        variants = {}
        variants["plain_fp64"], u_ref = run_path(wl, st0, {}, keep_u=True)
        log(f"{name} plain_fp64: {variants['plain_fp64']}")
        for lp in ("fp32", "bf16"):
            r, uu = run_path(wl, st0, {"local_prec": _ep.EP_FP32 if lp == "fp32" else _ep.EP_BF16},
                             keep_u=True)
            r["du_rel_vs_plain"] = _du(uu, u_ref)
            variants[f"local_{lp}"] = r
            log(f"{name} local_{lp}: {r}")
        r, uu = run_path(wl, st0, {"operator_form": _ep.EP_OPERATOR_SPLIT}, keep_u=True)
        r["du_rel_vs_plain"] = _du(uu, u_ref)
        variants["split_operator"] = r
        log(f"{name} split_operator: {r}")
        base = variants["plain_fp64"]["seconds"]
        for v in variants.values():
            v["speedup_vs_plain"] = round(base / v["seconds"], 3)
        rep[name] = {"workload": f"2x1x1 block, {block[0]}x{block[1]}x{block[2]} "
                                 f"{'27-node hexahedra' if name == 'q2_block' else 'P2 tetrahedra'} "
                                 f"({wl.mesh.n_int} points), Drucker-Prager with linear "
                                 "hardening, strip pressure ramped to 4000 in 20 steps",
                     "variants": variants}
    return rep


def time_pass(ctx, u, F, steps):
    """Mean wall time (ms) of `steps` passes (constitutive + compaction +
    assembly + force) after 2 warm-up passes."""
    import torch
    from paper_1805_04155_amd import _ep

    def step():
        _ep.ep_constitutive(ctx.h, u)
        _ep.ep_assemble_tangent(ctx.h)
        _ep.ep_internal_force(ctx.h, F)
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps


def lshape_report(level, steps, assembly="colours"):
    """The paper's von Mises example (Section 8.2) on the L-shaped domain of
    20-node serendipity hexahedra: tangent-assembly time of every Newton
    iteration against its number of plastic points, a least-squares line
    through them, the tangent assembly with every point plastic (seeded),
    and the K_elast assembly time for comparison; plus the hysteresis data
    (load factor, work f_max^T u) of the load path."""
    import numpy as np
    import torch
    from paper_1805_04155_amd import _ep
    from paper_1805_04155_amd import workloads as W
    wl = W.workload_lshape_vm(level, steps)
    mesh = wl.mesh
    ctx = _ep.Context(mesh, wl.free, wl.material, options={
        "newton_rtol": 1e-10,
        "assembly": _ep.ASSEMBLY[assembly]})
    u = torch.zeros(mesh.n_dof, dtype=torch.float64, device="cuda")
    _ep.ep_profile(ctx.h, 1)
    for _ in range(5):
        _ep.ep_assemble_elastic(ctx.h)
    el_ms = _ep.ep_profile_read(ctx.h, "elastic")[0] / 5
    _ep.ep_profile_read(ctx.h, "assembly")
    fmax = torch.tensor(200.0 * wl.f_unit, dtype=torch.float64, device="cuda")
    pts, hyst, its = [], [], 0
    t0 = time.perf_counter()
    for k in range(len(wl.load_factors)):
        f = ctx.tensor(wl.f(k))
        for _ in range(50):
            st, info = ctx.newton_step(f, u)
            ms = _ep.ep_profile_read(ctx.h, "assembly")[0]
            if info["converged"]:
                break
            its += 1
            pts.append((info["n_plastic_ip"], ms))
        ctx.commit_step(u)
        hyst.append((round(float(wl.load_factors[k] / 200.0), 4),
                     round(float(torch.dot(fmax, u).item()), 6)))
    t = time.perf_counter() - t0
    # every point plastic (all elements seeded at u = 0): the tangent
    # assembly measured, one untimed pass first (it also restores the path's
    # last plastic set)
    ep, beta, _, _ = W.seeded_state(wl, 1.0, seed=0)
    ctx.set_state(ep, beta, None)
    u.zero_()
    for k in range(6):
        _ep.ep_constitutive(ctx.h, u)
        _ep.ep_assemble_tangent(ctx.h)
        if k == 0:
            _ep.ep_profile_read(ctx.h, "assembly")
    all_ms = _ep.ep_profile_read(ctx.h, "assembly")[0] / 5
    all_ip, _ = _ep.ep_get_plastic(ctx.h)
    _ep.ep_profile(ctx.h, 0)
    ctx.close()
    n = np.array([p[0] for p in pts], dtype=np.float64)
    ms = np.array([p[1] for p in pts])
    A = np.vstack([np.ones_like(n), n]).T
    (a0, a1), *_ = np.linalg.lstsq(A, ms, rcond=None)
    pred = a0 + a1 * n
    r2 = 1.0 - ((ms - pred) ** 2).sum() / max(((ms - ms.mean()) ** 2).sum(), 1e-30)
    full = a0 + a1 * mesh.n_int
    small = [b for a, b in pts if 0 < a <= 30]
    out = {"workload": f"L-shaped domain, level {level}: {mesh.n_elems} 20-node serendipity "
                       f"hexahedra, {mesh.n_nodes} nodes, {mesh.n_int} points; von Mises "
                       f"kinematic, cyclic top traction 200 zeta(t), {steps} steps",
           "assembly": assembly,
           "newton_iterations": its, "path_seconds_profiled": round(t, 3),
           "elastic_assembly_ms": round(el_ms, 4),
           "tangent_assembly_ms_vs_plastic_points": [[int(a), round(b, 4)] for a, b in pts],
           "fit_ms": {"intercept": round(float(a0), 5), "per_1000_points": round(float(a1) * 1e3, 6),
                      "r2": round(float(r2), 4)},
           "extrapolated_all_plastic_ms": round(float(full), 4),
           "median_ms_at_1_to_30_plastic_points": round(float(np.median(small)), 4)
           if small else None,
           "assemblies_without_plastic_points_skipped": int(sum(1 for a, _ in pts if a == 0)),
           "ratio_all_plastic_to_elastic": round(float(full / el_ms), 3) if el_ms > 0 else None,
           "measured_all_plastic": {"plastic_points": int(all_ip), "tangent_assembly_ms":
                                    round(all_ms, 4), "ratio_to_elastic":
                                    round(all_ms / el_ms, 3) if el_ms > 0 else None},
           "hysteresis_zeta_work": hyst}
    log(f"lshape {assembly}: {len(pts)} assemblies, fit {out['fit_ms']}, elastic "
        f"{el_ms:.4f} ms, extrapolated {full:.4f} ms, measured all plastic {all_ms:.4f} ms "
        f"({all_ip} points)")
    return out


def footing_report(n, ud_max, du_max, max_steps):
    """The strip-footing example (Section 8.3), 9-node quadrilaterals on an
    n x n grid: displacement-controlled path with the paper's doubling of
    the increment, the normalised footing pressure p/c0 along it; with full
    Newton steps and with the damped Newton method (theta = 1/4)."""
    import torch
    from paper_1805_04155_amd import _ep, solver
    from paper_1805_04155_amd import workloads as W
    wl = W.workload_strip_footing(n, "Q2_2D")
    c0 = 450.0
    out = {"workload": f"plane strain [0,10]^2, {n}x{n} 9-node quadrilaterals "
                       f"({wl.mesh.n_dof} dofs), Drucker-Prager perfect E=1e7 nu=0.48 c0=450 "
                       "phi=pi/9, footing 0<=x1<=1 pushed down by u_D"}
    for name, theta in (("full_steps", 0.0), ("damped", 0.25)):
        ctx = _ep.Context(wl.mesh, wl.free, wl.material,
                          options={"newton_rtol": 1e-10, "newton_damping": theta})
        u = torch.zeros(wl.mesh.n_dof, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = solver.displacement_path(ctx, wl, u, ud_max=ud_max, du0=1e-3, du_max=du_max,
                                        max_steps=max_steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ctx.close()
        out[name] = {
            "newton_damping": theta, "seconds": round(t, 3), "steps": len(recs),
            "newton_its": sum(r["newton_its"] for r in recs),
            "pcg_its": sum(r["pcg_its"] for r in recs),
            "line_search_evals": sum(r["ls_evals"] for r in recs),
            "final_u_D": recs[-1]["u_D"] if recs else 0.0,
            "final_pressure_over_c0": round(recs[-1]["pressure"] / c0, 4) if recs else None,
            "path_u_D_p_over_c0_plastic": [[round(r["u_D"], 6), round(r["pressure"] / c0, 4),
                                           r["n_plastic_ip"]] for r in recs]}
        log(f"footing {name}: {out[name]['steps']} steps to u_D = {out[name]['final_u_D']}, "
            f"p/c0 = {out[name]['final_pressure_over_c0']}, {t:.1f} s")
    return out


def plastic_sweep(steps):
    """Throughput on the 64^3 Q1 cube (von Mises) against the seeded plastic
    fraction and the tangent value type, at u = 0 and at the first Newton
    iterate of load step 6 (t = 324)."""
    import torch
    from paper_1805_04155_amd import _ep
    from paper_1805_04155_amd import workloads as W
    wl = W.workload_q1_cube(64)
    mesh, mat = wl.mesh, wl.material
    out = {"workload": "unit cube, 64^3 Q1 hexahedra (2097152 points), von Mises kinematic",
           "unit": "M integration pts/s", "rows": []}
    F = torch.empty(mesh.n_dof, dtype=torch.float64, device="cuda")
    f6 = torch.as_tensor(wl.f(5), dtype=torch.float64, device="cuda")
    for tang in ("fp64", "fp32"):
        ctx = _ep.Context(mesh, wl.free, mat, options={
            "tangent_prec": _ep.EP_FP64 if tang == "fp64" else _ep.EP_FP32})
        for frac in (0.0, 0.25, 0.5, 1.0):
            ep, beta, kappa, _ = W.seeded_state(wl, frac, seed=0)
            ctx.set_state(ep, beta, None)
            u = torch.zeros(mesh.n_dof, dtype=torch.float64, device="cuda")
            ms0 = time_pass(ctx, u, F, steps)
            n_ip0, _ = _ep.ep_get_plastic(ctx.h)
            _ep.ep_newton_step(ctx.h, f6, u)
            ms1 = time_pass(ctx, u, F, steps)
            n_ip1, _ = _ep.ep_get_plastic(ctx.h)
            row = {"tangent": tang, "seeded_fraction": frac,
                   "u0": {"ms": round(ms0, 4), "value": round(mesh.n_int / ms0 / 1e3, 1),
                          "plastic_points": n_ip0},
                   "first_iterate": {"ms": round(ms1, 4),
                                     "value": round(mesh.n_int / ms1 / 1e3, 1),
                                     "plastic_points": n_ip1}}
            out["rows"].append(row)
            log(f"sweep {row}")
        ctx.close()
    return out


def local_precision_report(block):
    """Matrix-core local products on the blocks at a seeded state: tangent
    error against the FP64 path (relative Frobenius norm, and the largest
    entry error relative to its row scale) and the assembly kernel's rate."""
    import numpy as np
    import torch
    from paper_1805_04155_amd import _ep
    from paper_1805_04155_amd import workloads as W
    out = {}
    for name, fn, et in (("q2_block", W.workload_q2_block, "Q2_3D"),
                         ("p2_block", W.workload_p2_block, "P2_3D")):
        wl = fn(*block)
        mesh, mat = wl.mesh, wl.material
        ep, beta, kappa, _ = W.seeded_state(wl, 0.5, seed=0)
        rec = {}
        K64 = None
        for lp in ("fp64", "fp32", "bf16"):
            ctx = _ep.Context(mesh, wl.free, mat, options={
                "local_prec": {"fp64": _ep.EP_FP64, "fp32": _ep.EP_FP32, "bf16": _ep.EP_BF16}[lp]})
            ctx.set_state(*_state_args(mat, ep, beta, kappa))
            u = torch.zeros(mesh.n_dof, dtype=torch.float64, device="cuda")
            for _ in range(3):
                _ep.ep_constitutive(ctx.h, u)
                _ep.ep_assemble_tangent(ctx.h)
            torch.cuda.synchronize()
            n_ip, n_el = _ep.ep_get_plastic(ctx.h)
            _ep.ep_profile(ctx.h, 1)
            reps = 10
            for _ in range(reps):
                _ep.ep_constitutive(ctx.h, u)
                _ep.ep_assemble_tangent(ctx.h)
            torch.cuda.synchronize()
            ms, cnt = _ep.ep_profile_read(ctx.h, "assembly")
            _ep.ep_profile(ctx.h, 0)
            _, _, val = ctx.csr(1)
            r = {"assembly_ms": round(ms / reps, 4), "plastic_points": n_ip}
            flops = LOCAL_FLOPS_PER_IP[et] * n_ip
            r["local_product_TFLOP_s"] = round(flops / (ms / reps / 1e3) / 1e12, 2)
            if lp == "fp64":
                K64 = val.clone()
            else:
                r["mfma_utilization_lower_bound"] = round(
                    r["local_product_TFLOP_s"] / MFMA_PEAK_TFLOPS[lp], 5)
                r["K_rel_frobenius_error_vs_fp64"] = float(
                    (torch.linalg.norm(val - K64) / torch.linalg.norm(K64)).item())
            rec[lp] = r
            log(f"local precision {name} {lp}: {r}")
            ctx.close()
            del val, u
        del K64
        torch.cuda.empty_cache()
        out[name] = {"workload": f"{block[0]}x{block[1]}x{block[2]} block, "
                                 f"{mesh.n_int} points, half of the elements seeded plastic",
                     "local_flops_per_plastic_point": LOCAL_FLOPS_PER_IP[et],
                     "note": "matrix-core rate = useful local-product flops / whole assembly "
                             "kernel time (scatter included): a lower bound on the matrix "
                             "cores' utilisation",
                     "precisions": rec}
    return out


MDESC = {
    "q1_cube": "unit cube, 64^3 Q1 hexahedra (262144 elements, 2097152 points, 823875 dofs), "
               "von Mises kinematic E=206900 nu=0.29 sigma_y=450 H=10000",
    "q2_slope": "plane strain 40x20 rectangle, 512x256 9-node Q2 quads (131072 elements, "
                "1179648 points), Drucker-Prager perfect c0=450 phi=20deg E=20000 nu=0.49",
}


def copy_calibration():
    """Plain copy of 512 MiB (for scaling hardware byte counters) and the
    measured copy rate (read + write bytes over time) as the practical HBM
    ceiling beside the published peak."""
    import torch
    a = torch.empty(64 * 2 ** 20, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_ms = e0.elapsed_time(e1) / 20
    gbs = round(2 * a.numel() * 8 / (copy_ms / 1e3) / 1e9, 1)
    log(f"copy of 512 MiB: {copy_ms:.4f} ms, {gbs} GB/s read + write")
    return gbs


def measure_pass(name, frac, tangent, local_prec, steps, warmup, copy_gbs=None, keep=False,
                 assembly="colours"):
    """Timed passes of the hot path on workload `name` with `frac` of the
    elements seeded plastic: per-kernel breakdown (every kernel timed), then
    the timed region with HIP events on the dominant kernel only.  Returns
    the record (and, with keep, the inputs for the CPU baseline)."""
    import numpy as np
    import torch
    from paper_1805_04155_amd import _ep
    from paper_1805_04155_amd import workloads as W
    wl = getattr(W, WORKLOADS[name])()
    mesh, mat = wl.mesh, wl.material
    ep, beta, kappa, _ = W.seeded_state(wl, frac, seed=0)
    h = (np.prod(mesh.coord.max(axis=1) - mesh.coord.min(axis=1)) / mesh.n_elems) ** (1 / mesh.dim)
    u_np = W.random_displacement(mesh, 1, 1e-6 * h, wl.free)
    tb = 8 if tangent == "fp64" else 4
    lp = {"fp64": _ep.EP_FP64, "fp32": _ep.EP_FP32, "bf16": _ep.EP_BF16}[local_prec]
    ctx = _ep.Context(mesh, wl.free, mat,
                      options={"tangent_prec": _ep.EP_FP64 if tb == 8 else _ep.EP_FP32,
                               "local_prec": lp,
                               "assembly": _ep.ASSEMBLY[assembly]})
    ctx.set_state(ep, beta if mat.model == "VM" else None, kappa if mat.model == "DP" else None)
    u = ctx.tensor(u_np)
    F = torch.empty(mesh.n_dof, dtype=torch.float64, device="cuda")

    def step():
        _ep.ep_constitutive(ctx.h, u)
        _ep.ep_assemble_tangent(ctx.h)
        _ep.ep_internal_force(ctx.h, F)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    n_ip, n_el = _ep.ep_get_plastic(ctx.h)
    counts = {"plastic_elems": n_el, "plastic_ips": n_ip, "listed": n_el,
              "n_perm": mesh.n_elems}
    kb = kernel_bytes(mesh, mat, counts, tb)

    def kernel_row(kname, tms, n):
        t_step = tms / steps / 1e3
        return {"ms_per_step": round(tms / steps, 4), "launches_per_step": n // steps,
                "bytes_per_step": kb[kname],
                "GB_s": round(kb[kname] / t_step / 1e9, 1) if t_step > 0 else None}

    # per-kernel breakdown, every kernel timed: each timed dispatch costs a
    # few microseconds, so these passes are not the timed region
    _ep.ep_profile(ctx.h, 1)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof = {k: _ep.ep_profile_read(ctx.h, k) for k in _ep.PROF}
    _ep.ep_profile(ctx.h, 0)
    per_kernel = {k: kernel_row(k, *prof[k])
                  for k in ("constitutive", "compaction", "assembly", "force") if prof[k][1] > 0}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_step"])

    # timed region: HIP events on the dominant kernel's launches only
    _ep.ep_profile(ctx.h, 1, kernels=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    dom_ms, dom_n = _ep.ep_profile_read(ctx.h, dom)
    _ep.ep_profile(ctx.h, 0)
    ms = 1e3 * t / steps
    value = mesh.n_int / (ms / 1e3) / 1e6
    per_kernel[dom] = kernel_row(dom, dom_ms, dom_n)
    per_kernel[dom]["timed_region"] = True
    d = per_kernel[dom]
    n_launch = max(1, d["launches_per_step"])
    t_launch_s = d["ms_per_step"] / n_launch / 1e3
    roofline = {"bound": "hbm", "kernel": dom, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "avg_launch_ms": round(d["ms_per_step"] / n_launch, 5),
                "launches_per_step": n_launch, "copy_GB_s": copy_gbs}
    if dom == "assembly":
        scalar = assembly_bytes_scalar_model(mesh, counts, tb) / n_launch
        design = kb["assembly"] / n_launch if assembly == "colours" else None
        roofline.update({
            "bytes_model": "scalar-CSR model: per plastic point 8 (d n_p + 1) + 64 B, per "
                           "plastic element (d n_p)^2 (4 + 2 s) x 2 (restore + add)",
            "algorithmic_bytes_per_launch": int(scalar),
            "achieved": round(scalar / t_launch_s / 1e9, 1),
            "design_model": None if design is None else {
                "what": "node-block CSR of this build: per listed element n_p^2 block "
                        "position map entries, one-byte stamps, base value read and value "
                        "write; per plastic element its nodes; per plastic point its tangent "
                        "descriptor",
                "algorithmic_bytes_per_launch": int(design),
                "achieved": round(design / t_launch_s / 1e9, 1),
                "frac": round(design / t_launch_s / 1e9 / HBM_PEAK_GBS, 4)}})
    else:
        roofline.update({"algorithmic_bytes_per_launch": int(d["bytes_per_step"] / n_launch),
                         "achieved": d["GB_s"]})
    roofline["frac"] = round(roofline["achieved"] / HBM_PEAK_GBS, 4)
    roofline["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 4) if copy_gbs else None
    roofline["traffic"] = None
    if os.path.exists(TRAFFIC_FILE):
        for tr in json.load(open(TRAFFIC_FILE)):
            if tr.get("kernel_src_sha256") == src_hash() and tr.get("kernel") == dom and \
                    tr.get("tangent") == tangent and tr.get("workload") == name:
                roofline["traffic"] = tr.get("bytes_per_launch")
    ctx.close()
    del ctx, F, u
    torch.cuda.empty_cache()
    rec = {"workload": f"{name}: {MDESC.get(name, name)}", "plastic_fraction_seeded": frac,
           "plastic_elements": n_el, "plastic_points": n_ip, "tangent": tangent,
           "local_products": local_prec, "value": round(value, 2), "ms_per_step": round(ms, 4),
           "roofline": roofline, "kernels": per_kernel}
    log(f"pass {name} {tangent}: {value:.1f} M points/s, {ms:.4f} ms, {dom} "
        f"{roofline['achieved']} GB/s")
    return (rec, (wl, ep, beta, kappa, u_np)) if keep else rec


def p1_square_newton():
    """Time to |Q(f - F)| <= 1e-10 |Q f| over the ten load steps of the P1
    square (FP64), from the first Newton evaluation of step 1 to the last
    commit; one untimed run first."""
    import torch
    from paper_1805_04155_amd import _ep, solver
    from paper_1805_04155_amd import workloads as W
    wl = W.workload_p1_square()
    rec = None
    for rep in range(2):
        ctx = _ep.Context(wl.mesh, wl.free, wl.material, options={"newton_rtol": 1e-10})
        u = torch.zeros(wl.mesh.n_dof, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = solver.solve_load_path(ctx, wl, u)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ctx.close()
        rec = {"workload": "plane strain 10x10 square, 32x32 squares split into 2048 P1 "
                           "triangles (2048 points), von Mises kinematic, top traction 54k, "
                           "k = 1..10",
               "seconds": round(t, 4), "steps": len(recs),
               "newton_its": sum(r["newton_its"] for r in recs),
               "pcg_its": sum(r["pcg_its"] for r in recs),
               "max_final_res_rel": max(r["res_rel"] for r in recs),
               "plastic_points_last_step": recs[-1]["n_plastic_ip"]}
    log(f"p1 square newton: {rec}")
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="q1_cube", choices=list(WORKLOADS))
    ap.add_argument("--plastic-fraction", type=float, default=0.5)
    ap.add_argument("--tangent", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-calibration-copy", action="store_true")
    ap.add_argument("--local-prec", choices=["fp64", "fp32", "bf16"], default="fp64",
                    help="element-local products (27-node hexahedra, P2 tetrahedra only)")
    ap.add_argument("--assembly", choices=["colours", "rows", "fused"], default="colours",
                    help="colour rounds with stamps, element matrices + node-row gather, or "
                         "node rows with the element terms formed in place")
    ap.add_argument("--no-slope", action="store_true",
                    help="skip the slope passes (FP64 and FP32 tangent values)")
    ap.add_argument("--no-newton", action="store_true",
                    help="skip the time-to-1e-10 load paths and the local-precision report")
    ap.add_argument("--newton-cube-n", type=int, default=64)
    ap.add_argument("--newton-samples", type=float, default=20e6)
    ap.add_argument("--newton-block", default="32,16,16")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the plastic-fraction sweep on the Q1 cube")
    ap.add_argument("--no-lshape", action="store_true",
                    help="skip the L-shape von Mises example (assembly time vs plastic points)")
    ap.add_argument("--lshape-level", type=int, default=2)
    ap.add_argument("--no-footing", action="store_true",
                    help="skip the strip-footing example (displacement control)")
    ap.add_argument("--footing-n", type=int, default=64)
    ap.add_argument("--lshape-steps", type=int, default=40)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path is built and timed on a single "
              "MI355X (multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    copy_gbs = None if args.no_calibration_copy else copy_calibration()
    head, inputs = measure_pass(args.workload, args.plastic_fraction, args.tangent,
                                args.local_prec, args.steps, args.warmup, copy_gbs, keep=True,
                                assembly=args.assembly)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(*inputs)
    del inputs
    slope = p1 = newton = local = sweep = lshape = footing = None
    if not args.no_slope and args.workload != "q2_slope":
        slope = {t: measure_pass("q2_slope", 0.5, t, "fp64", args.steps, args.warmup, copy_gbs)
                 for t in ("fp64", "fp32")}
    if not args.no_newton:
        p1 = p1_square_newton()
    if not args.no_sweep:
        sweep = plastic_sweep(max(5, args.steps // 2))
    if not args.no_lshape:
        lshape = {m: lshape_report(args.lshape_level, args.lshape_steps, m)
                  for m in ("colours", "rows")}
    if not args.no_footing:
        footing = footing_report(args.footing_n, 0.1, 0.016, 40)
    if not args.no_newton:
        block = tuple(int(x) for x in args.newton_block.split(","))
        local = local_precision_report(block)
        newton = newton_report(args.newton_cube_n, int(args.newton_samples), block)

    line = {
        "metric": "M integration pts/s (return map + K assembly)",
        "value": head["value"], "unit": "M integration pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.tangent == "fp64" else
                 "f64 (return map, force) / f32 (tangent values)",
        "data": "synthetic",
        "config": {"workload": head["workload"],
                   "plastic_fraction_seeded": args.plastic_fraction,
                   "plastic_elements": head["plastic_elements"],
                   "plastic_points": head["plastic_points"], "tangent": args.tangent,
                   "local_products": args.local_prec, "assembly": args.assembly,
                   "step": "constitutive + compaction + incremental K assembly + internal "
                           "force"},
        "roofline": head["roofline"],
        "kernels": head["kernels"],
        "cpu_baseline": cpu,
        "q2_slope": slope,
        "p1_square_newton": p1,
        "newton": newton,
        "local_precision": local,
        "plastic_sweep": sweep,
        "lshape_vm": lshape,
        "strip_footing": footing,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
