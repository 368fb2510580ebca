#!/usr/bin/env python3
"""Throughput of the elastoplastic Newton hot path on one MI355X.

A step is one pass of the hot path over the whole workload: strain and return
map at every integration point with the fused constitutive kernel, plastic-
element compaction, the incremental tangent K_elast + B^T (D - D_elast) B
(colour rounds over the plastic work list) and the internal force / residual.  The metric is
millions of integration points per second.  Inputs are resident in HBM when
the timed region starts.

Workload (default): plane strain 40 x 20 rectangle, 512 x 256 nine-node Q2
quadrilaterals (131072 elements, 1179648 integration points), Drucker-Prager
perfect plasticity (c0 = 450, phi = 20 deg, E = 20000, nu = 0.49), half of the
elements seeded plastic.

Prints one JSON line (rank 0, one GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1805_04155_amd", "csrc", "ep_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_q2_slope.json")

WORKLOADS = {
    "q2_slope": "workload_q2_slope",
    "q1_cube": "workload_q1_cube",
    "p1_square": "workload_p1_square",
    "q2_block": "workload_q2_block",
    "p2_block": "workload_p2_block",
}


def kernel_bytes(mesh, mat, counts, tangent_bytes):
    """Algorithmic HBM bytes per step of each kernel (every array read or
    written once at the granularity the design moves it).  counts: plastic
    elements, plastic integration points, elements restored."""
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
        # flag, descriptor of plastic points, element force vectors, mask
        "constitutive": 2 * 8 * n_dof + 4 * NP * n_e + state * n_int + n_int
        + 8 * ndesc * pi + 8 * D * NP * n_e + 4 * n_e,
        # per listed element: position map, epoch read + write, base value
        # read, tangent write, mask; per plastic element its connectivity and
        # coordinates; per plastic point its tangent descriptor
        "assembly": listed * (blk * (4 + 8 + 2 * D * D * s) + 4) + pe * NP * (4 + 8 * D)
        + 8 * ndesc * pi,
        # colour-major order and two masks read, list written
        "compaction": counts["n_perm"] * 4 + 8 * n_e + 4 * listed,
        "force": 4 * (n_n + 1) + 4 * NP * n_e + 8 * D * NP * n_e + n_dof * (8 + 1 + 8),
    }


def src_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()


def cpu_baseline(wl, ep, beta, kappa, u):
    """The FP64 oracle timed on the host for one full pass of the same
    workload (strain, return map, plain sum w B^T D B assembled by COO sort,
    internal force), single thread."""
    import numpy as np
    from oracle import oracle as O
    mesh, mat = wl.mesh, wl.material
    dphi, w = O.geometry(mesh)
    pat = O.pattern(mesh)
    dim = mesh.dim
    ep6 = O.state_to_ip6(ep, dim)
    beta6 = O.state_to_ip6(beta, dim)
    t0 = time.perf_counter()
    eps = O.strain(mesh, dphi, u)
    out = O.constitutive(mat, eps, ep6, beta6, kappa)
    O.assemble(mesh, dphi, w, out["D"], *pat)
    O.internal_force(mesh, dphi, w, out["sig"])
    t = time.perf_counter() - t0
    del np
    return {"value": mesh.n_int / t / 1e6, "unit": "M integration pts/s", "cores": 1,
            "kind": "oracle", "seconds": round(t, 3),
            "sample": f"one full pass over all {mesh.n_elems} elements ({mesh.n_int} points): "
                      "strain, return map, COO-sorted K assembly, internal force; geometry "
                      "and sparsity pattern precomputed"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="q2_slope", choices=list(WORKLOADS))
    ap.add_argument("--plastic-fraction", type=float, default=0.5)
    ap.add_argument("--tangent", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-calibration-copy", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path is built and timed on a single "
              "MI355X (multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1805_04155_amd import _ep
    from paper_1805_04155_amd import workloads as W

    torch.cuda.set_device(0)
    wl = getattr(W, WORKLOADS[args.workload])()
    mesh, mat = wl.mesh, wl.material
    ep, beta, kappa, _ = W.seeded_state(wl, args.plastic_fraction, seed=0)
    h = (np.prod(mesh.coord.max(axis=1) - mesh.coord.min(axis=1)) / mesh.n_elems) ** (1 / mesh.dim)
    u_np = W.random_displacement(mesh, 1, 1e-6 * h, wl.free)

    tb = 8 if args.tangent == "fp64" else 4
    ctx = _ep.Context(mesh, wl.free, mat,
                      options={"tangent_prec": _ep.EP_FP64 if tb == 8 else _ep.EP_FP32})
    ctx.set_state(ep, beta if mat.model == "VM" else None, kappa if mat.model == "DP" else None)
    u = ctx.tensor(u_np)
    F = torch.empty(mesh.n_dof, dtype=torch.float64, device="cuda")

    if not args.no_calibration_copy:
        # plain copy of a known size, for scaling hardware byte counters
        a = torch.empty(64 * 2 ** 20, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step():
        _ep.ep_constitutive(ctx.h, u)
        _ep.ep_assemble_tangent(ctx.h)
        _ep.ep_internal_force(ctx.h, F)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    n_ip, n_el = _ep.ep_get_plastic(ctx.h)
    _ep.ep_profile(ctx.h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    prof = {k: _ep.ep_profile_read(ctx.h, k) for k in _ep.PROF}
    _ep.ep_profile(ctx.h, 0)
    ms = 1e3 * t / args.steps
    value = mesh.n_int / (ms / 1e3) / 1e6

    counts = {"plastic_elems": n_el, "plastic_ips": n_ip, "listed": n_el,
              "n_perm": mesh.n_elems}
    kb = kernel_bytes(mesh, mat, counts, tb)
    per_kernel = {}
    for name, key in (("constitutive", "constitutive"), ("compaction", "compaction"),
                      ("assembly", "assembly"), ("force", "force")):
        tms, n = prof[key]
        if n == 0:
            continue
        t_step = tms / args.steps / 1e3
        per_kernel[name] = {"ms_per_step": round(tms / args.steps, 4),
                            "launches_per_step": n // args.steps,
                            "bytes_per_step": kb[name],
                            "GB_s": round(kb[name] / t_step / 1e9, 1) if t_step > 0 else None}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_step"])
    d = per_kernel[dom]
    n_launch = max(1, d["launches_per_step"])
    achieved = d["GB_s"]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_src_sha256") == src_hash() and tr.get("kernel") == dom and \
                tr.get("tangent") == args.tangent and tr.get("workload") == args.workload:
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "algorithmic_bytes_per_launch": int(d["bytes_per_step"] / n_launch),
                "avg_launch_ms": round(d["ms_per_step"] / n_launch, 5),
                "traffic": traffic}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, ep, beta, kappa, u_np)

    mdesc = {"q2_slope": "plane strain 40x20 rectangle, 512x256 9-node Q2 quads (131072 elements, "
                         "1179648 points), Drucker-Prager perfect c0=450 phi=20deg E=20000 nu=0.49",
             "q1_cube": "unit cube, 64^3 Q1 hexahedra (2097152 points), von Mises kinematic "
                        "E=206900 nu=0.29 sigma_y=450 H=10000"}.get(args.workload, args.workload)
    line = {
        "metric": "M integration pts/s (return map + K assembly)",
        "value": round(value, 2), "unit": "M integration pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if tb == 8 else "f64 (return map, force) / f32 (tangent values)",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {mdesc}", "plastic_fraction_seeded": args.plastic_fraction,
                   "plastic_elements": n_el, "plastic_points": n_ip, "tangent": args.tangent,
                   "step": "constitutive + compaction + incremental K assembly + internal force"},
        "roofline": roofline,
        "kernels": per_kernel,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
