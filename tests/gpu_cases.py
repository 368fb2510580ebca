"""Small seeded cases shared by the GPU parity tests: every element kind and
material model, sized to span several blocks of every kernel with ragged
tails, with mixed elastic / plastic (and, for Drucker-Prager, apex) points."""
import numpy as np

from paper_1805_04155_amd import workloads as W

DPH = W.dp_material_3d_hardening()
DP3 = W.Material("DP", E=20000.0, nu=0.3, eta=DPH.eta, c=DPH.c, a=0.0)

CASES = {
    # name: (mesh factory, material)
    "p1_2d_vm": (lambda: W.mesh_p1_2d(41, 29, 10.0, 7.0), W.VM_MATERIAL),
    "q1_2d_dp": (lambda: W.mesh_q1_2d(37, 23, 3.0, 2.0), W.dp_material_2d()),
    "q2_2d_dp": (lambda: W.mesh_q2_2d(25, 19, 4.0, 3.0), W.dp_material_2d()),
    "p1_3d_vm": (lambda: W.mesh_tet_3d(7, 6, 5, 1.0, 0.9, 0.8, order=1), W.VM_MATERIAL),
    "p2_3d_dph": (lambda: W.mesh_tet_3d(5, 4, 3, 1.0, 0.8, 0.6, order=2), DPH),
    "q1_3d_vm": (lambda: W.mesh_q1_3d(11, 9, 8, 1.1, 0.9, 0.8), W.VM_MATERIAL),
    "q1_3d_dp": (lambda: W.mesh_q1_3d(9, 7, 6, 0.9, 0.7, 0.6), DP3),
    "q2_3d_dph": (lambda: W.mesh_q2_3d(5, 4, 3, 1.0, 0.8, 0.6), DPH),
    "q2s_2d_vm": (lambda: W.mesh_q2s_2d(23, 17, 3.0, 2.0), W.VM_MATERIAL),
    "q2s_3d_dph": (lambda: W.mesh_q2s_3d(6, 4, 3, 1.0, 0.7, 0.5), DPH),
}


def distort(mesh, amp=0.04, seed=0):
    """Smooth interior node perturbation (keeps boundary planes); straight
    simplices stay valid, curved hexahedra exercise the non-affine map."""
    x = mesh.coord.copy()
    lo, hi = x.min(axis=1, keepdims=True), x.max(axis=1, keepdims=True)
    inside = np.all((x > lo + 1e-9) & (x < hi - 1e-9), axis=0)
    h = (np.prod(hi - lo) / mesh.n_elems) ** (1.0 / mesh.dim)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, mesh.dim)
    for d in range(mesh.dim):
        x[d, inside] += amp * h * np.sin(3.0 * x[(d + 1) % mesh.dim, inside] / (hi[0, 0] - lo[0, 0]) * 6.28 + ph[d])
    return W.Mesh(mesh.etype, x, mesh.elem)


def make_case(name, seed=0, plastic_scale=1.0):
    make, mat = CASES[name]
    mesh = distort(make(), seed=seed)
    rng = np.random.default_rng(seed + 100)
    free = np.ones(mesh.n_dof, dtype=np.uint8)
    # fix the nodes of the x1 = min plane (keeps K_t non-singular for PCG)
    x0 = mesh.coord[0].min()
    on = np.abs(mesh.coord[0] - x0) < 1e-12
    for c in range(mesh.dim):
        free[mesh.dim * np.nonzero(on)[0] + c] = 0
    scale = (mat.Y if mat.model == "VM" else mat.c) / mat.E
    ep, beta, kappa = W.random_state(mesh, mat, seed + 1, 0.4 * scale)
    if mat.model == "VM":
        n3 = 3
        m = ep[:n3].mean(axis=0)
        ep[:n3] -= m
        beta[:n3] -= mat.a * m
    ext = mesh.coord.max(axis=1) - mesh.coord.min(axis=1)
    h = (np.prod(ext) / mesh.n_elems) ** (1.0 / mesh.dim)
    u = W.random_displacement(mesh, seed + 2, 0.5 * plastic_scale * scale * h)
    # volumetric stretch graded along x1: drives part of the Drucker-Prager
    # points to the apex, leaves others on the cone or elastic
    if mat.model == "DP":
        x = mesh.coord
        t = (x[0] - x[0].min()) / (x[0].max() - x[0].min())
        amp = 2.0 * plastic_scale * mat.c / (mat.eta * mat.bulk * mesh.dim)
        u += (amp * t * (x - x.mean(axis=1, keepdims=True))).T.reshape(-1) * rng.uniform(0.8, 1.0)
    return mesh, free, mat, u, (ep, beta, kappa)
