"""Pins of the oracle's assembly (K = sum w B^T D B, F = B^T W sigma, the CSR
pattern and the position map) against closed-form counts, invariants and
finite differences."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1805_04155_amd import workloads as W


def nnz_closed_form(kind, n):
    """Number of stored entries of the dof-pair pattern on structured grids.
    Q1: every node couples to the nodes of the up to 2^d cells around it, a
    count of 3 per axis inside and 2 on the boundary.  Q2 (doubled grid):
    vertex nodes reach +-2 grid steps (5 inside, 3 on the boundary), the
    other nodes +-1 (3).  P1 squares split along (0,0)-(1,1): every node
    couples to itself, its 4 axis neighbours and the two diagonal ones."""
    if kind == "Q1_3D":
        return 9 * np.prod([3 * m + 1 for m in n])
    if kind == "Q2_3D":
        return 9 * np.prod([8 * m + 1 for m in n])
    if kind == "Q2_2D":
        return 4 * np.prod([8 * m + 1 for m in n])
    if kind == "P1_2D":
        nx, ny = n
        edges = nx * (ny + 1) + ny * (nx + 1) + nx * ny
        return 4 * ((nx + 1) * (ny + 1) + 2 * edges)
    raise KeyError(kind)


def test_nnz_closed_forms_of_the_workloads():
    # sizes of the workloads' meshes
    assert nnz_closed_form("P1_2D", (32, 32)) == 29444
    assert nnz_closed_form("Q2_2D", (512, 256)) == 33579012
    assert nnz_closed_form("Q1_3D", (64, 64, 64)) == 64701513
    assert nnz_closed_form("Q2_3D", (32, 16, 16)) == 38490633


SMALL = {
    "P1_2D": (lambda: W.mesh_p1_2d(5, 4, 1.0, 0.8), (5, 4)),
    "Q2_2D": (lambda: W.mesh_q2_2d(4, 3, 1.0, 0.75), (4, 3)),
    "Q1_3D": (lambda: W.mesh_q1_3d(3, 2, 4, 0.75, 0.5, 1.0), (3, 2, 4)),
    "Q2_3D": (lambda: W.mesh_q2_3d(2, 3, 2, 0.5, 0.75, 0.5), (2, 3, 2)),
}


@pytest.mark.parametrize("etype", list(SMALL))
def test_pattern_counts_and_brute_force(etype):
    make, n = SMALL[etype]
    mesh = make()
    row_ptr, col_idx = O.pattern(mesh)
    assert col_idx.shape[0] == nnz_closed_form(etype, n)
    # brute force set of dof pairs
    d = mesh.dim
    pairs = set()
    for e in mesh.elem:
        dofs = [d * int(v) + c for v in e for c in range(d)]
        for a in dofs:
            for b in dofs:
                pairs.add((a, b))
    rows = np.repeat(np.arange(mesh.n_dof), np.diff(row_ptr))
    assert set(zip(rows.tolist(), col_idx.tolist())) == pairs
    assert np.all(np.diff(col_idx)[np.diff(rows) == 0] > 0)


def test_pattern_p2_brute_force():
    mesh = W.mesh_tet_3d(2, 1, 2, 1.0, 0.5, 1.0, order=2)
    row_ptr, col_idx = O.pattern(mesh)
    pairs = set()
    for e in mesh.elem:
        dofs = [3 * int(v) + c for v in e for c in range(3)]
        pairs.update((a, b) for a in dofs for b in dofs)
    assert col_idx.shape[0] == len(pairs)


@pytest.mark.parametrize("etype", list(SMALL))
def test_position_map(etype):
    mesh = SMALL[etype][0]()
    row_ptr, col_idx = O.pattern(mesh)
    pos = O.position_map(mesh, row_ptr, col_idx)
    d = mesh.dim
    dof = (d * mesh.elem[:, :, None] + np.arange(d)).reshape(mesh.n_elems, -1)
    rows = np.repeat(np.arange(mesh.n_dof), np.diff(row_ptr))
    assert np.all(pos >= 0)
    assert np.array_equal(col_idx[pos], np.broadcast_to(dof[:, None, :], pos.shape))
    assert np.array_equal(rows[pos], np.broadcast_to(dof[:, :, None], pos.shape))


def _elastic_D(mat, n):
    out = O.constitutive(mat, np.zeros((n, 6)), np.zeros((n, 6)))
    return out["D"]


def rigid_modes(mesh):
    x = mesh.coord
    d = mesh.dim
    modes = []
    for c in range(d):
        u = np.zeros((mesh.n_nodes, d))
        u[:, c] = 1
        modes.append(u.reshape(-1))
    if d == 2:
        modes.append(np.stack([-x[1], x[0]], axis=1).reshape(-1))
    else:
        for a, b in ((0, 1), (1, 2), (0, 2)):
            u = np.zeros((mesh.n_nodes, 3))
            u[:, a] = -x[b]
            u[:, b] = x[a]
            modes.append(u.reshape(-1))
    return modes


MIXED = {
    "P1_2D": lambda: (W.mesh_p1_2d(4, 4, 1.0, 1.0), W.VM_MATERIAL),
    "Q2_2D": lambda: (W.mesh_q2_2d(3, 2, 1.0, 0.7), W.dp_material_2d()),
    "Q1_3D": lambda: (W.mesh_q1_3d(2, 2, 2, 1.0, 1.0, 1.0), W.VM_MATERIAL),
    "Q2_3D": lambda: (W.mesh_q2_3d(2, 1, 1, 1.0, 0.5, 0.5), W.dp_material_3d_hardening()),
    "P2_3D": lambda: (W.mesh_tet_3d(1, 1, 1, 1.0, 1.0, 1.0, order=2), W.dp_material_3d_hardening()),
}


def _state(mesh, mat, seed):
    """Random displacement + random history so that a good share of the
    points are plastic."""
    scale = (mat.Y if mat.model == "VM" else mat.c) / mat.E
    ep, beta, kappa = W.random_state(mesh, mat, seed, 0.5 * scale)
    if mat.model == "VM":  # keep von Mises plastic strains deviatoric
        n3 = 3
        m = ep[:n3].mean(axis=0)
        ep[:n3] -= m
        beta[:n3] -= mat.a * m
    ext = mesh.coord.max(axis=1) - mesh.coord.min(axis=1)
    h = (np.prod(ext) / mesh.n_elems) ** (1.0 / mesh.dim)
    u = W.random_displacement(mesh, seed + 1, 0.6 * scale * h)
    return u, O.state_to_ip6(ep, mesh.dim), O.state_to_ip6(beta, mesh.dim), kappa


@pytest.mark.parametrize("etype", list(MIXED))
def test_symmetry_and_rigid_modes(etype):
    mesh, mat = MIXED[etype]()
    dphi, w = O.geometry(W.Mesh(mesh.etype, mesh.coord * 1.0, mesh.elem))
    u, ep6, beta6, kappa = _state(mesh, mat, 3)
    out = O.constitutive(mat, O.strain(mesh, dphi, u), ep6, beta6, kappa)
    assert 0 < np.count_nonzero(out["flag"]) < mesh.n_int
    for D in (_elastic_D(mat, mesh.n_int), out["D"]):
        rp, ci, val = O.assemble(mesh, dphi, w, D)
        K = O.csr_to_scipy(rp, ci, val, mesh.n_dof).toarray()
        nrm = np.abs(K).max()
        assert np.abs(K - K.T).max() < 1e-12 * nrm
        for r in rigid_modes(mesh):
            assert np.abs(K @ r).max() < 1e-12 * nrm * np.abs(r).max()


@pytest.mark.parametrize("etype", list(MIXED))
def test_internal_force_linear_in_elastic_range(etype):
    """F(u) = K_elast u when every point stays elastic."""
    mesh, mat = MIXED[etype]()
    dphi, w = O.geometry(mesh)
    u = W.random_displacement(mesh, 0, 1e-7)
    out = O.constitutive(mat, O.strain(mesh, dphi, u), np.zeros((mesh.n_int, 6)))
    assert np.all(out["flag"] == 0)
    F = O.internal_force(mesh, dphi, w, out["sig"])
    rp, ci, val = O.assemble(mesh, dphi, w, _elastic_D(mat, mesh.n_int))
    K = O.csr_to_scipy(rp, ci, val, mesh.n_dof)
    assert np.abs(F - K @ u).max() < 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("etype", list(MIXED))
def test_tangent_is_derivative_of_internal_force(etype):
    """K_t = dF/du, by central differences of the whole chain (strain,
    return map, B^T W sigma) at a state with mixed elastic/plastic points."""
    mesh, mat = MIXED[etype]()
    dphi, w = O.geometry(mesh)
    u, ep6, beta6, kappa = _state(mesh, mat, 5)
    out = O.constitutive(mat, O.strain(mesh, dphi, u), ep6, beta6, kappa)
    rp, ci, val = O.assemble(mesh, dphi, w, out["D"])
    K = O.csr_to_scipy(rp, ci, val, mesh.n_dof)
    rng = np.random.default_rng(9)
    v = rng.standard_normal(mesh.n_dof)
    h = 1e-6 * np.abs(u).max()

    def F(x):
        o = O.constitutive(mat, O.strain(mesh, dphi, x), ep6, beta6, kappa)
        return O.internal_force(mesh, dphi, w, o["sig"]), o["flag"]

    Fp, fp = F(u + h * v)
    Fm, fm = F(u - h * v)
    assert np.array_equal(fp, out["flag"]) and np.array_equal(fm, out["flag"])
    fd = (Fp - Fm) / (2 * h)
    Kv = K @ v
    assert np.abs(fd - Kv).max() < 1e-6 * np.abs(Kv).max()


def test_patch_test_solution():
    """Elastic patch test on a distorted Q2 mesh: with the exact linear field
    prescribed on the whole boundary and no load, the discrete solution is
    that linear field at every node."""
    import scipy.sparse.linalg as spla
    mesh = W.mesh_q2_3d(2, 2, 2, 1.0, 1.0, 1.0)
    x = mesh.coord.copy()
    interior = np.all((x > 1e-12) & (x < 1 - 1e-12), axis=0)
    x[:, interior] += 0.05 * np.sin(7.0 * x[:, interior])
    mesh = W.Mesh(mesh.etype, x, mesh.elem)
    dphi, w = O.geometry(mesh)
    rp, ci, val = O.assemble(mesh, dphi, w, _elastic_D(W.VM_MATERIAL, mesh.n_int))
    K = O.csr_to_scipy(rp, ci, val, mesh.n_dof).tocsc()
    G = np.array([[1e-3, 2e-4, -1e-4], [0.5e-3, -2e-3, 3e-4], [1e-4, 0, 1e-3]])
    u_lin = (G @ x).T.reshape(-1)
    free = np.repeat(interior, 3)
    u = u_lin.copy()
    u[free] = 0
    rhs = -(K @ u)
    u[free] = spla.spsolve(K[free][:, free], rhs[free])
    assert np.abs(u - u_lin).max() < 1e-12
