"""Pins of the oracle's reference elements, quadrature and geometry against
the paper's Appendix tables and against closed-form integrals."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1805_04155_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")

REF_VOLUME = {"P1_2D": 0.5, "Q1_2D": 4.0, "Q2_2D": 4.0, "P1_3D": 1 / 6,
              "P2_3D": 1 / 6, "Q1_3D": 8.0, "Q2_3D": 8.0, "Q2S_2D": 4.0, "Q2S_3D": 8.0}
# polynomial degree integrated exactly by each rule
EXACT_DEGREE = {"P1_2D": 1, "Q1_2D": 3, "Q2_2D": 5, "P1_3D": 1, "P2_3D": 4,
                "Q1_3D": 3, "Q2_3D": 5, "Q2S_2D": 5, "Q2S_3D": 5}


def _exact_monomial(etype, powers):
    if etype.startswith("Q"):
        out = 1.0
        for k in powers:
            out *= 0.0 if k % 2 else 2.0 / (k + 1)
        return out
    # simplex: int x^a y^b (z^c) = a! b! c! / (a + b + c + d)!
    d = len(powers)
    num = np.prod([math.factorial(k) for k in powers])
    return num / math.factorial(sum(powers) + d)


@pytest.mark.parametrize("etype", list(REF_VOLUME))
def test_quadrature_exactness(etype):
    xi, w = O.quadrature(etype)
    dim = xi.shape[1]
    assert abs(w.sum() - REF_VOLUME[etype]) < 1e-15
    deg = EXACT_DEGREE[etype]
    rng = range(deg + 1)
    for powers in np.ndindex(*([deg + 1] * dim)):
        if etype.startswith("P") and sum(powers) > deg:
            continue
        if etype.startswith("Q") and max(powers) > deg:
            continue
        approx = np.sum(w * np.prod(xi ** np.array(powers), axis=1))
        assert abs(approx - _exact_monomial(etype, powers)) < 1e-14, powers
    del rng


def test_keast_matches_printed_table():
    """The oracle uses exact surds; the paper prints 15 digits."""
    tab = np.loadtxt(os.path.join(GOLD, "keast_tet11.txt"))
    xi, w = O.quadrature("P2_3D")
    assert np.max(np.abs(xi - tab[:, :3])) < 1e-14
    assert np.max(np.abs(w - tab[:, 3])) < 2e-15
    # the printed weights sum to 1/6 only up to their truncation
    assert abs(-74 / 5625 + 4 * 343 / 45000 + 6 * 56 / 2250 - 1 / 6) < 1e-16


def _golden_nodes():
    out = {}
    for line in open(os.path.join(GOLD, "ref_nodes.txt")):
        if line.startswith("#") or not line.strip():
            continue
        et, k, *x = line.split()
        out.setdefault(et, {})[int(k)] = np.array([float(v) for v in x])
    return out


def _node_coords(etype):
    if etype == "Q2S_3D":
        g = _golden_nodes()
        return np.array([g["Q1_3D"][k] for k in range(1, 9)] +
                        [g["Q2_3D"][k] for k in range(9, 21)])
    if etype == "Q2S_2D":
        return W.QUAD9_LOCAL[:8].astype(float)
    if etype == "Q2_3D":
        return W.HEX27_LOCAL.astype(float)
    if etype == "Q1_3D":
        return W.HEX8_LOCAL.astype(float)
    if etype == "Q2_2D":
        return W.QUAD9_LOCAL.astype(float)
    if etype == "Q1_2D":
        return np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], float)
    if etype == "P1_2D":
        return np.array([[0, 0], [1, 0], [0, 1]], float)
    g = _golden_nodes()[etype]
    return np.array([g[k + 1] for k in range(len(g))])


def test_golden_nodes_agree_with_input_convention():
    g = _golden_nodes()
    for k in range(1, 9):
        assert np.array_equal(g["Q1_3D"][k], W.HEX27_LOCAL[k - 1])
    for k in range(9, 21):
        assert np.array_equal(g["Q2_3D"][k], W.HEX27_LOCAL[k - 1])


@pytest.mark.parametrize("etype", list(REF_VOLUME))
def test_basis_kronecker_unity_gradients(etype):
    nodes = _node_coords(etype)
    n_p = nodes.shape[0]
    dim = nodes.shape[1]
    for k in range(n_p):
        phi, _ = O.basis(etype, nodes[k])
        e = np.zeros(n_p)
        e[k] = 1.0
        assert np.max(np.abs(phi - e)) < 1e-14
    rng = np.random.default_rng(1)
    for _ in range(5):
        x = rng.uniform(0, 0.3, dim) if etype.startswith("P") else rng.uniform(-1, 1, dim)
        phi, dphi = O.basis(etype, x)
        assert abs(phi.sum() - 1) < 1e-14
        assert np.max(np.abs(dphi.sum(axis=0))) < 1e-13
        # gradients against central differences of the values
        h = 1e-6
        for d in range(dim):
            xp, xm = x.copy(), x.copy()
            xp[d] += h
            xm[d] -= h
            fd = (O.basis(etype, xp)[0] - O.basis(etype, xm)[0]) / (2 * h)
            assert np.max(np.abs(fd - dphi[:, d])) < 1e-8


@pytest.mark.parametrize("etype", ["Q2_2D", "Q2_3D", "P1_3D", "Q1_3D"])
def test_basis_reproduces_polynomials(etype):
    """Lagrange interpolation reproduces the element's polynomial space."""
    nodes = _node_coords(etype)
    dim = nodes.shape[1]
    rng = np.random.default_rng(2)
    if etype in ("Q2_2D", "Q2_3D"):
        def f(x):  # tensor-quadratic
            return np.prod([1 + 0.3 * x[d] - 0.7 * x[d] ** 2 for d in range(dim)])
    else:
        def f(x):
            return 0.4 - 0.2 * x[0] + 1.1 * x[-1]
    vals = np.array([f(n) for n in nodes])
    for _ in range(5):
        x = rng.uniform(-1, 1, dim) if etype.startswith("Q") else rng.uniform(0, 0.3, dim)
        phi, _ = O.basis(etype, x)
        assert abs(phi @ vals - f(x)) < 1e-13


@pytest.mark.parametrize("etype", ["Q2S_2D", "Q2S_3D"])
def test_serendipity_space(etype):
    """The serendipity basis reproduces every complete quadratic and the
    cubic terms of its space (x^2 y, x y^2; in 3D also x y z and the
    x_i^2 x_j products), but not the biquadratic x^2 y^2 (that is the
    9- / 27-node space): interpolation at the nodes is exact for the first,
    not for the second."""
    nodes = _node_coords(etype)
    dim = nodes.shape[1]
    rng = np.random.default_rng(6)
    c = rng.standard_normal(20)
    if dim == 2:
        def f(x):
            a, b = x
            return (c[0] + c[1] * a + c[2] * b + c[3] * a * a + c[4] * a * b + c[5] * b * b
                    + c[6] * a * a * b + c[7] * a * b * b)

        def g(x):
            return x[0] ** 2 * x[1] ** 2
    else:
        def f(x):
            a, b, z = x
            return (c[0] + c[1] * a + c[2] * b + c[3] * z + c[4] * a * a + c[5] * b * b
                    + c[6] * z * z + c[7] * a * b + c[8] * b * z + c[9] * a * z + c[10] * a * b * z
                    + c[11] * a * a * b + c[12] * a * a * z + c[13] * b * b * a
                    + c[14] * b * b * z + c[15] * z * z * a + c[16] * z * z * b)

        def g(x):
            return x[0] ** 2 * x[1] ** 2
    vals = np.array([f(n) for n in nodes])
    gv = np.array([g(n) for n in nodes])
    miss = 0.0
    for _ in range(5):
        x = rng.uniform(-1, 1, dim)
        phi, _ = O.basis(etype, x)
        assert abs(phi @ vals - f(x)) < 1e-13
        miss = max(miss, abs(phi @ gv - g(x)))
    assert miss > 1e-3


def test_serendipity_face_integrals():
    """Integrals of the 8-node serendipity functions over the reference
    square: -1/3 for a vertex, 4/3 for an edge midpoint (closed form); the
    consistent load of a uniform traction on such a face is -A/12 per
    vertex and A/3 per midpoint."""
    xi, w = O.quadrature("Q2S_2D")
    tot = np.zeros(8)
    for q in range(len(w)):
        phi, _ = O.basis("Q2S_2D", xi[q])
        tot += w[q] * phi
    assert np.max(np.abs(tot[:4] + 1 / 3)) < 1e-14
    assert np.max(np.abs(tot[4:] - 4 / 3)) < 1e-14


def test_p2_reproduces_quadratics():
    nodes = _node_coords("P2_3D")

    def f(x):
        return 1 + x[0] - 2 * x[1] * x[2] + 0.5 * x[0] ** 2 + 3 * x[1] ** 2

    vals = np.array([f(n) for n in nodes])
    rng = np.random.default_rng(3)
    for _ in range(5):
        x = rng.uniform(0, 0.3, 3)
        phi, _ = O.basis("P2_3D", x)
        assert abs(phi @ vals - f(x)) < 1e-13


MESHES = {
    "P1_2D": lambda: W.mesh_p1_2d(3, 2, 1.5, 1.0),
    "Q1_2D": lambda: W.mesh_q1_2d(3, 2, 1.5, 1.0),
    "Q2_2D": lambda: W.mesh_q2_2d(3, 2, 1.5, 1.0),
    "P1_3D": lambda: W.mesh_tet_3d(2, 2, 1, 1.0, 1.0, 0.5, order=1),
    "P2_3D": lambda: W.mesh_tet_3d(2, 2, 1, 1.0, 1.0, 0.5, order=2),
    "Q1_3D": lambda: W.mesh_q1_3d(2, 2, 1, 1.0, 1.0, 0.5),
    "Q2_3D": lambda: W.mesh_q2_3d(2, 2, 1, 1.0, 1.0, 0.5),
    "Q2S_2D": lambda: W.mesh_q2s_2d(3, 2, 1.5, 1.0),
    "Q2S_3D": lambda: W.mesh_q2s_3d(2, 2, 1, 1.0, 1.0, 0.5),
}


def _distort(mesh, seed=0, amp=0.08):
    """Move every node by a smooth map (keeps straight-sided simplices only
    affine-consistent when amp=0)."""
    x = mesh.coord.copy()
    if mesh.dim == 2:
        x[0] += amp * np.sin(2.0 * x[1]) * x[0]
        x[1] += amp * np.cos(1.5 * x[0]) * x[1]
    else:
        x[0] += amp * np.sin(2.0 * x[1]) * x[0]
        x[1] += amp * np.cos(1.5 * x[2]) * x[1]
        x[2] += amp * np.sin(x[0]) * x[2]
    return W.Mesh(mesh.etype, x, mesh.elem)


@pytest.mark.parametrize("etype", list(MESHES))
def test_geometry_volume_and_affine(etype):
    mesh = MESHES[etype]()
    dphi, w = O.geometry(mesh)
    lo, hi = mesh.coord.min(axis=1), mesh.coord.max(axis=1)
    assert abs(w.sum() - np.prod(hi - lo)) < 1e-13
    # affine image of the mesh: x -> A x + b scales weights by det A and maps
    # gradients by A^{-T}
    A = np.array([[1.2, 0.3, 0.1], [-0.2, 0.9, 0.05], [0.1, 0.0, 1.1]])[:mesh.dim, :mesh.dim]
    m2 = W.Mesh(mesh.etype, A @ mesh.coord + 0.7, mesh.elem)
    dphi2, w2 = O.geometry(m2)
    assert np.allclose(w2, w * np.linalg.det(A), rtol=1e-13, atol=0)
    assert np.allclose(dphi2, dphi @ np.linalg.inv(A), rtol=0, atol=1e-12)


@pytest.mark.parametrize("etype", list(MESHES))
def test_patch_test_strain(etype):
    """A linear displacement field gives the constant strain sym(G) at every
    integration point, also on a distorted mesh (isoparametric elements
    reproduce linear fields)."""
    mesh = MESHES[etype]()
    if etype.startswith("Q"):
        mesh = _distort(mesh)
    dphi, w = O.geometry(mesh)
    rng = np.random.default_rng(4)
    d = mesh.dim
    Gm = rng.standard_normal((d, d))
    u = (Gm @ mesh.coord).T.reshape(-1)
    eps = O.strain(mesh, dphi, u)
    S = 0.5 * (Gm + Gm.T)
    if d == 3:
        ref = np.array([S[0, 0], S[1, 1], S[2, 2], 2 * S[0, 1], 2 * S[1, 2], 2 * S[0, 2]])
    else:
        ref = np.array([S[0, 0], S[1, 1], 0, 2 * S[0, 1], 0, 0])
    assert np.max(np.abs(eps - ref)) < 1e-12


def test_structured_p1_counts():
    """Element / node / integration-point counts of the P1 square workload."""
    wl = W.workload_p1_square()
    assert (wl.mesh.n_elems, wl.mesh.n_nodes, wl.mesh.n_int) == (2048, 1089, 2048)


def _lshape_table():
    rows = []
    for line in open(os.path.join(GOLD, "lshape_sizes.txt")):
        if line.startswith("#") or not line.strip():
            continue
        d, lev, el, n = line.split()
        rows.append((int(d), int(lev), el, int(n)))
    return rows


LSHAPE_ETYPE = {(2, "P1"): "P1_2D", (2, "Q1"): "Q1_2D", (2, "Q2"): "Q2S_2D",
                (3, "P1"): "P1_3D", (3, "P2"): "P2_3D", (3, "Q1"): "Q1_3D", (3, "Q2"): "Q2S_3D"}


@pytest.mark.parametrize("row", [r for r in _lshape_table() if (r[0] == 2 and r[1] <= 5) or
                                 (r[0] == 3 and r[1] <= 2)], ids=str)
def test_lshape_mesh_sizes_match_paper_tables(row):
    """The L-shaped domain generator reproduces the matrix sizes printed in
    the paper's Tables 1 and 2 (levels small enough to build in a test)."""
    dim, level, el, n = row
    mesh = W.mesh_lshape(LSHAPE_ETYPE[(dim, el)], level)
    assert mesh.n_dof == n
    # the domain: area 75 (2D) or volume 75 (3D), covered exactly once
    dphi, w = O.geometry(mesh)
    assert abs(w.sum() - 75.0) < 1e-9


def test_lshape_vm_mesh_is_the_papers():
    """The von Mises experiment of Section 8.2 runs on the level-2 3D mesh of
    20-node hexahedra with 23,929 nodes."""
    mesh = W.mesh_lshape("Q2S_3D", 2)
    assert mesh.n_nodes == 23929
