"""Seeded synthetic inputs for the elastoplastic hot path.

This module is the only code shared by the HIP path and the FP64 oracle.  It
produces *inputs* only: node coordinates, element connectivity, Dirichlet
masks, consistent nodal load vectors for uniform tractions / body forces on
structured grids, and seeded initial plastic states.  It contains none of the
method's arithmetic (no basis-function gradients, no Jacobians, no return
mapping, no assembly).

Conventions (shared input format):
  * coord : float64 array (dim, n_nodes), Cartesian node coordinates.
  * elem  : int32 array (n_elems, n_p), 0-based node ids per element, in the
            local node order of the reference element (paper Appendix for P1,
            P2 tetrahedra, Q1 hexahedra and the 20-node serendipity
            hexahedron; tensor Lagrange orders for the 9-node quadrilateral
            and the 27-node hexahedron, listed below; the serendipity
            elements use the first 8 / 20 of those nodes).
  * dof numbering is interleaved: dof = dim * node + component (the paper's
            column-major U(:) of a dim x n_n array, Section 5).
  * free  : uint8 array (dim * n_nodes), 1 = free, 0 = Dirichlet.
  * Voigt order 11, 22, 33, 12, 23, 13; strain-type vectors carry doubled
    shears, stress-type vectors do not (Section 5).  Plane-strain state is
    stored with the four components 11, 22, 33, 12.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# Local node coordinates of the 27-node hexahedron: the 20 nodes of the
# paper's Q2 hexahedron (Appendix) followed by the six face centres
# (-xi3, +xi3, -xi2, +xi1, +xi2, -xi1) and the element centre.
HEX27_LOCAL = np.array(
    [[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
     [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1],
     [0, -1, -1], [1, 0, -1], [0, 1, -1], [-1, 0, -1],
     [0, -1, 1], [1, 0, 1], [0, 1, 1], [-1, 0, 1],
     [-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0],
     [0, 0, -1], [0, 0, 1], [0, -1, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0],
     [0, 0, 0]], dtype=np.int64)

# Local node coordinates of the 9-node quadrilateral: vertices
# counter-clockwise, edge midpoints (bottom, right, top, left), centre.
QUAD9_LOCAL = np.array(
    [[-1, -1], [1, -1], [1, 1], [-1, 1],
     [0, -1], [1, 0], [0, 1], [-1, 0], [0, 0]], dtype=np.int64)

# Q1 hexahedron vertex order of the paper's Appendix.
HEX8_LOCAL = HEX27_LOCAL[:8]

# P2 tetrahedron edge nodes of the paper's Appendix: (vertex a, vertex b).
TET10_EDGES = [(0, 1), (1, 2), (0, 2), (1, 3), (2, 3), (0, 3)]

ELEMENT_INFO = {
    # name: (dim, n_p, n_q)
    "P1_2D": (2, 3, 1),
    "Q1_2D": (2, 4, 4),
    "Q2_2D": (2, 9, 9),
    "P1_3D": (3, 4, 1),
    "P2_3D": (3, 10, 11),
    "Q1_3D": (3, 8, 8),
    "Q2_3D": (3, 27, 27),
    "Q2S_2D": (2, 8, 9),     # serendipity (the paper's Q2): 3x3 Gauss points
    "Q2S_3D": (3, 20, 27),   # serendipity 20-node hexahedron: 3x3x3
}


@dataclass
class Mesh:
    etype: str              # key of ELEMENT_INFO
    coord: np.ndarray       # (dim, n_n) float64
    elem: np.ndarray        # (n_e, n_p) int32
    dim: int = field(init=False)
    n_p: int = field(init=False)
    n_q: int = field(init=False)

    def __post_init__(self):
        self.dim, self.n_p, self.n_q = ELEMENT_INFO[self.etype]
        self.coord = np.ascontiguousarray(self.coord, dtype=np.float64)
        self.elem = np.ascontiguousarray(self.elem, dtype=np.int32)
        assert self.coord.shape[0] == self.dim
        assert self.elem.shape[1] == self.n_p

    @property
    def n_nodes(self) -> int:
        return self.coord.shape[1]

    @property
    def n_elems(self) -> int:
        return self.elem.shape[0]

    @property
    def n_int(self) -> int:
        return self.n_elems * self.n_q

    @property
    def n_dof(self) -> int:
        return self.dim * self.n_nodes


# --------------------------------------------------------------------------
# Structured meshes
# --------------------------------------------------------------------------

def _grid2(nx, ny, lx, ly):
    x = np.linspace(0.0, lx, nx + 1)
    y = np.linspace(0.0, ly, ny + 1)
    X, Y = np.meshgrid(x, y, indexing="xy")  # (ny+1, nx+1), i fastest when flattened
    return np.vstack([X.ravel(), Y.ravel()])


def _grid3(nx, ny, nz, lx, ly, lz):
    x = np.linspace(0.0, lx, nx + 1)
    y = np.linspace(0.0, ly, ny + 1)
    z = np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")  # (nz+1, ny+1, nx+1)
    return np.vstack([X.ravel(), Y.ravel(), Z.ravel()])


def mesh_p1_2d(nx, ny, lx, ly) -> Mesh:
    """Squares split into (n00, n10, n11) and (n00, n11, n01)."""
    coord = _grid2(nx, ny, lx, ly)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i, j = i.ravel(), j.ravel()
    n00 = i + (nx + 1) * j
    n10 = n00 + 1
    n01 = n00 + nx + 1
    n11 = n01 + 1
    t1 = np.stack([n00, n10, n11], axis=1)
    t2 = np.stack([n00, n11, n01], axis=1)
    elem = np.stack([t1, t2], axis=1).reshape(-1, 3)
    return Mesh("P1_2D", coord, elem)


def mesh_q1_2d(nx, ny, lx, ly) -> Mesh:
    coord = _grid2(nx, ny, lx, ly)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    n00 = (i + (nx + 1) * j).ravel()
    elem = np.stack([n00, n00 + 1, n00 + nx + 2, n00 + nx + 1], axis=1)
    return Mesh("Q1_2D", coord, elem)


def mesh_q2_2d(nx, ny, lx, ly) -> Mesh:
    """9-node quadrilaterals on the doubled grid of (2nx+1) x (2ny+1) nodes."""
    coord = _grid2(2 * nx, 2 * ny, lx, ly)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ci, cj = (2 * i + 1).ravel(), (2 * j + 1).ravel()
    cols = []
    for a, b in QUAD9_LOCAL:
        cols.append((ci + a) + (2 * nx + 1) * (cj + b))
    return Mesh("Q2_2D", coord, np.stack(cols, axis=1))


def mesh_q1_3d(nx, ny, nz, lx, ly, lz) -> Mesh:
    coord = _grid3(nx, ny, nz, lx, ly, lz)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sx, sy = nx + 1, (nx + 1) * (ny + 1)
    cols = []
    for a, b, c in HEX8_LOCAL:
        cols.append(((i + (a + 1) // 2) + sx * (j + (b + 1) // 2) + sy * (k + (c + 1) // 2)).ravel())
    return Mesh("Q1_3D", coord, np.stack(cols, axis=1))


def mesh_q2_3d(nx, ny, nz, lx, ly, lz) -> Mesh:
    """27-node hexahedra on the doubled grid."""
    coord = _grid3(2 * nx, 2 * ny, 2 * nz, lx, ly, lz)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sx, sy = 2 * nx + 1, (2 * nx + 1) * (2 * ny + 1)
    ci, cj, ck = (2 * i + 1).ravel(), (2 * j + 1).ravel(), (2 * k + 1).ravel()
    cols = [(ci + a) + sx * (cj + b) + sy * (ck + c) for a, b, c in HEX27_LOCAL]
    return Mesh("Q2_3D", coord, np.stack(cols, axis=1))


def _compact(etype, coord, elem):
    """Drop the nodes no element uses; the kept nodes keep their order."""
    used = np.zeros(coord.shape[1], dtype=bool)
    used[elem.ravel()] = True
    new_id = np.cumsum(used) - 1
    return Mesh(etype, coord[:, used], new_id[elem].astype(np.int32))


def mesh_q2s_2d(nx, ny, lx, ly) -> Mesh:
    """8-node serendipity quadrilaterals: the 9-node mesh without the
    element centres."""
    m = mesh_q2_2d(nx, ny, lx, ly)
    return _compact("Q2S_2D", m.coord, m.elem[:, :8])


def mesh_q2s_3d(nx, ny, nz, lx, ly, lz) -> Mesh:
    """20-node serendipity hexahedra (the paper's Q2 element, Appendix): the
    27-node mesh without the face and element centres."""
    m = mesh_q2_3d(nx, ny, nz, lx, ly, lz)
    return _compact("Q2S_3D", m.coord, m.elem[:, :20])


def _kuhn_tets():
    """Six tetrahedra of the unit cube along the diagonal v000 -> v111, each
    positively oriented (vertex lists in unit-cube corner coordinates)."""
    tets = []
    for perm in itertools.permutations(range(3)):
        v = [np.zeros(3, dtype=np.int64)]
        for ax in perm:
            nv = v[-1].copy()
            nv[ax] = 1
            v.append(nv)
        M = np.array([v[1] - v[0], v[2] - v[0], v[3] - v[0]])
        if round(np.linalg.det(M)) < 0:
            v[2], v[3] = v[3], v[2]
        tets.append(v)
    return tets


def mesh_tet_3d(nx, ny, nz, lx, ly, lz, order) -> Mesh:
    """Kuhn split (6 tetrahedra per cube).  order=2 puts the P2 nodes on the
    doubled grid; order=1 uses the plain grid."""
    m = 2 if order == 2 else 1
    coord = _grid3(m * nx, m * ny, m * nz, lx, ly, lz)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = (m * i).ravel(), (m * j).ravel(), (m * k).ravel()
    sx, sy = m * nx + 1, (m * nx + 1) * (m * ny + 1)

    def nid(p):
        return (i + p[0]) + sx * (j + p[1]) + sy * (k + p[2])

    out = []
    for tet in _kuhn_tets():
        vv = [m * np.asarray(v) for v in tet]
        cols = [nid(v) for v in vv]
        if order == 2:
            for a, b in TET10_EDGES:
                cols.append(nid((vv[a] + vv[b]) // 2))
        out.append(np.stack(cols, axis=1))
    n_p = 10 if order == 2 else 4
    elem = np.stack(out, axis=1).reshape(-1, n_p)
    return Mesh("P2_3D" if order == 2 else "P1_3D", coord, elem)


# --------------------------------------------------------------------------
# The paper's L-shaped domain (Section 8.1, the figure of the elastic
# problem): [0,10]^2 without [0,5)x[0,5), extruded over [0,1] in 3D.  Level l
# has element size h = 2^-l (10*2^l elements per box side in plane, 2^l
# through the thickness), which reproduces the matrix sizes of the paper's
# Tables 1 and 2.
# --------------------------------------------------------------------------

LSHAPE_GENERATORS = {
    "P1_2D": lambda n, m: mesh_p1_2d(n, n, 10.0, 10.0),
    "Q1_2D": lambda n, m: mesh_q1_2d(n, n, 10.0, 10.0),
    "Q2_2D": lambda n, m: mesh_q2_2d(n, n, 10.0, 10.0),
    "Q2S_2D": lambda n, m: mesh_q2s_2d(n, n, 10.0, 10.0),
    "P1_3D": lambda n, m: mesh_tet_3d(n, n, m, 10.0, 10.0, 1.0, order=1),
    "P2_3D": lambda n, m: mesh_tet_3d(n, n, m, 10.0, 10.0, 1.0, order=2),
    "Q1_3D": lambda n, m: mesh_q1_3d(n, n, m, 10.0, 10.0, 1.0),
    "Q2_3D": lambda n, m: mesh_q2_3d(n, n, m, 10.0, 10.0, 1.0),
    "Q2S_3D": lambda n, m: mesh_q2s_3d(n, n, m, 10.0, 10.0, 1.0),
}


def mesh_lshape(etype, level) -> Mesh:
    """Structured mesh of the L-shaped domain: the box mesh with the
    elements whose vertex centroid lies in [0,5)x[0,5) removed, unused nodes
    dropped."""
    n, m = 10 * 2 ** level, 2 ** level
    box = LSHAPE_GENERATORS[etype](n, m)
    nv = {"P1_2D": 3, "P1_3D": 4, "P2_3D": 4, "Q1_2D": 4, "Q2_2D": 4,
          "Q2S_2D": 4, "Q1_3D": 8, "Q2_3D": 8, "Q2S_3D": 8}[etype]
    cen = box.coord[:, box.elem[:, :nv]].mean(axis=2)  # (dim, n_e)
    keep = ~((cen[0] < 5.0) & (cen[1] < 5.0))
    return _compact(etype, box.coord, box.elem[keep])


# --------------------------------------------------------------------------
# Boundary masks and loads
# --------------------------------------------------------------------------

def free_mask(mesh: Mesh, fixed) -> np.ndarray:
    """fixed: list of (axis, value, components) -> components fixed on the
    plane coord[axis] == value."""
    free = np.ones((mesh.n_nodes, mesh.dim), dtype=np.uint8)
    for axis, value, comps in fixed:
        on = np.abs(mesh.coord[axis] - value) < 1e-12
        for c in comps:
            free[on, c] = 0
    return free.reshape(-1)


def _tensor_face_weights(order):
    # integrals of the 1D Lagrange basis over [0, 1]: linear (1/2, 1/2),
    # quadratic at nodes 0, 1/2, 1: (1/6, 2/3, 1/6)
    return {1: np.array([0.5, 0.5]), 2: np.array([1 / 6, 2 / 3, 1 / 6])}[order]


def nodal_load_structured_face(mesh: Mesh, grid_shape, order, axis, value,
                               direction, magnitude, region=None):
    """Consistent nodal loads of a uniform traction `magnitude` in direction
    `direction` on the face coord[axis]==value of a structured tensor grid
    (Q1 / Q2 elements).  grid_shape = number of elements per axis.

    The face is covered by tensor cells; each cell's nodes get the tensor
    product of the 1D Lagrange integrals times the cell size.  `region`
    optionally restricts to cells whose centre satisfies region(centre)."""
    dim = mesh.dim
    f = np.zeros((mesh.n_nodes, dim))
    npts = [order * n + 1 for n in grid_shape]
    strides = [1, npts[0]] + ([npts[0] * npts[1]] if dim == 3 else [])
    lo = mesh.coord.min(axis=1)
    hi = mesh.coord.max(axis=1)
    hcell = [(hi[a] - lo[a]) / grid_shape[a] for a in range(dim)]
    other = [a for a in range(dim) if a != axis]
    w1 = _tensor_face_weights(order)
    fixed_idx = 0 if abs(value - lo[axis]) < 1e-12 else npts[axis] - 1
    ranges = [range(grid_shape[a]) for a in other]
    for cell in itertools.product(*ranges):
        centre = np.zeros(dim)
        centre[axis] = value
        for a, c in zip(other, cell):
            centre[a] = lo[a] + (c + 0.5) * hcell[a]
        if region is not None and not region(centre):
            continue
        area = np.prod([hcell[a] for a in other])
        for loc in itertools.product(range(order + 1), repeat=len(other)):
            idx = fixed_idx * strides[axis]
            wt = area
            for a, c, l in zip(other, cell, loc):
                idx += (order * c + l) * strides[a]
                wt *= w1[l]
            f[idx, direction] += magnitude * wt
    return f.reshape(-1)


def nodal_load_serendipity_face(mesh: Mesh, axis, value, direction, magnitude):
    """Uniform traction on an axis-aligned boundary plane of a serendipity
    mesh: an 8-node quadrilateral edge of length L gives L/6 to each vertex
    and 2L/3 to the midpoint; a 20-node hexahedron face of area A gives
    -A/12 to each vertex and A/3 to each edge midpoint (the integrals of the
    8-node face functions)."""
    dim = mesh.dim
    nv, nface = (4, 3) if dim == 2 else (8, 8)
    on = np.abs(mesh.coord[axis] - value) < 1e-12
    on_e = on[mesh.elem]                          # (n_e, n_p)
    faces = np.nonzero(on_e.sum(axis=1) == nface)[0]
    f = np.zeros((mesh.n_nodes, dim))
    others = [a for a in range(dim) if a != axis]
    for e in faces:
        nodes = mesh.elem[e]
        sel = np.nonzero(on_e[e])[0]
        x = mesh.coord[:, nodes[sel]]
        size = np.prod([x[a].max() - x[a].min() for a in others])
        for loc in sel:
            if dim == 2:
                wgt = size / 6.0 if loc < nv else 2.0 * size / 3.0
            else:
                wgt = -size / 12.0 if loc < nv else size / 3.0
            f[nodes[loc], direction] += magnitude * wgt
    return f.reshape(-1)


def nodal_load_p1_edge_2d(mesh: Mesh, axis, value, direction, magnitude):
    """Uniform traction on a straight boundary line of a P1 triangle mesh:
    each boundary edge of length L gives L/2 to each end node."""
    on = np.abs(mesh.coord[axis] - value) < 1e-12
    idx = np.nonzero(on)[0]
    other = 1 - axis
    order = idx[np.argsort(mesh.coord[other, idx])]
    f = np.zeros((mesh.n_nodes, 2))
    for a, b in zip(order[:-1], order[1:]):
        L = abs(mesh.coord[other, b] - mesh.coord[other, a])
        f[a, direction] += magnitude * L / 2
        f[b, direction] += magnitude * L / 2
    return f.reshape(-1)


def nodal_load_body_q2_2d(mesh: Mesh, nx, ny, direction, magnitude):
    """Uniform body force on 9-node quadrilaterals of a structured grid:
    nodal weights are tensor products of (1/6, 2/3, 1/6) times the cell area."""
    lx = mesh.coord[0].max() - mesh.coord[0].min()
    ly = mesh.coord[1].max() - mesh.coord[1].min()
    area = (lx / nx) * (ly / ny)
    w1 = _tensor_face_weights(2)
    wl = np.array([w1[a + 1] * w1[b + 1] for a, b in QUAD9_LOCAL]) * area
    f = np.zeros((mesh.n_nodes, 2))
    np.add.at(f[:, direction], mesh.elem.ravel(), np.tile(wl, mesh.n_elems) * magnitude)
    return f.reshape(-1)


def nodal_load_p2_face_3d(mesh: Mesh, nx, ny, nz, axis, value, direction,
                          magnitude, region=None):
    """Uniform traction on a boundary plane of the Kuhn P2 tetrahedral mesh.
    The six-node boundary triangles carry 0 at vertices and area/3 at edge
    midpoints.  Boundary triangles are the faces of tetrahedra whose three
    vertices lie on the plane."""
    f = np.zeros((mesh.n_nodes, 3))
    faces = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
    # local edge node index for vertex pair
    edge_node = {}
    for k, (a, b) in enumerate(TET10_EDGES):
        edge_node[(a, b)] = 4 + k
        edge_node[(b, a)] = 4 + k
    X = mesh.coord
    for e in range(mesh.n_elems):
        nodes = mesh.elem[e]
        for fc in faces:
            vs = nodes[list(fc)]
            if not np.all(np.abs(X[axis, vs] - value) < 1e-12):
                continue
            centre = X[:, vs].mean(axis=1)
            if region is not None and not region(centre):
                continue
            p = X[:, vs].T
            area = 0.5 * np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[0]))
            for a, b in ((0, 1), (1, 2), (0, 2)):
                n = nodes[edge_node[(fc[a], fc[b])]]
                f[n, direction] += magnitude * area / 3.0
    return f.reshape(-1)


# --------------------------------------------------------------------------
# Materials (input parameters only)
# --------------------------------------------------------------------------

@dataclass
class Material:
    model: str          # "VM" (von Mises, linear kinematic hardening),
                        # "DP" (Drucker-Prager, linear cohesion hardening, a=0 perfect)
    E: float
    nu: float
    Y: float = 0.0      # VM yield level on |dev(sigma) - beta|
    a: float = 0.0      # hardening modulus
    eta: float = 0.0    # DP friction parameter
    c: float = 0.0      # DP cohesion parameter

    @property
    def shear(self):
        return self.E / (2.0 * (1.0 + self.nu))

    @property
    def bulk(self):
        return self.E / (3.0 * (1.0 - 2.0 * self.nu))


def dp_parameters(c0, phi, plane_strain):
    """eta and c from cohesion c0 and friction angle phi (Section 8.3)."""
    if plane_strain:
        t = math.tan(phi)
        s = math.sqrt(9.0 + 12.0 * t * t)
        return 3.0 * t / s, 3.0 * c0 / s
    sphi = math.sin(phi)
    d = math.sqrt(3.0) * (3.0 + sphi)
    return 6.0 * sphi / d, c0 * 6.0 * math.cos(phi) / d


VM_MATERIAL = Material("VM", E=206900.0, nu=0.29, Y=450.0 * math.sqrt(2.0 / 3.0), a=10000.0)


def dp_material_2d():
    eta, c = dp_parameters(450.0, math.pi / 9.0, plane_strain=True)
    return Material("DP", E=20000.0, nu=0.49, eta=eta, c=c, a=0.0)


def dp_material_3d_hardening():
    eta, c = dp_parameters(450.0, math.pi / 9.0, plane_strain=False)
    return Material("DP", E=20000.0, nu=0.3, eta=eta, c=c, a=2000.0)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    mesh: Mesh
    material: Material
    free: np.ndarray
    f_unit: np.ndarray            # load vector for unit load factor
    load_factors: np.ndarray      # one factor per load step
    note: str = ""
    u_dir_unit: np.ndarray = None  # displacement control: prescribed u per unit u_D

    def f(self, k):
        return self.load_factors[k] * self.f_unit


def workload_p1_square(n=32) -> Workload:
    """Plane strain 10x10 square of P1 triangles, von Mises linear kinematic
    hardening; sliding left / bottom, top traction ramped to 1.2*sigma_y = 540
    in 10 steps."""
    mesh = mesh_p1_2d(n, n, 10.0, 10.0)
    free = free_mask(mesh, [(0, 0.0, [0]), (1, 0.0, [1])])
    f = nodal_load_p1_edge_2d(mesh, 1, 10.0, 1, 1.0)
    return Workload("p1_square_vm", mesh, VM_MATERIAL, free, f,
                    54.0 * np.arange(1, 11, dtype=np.float64))


def workload_q2_slope(nx=512, ny=256, gamma_max=60.0, steps=20) -> Workload:
    """Plane strain 40x20 rectangle of 9-node Q2 quads, Drucker-Prager perfect
    plasticity; bottom fixed, body force (0, -gamma) ramped over 20 steps."""
    mesh = mesh_q2_2d(nx, ny, 40.0, 20.0)
    free = free_mask(mesh, [(1, 0.0, [0, 1])])
    f = nodal_load_body_q2_2d(mesh, nx, ny, 1, -1.0)
    lf = gamma_max * np.arange(1, steps + 1, dtype=np.float64) / steps
    return Workload("q2_slope_dp", mesh, dp_material_2d(), free, f, lf)


def workload_q1_cube(n=64) -> Workload:
    """Unit cube of Q1 hexahedra, von Mises as the P1 square; sliding on the
    three coordinate planes; top traction +x3 ramped 54k, k=1..10."""
    mesh = mesh_q1_3d(n, n, n, 1.0, 1.0, 1.0)
    free = free_mask(mesh, [(0, 0.0, [0]), (1, 0.0, [1]), (2, 0.0, [2])])
    f = nodal_load_structured_face(mesh, (n, n, n), 1, 2, 1.0, 2, 1.0)
    return Workload("q1_cube_vm", mesh, VM_MATERIAL, free, f,
                    54.0 * np.arange(1, 11, dtype=np.float64))


def cyclic_factors(steps: int = 30, t_max: float = 540.0):
    """Traction history zeta(t) * t_max at t_k = 4k/steps, k = 1..steps, with
    zeta piecewise linear: 0 -> 1 on [0, 1], down to -1 at t = 3, back to 0
    at t = 4 (the loading / unloading / reverse loading history of the
    paper's von Mises example, Section 8.2)."""
    out = []
    for k in range(1, steps + 1):
        t = 4.0 * k / steps
        z = t if t <= 1.0 else (1.0 - (t - 1.0) if t <= 3.0 else -1.0 + (t - 3.0))
        out.append(z * t_max)
    return np.array(out)


def workload_q1_cube_cyclic(n=64, steps=30) -> Workload:
    """The Q1 cube under the cyclic traction history (learned warm start
    workload): same mesh, material and supports as workload_q1_cube."""
    wl = workload_q1_cube(n)
    return Workload("q1_cube_vm_cyclic", wl.mesh, wl.material, wl.free, wl.f_unit,
                    cyclic_factors(steps, 540.0))


def workload_lshape_vm(level=2, steps=40) -> Workload:
    """The paper's von Mises example (Section 8.2): the L-shaped domain of
    20-node serendipity hexahedra (level 2: 23,929 nodes), von Mises with
    linear kinematic hardening (E = 206900, nu = 0.29, a = 10000,
    Y = 450 sqrt(2/3)), symmetry conditions on x1 = 0 and x2 = 0 (and
    u3 = 0 on x3 = 0), traction zeta(t) * 200 on the top x2 = 10 in +x2
    along the cyclic history at t_k = 4k/steps."""
    mesh = mesh_lshape("Q2S_3D", level)
    free = free_mask(mesh, [(0, 0.0, [0]), (1, 0.0, [1]), (2, 0.0, [2])])
    f = nodal_load_serendipity_face(mesh, 1, 10.0, 1, 1.0)
    return Workload("lshape_vm_cyclic", mesh, VM_MATERIAL, free, f, cyclic_factors(steps, 200.0))


def dp_strip_footing_material(phi=math.pi / 9, c0=450.0, E=1e7, nu=0.48, plane=True):
    """Drucker-Prager parameters of the strip-footing example (Section 8.3):
    eta and c from the friction angle phi and the cohesion c0 by
    dp_parameters (the plane strain fit or the 3D fit)."""
    eta, c = dp_parameters(c0, phi, plane_strain=plane)
    return Material("DP", E=E, nu=nu, eta=eta, c=c, a=0.0)


def workload_strip_footing(n=32, etype="Q2_2D", phi=math.pi / 9, c0=450.0) -> Workload:
    """The strip-footing example of Section 8.3 in plane strain: the square
    [0,10]^2 on n x n elements, zero normal displacement on the left, right
    and bottom sides, the footing 0 <= x1 <= 1 on the top pushed down by the
    prescribed vertical displacement u_D (no forces), Drucker-Prager perfect
    plasticity E = 1e7, nu = 0.48, c0 = 450, phi = pi/9."""
    make = {"Q2_2D": mesh_q2_2d, "Q2S_2D": mesh_q2s_2d, "Q1_2D": mesh_q1_2d,
            "P1_2D": mesh_p1_2d}[etype]
    mesh = make(n, n, 10.0, 10.0)
    free = free_mask(mesh, [(0, 0.0, [0]), (0, 10.0, [0]), (1, 0.0, [1])])
    x = mesh.coord
    foot = np.nonzero((np.abs(x[1] - 10.0) < 1e-12) & (x[0] <= 1.0 + 1e-12))[0]
    free[2 * foot + 1] = 0
    ud = np.zeros(mesh.n_dof)
    ud[2 * foot + 1] = -1.0
    return Workload("strip_footing_dp", mesh, dp_strip_footing_material(phi, c0), free,
                    np.zeros(mesh.n_dof), np.zeros(0), note=f"footing nodes {len(foot)}",
                    u_dir_unit=ud)


def _block_bcs(mesh):
    return free_mask(mesh, [(2, 0.0, [0, 1, 2]), (0, 0.0, [0]), (0, 2.0, [0]),
                            (1, 0.0, [1]), (1, 1.0, [1])])


def workload_q2_block(nx=32, ny=16, nz=16, q_max=4000.0, steps=20) -> Workload:
    """2x1x1 block of 27-node hexahedra, Drucker-Prager with linear hardening;
    bottom fixed, sides sliding, downward pressure on the strip x1 <= 0.5 of
    the top face."""
    mesh = mesh_q2_3d(nx, ny, nz, 2.0, 1.0, 1.0)
    free = _block_bcs(mesh)
    f = nodal_load_structured_face(mesh, (nx, ny, nz), 2, 2, 1.0, 2, -1.0,
                                   region=lambda c: c[0] <= 0.5)
    lf = q_max * np.arange(1, steps + 1, dtype=np.float64) / steps
    return Workload("q2_block_dph", mesh, dp_material_3d_hardening(), free, f, lf)


def workload_p2_block(nx=32, ny=16, nz=16, q_max=4000.0, steps=20) -> Workload:
    mesh = mesh_tet_3d(nx, ny, nz, 2.0, 1.0, 1.0, order=2)
    free = _block_bcs(mesh)
    f = nodal_load_p2_face_3d(mesh, nx, ny, nz, 2, 1.0, 2, -1.0,
                              region=lambda c: c[0] <= 0.5)
    lf = q_max * np.arange(1, steps + 1, dtype=np.float64) / steps
    return Workload("p2_block_dph", mesh, dp_material_3d_hardening(), free, f, lf)


# --------------------------------------------------------------------------
# Seeded initial states
# --------------------------------------------------------------------------

def _unit_deviatoric_strain_voigt(rng, n, plane):
    """n random symmetric deviatoric tensors of unit Frobenius norm, written
    as strain-type Voigt vectors (doubled shears).  plane=True keeps the 13
    and 23 components zero (plane strain)."""
    A = rng.standard_normal((n, 3, 3))
    A = 0.5 * (A + np.transpose(A, (0, 2, 1)))
    if plane:
        A[:, 0, 2] = A[:, 2, 0] = A[:, 1, 2] = A[:, 2, 1] = 0.0
    tr = np.trace(A, axis1=1, axis2=2) / 3.0
    for d in range(3):
        A[:, d, d] -= tr
    nrm = np.sqrt(np.einsum("nij,nij->n", A, A))
    A /= nrm[:, None, None]
    v = np.stack([A[:, 0, 0], A[:, 1, 1], A[:, 2, 2],
                  2 * A[:, 0, 1], 2 * A[:, 1, 2], 2 * A[:, 0, 2]], axis=1)
    return v


def seeded_state(wl: Workload, fraction: float, seed: int = 0):
    """Initial state with the first floor(fraction*n_e) elements of a seeded
    permutation plastic at u = 0.

    von Mises: eps_p0 = (1.5 Y/(2G+a)) * N (N unit deviatoric), beta0 = a*eps_p0
    (as tensors), so the trial deviator norm at u = 0 is exactly 1.5 Y.

    Drucker-Prager: eps_p0 = r * N + v * I/3 with r chosen so that the trial
    deviatoric norm at u = 0 is 1.5*sqrt(2)*c and v = -zeta*c/(eta*K) with
    zeta ~ U(0, 2), so seeded points fall on both the smooth and the apex
    branches where the bulk modulus allows (nu = 0.3); at nu = 0.49 the
    apex test is out of reach and every seeded point is on the cone.

    Returns (ep, beta, kappa) as SoA arrays (n_sc, n_int) / (n_int,), with
    n_sc = 6 in 3D and 4 (11, 22, 33, 12) in plane strain."""
    mesh, mat = wl.mesh, wl.material
    rng = np.random.default_rng(seed)
    n_e, n_q = mesh.n_elems, mesh.n_q
    n_seed = int(math.floor(fraction * n_e))
    seeded = np.zeros(n_e, dtype=bool)
    seeded[rng.permutation(n_e)[:n_seed]] = True
    ip_mask = np.repeat(seeded, n_q)
    n_int = mesh.n_int
    plane = mesh.dim == 2
    N = _unit_deviatoric_strain_voigt(rng, n_int, plane)
    G, K = mat.shear, mat.bulk
    ep6 = np.zeros((n_int, 6))
    beta6 = np.zeros((n_int, 6))
    kappa = np.zeros(n_int)
    if mat.model == "VM":
        ep6 = (1.5 * mat.Y / (2 * G + mat.a)) * N
        beta6 = mat.a * ep6
        beta6[:, 3:] *= 0.5  # stress-type shears
    else:
        r = 1.5 * math.sqrt(2.0) * mat.c / (2 * G)
        zeta = rng.uniform(0.0, 2.0, n_int)
        v = -zeta * mat.c / (mat.eta * K)
        ep6 = r * N
        ep6[:, :3] += (v / 3.0)[:, None]
    ep6[~ip_mask] = 0.0
    beta6[~ip_mask] = 0.0
    if plane:
        sel = [0, 1, 2, 3]
        ep, beta = ep6[:, sel], beta6[:, sel]
    else:
        ep, beta = ep6, beta6
    return (np.ascontiguousarray(ep.T), np.ascontiguousarray(beta.T),
            kappa, seeded)


def random_state(mesh: Mesh, mat: Material, seed: int, scale: float):
    """Generic random history state (for parity tests): eps_p ~ scale*N(0,1)
    per component, beta = a*eps_p as tensors (von Mises) and kappa ~ U(0,
    scale) (Drucker-Prager hardening)."""
    rng = np.random.default_rng(seed)
    n_int = mesh.n_int
    plane = mesh.dim == 2
    ep6 = scale * rng.standard_normal((n_int, 6))
    if plane:
        ep6[:, 4:] = 0.0
    beta6 = np.zeros_like(ep6)
    if mat.model == "VM":
        beta6 = mat.a * ep6
        beta6[:, 3:] *= 0.5
    kappa = scale * rng.uniform(0.0, 1.0, n_int)
    sel = [0, 1, 2, 3] if plane else list(range(6))
    return (np.ascontiguousarray(ep6[:, sel].T), np.ascontiguousarray(beta6[:, sel].T),
            kappa)


def random_displacement(mesh: Mesh, seed: int, scale: float, free=None):
    rng = np.random.default_rng(seed)
    u = scale * rng.standard_normal(mesh.n_dof)
    if free is not None:
        u = u * free
    return u


# --------------------------------------------------------------------------
# Seeded initial weights of the warm-start network
# --------------------------------------------------------------------------

MLP_SIZES = [("W1", (128, 13)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
             ("W3", (7, 128)), ("b3", (7,))]


def mlp_he_uniform(seed):
    """He-uniform initial parameters of the 13-128-128-7 network in the
    library's layout (W[out][in], then bias, per layer): weights uniform in
    +-sqrt(6 / fan_in), biases zero.  float64 vector of 19207 values."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in MLP_SIZES:
        if name.startswith("W"):
            parts.append((rng.uniform(-1.0, 1.0, shape) * math.sqrt(6.0 / shape[1])).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts)
