"""Degenerate and extreme inputs through the C ABI against the oracle: the
smallest mesh of every element kind (one element, or one cell split into
simplices), a state with no plastic point, and one with every point plastic.
Integer outputs bit for bit, FP64 outputs within 1e-12 of the field's scale."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_cases import DPH  # noqa: E402
from paper_1805_04155_amd import _ep  # noqa: E402
from paper_1805_04155_amd import workloads as W  # noqa: E402

RTOL = 1e-12

TINY = {
    "p1_2d": lambda: W.mesh_p1_2d(1, 1, 1.0, 0.8),
    "q1_2d": lambda: W.mesh_q1_2d(1, 1, 1.0, 0.8),
    "q2_2d": lambda: W.mesh_q2_2d(1, 1, 1.0, 0.8),
    "q2s_2d": lambda: W.mesh_q2s_2d(1, 1, 1.0, 0.8),
    "p1_3d": lambda: W.mesh_tet_3d(1, 1, 1, 1.0, 0.8, 0.7, order=1),
    "p2_3d": lambda: W.mesh_tet_3d(1, 1, 1, 1.0, 0.8, 0.7, order=2),
    "q1_3d": lambda: W.mesh_q1_3d(1, 1, 1, 1.0, 0.8, 0.7),
    "q2_3d": lambda: W.mesh_q2_3d(1, 1, 1, 1.0, 0.8, 0.7),
    "q2s_3d": lambda: W.mesh_q2s_3d(1, 1, 1, 1.0, 0.8, 0.7),
}
MATERIALS = {"vm": W.VM_MATERIAL, "dph": DPH}


def _np(t):
    return t.detach().cpu().numpy()


def _setup(name, matname):
    mesh = TINY[name]()
    mat = MATERIALS[matname]
    free = np.ones(mesh.n_dof, dtype=np.uint8)
    on = np.abs(mesh.coord[0] - mesh.coord[0].min()) < 1e-12
    for c in range(mesh.dim):
        free[mesh.dim * np.nonzero(on)[0] + c] = 0
    return mesh, free, mat


def _oracle(mesh, mat, u):
    dphi, w = O.geometry(mesh)
    n = mesh.n_int
    z = np.zeros((n, 6))
    ref = O.constitutive(mat, O.strain(mesh, dphi, u), z, z, np.zeros(n), crit=True)
    rp, ci = O.pattern(mesh)
    _, _, K = O.assemble(mesh, dphi, w, ref["D"], rp, ci)
    F = O.internal_force(mesh, dphi, w, ref["sig"])
    return ref, rp, K, F


def _check_rows(a, b, rp):
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    rmax = np.zeros(len(rp) - 1)
    np.maximum.at(rmax, rows, np.abs(b))
    assert (np.abs(a - b) / rmax[rows]).max() <= RTOL


@pytest.mark.parametrize("mode", ["colours", "rows", "fused"])
@pytest.mark.parametrize("matname", list(MATERIALS))
@pytest.mark.parametrize("name", list(TINY))
@pytest.mark.parametrize("amp", [0.3, 0.6, 300.0])
def test_smallest_mesh(name, matname, amp, mode):
    """One element (or one cell of simplices): mixed plastic sets at amp 0.3
    and 0.6 (none to most points, depending on the element); at amp 300 (times the yield strain) every von Mises point is plastic
    (Drucker-Prager points under strong compression may stay elastic)."""
    mesh, free, mat = _setup(name, matname)
    yld = (mat.Y if mat.model == "VM" else mat.c) / mat.E
    u = W.random_displacement(mesh, 7, amp * yld)
    ref, rp, K, F = _oracle(mesh, mat, u)
    if amp > 1.0 and mat.model == "VM":
        assert ref["flag"].all()  # the input really makes every point plastic
    ctx = _ep.Context(mesh, free, mat, options={
        "assembly": _ep.ASSEMBLY[mode]})
    try:
        sig, _, flag = ctx.constitutive(ctx.tensor(u), D=False)
        assert not O.tie_band(mat, ref["crit"]).any()  # exact branch decisions are meaningful
        assert np.array_equal(_np(flag), ref["flag"])
        ip, el = ctx.plastic()
        pl = np.nonzero(ref["flag"])[0]
        assert np.array_equal(_np(ip), pl)
        assert np.array_equal(_np(el), np.unique(pl // mesh.n_q))
        ctx.assemble_tangent()
        rpg, cig, val = (_np(t) for t in ctx.csr(1))
        assert np.array_equal(rpg, rp) and np.array_equal(cig, ci_of(mesh))
        _check_rows(val, K, rp)
        Fg = _np(ctx.internal_force())
        assert np.abs(Fg - F).max() <= RTOL * np.abs(F).max()
    finally:
        ctx.close()


def ci_of(mesh):
    return O.pattern(mesh)[1]


@pytest.mark.parametrize("name", list(TINY))
def test_no_plastic_point(name):
    """u = 0 from the zero state: no plastic point, empty lists, K_tangent is
    K_elast bit for bit and F = 0 exactly."""
    mesh, free, mat = _setup(name, "vm")
    ctx = _ep.Context(mesh, free, mat)
    try:
        u = torch.zeros(mesh.n_dof, dtype=torch.float64, device="cuda")
        ctx.constitutive(u, sig=False, D=False, flag=False)
        ip, el = ctx.plastic()
        assert ip.numel() == 0 and el.numel() == 0
        ctx.assemble_tangent()
        assert np.array_equal(_np(ctx.csr(1)[2]), _np(ctx.csr(0)[2]))
        assert not _np(ctx.internal_force()).any()
    finally:
        ctx.close()


@pytest.mark.parametrize("order", [1, 2])
def test_fused_rows_many_slots(order):
    """Fused node rows where a node has more plastic elements than one chunk
    of the wavefront holds (Kuhn tetrahedra: 24 around an interior vertex;
    chunks of 16 P1 or 6 P2 elements): every point plastic, K_tangent and
    the row-by-row order of the chunks against the oracle."""
    mesh = W.mesh_tet_3d(3, 3, 3, 1.0, 0.8, 0.7, order=order)
    mat = W.VM_MATERIAL
    n2e = np.bincount(mesh.elem.ravel(), minlength=mesh.n_nodes)
    assert n2e.max() > (16 if order == 1 else 6)
    free = np.ones(mesh.n_dof, dtype=np.uint8)
    on = np.abs(mesh.coord[0] - mesh.coord[0].min()) < 1e-12
    for c in range(mesh.dim):
        free[mesh.dim * np.nonzero(on)[0] + c] = 0
    u = W.random_displacement(mesh, 7, 300.0 * mat.Y / mat.E)
    ref, rp, K, _ = _oracle(mesh, mat, u)
    assert ref["flag"].all()
    ctx = _ep.Context(mesh, free, mat, options={"assembly": _ep.EP_ASSEMBLY_FUSED})
    try:
        ctx.constitutive(ctx.tensor(u), sig=False, D=False, flag=False)
        ctx.assemble_tangent()
        _check_rows(_np(ctx.csr(1)[2]), K, rp)
    finally:
        ctx.close()
