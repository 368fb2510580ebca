"""Matrix-core element-local products (27-node hexahedra and 10-node
tetrahedra): the incremental tangent with BF16 or FP32 operands and FP32
accumulation against the oracle's FP64 sum w B^T D B, and the converged Newton
solution unchanged (the residual and stopping test stay FP64)."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_cases import make_case  # noqa: E402
from paper_1805_04155_amd import _ep, solver  # noqa: E402
from paper_1805_04155_amd import workloads as W  # noqa: E402

# Per-entry error bounds relative to the row scale max(|K_t|, |K_elast|):
# operands are rounded to the product precision (unit roundoff u = 2^-24 for
# FP32, 2^-9 for BF16 with round-to-nearest), each entry sums 6 n_q <= 162
# products of two rounded operands, accumulated in FP32: |err| <~ 162 * 2u *
# max|term|, and max|term| is below the row scale.
TOL = {"fp32": 162 * 2 * 2.0 ** -24 * 2, "bf16": 3e-2}


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("mode", ["colours", "rows"])
@pytest.mark.parametrize("case", ["q2_3d_dph", "q2s_3d_dph", "p2_3d_dph"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16_f32values"])
def test_incremental_tangent_matrix_cores(case, prec, mode):
    """bf16_f32values: BF16 local products with K stored in FP32.  rows:
    the element matrices (FP32) go through the buffer of the row gather."""
    mesh, free, mat, u, (ep, beta, kappa) = make_case(case)
    opts = {"local_prec": _ep.EP_FP32 if prec == "fp32" else _ep.EP_BF16,
            "assembly": _ep.ASSEMBLY[mode]}
    if prec == "bf16_f32values":
        opts["tangent_prec"] = _ep.EP_FP32
    prec = prec.split("_")[0]
    ctx = _ep.Context(mesh, free, mat, options=opts)
    try:
        ctx.set_state(ep, None, kappa)
        _, _, Ke = ctx.csr(0)
        Ke = _np(Ke)
        dphi, w = O.geometry(mesh)
        pat = O.pattern(mesh)
        errs = []
        for s in (1.0, 0.4, 1.0):
            ctx.constitutive(ctx.tensor(u * s), sig=False, D=False, flag=False)
            ctx.assemble_tangent()
            _, _, val = ctx.csr(1)
            ref = O.constitutive(mat, O.strain(mesh, dphi, u * s), O.state_to_ip6(ep, 3), None, kappa)
            _, _, Kt = O.assemble(mesh, dphi, w, ref["D"], *pat)
            rows = np.repeat(np.arange(mesh.n_dof), np.diff(pat[0]))
            scale = np.zeros(mesh.n_dof)
            np.maximum.at(scale, rows, np.maximum(np.abs(Kt), np.abs(Ke)))
            e = np.abs(_np(val) - Kt) / scale[rows]
            errs.append(e.max())
            # blocks of elastic elements are exactly K_elast
        assert max(errs) <= TOL[prec], errs
        assert max(errs) > 0  # the reduced precision is really used
    finally:
        ctx.close()


def test_matrix_cores_refused_for_other_elements():
    mesh = W.mesh_q1_3d(2, 2, 2, 1.0, 1.0, 1.0)
    with pytest.raises(_ep.EpError):
        _ep.Context(mesh, np.ones(mesh.n_dof, np.uint8), W.VM_MATERIAL,
                    options={"local_prec": _ep.EP_BF16})


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_newton_solution_unchanged_by_local_precision(prec):
    """Q2 block with Drucker-Prager hardening: the converged displacement with
    reduced-precision local products equals the FP64 one (the tangent only
    changes the convergence rate)."""
    wl = W.workload_q2_block(4, 2, 2, q_max=4000.0, steps=4)
    res = {}
    for lp in ("fp64", prec):
        opts = {"newton_rtol": 1e-12,
                "local_prec": {"fp64": _ep.EP_FP64, "fp32": _ep.EP_FP32, "bf16": _ep.EP_BF16}[lp]}
        ctx = _ep.Context(wl.mesh, wl.free, wl.material, options=opts)
        u = torch.zeros(wl.mesh.n_dof, dtype=torch.float64, device="cuda")
        recs = solver.solve_load_path(ctx, wl, u)
        res[lp] = (_np(u), sum(r["newton_its"] for r in recs))
        ctx.close()
    ua, ub = res["fp64"][0], res[prec][0]
    assert np.abs(ua - ub).max() <= 1e-9 * np.abs(ua).max()
    assert res[prec][1] >= res["fp64"][1]


def test_fused_rows_refuse_reduced_local_precision():
    """The fused row assembly forms its element terms in FP64 only."""
    mesh = W.mesh_q2_3d(2, 1, 1, 1.0, 1.0, 1.0)
    with pytest.raises(_ep.EpError):
        _ep.Context(mesh, np.ones(mesh.n_dof, np.uint8), W.VM_MATERIAL,
                    options={"local_prec": _ep.EP_FP32, "assembly": _ep.EP_ASSEMBLY_FUSED})


@pytest.mark.parametrize("case", ["q2_3d_dph", "p2_3d_dph"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_matrix_core_products_through_the_row_route(case, prec):
    """Colour mode inside Newton steps with matrix-core products: a work
    list that fits the element-matrix buffer (every list of these small
    meshes) goes through the matrix-core element matrices, stored at the
    elements' work-list positions, and the node-row gather (two launches);
    K_tangent equals the oracle's at each step's displacement to the
    per-entry bound, over steps whose plastic sets differ."""
    mesh, free, mat, u, (ep, beta, kappa) = make_case(case)
    ctx = _ep.Context(mesh, free, mat, options={
        "local_prec": _ep.EP_FP32 if prec == "fp32" else _ep.EP_BF16})
    try:
        ctx.set_state(ep, None, kappa)
        _, _, Ke = ctx.csr(0)
        Ke = _np(Ke)
        dphi, w = O.geometry(mesh)
        pat = O.pattern(mesh)
        rows = np.repeat(np.arange(mesh.n_dof), np.diff(pat[0]))
        f = np.zeros(mesh.n_dof)
        f[-1] = 1e-9  # a nonzero load: the step is not converged
        _ep.ep_profile(ctx.h, True, ["assembly"])
        errs, listed = [], []
        for s in (1.0, 0.1, 1.0, 0.02):
            _ep.ep_profile_read(ctx.h, "assembly")
            st, info = _ep.ep_newton_step(ctx.h, ctx.tensor(f), ctx.tensor(u * s))
            assert _ep.ep_profile_read(ctx.h, "assembly")[1] == 2, s
            listed.append(info["n_plastic_elem"])
            _, _, val = ctx.csr(1)
            ref = O.constitutive(mat, O.strain(mesh, dphi, u * s), O.state_to_ip6(ep, 3), None,
                                 kappa)
            _, _, Kt = O.assemble(mesh, dphi, w, ref["D"], *pat)
            scale = np.zeros(mesh.n_dof)
            np.maximum.at(scale, rows, np.maximum(np.abs(Kt), np.abs(Ke)))
            errs.append((np.abs(_np(val) - Kt) / scale[rows]).max())
        _ep.ep_profile(ctx.h, 0)
        assert min(listed) > 0 and len(set(listed)) > 1, listed
        assert max(errs) <= TOL[prec], errs
        assert max(errs) > 0
    finally:
        ctx.close()
