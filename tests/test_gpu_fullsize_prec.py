"""Parity at the full workload sizes for the setup arrays and the
reduced-precision tangents: the whole CSR pattern and scalar position map of
the slope and of the 27-node block, bit for bit, against the oracle's
independent sort-unique and binary search; sampled rows of K_tangent built
with matrix-core local products (FP32, BF16 operands) on the full 27-node
and P2 blocks, and with FP32 tangent storage on the full slope and cube,
each at its per-entry bound against the oracle's FP64 rows."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

from paper_1805_04155_amd import _ep  # noqa: E402
from paper_1805_04155_amd import workloads as W  # noqa: E402

# per-entry bounds relative to the row scale max(|K_t|, |K_elast|) (see
# test_gpu_mfma: 6 n_q <= 162 products of two rounded operands accumulated
# in FP32); FP32 storage rounds K_elast and the sum once each
TOL = {"fp32": 162 * 2 * 2.0 ** -24 * 2, "bf16": 3e-2, "store32": 4 * 2.0 ** -24}


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", ["q2_slope", "q2_block"])
def test_pattern_and_position_map_full(name):
    """Every row pointer, column index and position-map entry of the full
    mesh equals the oracle's (33 579 012 and 38 490 633 non-zeros)."""
    wl = {"q2_slope": W.workload_q2_slope, "q2_block": W.workload_q2_block}[name]()
    mesh = wl.mesh
    ctx = _ep.Context(mesh, wl.free, wl.material)
    try:
        rp, ci, _ = ctx.csr(0)
        rp, ci = _np(rp), _np(ci)
        pos = _np(ctx.position_map())
    finally:
        ctx.close()
    rpo, cio = O.pattern(mesh)
    assert np.array_equal(rp, rpo)
    assert np.array_equal(ci, cio)
    del cio
    poso = O.position_map(mesh, rpo, ci)
    assert np.array_equal(pos, poso)


def _seeded(wl):
    mesh = wl.mesh
    ep, beta, kappa, _ = W.seeded_state(wl, 0.5, seed=0)
    h = (np.prod(mesh.coord.max(axis=1) - mesh.coord.min(axis=1)) / mesh.n_elems) ** (1 / mesh.dim)
    u = W.random_displacement(mesh, 1, 1e-6 * h, wl.free)
    return ep, beta, kappa, u


def _rows_check(wl, options, tol, n_rows=24, seed=11):
    """K_tangent rows from sampled plastic and elastic elements' nodes
    against the oracle's rows; returns the largest relative entry error."""
    mesh, mat = wl.mesh, wl.material
    ep, beta, kappa, u = _seeded(wl)
    d = mesh.dim
    ctx = _ep.Context(mesh, wl.free, mat, options=options)
    try:
        ctx.set_state(ep, beta if mat.model == "VM" else None, kappa if mat.model == "DP" else None)
        ctx.constitutive(ctx.tensor(u), sig=False, D=False, flag=False)
        ctx.assemble_tangent()
        _, el = ctx.plastic()
        el = _np(el)
        rp, ci, val = ctx.csr(1)
        Ke = ctx.csr(0)[2]
        rng = np.random.default_rng(seed)
        elastic = np.setdiff1d(np.arange(mesh.n_elems), el)
        elems = np.concatenate([rng.choice(el, 3, replace=False), rng.choice(elastic, 1)])
        rows = np.unique((d * mesh.elem[elems][:, :, None] + np.arange(d)).ravel())
        rows = rng.choice(rows, size=min(n_rows, len(rows)), replace=False)
        rp_h = _np(rp)
        got = []
        for r in rows:
            a, b = int(rp_h[r]), int(rp_h[r + 1])
            got.append((_np(ci[a:b]), _np(val[a:b]), _np(Ke[a:b])))
    finally:
        ctx.close()
    dphi, w = O.geometry(mesh)
    eps = O.strain(mesh, dphi, u)
    ref = O.constitutive(mat, eps, O.state_to_ip6(ep, d), O.state_to_ip6(beta, d), kappa)
    orows = O.K_rows(mesh, dphi, w, ref["D"], rows)
    worst = 0.0
    for r, (gc, gv, gk), (oc, ov) in zip(rows, got, orows):
        assert np.array_equal(gc, oc), r
        scale = max(np.abs(ov).max(), np.abs(gk).max())
        err = np.abs(gv - ov).max() / scale
        assert err <= tol, (r, err, tol)
        worst = max(worst, err)
    return worst


@pytest.mark.parametrize("name", ["q2_block", "p2_block"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_matrix_core_tangent_rows_full(name, prec):
    wl = {"q2_block": W.workload_q2_block, "p2_block": W.workload_p2_block}[name]()
    worst = _rows_check(wl, {"local_prec": _ep.EP_FP32 if prec == "fp32" else _ep.EP_BF16},
                        TOL[prec])
    assert worst > 0.0  # the reduced precision is really used


@pytest.mark.parametrize("name", ["q2_slope", "q1_cube"])
def test_fp32_tangent_storage_rows_full(name):
    wl = {"q2_slope": W.workload_q2_slope, "q1_cube": W.workload_q1_cube}[name]()
    worst = _rows_check(wl, {"tangent_prec": _ep.EP_FP32}, TOL["store32"])
    assert worst > 0.0


@pytest.mark.parametrize("name", ["q1_cube", "p2_block"])
def test_row_gather_assembly_rows_full(name):
    """The node-row gather assembly (FP64) at full size: sampled rows of
    K_tangent at the FP64 bound of the colour-round assembly."""
    wl = {"q1_cube": W.workload_q1_cube, "p2_block": W.workload_p2_block}[name]()
    _rows_check(wl, {"assembly": _ep.EP_ASSEMBLY_ROWS}, 1e-12)


@pytest.mark.parametrize("name", ["q1_cube", "q2_slope"])
def test_fused_row_assembly_rows_full(name):
    """The fused node-row assembly (FP64, every row scanned) at full size:
    sampled rows of K_tangent at the FP64 bound of the colour-round
    assembly."""
    wl = {"q1_cube": W.workload_q1_cube, "q2_slope": W.workload_q2_slope}[name]()
    _rows_check(wl, {"assembly": _ep.EP_ASSEMBLY_FUSED}, 1e-12)


def test_fused_row_assembly_fp32_values_full():
    """Fused rows with FP32 tangent values on the full slope: sampled rows
    at the FP32 storage bound."""
    wl = W.workload_q2_slope()
    worst = _rows_check(wl, {"assembly": _ep.EP_ASSEMBLY_FUSED, "tangent_prec": _ep.EP_FP32},
                        TOL["store32"])
    assert worst > 0.0
