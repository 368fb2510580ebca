"""Parity at the full workload sizes, in the configuration bench.py times
(seeded plastic state, FP64), on outputs the oracle can compute one by one:
stresses, tangents and flags at sampled points; the plastic point and
element sets in full (the oracle's return map runs over every point); rows
of K_tangent and the position map of sampled elements; F at sampled nodes
(from the oracle's force over only the elements touching them)."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

from paper_1805_04155_amd import _ep  # noqa: E402
from paper_1805_04155_amd import workloads as W  # noqa: E402

WORKLOADS = {
    "q2_slope": W.workload_q2_slope,
    "q1_cube": W.workload_q1_cube,
    "q2_block": W.workload_q2_block,
    "p2_block": W.workload_p2_block,
}


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", params=list(WORKLOADS))
def full(request):
    name = request.param
    wl = WORKLOADS[name]()
    mesh, mat = wl.mesh, wl.material
    ep, beta, kappa, _ = W.seeded_state(wl, 0.5, seed=0)
    h = (np.prod(mesh.coord.max(axis=1) - mesh.coord.min(axis=1)) / mesh.n_elems) ** (1 / mesh.dim)
    u = W.random_displacement(mesh, 1, 1e-6 * h, wl.free)  # the input bench.py times
    ctx = _ep.Context(mesh, wl.free, mat)
    ctx.set_state(ep, beta if mat.model == "VM" else None, kappa if mat.model == "DP" else None)
    sig, D, flag = ctx.constitutive(ctx.tensor(u))
    ctx.assemble_tangent()
    out = dict(name=name, wl=wl, mesh=mesh, mat=mat, u=u, ep=ep, beta=beta, kappa=kappa, ctx=ctx,
               sig=_np(sig), D=_np(D), flag=_np(flag))
    yield out
    ctx.close()


def _oracle_points(f, elems):
    mesh = f["mesh"]
    sub = np.ascontiguousarray(mesh.elem[elems])
    dphi, w = O.geometry(mesh, sub)
    eps = O.strain(mesh, dphi, f["u"], sub)
    ips = (elems[:, None] * mesh.n_q + np.arange(mesh.n_q)).ravel()
    ep6 = O.state_to_ip6(f["ep"][:, ips], mesh.dim)
    beta6 = O.state_to_ip6(f["beta"][:, ips], mesh.dim)
    return (ips, O.constitutive(f["mat"], eps, ep6, beta6, f["kappa"][ips], crit=True), dphi, w,
            sub)


def test_points_sampled(full):
    mesh = full["mesh"]
    rng = np.random.default_rng(7)
    elems = np.sort(rng.choice(mesh.n_elems, size=min(3000, mesh.n_elems), replace=False))
    ips, ref, _, _, _ = _oracle_points(full, elems)
    # exact outside the tie band of the yield tests, which is empty here
    band = O.tie_band(full["mat"], ref["crit"])
    assert np.array_equal(full["flag"][ips][~band], ref["flag"][~band])
    assert not band.any(), f"{int(band.sum())} sampled points in the tie band"
    d = mesh.dim
    sig = full["sig"][:, ips].T
    rs = ref["sig"] if d == 3 else ref["sig"][:, :4]
    assert np.abs(sig - rs).max() <= 1e-12 * np.abs(rs).max()
    ns = 6 if d == 3 else 3
    Dg = full["D"][:, ips].T.reshape(-1, ns, ns)
    Dr = ref["D"] if d == 3 else ref["D"][:, [0, 1, 3]][:, :, [0, 1, 3]]
    assert np.abs(Dg - Dr).max() <= 1e-12 * full["mat"].E


def _oracle_all(f):
    if "all" not in f:
        f["all"] = _oracle_points(f, np.arange(f["mesh"].n_elems))
    return f["all"]


def test_plastic_sets_full(full):
    mesh = full["mesh"]
    ips, ref, _, _, _ = _oracle_all(full)
    pl = np.nonzero(ref["flag"])[0]
    ip, el = full["ctx"].plastic()
    assert np.array_equal(_np(ip), pl)
    assert np.array_equal(_np(el), np.unique(pl // mesh.n_q))
    assert 0 < len(pl) < mesh.n_int


def test_tangent_rows_and_position_map_sampled(full):
    mesh, ctx = full["mesh"], full["ctx"]
    d = mesh.dim
    rp, ci, val = ctx.csr(1)
    rp_h = _np(rp)
    # nnz by brute force: dim^2 times the distinct node pairs of all elements
    e = mesh.elem.astype(np.int64)
    keys = np.unique((e[:, :, None] * mesh.n_nodes + e[:, None, :]).ravel())
    assert rp_h[-1] == d * d * len(keys)
    rng = np.random.default_rng(11)
    # rows of nodes of a few sampled elements (plastic and elastic ones)
    elems = rng.choice(mesh.n_elems, size=4, replace=False)
    rows = np.unique((d * mesh.elem[elems][:, :, None] + np.arange(d)).ravel())[:24]
    ips, ref, dphi, w, _ = _oracle_all(full)
    orows = O.K_rows(mesh, dphi, w, ref["D"], rows)
    Ke = _np(ctx.csr(0)[2])
    for r, (oc, ov) in zip(rows, orows):
        a, b = rp_h[r], rp_h[r + 1]
        gc = _np(ci[a:b])
        assert np.array_equal(gc, oc), r
        gv = _np(val[a:b])
        scale = max(np.abs(ov).max(), np.abs(Ke[a:b]).max())
        assert np.abs(gv - ov).max() <= 1e-12 * scale, r
    pos = _np(ctx.position_map()[torch.as_tensor(elems, device="cuda")])
    nl = d * mesh.n_p
    for k, e in enumerate(elems):
        dof = (d * mesh.elem[e][:, None] + np.arange(d)).ravel()
        for a_ in range(nl):
            cols = _np(ci[rp_h[dof[a_]]:rp_h[dof[a_] + 1]])
            expect = rp_h[dof[a_]] + np.searchsorted(cols, dof)
            assert np.array_equal(pos[k, a_], expect)
            assert np.array_equal(cols[expect - rp_h[dof[a_]]], dof)


def test_internal_force_sampled(full):
    mesh, ctx = full["mesh"], full["ctx"]
    F = _np(ctx.internal_force())
    rng = np.random.default_rng(5)
    nodes = rng.choice(mesh.n_nodes, size=40, replace=False)
    touch = np.nonzero(np.isin(mesh.elem, nodes).any(axis=1))[0]
    ips, ref, dphi, w, sub = _oracle_points(full, touch)
    Fo = O.internal_force(mesh, dphi, w, ref["sig"], sub)
    d = mesh.dim
    dofs = (d * nodes[:, None] + np.arange(d)).ravel()
    scale = np.abs(Fo[dofs]).max() + 1e-300
    assert np.abs(F[dofs] - Fo[dofs]).max() <= 1e-11 * max(scale, np.abs(F).max() * 1e-3)
