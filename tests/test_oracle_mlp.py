"""Pins of the learned-warm-start oracle (oracle/mlp.py) against what the
mathematics fixes: finite differences of the loss, networks wired to compute
known functions, closed forms of the loss and of Adam under a constant
gradient, the return-map closed forms behind the training targets, limits of
the consistent tangent for the predicted-branch tangent, and one exact Newton
step for the warm start with an exact network."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from oracle import oracle as O
from paper_1805_04155_amd import workloads as W


def trial_stress(mat, e):
    """C e for strain-type Voigt rows e (Lame form)."""
    G, K = mat.shear, mat.bulk
    lam = K - 2 * G / 3
    sig = np.zeros_like(e)
    sig[:, :3] = lam * e[:, :3].sum(axis=1, keepdims=True) + 2 * G * e[:, :3]
    sig[:, 3:] = G * e[:, 3:]
    return sig


def _batch(seed, n=24):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, M.XS))
    X[:, :M.NI] = rng.standard_normal((n, M.NI))
    T = np.zeros((n, M.YS))
    T[:, :6] = rng.standard_normal((n, 6))
    T[:, 6] = rng.integers(0, 2, n)
    return X, T


def test_parameter_count():
    assert M.NPARAM == 13 * 128 + 128 + 128 * 128 + 128 + 7 * 128 + 7 == 19207


def test_gradient_matches_central_differences():
    """Backpropagation against central differences of the loss in FP64 at
    every bias of the output layer and a random sample of all parameters."""
    X, T = _batch(0)
    p = W.mlp_he_uniform(1)
    p += 0.05 * np.random.default_rng(2).standard_normal(p.shape)  # nonzero biases
    L, g = M.loss_grad(p, X, T)
    assert abs(L - M.loss(p, X, T)) <= 1e-15 * abs(L)
    rng = np.random.default_rng(3)
    off_b3 = M.NPARAM - 7
    idx = np.concatenate([np.arange(off_b3, M.NPARAM), rng.choice(M.NPARAM, 120, replace=False)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (M.loss(p + e, X, T) - M.loss(p - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_wiring_computes_known_function():
    """relu(x) - relu(-x) = x: a network wired to output y0 = x0, y1 = 2 x5,
    y6 = x12 - 1 reproduces them exactly (checks W[out][in] order, ReLU and
    the parameter layout)."""
    d = {name: np.zeros(shape) for name, shape in M.SIZES}
    for h, (i, s) in enumerate([(0, 1), (0, -1), (5, 1), (5, -1), (12, 1), (12, -1)]):
        d["W1"][h, i] = s
        d["W2"][h, h] = 1.0
    d["W3"][0, 0], d["W3"][0, 1] = 1.0, -1.0
    d["W3"][1, 2], d["W3"][1, 3] = 2.0, -2.0
    d["W3"][6, 4], d["W3"][6, 5] = 1.0, -1.0
    d["b3"][6] = -1.0
    X, _ = _batch(4, 50)
    y, _ = M.forward(M.pack(d), X)
    assert np.array_equal(y[:, 0], X[:, 0])
    assert np.array_equal(y[:, 1], 2 * X[:, 5])
    assert np.array_equal(y[:, 6], X[:, 12] - 1.0)
    assert not y[:, 2:6].any()


def test_loss_closed_forms():
    """Outputs equal to the stress targets and a zero logit: L = log 2; a
    logit z with flag t: the logistic loss log(1 + e^z) - t z."""
    d = {name: np.zeros(shape) for name, shape in M.SIZES}
    d["b3"][:6] = [0.5, -1.0, 2.0, 0.0, 0.25, -0.75]
    X, T = _batch(5, 10)
    T[:, :6] = d["b3"][:6]
    assert abs(M.loss(M.pack(d), X, T) - math.log(2.0)) <= 1e-15
    for z, t in [(3.0, 1.0), (-2.0, 0.0), (40.0, 0.0), (-40.0, 1.0)]:
        d["b3"][6] = z
        ref = math.log1p(math.exp(z)) - t * z
        T[:, 6] = t
        assert abs(M.loss(M.pack(d), X, T) - ref) <= 1e-14 * max(1.0, abs(ref))


def test_adam_under_constant_gradient():
    """With a constant gradient g the bias-corrected moments are g and g^2,
    so every step moves each parameter by lr g / (|g| + eps)."""
    rng = np.random.default_rng(6)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    lr = 1e-3
    for t in range(1, 6):
        p, m, v = M.adam_step(p, m, v, g, lr, t)
        assert np.allclose(p, p0 - t * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_he_uniform_bounds_and_variance():
    P = M.unpack(W.mlp_he_uniform(7))
    for name, fan in (("W1", 13), ("W2", 128), ("W3", 128)):
        w = P[name]
        assert np.abs(w).max() <= math.sqrt(6.0 / fan)
        assert abs(w.var() / (2.0 / fan) - 1.0) < 0.2
    assert not P["b1"].any() and not P["b2"].any() and not P["b3"].any()


def _pool(material, n, seed, plastic_scale):
    rng = np.random.default_rng(seed)
    eps = plastic_scale * rng.standard_normal((6, n))
    ep = 0.3 * plastic_scale * rng.standard_normal((6, n))
    if material.model == "VM":
        ep[:3] -= ep[:3].mean(axis=0)
    kappa = plastic_scale * rng.uniform(0, 1, n)
    return eps, ep, kappa


def test_datagen_targets_and_features():
    """Targets are sigma - sigma_tr: zero at elastic samples; plastic von
    Mises samples follow the radial return: dev sigma - beta_prev is parallel
    to the trial s_tr with norm Y + a (|s_tr| - Y) / (2G + a); features give
    back the total strain; out-of-pool indices give zero rows."""
    mat = W.VM_MATERIAL
    s_in, s_out = M.scales(mat)
    assert abs(s_out * math.sqrt(1.5) * mat.Y - 1.0) < 1e-15
    eps, ep, _ = _pool(mat, 400, 8, 0.6 * mat.Y / mat.E)
    idx = np.arange(-3, 420)
    deps = 1e-4 * np.random.default_rng(9).standard_normal((6, len(idx)))
    X, T = M.datagen(mat, idx, eps, ep, None, None, deps)
    ok = (idx >= 0) & (idx < 400)
    assert not X[~ok].any() and not T[~ok].any()
    i = idx[ok]
    etot = eps[:, i] + deps[:, ok]
    rec = (X[ok, 0:6].astype(np.float64) + X[ok, 6:12]) / s_in
    assert np.abs(rec - etot.T).max() <= 2e-7 * np.abs(etot).max()
    G = mat.shear
    e = (etot - ep[:, i]).T
    sig_el = trial_stress(mat, e)
    el = T[ok, 6] == 0
    pl = ~el
    assert el.sum() > 20 and pl.sum() > 20
    assert np.abs(T[ok][el, :6] / s_out).max() <= 1e-12 * np.abs(sig_el).max()
    sig = T[ok][pl, :6].astype(np.float64) / s_out + sig_el[pl]
    beta = M.back_stress(mat, ep[:, i].T)[pl]
    dev = sig.copy()
    dev[:, :3] -= sig[:, :3].mean(axis=1, keepdims=True)
    s = dev - beta

    def nrm(v):
        return np.sqrt((v[:, :3] ** 2).sum(axis=1) + 2 * (v[:, 3:] ** 2).sum(axis=1))

    ed = e[pl].copy()
    ed[:, :3] -= ed[:, :3].mean(axis=1, keepdims=True)
    ed[:, 3:] *= 0.5
    s_tr = 2 * G * ed - beta
    ntr = nrm(s_tr)
    expect = mat.Y + mat.a * (ntr - mat.Y) / (2 * G + mat.a)
    assert np.abs(nrm(s) / expect - 1.0).max() < 1e-5
    cos = (s[:, :3] * s_tr[:, :3]).sum(1) + 2 * (s[:, 3:] * s_tr[:, 3:]).sum(1)
    assert np.abs(cos / (nrm(s) * ntr) - 1.0).max() < 1e-5


def _vm_states(mat, n, seed, radius):
    """Trial states with |s_tr| = radius * Y (random directions)."""
    rng = np.random.default_rng(seed)
    G = mat.shear
    ep = np.zeros((n, 6))
    beta = M.back_stress(mat, ep)
    N = W._unit_deviatoric_strain_voigt(rng, n, False)
    # s_tr = 2G dev(eps) for eps = r N (N strain-type unit): |s_tr| = 2G r |N|_stress
    nst = N.copy()
    nst[:, 3:] *= 0.5
    norm = np.sqrt((nst[:, :3] ** 2).sum(1) + 2 * (nst[:, 3:] ** 2).sum(1))
    eps = N * (radius * mat.Y / (2 * G * norm))[:, None]
    eps[:, :3] += 1e-4 * rng.standard_normal((n, 1))  # volumetric part
    return eps, ep, beta


def test_predicted_tangent_von_mises():
    """Outside the yield surface it is the consistent tangent of the exact
    return map; inside it is the limit of that tangent at the surface."""
    mat = W.VM_MATERIAL
    eps, ep, beta = _vm_states(mat, 30, 10, 1.7)
    ref = O.constitutive(mat, eps, ep, beta)
    assert ref["flag"].all()
    D = M.predicted_tangent(mat, eps, ep, beta, np.zeros(30))
    assert np.abs(D - ref["D"]).max() <= 1e-12 * mat.E
    inside, _, _ = _vm_states(mat, 30, 11, 0.6)
    Dc = M.predicted_tangent(mat, inside, ep, beta, np.zeros(30))
    # the same directions just outside the surface
    vol = inside[:, :3].mean(axis=1, keepdims=True)
    dev = inside.copy()
    dev[:, :3] -= vol
    edge = dev * ((1.0 + 1e-9) / 0.6)
    edge[:, :3] += vol
    lim = O.constitutive(mat, edge, ep, beta)
    assert lim["flag"].all()
    assert np.abs(Dc - lim["D"]).max() <= 1e-6 * mat.E


@pytest.mark.parametrize("a", [0.0, 2000.0])
def test_predicted_tangent_drucker_prager(a):
    """Cone and apex points (CRIT1 > 0) get the exact consistent tangent;
    an elastic point taken as plastic gets the limit of the cone tangent at
    CRIT1 -> 0+."""
    base = W.dp_material_3d_hardening()
    mat = W.Material("DP", E=base.E, nu=base.nu, eta=base.eta, c=base.c, a=a)
    rng = np.random.default_rng(12)
    n = 200
    scale = mat.c / mat.E
    eps = 3 * scale * rng.standard_normal((n, 6))
    eps[:, :3] += scale * rng.uniform(-2, 6, (n, 1))
    ep = np.zeros((n, 6))
    kappa = scale * rng.uniform(0, 1, n)
    ref = O.constitutive(mat, eps, ep, None, kappa)
    f = ref["flag"]
    assert (f == 1).sum() > 10 and (f == 2).sum() > 10 and (f == 0).sum() > 10
    D = M.predicted_tangent(mat, eps, ep, np.zeros((n, 6)), kappa)
    pl = f != 0
    assert np.abs(D[pl] - ref["D"][pl]).max() <= 1e-11 * mat.E
    # elastic points: scale the deviatoric part up to just past the cone
    el = np.nonzero(f == 0)[0][:10]
    for k in el:
        e = eps[k].copy()
        vol = e[:3].mean()
        dv = e.copy()
        dv[:3] -= vol
        lo, hi = 1.0, 1.0
        while True:
            hi *= 2.0
            t = dv * hi
            t[:3] += vol
            if O.constitutive(mat, t[None], ep[:1], None, kappa[k:k + 1])["flag"][0]:
                break
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            t = dv * mid
            t[:3] += vol
            if O.constitutive(mat, t[None], ep[:1], None, kappa[k:k + 1])["flag"][0]:
                hi = mid
            else:
                lo = mid
        t = dv * hi
        t[:3] += vol
        lim = O.constitutive(mat, t[None], ep[:1], None, kappa[k:k + 1])
        if lim["flag"][0] != 1:
            continue  # the ray reached the apex first
        Dt = M.predicted_tangent(mat, t[None], ep[:1], np.zeros((1, 6)), kappa[k:k + 1])
        assert np.abs(Dt - lim["D"]).max() <= 1e-8 * mat.E
        # and at the elastic point itself the tangent is the same continuum one
        Dk = M.predicted_tangent(mat, eps[k:k + 1], ep[:1], np.zeros((1, 6)), kappa[k:k + 1])
        assert np.abs(Dk - Dt).max() <= 1e-8 * mat.E


def test_learned_constitutive_with_exact_outputs():
    """Network outputs equal to the exact targets reproduce the exact
    stress and consistent tangent at every point."""
    mat = W.VM_MATERIAL
    eps, ep, beta = _vm_states(mat, 40, 13, 1.0)
    eps[::2] *= 1.5
    ref = O.constitutive(mat, eps, ep, beta)
    _, s_out = M.scales(mat)
    Y = np.zeros((40, M.YS))
    Y[:, :6] = s_out * (ref["sig"] - trial_stress(mat, eps - ep))
    Y[:, 6] = np.where(ref["flag"] != 0, 1.0, -1.0)
    flag, sig, D = M.learned_constitutive(mat, eps, ep, beta, np.zeros(40), Y)
    assert np.array_equal(flag, ref["flag"] != 0)
    assert np.abs(sig - ref["sig"]).max() <= 1e-12 * np.abs(ref["sig"]).max()
    assert np.abs(D - ref["D"]).max() <= 1e-12 * mat.E


def test_warm_start_with_exact_network_is_a_newton_step():
    """With a network that returns the exact return map, the warm start is
    one exact Newton step from the extrapolated displacement, and the exact
    residual decides its acceptance."""
    wl = W.workload_q1_cube(3)
    mesh, mat = wl.mesh, wl.material
    ep, beta, kappa, _ = W.seeded_state(wl, 0.5, seed=2)
    ep6, beta6 = O.state_to_ip6(ep, 3), O.state_to_ip6(beta, 3)
    kap = np.zeros(mesh.n_int)
    dphi, w = O.geometry(mesh)
    u4, *_ = O.newton_solve(mesh, mat, wl.free, wl.f(4), np.zeros(mesh.n_dof), ep6, beta6, kap,
                            tol=1e-12)
    u5, *_ = O.newton_solve(mesh, mat, wl.free, wl.f(5), u4, ep6, beta6, kap, tol=1e-12)
    f = wl.f(6)
    extrap = (wl.load_factors[6] - wl.load_factors[5]) / (wl.load_factors[5] - wl.load_factors[4])
    u_pred = u5 + extrap * (u5 - u4) * wl.free
    _, s_out = M.scales(mat)

    def exact_network(X):
        eps = O.strain(mesh, dphi, u_pred)
        out = O.constitutive(mat, eps, ep6, beta6, kap)
        Y = np.zeros((mesh.n_int, M.YS))
        Y[:, :6] = s_out * (out["sig"] - trial_stress(mat, eps - ep6))
        Y[:, 6] = np.where(out["flag"] != 0, 1.0, -1.0)
        return Y

    u_ws, info = M.warm_start(mesh, mat, wl.free, f, u5, u4, extrap, ep6, beta6, kap,
                              exact_network)
    u_ref, it, res, _ = O.newton_solve(mesh, mat, wl.free, f, u_pred, ep6, beta6, kap, max_it=1,
                                       tol=0.0, raise_on_limit=False)
    assert it == 1
    assert info["accepted"] == 1
    assert np.abs(u_ws - u_ref).max() <= 1e-10 * np.abs(u_ref).max()
    assert abs(info["res_rel_pred"] - res[0]) <= 1e-10 * res[0]
    assert abs(info["res_rel_warm"] - res[1]) <= 1e-8 * max(res[1], 1e-14)
    assert info["res_rel_warm"] < info["res_rel_start"]
    # a network that predicts garbage is rejected: u_out = u_prev
    u_bad, info_bad = M.warm_start(mesh, mat, wl.free, f, u5, u4, extrap, ep6, beta6, kap,
                                   lambda X: np.full((X.shape[0], M.YS), 50.0))
    assert info_bad["accepted"] == 0 and np.array_equal(u_bad, u5)
