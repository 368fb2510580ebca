"""Pins of the oracle's return maps (paper Sections 2.2 and 2.3, and the
linear cohesion-hardening Drucker-Prager extension) against invariants,
special cases with independent closed forms, and finite differences."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1805_04155_amd import workloads as W

VM = W.VM_MATERIAL
DP2 = W.dp_material_2d()
DPH = W.dp_material_3d_hardening()
DP_PERFECT_3D = W.Material("DP", E=20000.0, nu=0.3, eta=DPH.eta, c=DPH.c, a=0.0)


def voigt_stress_tensor(v):
    return np.array([[v[0], v[3], v[5]], [v[3], v[1], v[4]], [v[5], v[4], v[2]]])


def voigt_strain_tensor(v):
    return np.array([[v[0], v[3] / 2, v[5] / 2], [v[3] / 2, v[1], v[4] / 2],
                     [v[5] / 2, v[4] / 2, v[2]]])


def dev(t):
    return t - np.trace(t) / 3 * np.eye(3)


def single(mat, eps, ep=None, beta=None, kappa=None):
    eps = np.atleast_2d(np.asarray(eps, float))
    n = eps.shape[0]
    ep = np.zeros((n, 6)) if ep is None else np.atleast_2d(ep)
    beta = np.zeros((n, 6)) if beta is None else np.atleast_2d(beta)
    kappa = np.zeros(n) if kappa is None else np.atleast_1d(kappa)
    return O.constitutive(mat, eps, ep, beta, kappa)


def random_states(mat, n, seed):
    rng = np.random.default_rng(seed)
    scale = (1.5 * mat.Y if mat.model == "VM" else 4 * mat.c) / mat.E
    eps = scale * rng.standard_normal((n, 6))
    ep = 0.3 * scale * rng.standard_normal((n, 6))
    beta = np.zeros((n, 6))
    if mat.model == "VM":
        # von Mises flow is deviatoric: admissible plastic strains are too
        ep[:, :3] -= ep[:, :3].mean(axis=1, keepdims=True)
        beta = mat.a * ep
        beta[:, 3:] *= 0.5
    kappa = 0.2 * scale * rng.uniform(size=n)
    return eps, ep, beta, kappa


def test_elastic_is_hooke():
    """Inside the yield surface the response is C(eps - ep) (eq. elastic_law):
    compared with E, nu Hooke's law in its compliance form."""
    rng = np.random.default_rng(0)
    eps = 1e-5 * rng.standard_normal((20, 6))
    out = single(VM, eps)
    assert np.all(out["flag"] == 0)
    E, nu = VM.E, VM.nu
    for k in range(20):
        s = voigt_stress_tensor(out["sig"][k])
        e_back = ((1 + nu) * s - nu * np.trace(s) * np.eye(3)) / E
        assert np.max(np.abs(e_back - voigt_strain_tensor(eps[k]))) < 1e-18


def test_vm_simple_shear_closed_form():
    """Simple shear reduces von Mises with linear kinematic hardening to a
    1D spring: tau = G (gamma - gamma_p), back stress a*gamma_p/2, yield
    sqrt(2) |tau - a gamma_p / 2| = Y."""
    G, a, Y = VM.shear, VM.a, VM.Y
    for gamma in [1e-3, 4e-3, 2e-2]:
        gp = max(0.0, (G * gamma - Y / math.sqrt(2)) / (G + a / 2))
        tau = G * (gamma - gp)
        out = single(VM, [0, 0, 0, gamma, 0, 0])
        assert abs(out["sig"][0, 3] - tau) < 1e-10 * tau
        assert np.max(np.abs(out["sig"][0, [0, 1, 2, 4, 5]])) < 1e-9
        assert abs(out["ep"][0, 3] - gp) < 1e-16 + 1e-12 * gp
        assert out["flag"][0] == (1 if gp > 0 else 0)


@pytest.mark.parametrize("seed", range(3))
def test_vm_yield_consistency_and_normality(seed):
    eps, ep, beta, kappa = random_states(VM, 400, seed)
    out = O.constitutive(VM, eps, ep, beta, kappa)
    pl = out["flag"] == 1
    assert 50 < pl.sum() < 390
    for k in np.nonzero(pl)[0]:
        s = dev(voigt_stress_tensor(out["sig"][k])) - voigt_stress_tensor(out["beta"][k])
        assert abs(np.linalg.norm(s) - VM.Y) < 1e-12 * VM.Y
        # plastic strain increment is parallel to the returned s (normality)
        dep = voigt_strain_tensor(out["ep"][k]) - voigt_strain_tensor(ep[k])
        cos = np.sum(dep * s) / (np.linalg.norm(dep) * np.linalg.norm(s))
        assert abs(cos - 1) < 1e-12
        # back stress moves by a times the plastic strain increment
        db = voigt_stress_tensor(out["beta"][k]) - voigt_stress_tensor(beta[k])
        assert np.max(np.abs(db - VM.a * dep)) < 1e-9
    for k in np.nonzero(~pl)[0]:
        s = dev(voigt_stress_tensor(out["sig"][k])) - voigt_stress_tensor(beta[k])
        assert np.linalg.norm(s) <= VM.Y


def test_vm_perfect_limit():
    """a = 0 is perfect plasticity: the returned deviator has norm Y and no
    back stress develops."""
    mat = W.Material("VM", E=VM.E, nu=VM.nu, Y=VM.Y, a=0.0)
    eps, ep, _, _ = random_states(mat, 200, 7)
    out = O.constitutive(mat, eps, ep, np.zeros_like(ep), None)
    pl = out["flag"] == 1
    assert pl.sum() > 20
    for k in np.nonzero(pl)[0]:
        assert abs(np.linalg.norm(dev(voigt_stress_tensor(out["sig"][k]))) - mat.Y) < 1e-12 * mat.Y
    assert np.all(out["beta"] == 0)


def dp_psi(mat, sig_v, kappa):
    s = voigt_stress_tensor(sig_v)
    p = np.trace(s) / 3
    return np.linalg.norm(dev(s)) / math.sqrt(2) + mat.eta * p - (mat.c + mat.a * kappa)


@pytest.mark.parametrize("mat", [DP2, DP_PERFECT_3D, DPH], ids=["dp2d", "dp3d", "dph"])
def test_dp_consistency_branches(mat):
    eps, ep, _, kappa = random_states(mat, 600, 11)
    # add volumetric tension to reach the apex on some points
    eps[:300, :3] += 3 * mat.c / (mat.eta * mat.bulk)
    out = O.constitutive(mat, eps, ep, None, kappa)
    f = out["flag"]
    assert (f == 1).sum() > 30 and (f == 2).sum() > 30 and (f == 0).sum() > 10
    for k in range(600):
        psi = dp_psi(mat, out["sig"][k], out["kappa"][k])
        if f[k] == 0:
            assert psi <= 0
            assert out["kappa"][k] == kappa[k]
        else:
            assert abs(psi) < 1e-11 * mat.c
            assert out["kappa"][k] > kappa[k]
        if f[k] == 2:
            s = voigt_stress_tensor(out["sig"][k])
            assert np.linalg.norm(dev(s)) < 1e-9
            if mat.a == 0:
                assert abs(s[0, 0] - mat.c / mat.eta) < 1e-11 * mat.c / mat.eta
                assert np.all(out["D"][k] == 0)
            # stress from the updated plastic strain (Hooke) equals the return
            e_el = voigt_strain_tensor(eps[k]) - voigt_strain_tensor(out["ep"][k])
            s_h = mat.bulk * np.trace(e_el) * np.eye(3) + 2 * mat.shear * dev(e_el)
            assert np.max(np.abs(s_h - s)) < 1e-9 * mat.c


def test_dp_hydrostatic_tension_apex():
    """Pure volumetric strain beyond c/(3 K eta) returns to the apex c/eta."""
    mat = DP_PERFECT_3D
    e = 2 * mat.c / (3 * mat.bulk * mat.eta)
    out = single(mat, [e, e, e, 0, 0, 0])
    assert out["flag"][0] == 2
    assert np.allclose(out["sig"][0], [mat.c / mat.eta] * 3 + [0] * 3, rtol=1e-14, atol=1e-12)


def test_dp_pure_shear_dilatancy():
    """Pure shear on the smooth cone: the shear stress drops to the yield
    value and the associated flow produces volumetric plastic strain
    eta*dl, i.e. a compressive mean stress -K*eta*dl."""
    mat = DP_PERFECT_3D
    G, K, eta, c = mat.shear, mat.bulk, mat.eta, mat.c
    gamma = 3 * c / G
    out = single(mat, [0, 0, 0, gamma, 0, 0])
    assert out["flag"][0] == 1
    dl = (G * gamma - c) / (G + K * eta ** 2)
    tr_ep = out["ep"][0, :3].sum()
    assert abs(tr_ep - eta * dl) < 1e-14
    s = voigt_stress_tensor(out["sig"][0])
    assert abs(np.trace(s) / 3 + K * eta * dl) < 1e-10
    assert abs(s[0, 1] - (G * gamma - G * dl)) < 1e-9


def test_dp_hardening_zero_equals_perfect():
    eps, ep, _, kappa = random_states(DP_PERFECT_3D, 300, 5)
    a = O.constitutive(DP_PERFECT_3D, eps, ep, None, kappa)
    b = O.constitutive(DP_PERFECT_3D, eps, ep, None, np.zeros_like(kappa))
    for key in ("sig", "D", "flag", "ep"):
        assert np.array_equal(a[key], b[key])


@pytest.mark.parametrize("mat", [DP2, DPH], ids=["dp", "dph"])
def test_dp_stress_continuous_across_apex(mat):
    """Along a ray of volumetric strain added to a sheared state the stress
    is continuous where the branch switches from smooth to apex."""
    G = mat.shear
    base = np.array([0, 0, 0, 2 * mat.c / G, 0, 0])
    ts = np.linspace(0, 30 * mat.c / (mat.eta * mat.bulk), 20001)
    eps = np.array([base + t * np.array([1, 1, 1, 0, 0, 0]) / 3 for t in ts])
    out = single(mat, eps)
    f = out["flag"]
    k = np.nonzero((f[:-1] == 1) & (f[1:] == 2))[0]
    assert len(k) == 1
    jump = np.max(np.abs(out["sig"][k[0] + 1] - out["sig"][k[0]]))
    step = np.max(np.abs(out["sig"][k[0]] - out["sig"][k[0] - 1]))
    assert jump < 3 * step + 1e-9


def _fd_tangent(mat, eps, ep, beta, kappa, h):
    D = np.zeros((6, 6))
    for j in range(6):
        ep_ = np.zeros(6)
        ep_[j] = h
        sp = single(mat, eps + ep_, ep, beta, kappa)["sig"][0]
        sm = single(mat, eps - ep_, ep, beta, kappa)["sig"][0]
        D[:, j] = (sp - sm) / (2 * h)
    return D


@pytest.mark.parametrize("mat", [VM, DP2, DP_PERFECT_3D, DPH], ids=["vm", "dp2d", "dp3d", "dph"])
def test_tangent_matches_finite_differences(mat):
    """The consistent tangent is the derivative of the stress (eqs.
    DT_kinematic and the Drucker-Prager tangents), checked by central
    differences away from the branch boundaries; it is symmetric."""
    eps, ep, beta, kappa = random_states(mat, 300, 3)
    if mat.model == "DP":
        eps[:150, :3] += 3 * mat.c / (mat.eta * mat.bulk)
    out = O.constitutive(mat, eps, ep, beta, kappa)
    scale = mat.Y if mat.model == "VM" else mat.c
    checked = {0: 0, 1: 0, 2: 0}
    for k in range(300):
        # distance to the branch boundaries, measured on slightly perturbed
        # states
        far = True
        for dlt in (1e-6, -1e-6):
            o2 = single(mat, eps[k] * (1 + dlt), ep[k], beta[k], kappa[k])
            if o2["flag"][0] != out["flag"][k]:
                far = False
        if not far:
            continue
        Dfd = _fd_tangent(mat, eps[k], ep[k], beta[k], kappa[k], 1e-9 * scale / mat.E * 1e3)
        D = out["D"][k]
        # floor: rounding noise of the central difference, ~eps_mach*|sigma|/h
        assert np.max(np.abs(D - Dfd)) < 1e-6 * np.max(np.abs(D)) + 1e-6 * mat.E
        assert np.max(np.abs(D - D.T)) < 1e-9 * mat.E
        checked[int(out["flag"][k])] += 1
    assert checked[0] > 5 and checked[1] > 5
    if mat.model == "DP":
        assert checked[2] > 5
