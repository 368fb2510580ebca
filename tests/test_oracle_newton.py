"""Pins of the oracle's semismooth Newton (ALG-NEWTON, Section 4)."""
import math

import numpy as np

from oracle import oracle as O
from paper_1805_04155_amd import workloads as W


def material_point_uniaxial(mat, t, ep6, beta6):
    """Plane-strain uniaxial stress: find (eps11, eps22) with sigma11 = 0,
    sigma22 = t (eps33 = shears = 0), by Newton on the point's return map."""
    e = np.zeros(2)
    for _ in range(50):
        eps = np.array([[e[0], e[1], 0, 0, 0, 0]])
        out = O.constitutive(mat, eps, ep6, beta6)
        r = np.array([0.0, t]) - out["sig"][0, :2]
        if np.abs(r).max() < 1e-12 * t:
            return eps[0], out
        e += np.linalg.solve(out["D"][0][:2, :2], r)
    raise RuntimeError("point solve did not converge")


def test_p1_square_homogeneous_load_path():
    """The P1 square workload (sliding left/bottom, free right edge, uniform
    top traction) has a homogeneous uniaxial solution on any mesh.  Steps
    1-9 are elastic with closed-form strains; step 10 (t = 540 > 505) is
    plastic and every point must equal the material-point solution."""
    wl = W.workload_p1_square()
    mesh, mat = wl.mesh, wl.material
    E, nu = mat.E, mat.nu
    n = mesh.n_int
    ep6, beta6 = np.zeros((n, 6)), np.zeros((n, 6))
    u = np.zeros(mesh.n_dof)
    dphi, w = O.geometry(mesh)
    pat = O.pattern(mesh)
    its = []
    for k in range(10):
        t = wl.load_factors[k]
        f = wl.f(k)
        u, it, res, out = O.newton_solve(mesh, mat, wl.free, f, u, ep6, beta6, None,
                                         dphi=dphi, w=w, pattern_=pat)
        its.append(it)
        eps = O.strain(mesh, dphi, u)
        if k < 9:
            assert np.all(out["flag"] == 0)
            e22 = t * (1 - nu ** 2) / E
            e11 = -t * nu * (1 + nu) / E
            assert np.abs(eps[:, 0] - e11).max() < 1e-12 * abs(e22)
            assert np.abs(eps[:, 1] - e22).max() < 1e-12 * abs(e22)
        else:
            assert np.all(out["flag"] == 1)
            e_pt, o_pt = material_point_uniaxial(mat, t, ep6[:1], beta6[:1])
            assert np.abs(eps - e_pt).max() < 1e-10 * abs(e_pt[1])
            assert np.abs(out["sig"] - o_pt["sig"][0]).max() < 1e-10 * t
        ep6, beta6 = out["ep"], out["beta"]
    # onset of yield: |dev sigma| = Y under plane-strain uniaxial stress t
    t_yield = mat.Y / (math.sqrt(6 * (1 - nu + nu ** 2)) / 3)
    assert 486 < t_yield < 540
    assert its[9] >= 2


def test_quadratic_local_convergence():
    """Semismooth Newton converges quadratically once the plastic set is
    fixed (paper Section 4; semismoothness of T_k): on a small non-uniform
    problem the residual exponent log r_{l+1} / log r_l approaches 2."""
    wl = W.workload_q1_cube(4)
    mesh, mat = wl.mesh, wl.material
    ep, beta, kappa, _ = W.seeded_state(wl, 0.5, seed=0)
    ep6, beta6 = O.state_to_ip6(ep, 3), O.state_to_ip6(beta, 3)
    hist = []
    u, it, res, out = O.newton_solve(mesh, mat, wl.free, wl.f(6), np.zeros(mesh.n_dof),
                                     ep6, beta6, None, tol=1e-14, history=hist)
    assert 0 < np.count_nonzero(out["flag"]) < mesh.n_int
    # last iterations with a frozen plastic set
    ratios = []
    for l in range(1, len(res) - 1):
        if hist[l]["n_plastic"] == hist[l + 1]["n_plastic"] and 1e-14 < res[l + 1] < res[l] < 1e-2:
            ratios.append(math.log(res[l + 1]) / math.log(res[l]))
    assert ratios, res
    assert max(ratios) > 1.7, (res, ratios)


def test_seeded_cyclic_cube_path_converges():
    """The cyclic traction history on the 8^3 cube from the seeded state
    (half of the elements plastic): every step, the zero-load instants
    included, reaches |Q(f - F)| <= 1e-10 |Q f| (or the reaction scale where
    Q f = 0: the seeded plastic strain leaves residual stresses), in a few
    Newton iterations per step."""
    wl = W.workload_q1_cube_cyclic(8, 30)
    mesh, mat = wl.mesh, wl.material
    ep, beta, _, _ = W.seeded_state(wl, 0.5, seed=0)
    ep6, beta6 = O.state_to_ip6(ep, 3), O.state_to_ip6(beta, 3)
    kappa = np.zeros(mesh.n_int)
    u = np.zeros(mesh.n_dof)
    dphi, w = O.geometry(mesh)
    pat = O.pattern(mesh)
    its = []
    for k in range(len(wl.load_factors)):
        f = wl.f_unit * wl.load_factors[k]
        u, it, res, out = O.newton_solve(mesh, mat, wl.free, f, u, ep6, beta6, kappa, tol=1e-10,
                                         dphi=dphi, w=w, pattern_=pat)
        assert res[-1] <= 1e-10
        ep6, beta6, kappa = out["ep"], out["beta"], out["kappa"]
        its.append(it)
    assert min(wl.load_factors) < 0.0 < max(wl.load_factors)
    assert 0.0 in [float(x) for x in wl.load_factors]
    assert sum(its) < 4 * len(its)
