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


# --------------------------------------------------------------------------
# damped Newton (Section 4) and the energy-norm increment of ALG-NEWTON
# --------------------------------------------------------------------------

def test_line_search_closed_forms():
    """g(a) = du . Q(f - F(u + a du)) is the negative derivative of the
    convex incremental energy along du.  Linear g (a quadratic energy): the
    full step is kept when the minimiser is at or beyond a = 1 / (1 + theta),
    and otherwise regula falsi lands on the exact root in one evaluation.
    A cubic g: the returned step meets |g| <= theta g(0)."""
    theta = 0.25
    for root in (1.0, 2.0, 1.0 / (1.0 + theta) + 1e-9):
        a, n = O.line_search(lambda x: 3.0 * (1.0 - x / root), 3.0, theta)
        assert (a, n) == (1.0, 1)
    for root in (0.7, 0.3, 0.05):
        a, n = O.line_search(lambda x: 3.0 * (1.0 - x / root), 3.0, theta)
        assert abs(a - root) <= 1e-15 and n == 2
    g = lambda x: 2.0 - 50.0 * x ** 3  # noqa: E731
    a, n = O.line_search(g, 2.0, theta)
    assert abs(g(a)) <= theta * 2.0 and 0 < a < 1 and n <= 12
    # no descent information (g(0) <= 0): the full step
    assert O.line_search(lambda x: -1.0, -1.0, theta) == (1.0, 1)


def test_energy_norm_increment_closed_forms():
    """|du|_e / (|u|_e + |u + du|_e): 1 from u = 0, 0 for du = 0, invariant
    under a common scaling, and equal to the plain Euclidean expression for
    K = I."""
    import scipy.sparse as sp
    rng = np.random.default_rng(0)
    n = 12
    A = rng.normal(size=(n, n))
    K = sp.csr_matrix(A @ A.T + n * np.eye(n))
    du, u = rng.normal(size=n), rng.normal(size=n)
    assert O.energy_norm_increment(K, du, np.zeros(n)) == 1.0
    assert O.energy_norm_increment(K, np.zeros(n), u) == 0.0
    e = O.energy_norm_increment(K, du, u)
    assert abs(O.energy_norm_increment(K, 7.0 * du, 7.0 * u) - e) <= 1e-15
    I = sp.identity(n, format="csr")
    want = np.linalg.norm(du) / (np.linalg.norm(u) + np.linalg.norm(u + du))
    assert abs(O.energy_norm_increment(I, du, u) - want) <= 1e-15


def test_damped_newton_keeps_full_steps_in_the_elastic_range():
    """On the elastic steps of the P1 square the problem is linear, the
    Newton step lands on the minimiser and the damped method takes it
    unchanged: the same iterates as the plain method, bit for bit; the
    energy-norm increment of the single correction from u = 0 is 1."""
    wl = W.workload_p1_square()
    mesh, mat = wl.mesh, wl.material
    n = mesh.n_int
    z = np.zeros((n, 6))
    h = []
    u1, it1, res1, _ = O.newton_solve(mesh, mat, wl.free, wl.f(0), np.zeros(mesh.n_dof), z, z,
                                      None, history=h)
    u2, it2, res2, _ = O.newton_solve(mesh, mat, wl.free, wl.f(0), np.zeros(mesh.n_dof), z, z,
                                      None, damping=0.25)
    assert it1 == it2 == 1
    assert np.array_equal(u1, u2) and res1 == res2
    assert h[0]["step"] == 1.0 and h[0]["energy_incr"] == 1.0


def test_damped_newton_converges_where_the_plain_method_fails():
    """The strip footing (Section 8.3) on 16 x 16 nine-node quadrilaterals,
    pushed to u_D = 0.5 in a single displacement step: the plain semismooth
    Newton method wanders without converging in 60 iterations, the damped
    one (line search on the incremental energy) reaches 1e-10; its step
    lengths leave 1 while the plastic zone forms and return to 1 for the
    final, quadratically converging iterations."""
    wl = W.workload_strip_footing(16, "Q2_2D")
    mesh, mat = wl.mesh, wl.material
    n = mesh.n_int
    u0 = wl.u_dir_unit * 0.5
    dphi, w = O.geometry(mesh)
    pat = O.pattern(mesh)
    args = (mesh, mat, wl.free, np.zeros(mesh.n_dof), u0, np.zeros((n, 6)), None, np.zeros(n))
    kw = dict(tol=1e-10, max_it=60, dphi=dphi, w=w, pattern_=pat)
    import pytest
    with pytest.raises(RuntimeError):
        O.newton_solve(*args, **kw)
    h = []
    u, it, res, out = O.newton_solve(*args, damping=0.25, history=h, **kw)
    assert res[-1] <= 1e-10 and it <= 60
    steps = [x["step"] for x in h if "step" in x]
    assert min(steps) < 0.5
    assert steps[-3:] == [1.0, 1.0, 1.0]
    # the stopping quantity of ALG-NEWTON falls with the residual at the end
    e = [x["energy_incr"] for x in h if "energy_incr" in x]
    assert e[-1] < 1e-6 and e[-1] < e[-2] < e[-3]
