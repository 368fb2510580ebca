"""Pins of the oracle pieces the GPU parity tests lean on at full size: the
sampled rows of K (against the oracle's own COO sort-and-sum assembly, bit
for bit), Jacobi-PCG (against a sparse direct solve and the closed-form
one-step case of a diagonal matrix), the Drucker-Prager parameter fits of
Section 8.3 (against the Mohr-Coulomb surfaces they are fitted to) and the
yield tests that decide the return-map branches (against the flags and the
trial yield functions)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_1805_04155_amd import workloads as W
from tests.gpu_cases import CASES, make_case


def _oracle_state(mesh, mat, u, state):
    ep, beta, kappa = state
    dphi, w = O.geometry(mesh)
    eps = O.strain(mesh, dphi, u)
    out = O.constitutive(mat, eps, O.state_to_ip6(ep, mesh.dim),
                         O.state_to_ip6(beta, mesh.dim) if mat.model == "VM" else None,
                         kappa if mat.model == "DP" else None, crit=True)
    return dphi, w, out


@pytest.mark.parametrize("name", list(CASES))
def test_K_rows_equal_assembled_rows_bit_for_bit(name):
    """or_K_rows (the reference of the full-size K-row parity) sums the same
    element contributions in the same element order as the COO sort-and-sum
    of or_assemble, so each sampled row must equal the assembled one exactly,
    at a state with elastic and plastic points."""
    mesh, free, mat, u, state = make_case(name, seed=3)
    dphi, w, out = _oracle_state(mesh, mat, u, state)
    flags = out["flag"]
    assert 0 < np.count_nonzero(flags) < flags.size, "want a mixed plastic state"
    row_ptr, col_idx, val = O.assemble(mesh, dphi, w, out["D"])
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([[0, mesh.n_dof - 1],
                                     rng.choice(mesh.n_dof, 24, replace=False)]))
    got = O.K_rows(mesh, dphi, w, out["D"], rows)
    for r, (cols, vals) in zip(rows, got):
        a, b = row_ptr[r], row_ptr[r + 1]
        assert np.array_equal(cols, col_idx[a:b]), f"row {r}: columns"
        assert np.array_equal(vals, val[a:b]), f"row {r}: values"


def test_K_rows_reports_a_short_buffer():
    mesh, free, mat, u, state = make_case("q1_3d_vm", seed=0)
    dphi, w, out = _oracle_state(mesh, mat, u, state)
    with pytest.raises(RuntimeError):
        O.K_rows(mesh, dphi, w, out["D"], [3 * 40], max_cols=5)


def _spd_tangent(name, seed):
    mesh, free, mat, u, state = make_case(name, seed=seed)
    dphi, w, out = _oracle_state(mesh, mat, u, state)
    row_ptr, col_idx, val = O.assemble(mesh, dphi, w, out["D"])
    return mesh, free, row_ptr, col_idx, val, out["flag"]


@pytest.mark.parametrize("name", ["q1_3d_vm", "p1_2d_vm", "q2s_2d_vm"])
def test_pcg_matches_direct_solve(name):
    """Jacobi-PCG on the free dofs of a tangent with plastic points equals
    scipy's sparse direct solve of the same restricted system to the
    accuracy its stopping test allows, and the returned relative residual is
    the true one."""
    mesh, free, row_ptr, col_idx, val, flags = _spd_tangent(name, 5)
    assert np.count_nonzero(flags) > 0
    n = mesh.n_dof
    q = free.astype(bool)
    K = sp.csr_matrix((val, col_idx, row_ptr), shape=(n, n))
    Kq = K[q][:, q].tocsc()
    b = np.random.default_rng(1).normal(size=n)
    x, its, rel = O.pcg(row_ptr, col_idx, val, free, b, 1e-12, 20000)
    assert its > 0
    assert np.all(x[~q] == 0.0)
    xd = spla.spsolve(Kq, b[q])
    res = np.linalg.norm(b[q] - Kq @ x[q]) / np.linalg.norm(b[q])
    # the recurred residual the stopping test reads drifts from the true one
    # by rounding only
    assert rel <= 1e-12
    assert res <= 2e-12
    assert abs(res - rel) <= 1e-12
    # error bounded by the condition number times the residual
    kappa = np.linalg.cond(Kq.toarray()) if Kq.shape[0] <= 3000 else 1e6
    assert np.linalg.norm(x[q] - xd) <= 2 * kappa * res * np.linalg.norm(xd)
    assert np.linalg.norm(x[q] - xd) <= 1e-7 * np.linalg.norm(xd)


def test_pcg_diagonal_matrix_is_one_step():
    """With a diagonal matrix the Jacobi preconditioner is the inverse: the
    first search direction is the exact solution, reached with step 1."""
    n = 37
    d = np.linspace(1.0, 40.0, n)
    row_ptr = np.arange(n + 1, dtype=np.int32)
    col_idx = np.arange(n, dtype=np.int32)
    free = np.ones(n, dtype=np.uint8)
    free[[0, 5]] = 0
    b = np.random.default_rng(2).normal(size=n)
    x, its, rel = O.pcg(row_ptr, col_idx, d, free, b, 1e-14, 50)
    assert its == 1
    want = np.where(free == 1, b / d, 0.0)
    assert np.abs(x - want).max() <= 4e-16 * np.abs(want).max()


def test_pcg_iteration_limit_reported():
    mesh, free, row_ptr, col_idx, val, _ = _spd_tangent("q1_3d_vm", 5)
    b = np.random.default_rng(1).normal(size=mesh.n_dof)
    x, its, rel = O.pcg(row_ptr, col_idx, val, free, b, 1e-14, 3)
    assert its == -1 and rel > 1e-14


# --------------------------------------------------------------------------
# Drucker-Prager parameters of Section 8.3
# --------------------------------------------------------------------------

PHI = math.pi / 9
C0 = 450.0


def _mohr_coulomb(s1, s3):
    """Mohr-Coulomb yield function with tension positive, s1 >= s3 the
    largest and smallest principal stresses."""
    return (s1 - s3) + (s1 + s3) * math.sin(PHI) - 2.0 * C0 * math.cos(PHI)


def _dp(sig, eta, c):
    p = sum(sig) / 3.0
    dev = [s - p for s in sig]
    return math.sqrt(sum(x * x for x in dev)) / math.sqrt(2.0) + eta * p - c


def test_dp_3d_parameters_are_the_cone_through_a_mohr_coulomb_meridian():
    """The 3D fit is the cone through the meridian sigma1 > sigma2 = sigma3
    of the Mohr-Coulomb pyramid: stresses on that meridian and on the
    Mohr-Coulomb surface satisfy the Drucker-Prager function with equality,
    stresses on the other meridian do not."""
    eta, c = W.dp_parameters(C0, PHI, plane_strain=False)
    for s in (-900.0, -100.0, 0.0, 150.0):
        # sigma = (s + d, s, s) on the Mohr-Coulomb surface
        d = (2.0 * C0 * math.cos(PHI) - 2.0 * s * math.sin(PHI)) / (1.0 + math.sin(PHI))
        assert abs(_mohr_coulomb(s + d, s)) < 1e-9
        assert abs(_dp((s + d, s, s), eta, c)) <= 1e-12 * C0
        # the other meridian, sigma = (s, s, s - d'), on the MC surface
        d2 = (2.0 * C0 * math.cos(PHI) - 2.0 * s * math.sin(PHI)) / (1.0 - math.sin(PHI))
        assert abs(_mohr_coulomb(s, s - d2)) < 1e-9
        assert _dp((s, s, s - d2), eta, c) > 1e-3 * C0
    assert (round(eta, 6), round(c, 3)) == (0.354514, 438.308)


def test_dp_plane_strain_parameters_reproduce_mohr_coulomb_in_plane_strain():
    """The plane-strain fit: at a Drucker-Prager yield state whose associated
    flow has no out-of-plane plastic strain rate, the in-plane principal
    stresses lie on the Mohr-Coulomb surface (for every mean stress)."""
    eta, c = W.dp_parameters(C0, PHI, plane_strain=True)
    for m in (-800.0, -200.0, 0.0, 100.0):
        # unknowns: in-plane difference d and out-of-plane offset x of the
        # stress diag(m + d/2, m - d/2, m + x); solve the flow constraint
        # (33 component of n/sqrt(2) + eta/3 I is 0) and the yield condition
        def residual(v):
            d, x = v
            sig = (m + d / 2, m - d / 2, m + x)
            p = sum(sig) / 3.0
            dev = [s - p for s in sig]
            nrm = math.sqrt(sum(t * t for t in dev))
            return [_dp(sig, eta, c), dev[2] / (math.sqrt(2.0) * nrm) + eta / 3.0]
        from scipy.optimize import fsolve
        d, x = fsolve(residual, [600.0, -50.0], xtol=1e-14)
        assert max(abs(r) for r in residual((d, x))) < 1e-9
        s1, s3 = m + d / 2, m - d / 2
        assert s3 <= m + x <= s1  # the out-of-plane stress is intermediate
        assert abs(_mohr_coulomb(s1, s3)) <= 1e-9 * C0
    assert (round(eta, 6), round(c, 3)) == (0.335541, 414.851)


def test_workload_materials_use_the_section_8_3_fits():
    eta, c = W.dp_parameters(C0, PHI, plane_strain=True)
    for mat in (W.dp_material_2d(), W.dp_strip_footing_material()):
        assert (mat.eta, mat.c) == (eta, c)
    eta3, c3 = W.dp_parameters(C0, PHI, plane_strain=False)
    mat = W.dp_strip_footing_material(plane=False)
    assert (mat.eta, mat.c) == (eta3, c3)
    assert (W.dp_material_3d_hardening().eta, W.dp_material_3d_hardening().c) == (eta3, c3)


# --------------------------------------------------------------------------
# yield tests (the branch decisions)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["q1_3d_vm", "q2_3d_dph", "q1_3d_dp", "q2_2d_dp"])
def test_yield_tests_decide_the_flags(name):
    mesh, free, mat, u, state = make_case(name, seed=4)
    _, _, out = _oracle_state(mesh, mat, u, state)
    c1, c2, f = out["crit"][:, 0], out["crit"][:, 1], out["flag"]
    if mat.model == "VM":
        assert np.array_equal(f == 1, c1 > 0)
    else:
        assert np.array_equal(f == 0, c1 <= 0)
        assert np.array_equal(f == 1, (c1 > 0) & (c2 <= 0))
        assert np.array_equal(f == 2, (c1 > 0) & (c2 > 0))
        assert np.count_nonzero(f == 1) > 0 and np.count_nonzero(f == 2) > 0
    # at elastic points the trial stress is the returned stress: the first
    # test is the yield function evaluated on it
    el = f == 0
    s = out["sig"][el]
    p = s[:, :3].sum(axis=1) / 3.0
    dev = s.copy()
    dev[:, :3] -= p[:, None]
    if mat.model == "VM":
        dev -= O.state_to_ip6(state[1], mesh.dim)[el]
        nrm = np.sqrt((dev[:, :3] ** 2).sum(1) + 2 * (dev[:, 3:] ** 2).sum(1))
        want = nrm - mat.Y
    else:
        nrm = np.sqrt((dev[:, :3] ** 2).sum(1) + 2 * (dev[:, 3:] ** 2).sum(1))
        want = nrm / math.sqrt(2.0) + mat.eta * p - (mat.c + mat.a * state[2][el])
    assert np.abs(c1[el] - want).max() <= 1e-11 * (mat.Y if mat.model == "VM" else mat.c)
    # the tie band is empty on these seeded inputs
    assert not O.tie_band(mat, out["crit"]).any()


def test_tie_band_marks_points_near_the_surface():
    mat = W.VM_MATERIAL
    crit = np.array([[0.0, 0.0], [1e-13 * mat.Y, 0.0], [1e-10 * mat.Y, 0.0], [-1e-14, 0.0]])
    assert O.tie_band(mat, crit).tolist() == [True, True, False, True]
    dp = W.dp_material_2d()
    crit = np.array([[1.0, 1e-14], [-1.0, 1e-14], [1e-13, -5.0], [1.0, -1.0]])
    assert O.tie_band(dp, crit).tolist() == [True, False, True, False]


def test_oracle_threads_do_not_change_results():
    """The oracle's parallel loops write disjoint outputs and its sums keep
    their serial order: strain, return map, internal force and K are bit
    for bit the same on 1 and on 4 threads."""
    wl = W.workload_q2_slope(8, 4)
    mesh, mat = wl.mesh, wl.material
    ep, beta, kappa, _ = W.seeded_state(wl, 0.5, seed=0)
    u = W.random_displacement(mesh, 3, 1e-3, wl.free)
    dphi, w = O.geometry(mesh)
    rp, ci = O.pattern(mesh)
    prev = O.set_threads(0)
    outs = []
    try:
        for nt in (1, 4):
            O.set_threads(nt)
            eps = O.strain(mesh, dphi, u)
            o = O.constitutive(mat, eps, O.state_to_ip6(ep, 2), None, kappa)
            F = O.internal_force(mesh, dphi, w, o["sig"])
            _, _, K = O.assemble(mesh, dphi, w, o["D"], rp, ci)
            outs.append((eps, o["sig"], o["D"], F, K))
    finally:
        O.set_threads(prev)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
