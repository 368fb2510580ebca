"""The seeded input recipes, checked with the oracle: the cyclic traction
history of the von Mises example (Section 8.2) and the seeded plastic states
whose plastic set at u = 0 is exactly the seeded elements' points (the
plastic-fraction sweep relies on it)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1805_04155_amd import workloads as W


def test_cyclic_history_turning_points():
    # t_k = 4k/steps: with 4 steps the samples are the turning points
    assert np.allclose(W.cyclic_factors(4, 540.0), [540.0, 0.0, -540.0, 0.0])
    f = W.cyclic_factors(40, 200.0)
    assert len(f) == 40
    assert f.max() == pytest.approx(200.0) and f.min() == pytest.approx(-200.0)
    assert f[9] == pytest.approx(200.0) and f[19] == pytest.approx(0.0, abs=1e-12)
    assert f[29] == pytest.approx(-200.0) and f[39] == pytest.approx(0.0, abs=1e-12)
    # piecewise linear: constant slope magnitude between the turning points
    d = np.diff(np.concatenate([[0.0], f]))
    assert np.allclose(np.abs(d), 200.0 / 10)


@pytest.mark.parametrize("make,fraction", [
    (lambda: W.workload_q1_cube(6), 0.25),
    (lambda: W.workload_q1_cube(6), 1.0),
    (lambda: W.workload_q2_slope(8, 4), 0.5),
    (lambda: W.workload_q2_block(4, 2, 2), 0.5),
])
def test_seeded_state_plastic_set_is_the_seeded_elements(make, fraction):
    """At u = 0 the points of the first floor(fraction * n_e) elements of
    the seeded permutation are plastic and no other point is."""
    wl = make()
    mesh, mat = wl.mesh, wl.material
    ep, beta, kappa, _ = W.seeded_state(wl, fraction, seed=0)
    dim, n = mesh.dim, mesh.n_int
    dphi, w = O.geometry(mesh)
    eps = O.strain(mesh, dphi, np.zeros(mesh.n_dof))
    out = O.constitutive(mat, eps, O.state_to_ip6(ep, dim), O.state_to_ip6(beta, dim),
                         kappa if mat.model == "DP" else np.zeros(n))
    plastic = out["flag"] != 0
    n_seed = int(math.floor(fraction * mesh.n_elems))
    assert plastic.sum() == n_seed * mesh.n_q
    # whole elements: every point of a seeded element, none of the others
    per_elem = plastic.reshape(mesh.n_elems, mesh.n_q)
    assert np.all(per_elem.all(axis=1) | ~per_elem.any(axis=1))
    if mat.model == "DP":
        # the apex branch is reached where the bulk modulus allows it: both
        # branches at nu = 0.3, the smooth cone only at nu = 0.49
        branches = set(int(x) for x in np.unique(out["flag"][plastic]))
        assert branches == ({1, 2} if mat.nu < 0.4 else {1})
