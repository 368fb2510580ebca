"""Kernel timing of the library's profiled sections (ep_profile,
ep_profile_read).  The section events travel with the kernel dispatches, so
each section that ran reports one positive time, the times fit inside the
wall time around them, and profiling changes no result bit."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_cases import make_case  # noqa: E402
from paper_1805_04155_amd import _ep  # noqa: E402


def _pass(ctx, u, F):
    _ep.ep_constitutive(ctx.h, u)
    _ep.ep_assemble_tangent(ctx.h)
    _ep.ep_internal_force(ctx.h, F)


@pytest.mark.parametrize("name", ["q2_2d_dp", "q1_3d_vm", "p2_3d_dph"])
def test_profile_sections(name):
    mesh, free, mat, u_np, state = make_case(name)
    ctx = _ep.Context(mesh, free, mat)
    try:
        ctx.set_state(*state)
        u = ctx.tensor(u_np)
        F = torch.empty(mesh.n_dof, dtype=torch.float64, device="cuda")
        runs = {}
        for prof in (0, 1, 0):
            _ep.ep_profile(ctx.h, prof)
            torch.cuda.synchronize()
            n = 3
            t0 = time.perf_counter()
            for _ in range(n):
                _pass(ctx, u, F)
            torch.cuda.synchronize()
            wall_ms = 1e3 * (time.perf_counter() - t0)
            b = u.clone()
            b[torch.from_numpy(free == 0).to(b.device)] = 0.0
            x = torch.zeros_like(u)
            st, its, _ = _ep.ep_pcg(ctx.h, b, x, 1e-8, 400)
            assert st in (_ep.EP_OK, _ep.EP_ENOTCONV) and its > 0
            torch.cuda.synchronize()
            prof_read = {k: _ep.ep_profile_read(ctx.h, k) for k in _ep.PROF}
            _ep.ep_profile(ctx.h, 0)
            runs[len(runs)] = (_np(ctx.csr(1)[2]), F.cpu().numpy(), x.cpu().numpy(), its)
            if prof:
                p = prof_read
                for k in ("constitutive", "compaction", "force"):
                    assert p[k][1] == n, (k, p[k])
                assert p["assembly"][1] > 0 and p["assembly"][1] % n == 0
                for k in ("constitutive", "compaction", "assembly", "force"):
                    assert 0.0 < p[k][0] < wall_ms, (k, p[k], wall_ms)
                assert sum(p[k][0] for k in ("constitutive", "compaction", "assembly",
                                              "force")) < wall_ms
                # iterations run in chunks: at least the converged count (small
                # systems: one single-workgroup launch per chunk)
                if mesh.n_dof <= 12288:
                    assert p["pcg_small"][1] >= its and p["pcg_small"][0] > 0.0
                    assert p["spmv"][1] == 0 and p["pcg_vec"][1] == 0
                else:
                    assert p["spmv"][1] >= its and p["pcg_vec"][1] == p["spmv"][1]
                    assert p["spmv"][0] > 0.0 and p["pcg_vec"][0] > 0.0
                assert p["split"][1] == 0 and p["elastic"][1] == 0
            else:
                assert all(v == (0.0, 0) for v in prof_read.values())
        for k in (1, 2):
            for a, b in zip(runs[0], runs[k]):
                assert np.array_equal(a, b)
    finally:
        ctx.close()


def test_profile_mask():
    """Only the selected kernel ids are timed."""
    mesh, free, mat, u_np, state = make_case("q1_3d_vm")
    ctx = _ep.Context(mesh, free, mat)
    try:
        ctx.set_state(*state)
        u = ctx.tensor(u_np)
        F = torch.empty(mesh.n_dof, dtype=torch.float64, device="cuda")
        for sel in (["assembly"], ["constitutive", "force"]):
            _ep.ep_profile(ctx.h, 1, kernels=sel)
            for _ in range(2):
                _pass(ctx, u, F)
            p = {k: _ep.ep_profile_read(ctx.h, k) for k in _ep.PROF}
            _ep.ep_profile(ctx.h, 0)
            for k, (ms, cnt) in p.items():
                if k in sel:
                    assert cnt > 0 and cnt % 2 == 0 and ms > 0.0, (k, ms, cnt)
                else:
                    assert (ms, cnt) == (0.0, 0), (k, ms, cnt)
    finally:
        ctx.close()


def test_profile_elastic_assembly():
    mesh, free, mat, u_np, state = make_case("q2_2d_dp")
    ctx = _ep.Context(mesh, free, mat)
    try:
        _ep.ep_profile(ctx.h, 1)
        _ep.ep_assemble_elastic(ctx.h)
        torch.cuda.synchronize()
        ms, cnt = _ep.ep_profile_read(ctx.h, "elastic")
        _ep.ep_profile(ctx.h, 0)
        assert cnt == 1 and ms > 0.0
    finally:
        ctx.close()


def _np(t):
    return t.detach().cpu().numpy()


def test_binding_checks_buffers():
    """The binding refuses a buffer of the wrong element type or one too
    small for the context before the library is called."""
    mesh, free, mat, u_np, state = make_case("q2_2d_dp")
    ctx = _ep.Context(mesh, free, mat)
    try:
        u = ctx.tensor(u_np)
        with pytest.raises(TypeError):
            _ep.ep_constitutive(ctx.h, u.float())
        with pytest.raises(ValueError):
            _ep.ep_constitutive(ctx.h, u[:-1])
        with pytest.raises(ValueError):
            _ep.ep_internal_force(ctx.h, torch.empty(mesh.n_dof - 2, dtype=torch.float64,
                                                     device="cuda"))
        with pytest.raises(TypeError):
            _ep.ep_get_plastic(ctx.h, torch.empty(mesh.n_int, dtype=torch.int64, device="cuda"))
        _ep.ep_constitutive(ctx.h, u)  # the right buffers still work
        torch.cuda.synchronize()
    finally:
        ctx.close()
