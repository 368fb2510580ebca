"""Python face of the plain FP64 CPU oracle (ep_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the HIP product path.

Every function takes the shared seeded inputs (paper_1805_04155_amd.workloads
arrays) and converts them to the oracle's own IP-major layouts.  Section and
equation references are to Cermak, Sysala, Valdman (arXiv 1805.04155).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ep_oracle.c")
LIB = os.path.join(HERE, "libep_oracle.so")

ETYPE = {"P1_2D": 1, "Q1_2D": 2, "Q2_2D": 3, "P1_3D": 4, "P2_3D": 5, "Q1_3D": 6, "Q2_3D": 7,
         "Q2S_2D": 8, "Q2S_3D": 9}
PLANE = [0, 1, 3]


def build(force=False):
    """Compile the oracle with gcc (no fused multiply-add contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-std=c99", SRC, "-o", LIB + ".tmp", "-lm"])
        os.replace(LIB + ".tmp", LIB)


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P, I64, I, D = C.c_void_p, C.c_int64, C.c_int, C.c_double
        L.or_elem_info.argtypes = [I, P, P, P]
        L.or_basis.argtypes = [I, P, P, P]
        L.or_quadrature.argtypes = [I, P, P]
        L.or_geometry.argtypes = [I, I64, I64, P, P, P, P]
        L.or_geometry.restype = I64
        L.or_strain.argtypes = [I, I64, P, P, P, P]
        L.or_constitutive.argtypes = [I, I64, P, P, P, P, D, D, D, D, D, D, P, P, P, P, P, P]
        L.or_constitutive_crit.argtypes = [I, I64, P, P, P, P, D, D, D, D, D, D, P, P, P, P,
                                           P, P, P]
        L.or_internal_force.argtypes = [I, I64, I64, P, P, P, P, P]
        L.or_pattern.argtypes = [I, I64, I64, P, P, P]
        L.or_pattern.restype = I64
        L.or_position_map.argtypes = [I, I64, P, P, P, P]
        L.or_assemble.argtypes = [I, I64, P, P, P, P, P, P, P]
        L.or_assemble.restype = I
        L.or_K_rows.argtypes = [I, I64, P, P, P, P, I64, P, I, P, P, P]
        L.or_K_rows.restype = I
        L.or_pcg.argtypes = [I64, P, P, P, P, P, P, D, I, P]
        L.or_pcg.restype = I
        L.or_set_threads.argtypes = [I]
        L.or_set_threads.restype = I
        L.or_set_threads(1)  # one thread unless a caller asks for more
        _lib = L
    return _lib


def set_threads(n=0):
    """Threads of the oracle's parallel loops (1 after loading; n <= 0:
    unchanged); returns the count in effect.  Results do not depend on it (only loops with
    disjoint outputs run in parallel, sums keep their serial order)."""
    return int(lib().or_set_threads(int(n)))


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def elem_info(etype):
    d, p, q = C.c_int(), C.c_int(), C.c_int()
    lib().or_elem_info(ETYPE[etype], C.byref(d), C.byref(p), C.byref(q))
    return d.value, p.value, q.value


def basis(etype, xi):
    """Basis values (n_p,) and reference gradients (n_p, dim) at xi."""
    dim, n_p, _ = elem_info(etype)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    phi = np.zeros(n_p)
    dphi = np.zeros((n_p, dim))
    lib().or_basis(ETYPE[etype], _p(xi), _p(phi), _p(dphi))
    return phi, dphi


def quadrature(etype):
    dim, _, n_q = elem_info(etype)
    xi = np.zeros((n_q, dim))
    w = np.zeros(n_q)
    lib().or_quadrature(ETYPE[etype], _p(xi), _p(w))
    return xi, w


def geometry(mesh, elem=None):
    """dphi (n_int, n_p, dim) and WEIGHT (n_int,) (Section 6.1)."""
    elem = mesh.elem if elem is None else np.ascontiguousarray(elem, dtype=np.int32)
    n_e = elem.shape[0]
    dphi = np.zeros((n_e * mesh.n_q, mesh.n_p, mesh.dim))
    w = np.zeros(n_e * mesh.n_q)
    bad = lib().or_geometry(ETYPE[mesh.etype], mesh.n_nodes, n_e, _p(mesh.coord),
                            _p(elem), _p(dphi), _p(w))
    if bad:
        raise ValueError(f"{bad} integration points with non-positive det J")
    return dphi, w


def strain(mesh, dphi, u, elem=None):
    """E = B u, (n_int, 6) engineering Voigt (Section 6.2)."""
    elem = mesh.elem if elem is None else np.ascontiguousarray(elem, dtype=np.int32)
    u = np.ascontiguousarray(u, dtype=np.float64)
    eps = np.zeros((elem.shape[0] * mesh.n_q, 6))
    lib().or_strain(ETYPE[mesh.etype], elem.shape[0], _p(elem), _p(dphi), _p(u), _p(eps))
    return eps


def state_to_ip6(arr, dim):
    """Shared SoA state (n_sc, n_int) -> oracle IP-major (n_int, 6)."""
    arr = np.asarray(arr, dtype=np.float64)
    out = np.zeros((arr.shape[1], 6))
    if dim == 3:
        out[:] = arr.T
    else:
        out[:, :4] = arr.T
    return out


def ip6_to_state(arr, dim):
    return np.ascontiguousarray(arr.T if dim == 3 else arr[:, :4].T)


def constitutive(material, eps, ep6, beta6=None, kappa=None, crit=False):
    """Return map at every point (Sections 2.2, 2.3 and the linear cohesion
    hardening extension).  Returns dict(sig (n,6), D (n,6,6), flag (n,),
    ep (n,6), beta (n,6), kappa (n,)); with crit=True also crit (n,2), the
    yield tests the branches are decided on (von Mises |s_tr| - Y;
    Drucker-Prager CRIT1 and CRIT2)."""
    n = eps.shape[0]
    model = 1 if material.model == "VM" else 2
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    ep6 = np.ascontiguousarray(ep6, dtype=np.float64)
    beta6 = np.zeros((n, 6)) if beta6 is None else np.ascontiguousarray(beta6, dtype=np.float64)
    kappa = np.zeros(n) if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
    out = dict(sig=np.zeros((n, 6)), D=np.zeros((n, 6, 6)), flag=np.zeros(n, np.uint8),
               ep=np.zeros((n, 6)), beta=np.zeros((n, 6)), kappa=np.zeros(n))
    if crit:
        out["crit"] = np.zeros((n, 2))
    lib().or_constitutive_crit(model, n, _p(eps), _p(ep6), _p(beta6), _p(kappa),
                               material.shear, material.bulk, material.a, material.Y,
                               material.eta, material.c,
                               _p(out["sig"]), _p(out["D"]), _p(out["flag"]),
                               _p(out["ep"]), _p(out["beta"]), _p(out["kappa"]),
                               _p(out["crit"]) if crit else None)
    return out


def tie_band(material, crit, rel=1e-12):
    """Points whose branch decision lies within rel of a tie: |CRIT| < rel*Y
    (von Mises), or |CRIT1| < rel*c, or CRIT1 > 0 with |CRIT2| < rel*c
    (Drucker-Prager).  Two codes that round the yield test differently may
    take different branches only there.  Returns a boolean mask."""
    crit = np.asarray(crit)
    if material.model == "VM":
        return np.abs(crit[:, 0]) < rel * material.Y
    s = rel * material.c
    return (np.abs(crit[:, 0]) < s) | ((crit[:, 0] > 0) & (np.abs(crit[:, 1]) < s))


def internal_force(mesh, dphi, w, sig, elem=None):
    """F = B^T (WEIGHT .* S) (Section 7)."""
    elem = mesh.elem if elem is None else np.ascontiguousarray(elem, dtype=np.int32)
    F = np.zeros(mesh.n_dof)
    lib().or_internal_force(ETYPE[mesh.etype], mesh.n_nodes, elem.shape[0], _p(elem),
                            _p(dphi), _p(w), _p(np.ascontiguousarray(sig)), _p(F))
    return F


def pattern(mesh, elem=None):
    """CSR pattern (row_ptr, col_idx) of all element dof pairs, sorted."""
    elem = mesh.elem if elem is None else np.ascontiguousarray(elem, dtype=np.int32)
    L = lib()
    nnz = L.or_pattern(ETYPE[mesh.etype], mesh.n_nodes, elem.shape[0], _p(elem), None, None)
    row_ptr = np.zeros(mesh.n_dof + 1, dtype=np.int32)
    col_idx = np.zeros(nnz, dtype=np.int32)
    L.or_pattern(ETYPE[mesh.etype], mesh.n_nodes, elem.shape[0], _p(elem), _p(row_ptr), _p(col_idx))
    return row_ptr, col_idx


def position_map(mesh, row_ptr, col_idx):
    nl = mesh.dim * mesh.n_p
    pos = np.zeros((mesh.n_elems, nl, nl), dtype=np.int32)
    lib().or_position_map(ETYPE[mesh.etype], mesh.n_elems, _p(mesh.elem), _p(row_ptr),
                          _p(col_idx), _p(pos))
    return pos


def assemble(mesh, dphi, w, D, row_ptr=None, col_idx=None):
    """K = sum_e sum_q w B^T D B (paper Section 9 form), COO sort-and-sum.
    Returns (row_ptr, col_idx, val)."""
    if row_ptr is None:
        row_ptr, col_idx = pattern(mesh)
    val = np.zeros(col_idx.shape[0])
    rc = lib().or_assemble(ETYPE[mesh.etype], mesh.n_elems, _p(mesh.elem), _p(dphi), _p(w),
                           _p(np.ascontiguousarray(D)), _p(row_ptr), _p(col_idx), _p(val))
    if rc:
        raise RuntimeError("triplet outside the pattern")
    return row_ptr, col_idx, val


def K_rows(mesh, dphi, w, D, rows, max_cols=None):
    """Sampled rows of K: list of (cols, vals)."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if max_cols is None:
        max_cols = mesh.dim * 125 * 2
    cols = np.zeros((len(rows), max_cols), dtype=np.int32)
    vals = np.zeros((len(rows), max_cols))
    n = np.zeros(len(rows), dtype=np.int32)
    rc = lib().or_K_rows(ETYPE[mesh.etype], mesh.n_elems, _p(mesh.elem), _p(dphi), _p(w),
                         _p(np.ascontiguousarray(D)), len(rows), _p(rows), max_cols,
                         _p(cols), _p(vals), _p(n))
    if rc:
        raise RuntimeError("max_cols too small")
    return [(cols[i, :n[i]].copy(), vals[i, :n[i]].copy()) for i in range(len(rows))]


def pcg(row_ptr, col_idx, val, free, b, rtol, max_it):
    n = row_ptr.shape[0] - 1
    x = np.zeros(n)
    rel = C.c_double()
    it = lib().or_pcg(n, _p(row_ptr), _p(col_idx), _p(val), _p(np.ascontiguousarray(free)),
                      _p(np.ascontiguousarray(b, dtype=np.float64)), _p(x), rtol, max_it,
                      C.byref(rel))
    return x, it, rel.value


# --------------------------------------------------------------------------
# Semismooth Newton (ALG-NEWTON, Section 4) on top of the oracle pieces
# --------------------------------------------------------------------------

def csr_to_scipy(row_ptr, col_idx, val, n):
    import scipy.sparse as sp
    return sp.csr_matrix((val, col_idx, row_ptr), shape=(n, n))


def energy_norm_increment(Ke, du, u_old):
    """The stopping quantity of ALG-NEWTON (Section 4):
    |du|_e / (|u_old|_e + |u_old + du|_e) with |v|_e^2 = v^T K_elast v."""
    u_new = u_old + du
    a = float(du @ (Ke @ du))
    b = float(u_old @ (Ke @ u_old))
    c = float(u_new @ (Ke @ u_new))
    den = math.sqrt(max(b, 0.0)) + math.sqrt(max(c, 0.0))
    return math.sqrt(max(a, 0.0)) / den if den > 0 else 0.0


def line_search(g, g0, theta, max_evals=12):
    """Step length of the damped Newton method (the damped variant Section 4
    mentions): the Newton correction du is scaled by the minimiser of the
    incremental energy J(u + a du) over a in (0, 1].  J is convex along the
    line (the models are associative), its derivative is -g(a) with
    g(a) = du . Q(f - F(u + a du)) and g(0) = g0 > 0.  The full step is kept
    if g(1) >= -theta g0 (the minimiser is not far before 1); otherwise the
    root of g in (0, 1) is bracketed and found by regula falsi with the
    Illinois modification to |g| <= theta g0.  g is a callable; returns
    (a, number of evaluations of g)."""
    g1 = g(1.0)
    n = 1
    if not (g0 > 0) or g1 >= -theta * g0:
        return 1.0, n
    a, ga, b, gb = 0.0, g0, 1.0, g1
    side = 0
    x = 1.0
    while n < max_evals:
        x = (a * gb - b * ga) / (gb - ga)
        gx = g(x)
        n += 1
        if abs(gx) <= theta * g0:
            break
        if gx > 0:
            a, ga = x, gx
            if side == 1:
                gb *= 0.5
            side = 1
        else:
            b, gb = x, gx
            if side == -1:
                ga *= 0.5
            side = -1
    return x, n


def newton_solve(mesh, material, free, f, u0, ep6, beta6, kappa, *, tol=1e-10,
                 max_it=50, linear="direct", dphi=None, w=None, pattern_=None,
                 history=None, raise_on_limit=True, damping=None):
    """Solve one load step: find u with |Q(f - F(u))| <= tol |Q f| (with
    Q f = 0, under pure displacement control, relative to the reactions
    |(I - Q) F(u)| instead).

    The first iterate is u0 (the previous step's displacement on free dofs;
    Dirichlet values are already in u0).  The linear solve is either a sparse
    direct solve (scipy, tiny meshes) or the oracle's Jacobi-PCG with
    forcing tolerance min(1e-2, |r|/|f|).  damping = theta turns on the
    damped Newton method (line_search with that theta).  history, if given,
    receives per iteration the relative residual, the plastic count and, for
    iterations that made a correction, the step length, the line-search
    evaluations and the energy-norm increment of ALG-NEWTON.  Returns (u,
    its, residual history, last constitutive output); at max_it iterations
    it raises, or returns the last iterate if raise_on_limit is False."""
    import scipy.sparse.linalg as spla
    if dphi is None:
        dphi, w = geometry(mesh)
    if pattern_ is None:
        pattern_ = pattern(mesh)
    row_ptr, col_idx = pattern_
    q = free.astype(bool)
    u = u0.copy()
    fq = np.linalg.norm(f[q])
    res = []
    Ke = None

    def evaluate(v):
        eps = strain(mesh, dphi, v)
        o = constitutive(material, eps, ep6, beta6, kappa)
        F = internal_force(mesh, dphi, w, o["sig"])
        return o, F, (f - F) * free

    for it in range(max_it + 1):
        out, F, r = evaluate(u)
        scale = fq if fq > 0 else np.linalg.norm(F[~q])
        rel = np.linalg.norm(r) / scale if scale > 0 else np.linalg.norm(r)
        res.append(rel)
        rec = dict(rel=rel, n_plastic=int((out["flag"] != 0).sum()))
        if history is not None:
            history.append(rec)
        if rel <= tol:
            return u, it, res, out
        if it == max_it:
            if not raise_on_limit:
                return u, it, res, out
            break
        _, _, val = assemble(mesh, dphi, w, out["D"], row_ptr, col_idx)
        if linear == "direct":
            K = csr_to_scipy(row_ptr, col_idx, val, mesh.n_dof)[q][:, q]
            du = np.zeros(mesh.n_dof)
            du[q] = spla.spsolve(K.tocsc(), r[q])
        else:
            du, pits, _ = pcg(row_ptr, col_idx, val, free, r, min(1e-2, rel), 100000)
            if pits < 0:
                raise RuntimeError("oracle PCG did not converge")
        du = du * free
        alpha, evals = 1.0, 0
        if damping is not None:
            alpha, evals = line_search(lambda a: float(du @ evaluate(u + a * du)[2]),
                                       float(du @ r), damping)
        if history is not None:
            if Ke is None:
                D0 = constitutive(material, np.zeros((mesh.n_int, 6)),
                                  np.zeros((mesh.n_int, 6)))["D"]
                _, _, kv = assemble(mesh, dphi, w, D0, row_ptr, col_idx)
                Ke = csr_to_scipy(row_ptr, col_idx, kv, mesh.n_dof)
            rec.update(step=alpha, ls_evals=evals,
                       energy_incr=energy_norm_increment(Ke, alpha * du, u))
        u = u + alpha * du
    raise RuntimeError(f"Newton did not converge: {res[-5:]}")
