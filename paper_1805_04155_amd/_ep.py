"""ctypes binding of libep.so (include/ep.h).  Argument marshalling only:
torch tensors supply device memory and the HIP stream, every step runs in the
library's kernels.  There is no fallback: if the library is missing or no
HIP device is visible the calls raise."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libep.so")

EP_OK, EP_EINVAL, EP_ENOMEM, EP_EDEVICE, EP_ENOTCONV, EP_ESTATE, EP_ENONFINITE = \
    0, -1, -2, -3, -4, -5, -6
EP_P1, EP_P2, EP_Q1, EP_Q2, EP_Q2S = 1, 2, 3, 4, 5
EP_VM, EP_DP = 1, 2
EP_FP64, EP_FP32, EP_BF16 = 0, 1, 2
EP_OPERATOR_ASSEMBLED, EP_OPERATOR_SPLIT = 0, 1
EP_ASSEMBLY_COLOURS, EP_ASSEMBLY_ROWS, EP_ASSEMBLY_FUSED = 0, 1, 2
ASSEMBLY = {"colours": EP_ASSEMBLY_COLOURS, "rows": EP_ASSEMBLY_ROWS, "fused": EP_ASSEMBLY_FUSED}
PROF = dict(constitutive=0, compaction=1, split=2, assembly=3, force=4, spmv=5, pcg_vec=6,
            elastic=7, pcg_small=8)

ETYPE = {"P1_2D": (2, EP_P1), "Q1_2D": (2, EP_Q1), "Q2_2D": (2, EP_Q2), "P1_3D": (3, EP_P1),
         "P2_3D": (3, EP_P2), "Q1_3D": (3, EP_Q1), "Q2_3D": (3, EP_Q2), "Q2S_2D": (2, EP_Q2S),
         "Q2S_3D": (3, EP_Q2S)}


class EpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ep status {status}: {msg}")
        self.status = status


class ep_mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("type", C.c_int32), ("n_nodes", C.c_int64),
                ("n_elems", C.c_int64), ("coord", C.c_void_p), ("elem", C.c_void_p),
                ("free_mask", C.c_void_p)]


class ep_quadrature(C.Structure):
    _fields_ = [("n_q", C.c_int32), ("xi", C.c_void_p), ("w", C.c_void_p)]


class ep_material(C.Structure):
    _fields_ = [("model", C.c_int32), ("E", C.c_double), ("nu", C.c_double), ("Y", C.c_double),
                ("a", C.c_double), ("eta", C.c_double), ("c", C.c_double)]


class ep_options(C.Structure):
    _fields_ = [("tangent_prec", C.c_int32), ("local_prec", C.c_int32),
                ("pcg_max_it", C.c_int32), ("pcg_check_every", C.c_int32),
                ("newton_rtol", C.c_double), ("pcg_forcing_max", C.c_double),
                ("operator_form", C.c_int32), ("newton_damping", C.c_double),
                ("ls_max_evals", C.c_int32), ("assembly", C.c_int32)]


class ep_sizes(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_p", C.c_int32), ("n_q", C.c_int32),
                ("n_str", C.c_int32), ("n_sc", C.c_int32), ("n_colours", C.c_int32),
                ("n_nodes", C.c_int64), ("n_elems", C.c_int64), ("n_int", C.c_int64),
                ("n_dof", C.c_int64), ("nnz", C.c_int64), ("nnz_blocks", C.c_int64)]


class ep_newton_info(C.Structure):
    _fields_ = [("res_rel", C.c_double), ("res_norm", C.c_double), ("f_norm", C.c_double),
                ("pcg_relres", C.c_double), ("pcg_its", C.c_int32), ("converged", C.c_int32),
                ("n_plastic_ip", C.c_int64), ("n_plastic_elem", C.c_int64),
                ("energy_incr", C.c_double), ("step", C.c_double), ("ls_evals", C.c_int32),
                ("pcg_breakdown", C.c_int32)]


class ep_warm_info(C.Structure):
    _fields_ = [("res_rel_pred", C.c_double), ("res_rel_start", C.c_double),
                ("res_rel_warm", C.c_double), ("pcg_its", C.c_int32), ("accepted", C.c_int32),
                ("n_plastic_pred", C.c_int64)]


MLP_IN, MLP_HID, MLP_OUT, MLP_XS, MLP_YS, MLP_NPARAM = 13, 128, 7, 16, 8, 19207
MLP_NOALLOC_MAX_BATCH = 2048

_lib = None


def lib():
    """Load libep.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(or python paper_1805_04155_amd/build.py) first")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sigs = {
            "ep_setup": [P, P, P, P, P, P],
            "ep_destroy": [P],
            "ep_last_error": [P],
            "ep_set_stream": [P, P],
            "ep_get_sizes": [P, P],
            "ep_set_state": [P, P, P, P],
            "ep_get_state": [P, P, P, P],
            "ep_geometry": [P, P, P],
            "ep_strain": [P, P, P],
            "ep_constitutive": [P, P, P, P, P],
            "ep_assemble_tangent": [P],
            "ep_assemble_elastic": [P],
            "ep_internal_force": [P, P],
            "ep_newton_step": [P, P, P, P],
            "ep_commit_step": [P, P],
            "ep_get_plastic": [P, P, P, P, P],
            "ep_get_csr": [P, I32, P, P, P],
            "ep_get_position_map": [P, P],
            "ep_spmv": [P, P, P],
            "ep_apply_tangent": [P, P, P],
            "ep_pcg": [P, P, P, D, I32, P, P],
            "ep_profile": [P, I32],
            "ep_profile_read": [P, I32, P, P],
            "ep_mlp_create": [I32, I64, P, P],
            "ep_mlp_destroy": [P],
            "ep_mlp_last_error": [P],
            "ep_mlp_set_params": [P, P],
            "ep_mlp_get_params": [P, P],
            "ep_mlp_forward": [P, P, I64, P],
            "ep_mlp_loss_grad": [P, P, P, I64, P, P],
            "ep_mlp_adam_step": [P, P, P, I64, C.c_float, P],
            "ep_mlp_datagen": [P, I64, P, I64, P, P, P, P, P, P, P, P],
            "ep_mlp_features": [P, P, P],
            "ep_warm_start": [P, P, P, P, P, D, D, P, P],
            "ep_predictor": [P, P, P, D, P],
            "ep_mlp_loss_grad_noalloc": [I32, P, P, P, I64, P, P, P],
            "ep_mlp_noalloc_last_error": [],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.ep_destroy.restype = None
        L.ep_last_error.restype = C.c_char_p
        L.ep_mlp_destroy.restype = None
        L.ep_mlp_last_error.restype = C.c_char_p
        L.ep_mlp_noalloc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


EXPORTED = ["ep_setup", "ep_destroy", "ep_last_error", "ep_set_stream", "ep_get_sizes",
            "ep_set_state", "ep_get_state", "ep_geometry", "ep_strain", "ep_constitutive",
            "ep_assemble_tangent", "ep_assemble_elastic", "ep_internal_force", "ep_newton_step",
            "ep_commit_step",
            "ep_get_plastic", "ep_get_csr", "ep_get_position_map", "ep_spmv",
            "ep_apply_tangent", "ep_pcg",
            "ep_profile", "ep_profile_read", "ep_mlp_create", "ep_mlp_destroy",
            "ep_mlp_last_error", "ep_mlp_set_params", "ep_mlp_get_params", "ep_mlp_forward",
            "ep_mlp_loss_grad", "ep_mlp_adam_step", "ep_mlp_datagen", "ep_mlp_features",
            "ep_warm_start", "ep_predictor", "ep_mlp_loss_grad_noalloc",
            "ep_mlp_noalloc_last_error"]


def _ptr(t):
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise TypeError("device pointers must be contiguous CUDA (HIP) tensors")
    return C.c_void_p(t.data_ptr())


_SIZES = {}


def _sizes(ctx):
    """Sizes of a live context (cached until ep_destroy)."""
    key = ctx.value if isinstance(ctx, C.c_void_p) else ctx
    sz = _SIZES.get(key)
    if sz is None:
        sz = _SIZES[key] = ep_get_sizes(ctx)
    return sz


def _dev(t, dtype, n, what):
    """Device pointer of t after checking its element type and that it holds
    at least the n elements the library reads or writes (None passes)."""
    if t is None:
        return None
    import torch
    want = {"f64": torch.float64, "f32": torch.float32, "i32": torch.int32,
            "i64": torch.int64, "u8": torch.uint8}[dtype]
    if not isinstance(t, torch.Tensor) or t.dtype != want:
        raise TypeError(f"{what}: expected a {want} tensor")
    if t.numel() < n:
        raise ValueError(f"{what}: {t.numel()} elements, the context needs {n}")
    return _ptr(t)


def _check(ctx, st):
    if st != EP_OK:
        msg = lib().ep_last_error(ctx)
        raise EpError(st, msg.decode() if msg else "")
    return st


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# --------------------------------------------------------------------------
# Same names as the C ABI
# --------------------------------------------------------------------------

def _material(material):
    return ep_material(EP_VM if material.model == "VM" else EP_DP, material.E, material.nu,
                       material.Y, material.a, material.eta, material.c)


def ep_setup(mesh, free, material, options=None, quadrature=None, stream=None):
    """mesh: workloads.Mesh; free: uint8 (n_dof,); material: workloads.Material;
    options: dict of ep_options fields."""
    dim, et = ETYPE[mesh.etype]
    coord = np.ascontiguousarray(mesh.coord, dtype=np.float64)
    elem = np.ascontiguousarray(mesh.elem, dtype=np.int32)
    free = np.ascontiguousarray(free, dtype=np.uint8)
    m = ep_mesh(dim, et, mesh.n_nodes, mesh.n_elems, coord.ctypes.data, elem.ctypes.data,
                free.ctypes.data)
    mat = _material(material)
    opt = ep_options(EP_FP64, EP_FP64, 20000, 50, 1e-10, 1e-2, EP_OPERATOR_ASSEMBLED, 0.0, 12,
                     EP_ASSEMBLY_COLOURS)
    for k, v in (options or {}).items():
        setattr(opt, k, v)
    q = None
    if quadrature is not None:
        xi = np.ascontiguousarray(quadrature[0], dtype=np.float64)
        w = np.ascontiguousarray(quadrature[1], dtype=np.float64)
        q = ep_quadrature(len(w), xi.ctypes.data, w.ctypes.data)
    h = C.c_void_p()
    st = lib().ep_setup(C.byref(m), C.byref(q) if q is not None else None, C.byref(mat),
                        C.byref(opt), stream if stream is not None else _stream(), C.byref(h))
    _check(None, st)
    return h


def ep_destroy(ctx):
    _SIZES.pop(ctx.value if isinstance(ctx, C.c_void_p) else ctx, None)
    lib().ep_destroy(ctx)


def ep_last_error(ctx):
    return lib().ep_last_error(ctx).decode()


def ep_set_stream(ctx, stream=None):
    _check(ctx, lib().ep_set_stream(ctx, stream if stream is not None else _stream()))


def ep_get_sizes(ctx):
    s = ep_sizes()
    _check(ctx, lib().ep_get_sizes(ctx, C.byref(s)))
    return {k: getattr(s, k) for k, _ in ep_sizes._fields_}


def _state_ptrs(ctx, ep, beta, kappa):
    s = _sizes(ctx)
    n = s["n_sc"] * s["n_int"]
    return (_dev(ep, "f64", n, "ep"), _dev(beta, "f64", n, "beta"),
            _dev(kappa, "f64", s["n_int"], "kappa"))


def ep_set_state(ctx, ep=None, beta=None, kappa=None):
    _check(ctx, lib().ep_set_state(ctx, *_state_ptrs(ctx, ep, beta, kappa)))


def ep_get_state(ctx, ep=None, beta=None, kappa=None):
    _check(ctx, lib().ep_get_state(ctx, *_state_ptrs(ctx, ep, beta, kappa)))


def ep_geometry(ctx, dphi=None, w=None):
    s = _sizes(ctx)
    _check(ctx, lib().ep_geometry(ctx, _dev(dphi, "f64", s["n_int"] * s["n_p"] * s["dim"], "dphi"),
                                  _dev(w, "f64", s["n_int"], "w")))


def ep_strain(ctx, u, eps):
    s = _sizes(ctx)
    _check(ctx, lib().ep_strain(ctx, _dev(u, "f64", s["n_dof"], "u"),
                                _dev(eps, "f64", s["n_str"] * s["n_int"], "eps")))


def ep_constitutive(ctx, u, sig=None, D=None, flag=None):
    s = _sizes(ctx)
    n = s["n_int"]
    _check(ctx, lib().ep_constitutive(ctx, _dev(u, "f64", s["n_dof"], "u"),
                                      _dev(sig, "f64", s["n_sc"] * n, "sig"),
                                      _dev(D, "f64", s["n_str"] ** 2 * n, "D"),
                                      _dev(flag, "u8", n, "flag")))


def ep_assemble_tangent(ctx):
    _check(ctx, lib().ep_assemble_tangent(ctx))


def ep_assemble_elastic(ctx):
    _check(ctx, lib().ep_assemble_elastic(ctx))


def _dof(ctx, t, what):
    return _dev(t, "f64", _sizes(ctx)["n_dof"], what)


def ep_internal_force(ctx, F):
    _check(ctx, lib().ep_internal_force(ctx, _dof(ctx, F, "F")))


def ep_newton_step(ctx, f, u):
    """Returns (status, info dict); EP_ENOTCONV is returned, not raised."""
    info = ep_newton_info()
    st = lib().ep_newton_step(ctx, _dof(ctx, f, "f"), _dof(ctx, u, "u"), C.byref(info))
    if st not in (EP_OK, EP_ENOTCONV):
        _check(ctx, st)
    return st, {k: getattr(info, k) for k, _ in ep_newton_info._fields_}


def ep_commit_step(ctx, u):
    _check(ctx, lib().ep_commit_step(ctx, _dof(ctx, u, "u")))


def ep_get_plastic(ctx, ip=None, elem=None):
    n_ip, n_el = C.c_int64(), C.c_int64()
    s = _sizes(ctx)
    _check(ctx, lib().ep_get_plastic(ctx, _dev(ip, "i32", s["n_int"], "ip"), C.byref(n_ip),
                                     _dev(elem, "i32", s["n_elems"], "elem"), C.byref(n_el)))
    return n_ip.value, n_el.value


def ep_get_csr(ctx, which, row_ptr=None, col_idx=None, val=None):
    s = _sizes(ctx)
    _check(ctx, lib().ep_get_csr(ctx, which, _dev(row_ptr, "i32", s["n_dof"] + 1, "row_ptr"),
                                 _dev(col_idx, "i32", s["nnz"], "col_idx"),
                                 _dev(val, "f64", s["nnz"], "val")))


def ep_get_position_map(ctx, pos):
    s = _sizes(ctx)
    n = s["n_elems"] * (s["dim"] * s["n_p"]) ** 2
    _check(ctx, lib().ep_get_position_map(ctx, _dev(pos, "i32", n, "pos")))


def ep_spmv(ctx, x, y):
    _check(ctx, lib().ep_spmv(ctx, _dof(ctx, x, "x"), _dof(ctx, y, "y")))


def ep_apply_tangent(ctx, x, y):
    _check(ctx, lib().ep_apply_tangent(ctx, _dof(ctx, x, "x"), _dof(ctx, y, "y")))


def ep_pcg(ctx, b, x, rtol, max_it):
    its, rel = C.c_int32(), C.c_double()
    st = lib().ep_pcg(ctx, _dof(ctx, b, "b"), _dof(ctx, x, "x"), rtol, max_it, C.byref(its),
                      C.byref(rel))
    if st not in (EP_OK, EP_ENOTCONV):
        _check(ctx, st)
    return st, its.value, rel.value


EP_PROFILE_ALL = 0x1FF


def ep_profile(ctx, enable, kernels=None):
    """Turns kernel timing on (every kernel id, or only the names in
    `kernels`, keys of PROF) or off."""
    mask = 0
    if enable:
        mask = EP_PROFILE_ALL if kernels is None else sum(1 << PROF[k] for k in set(kernels))
    _check(ctx, lib().ep_profile(ctx, mask))


def ep_profile_read(ctx, k):
    ms, n = C.c_double(), C.c_int64()
    _check(ctx, lib().ep_profile_read(ctx, PROF[k] if isinstance(k, str) else k,
                                      C.byref(ms), C.byref(n)))
    return ms.value, n.value


# --------------------------------------------------------------------------
# Convenience wrapper holding a context and allocating torch outputs
# --------------------------------------------------------------------------

class Context:
    def __init__(self, mesh, free, material, options=None, quadrature=None, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.mesh = mesh
        self.h = ep_setup(mesh, free, material, options, quadrature)
        self.sizes = ep_get_sizes(self.h)

    def close(self):
        if self.h is not None:
            ep_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty(self, shape, dtype=None):
        t = self.torch
        return t.empty(shape, dtype=dtype or t.float64, device=self.device)

    def tensor(self, a, dtype=None):
        t = self.torch
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype or t.float64).to(self.device)

    def set_state(self, ep=None, beta=None, kappa=None):
        ep_set_state(self.h, *(None if a is None else self.tensor(a) for a in (ep, beta, kappa)))

    def get_state(self):
        s = self.sizes
        ep = self._empty((s["n_sc"], s["n_int"]))
        beta = self._empty((s["n_sc"], s["n_int"]))
        kappa = self._empty((s["n_int"],))
        ep_get_state(self.h, ep, beta, kappa)
        return ep, beta, kappa

    def geometry(self):
        s = self.sizes
        dphi = self._empty((s["n_int"], s["n_p"], s["dim"]))
        w = self._empty((s["n_int"],))
        ep_geometry(self.h, dphi, w)
        return dphi, w

    def strain(self, u):
        eps = self._empty((self.sizes["n_str"], self.sizes["n_int"]))
        ep_strain(self.h, u, eps)
        return eps

    def constitutive(self, u, sig=True, D=True, flag=True):
        s = self.sizes
        t = self.torch
        so = self._empty((s["n_sc"], s["n_int"])) if sig else None
        Do = self._empty((s["n_str"] ** 2, s["n_int"])) if D else None
        fo = self._empty((s["n_int"],), t.uint8) if flag else None
        ep_constitutive(self.h, u, so, Do, fo)
        return so, Do, fo

    def assemble_tangent(self):
        ep_assemble_tangent(self.h)

    def internal_force(self):
        F = self._empty((self.sizes["n_dof"],))
        ep_internal_force(self.h, F)
        return F

    def newton_step(self, f, u):
        return ep_newton_step(self.h, f, u)

    def commit_step(self, u):
        ep_commit_step(self.h, u)

    def plastic(self):
        s = self.sizes
        t = self.torch
        ip = self._empty((max(1, s["n_int"]),), t.int32)
        el = self._empty((max(1, s["n_elems"]),), t.int32)
        n_ip, n_el = ep_get_plastic(self.h, ip, el)
        return ip[:n_ip], el[:n_el]

    def csr(self, which):
        s = self.sizes
        t = self.torch
        rp = self._empty((s["n_dof"] + 1,), t.int32)
        ci = self._empty((s["nnz"],), t.int32)
        v = self._empty((s["nnz"],))
        ep_get_csr(self.h, which, rp, ci, v)
        return rp, ci, v

    def position_map(self):
        s = self.sizes
        nl = s["dim"] * s["n_p"]
        pos = self._empty((s["n_elems"], nl, nl), self.torch.int32)
        ep_get_position_map(self.h, pos)
        return pos

    def spmv(self, x):
        y = self._empty((self.sizes["n_dof"],))
        ep_spmv(self.h, x, y)
        return y

    def apply_tangent(self, x):
        y = self._empty((self.sizes["n_dof"],))
        ep_apply_tangent(self.h, x, y)
        return y

    def pcg(self, b, rtol, max_it=100000):
        x = self._empty((self.sizes["n_dof"],))
        st, its, rel = ep_pcg(self.h, b, x, rtol, max_it)
        return x, st, its, rel

    def mlp_features(self, u):
        X = self._empty((self.sizes["n_int"], MLP_XS), self.torch.float32)
        ep_mlp_features(self.h, u, X)
        return X

    def warm_start(self, mlp, f, u_prev, u_prev2, extrap, pcg_rtol, u_out):
        return ep_warm_start(self.h, mlp.h, f, u_prev, u_prev2, extrap, pcg_rtol, u_out)


# ---- learned warm start ----

def _check_mlp(m, st):
    if st != EP_OK:
        msg = lib().ep_mlp_last_error(m)
        raise EpError(st, msg.decode() if msg else "")
    return st


def ep_mlp_create(prec, max_batch, stream=None):
    h = C.c_void_p()
    _check(None, lib().ep_mlp_create(prec, max_batch,
                                     stream if stream is not None else _stream(), C.byref(h)))
    return h


def ep_mlp_destroy(m):
    lib().ep_mlp_destroy(m)


def ep_mlp_last_error(m):
    return lib().ep_mlp_last_error(m).decode()


def ep_mlp_set_params(m, params):
    _check_mlp(m, lib().ep_mlp_set_params(m, _dev(params, "f32", MLP_NPARAM, "params")))


def ep_mlp_get_params(m, params):
    _check_mlp(m, lib().ep_mlp_get_params(m, _dev(params, "f32", MLP_NPARAM, "params")))


def ep_mlp_forward(m, X, n, Y):
    _check_mlp(m, lib().ep_mlp_forward(m, _dev(X, "f32", n * MLP_XS, "X"), n,
                                       _dev(Y, "f32", n * MLP_YS, "Y")))


def ep_mlp_loss_grad(m, X, T, n, grad=None, loss=None):
    _check_mlp(m, lib().ep_mlp_loss_grad(m, _dev(X, "f32", n * MLP_XS, "X"),
                                         _dev(T, "f32", n * MLP_YS, "T"), n,
                                         _dev(grad, "f32", MLP_NPARAM, "grad"),
                                         _dev(loss, "f32", 1, "loss")))


def ep_mlp_loss_grad_noalloc(prec, params, X, T, n, grad=None, loss=None, stream=None):
    """Loss gradient of the network given by its parameters (device, float32)
    with the library's static device scratch (allocates nothing)."""
    st = lib().ep_mlp_loss_grad_noalloc(int(prec), _dev(params, "f32", MLP_NPARAM, "params"),
                                        _dev(X, "f32", max(n, 0) * MLP_XS, "X"),
                                        _dev(T, "f32", max(n, 0) * MLP_YS, "T"), int(n),
                                        _dev(grad, "f32", MLP_NPARAM, "grad"),
                                        _dev(loss, "f32", 1, "loss"),
                                        stream if stream is not None else _stream())
    if st != EP_OK:
        raise EpError(st, lib().ep_mlp_noalloc_last_error().decode())


def ep_mlp_noalloc_last_error():
    return lib().ep_mlp_noalloc_last_error().decode()


def ep_mlp_adam_step(m, X, T, n, lr, loss=None):
    _check_mlp(m, lib().ep_mlp_adam_step(m, _dev(X, "f32", n * MLP_XS, "X"),
                                         _dev(T, "f32", n * MLP_YS, "T"), n, float(lr),
                                         _dev(loss, "f32", 1, "loss")))


def ep_mlp_datagen(material, n, idx, n_pool, eps_pool, ep_pool, beta_pool, kappa_pool, deps,
                   X, T, stream=None):
    mat = _material(material)
    pool = 6 * n_pool
    _check(None, lib().ep_mlp_datagen(C.byref(mat), n, _dev(idx, "i64", n, "idx"), n_pool,
                                      _dev(eps_pool, "f64", pool, "eps_pool"),
                                      _dev(ep_pool, "f64", pool, "ep_pool"),
                                      _dev(beta_pool, "f64", pool, "beta_pool"),
                                      _dev(kappa_pool, "f64", n_pool, "kappa_pool"),
                                      _dev(deps, "f64", 6 * n, "deps"),
                                      _dev(X, "f32", n * MLP_XS, "X"),
                                      _dev(T, "f32", n * MLP_YS, "T"),
                                      stream if stream is not None else _stream()))


def ep_mlp_features(ctx, u, X):
    _check(ctx, lib().ep_mlp_features(ctx, _dof(ctx, u, "u"),
                                      _dev(X, "f32", _sizes(ctx)["n_int"] * MLP_XS, "X")))


def ep_predictor(ctx, u_prev, u_prev2, extrap, u_out):
    _check(ctx, lib().ep_predictor(ctx, _dof(ctx, u_prev, "u_prev"), _dof(ctx, u_prev2, "u_prev2"),
                                   float(extrap), _dof(ctx, u_out, "u_out")))


def ep_warm_start(ctx, m, f, u_prev, u_prev2, extrap, pcg_rtol, u_out):
    info = ep_warm_info()
    st = lib().ep_warm_start(ctx, m, _dof(ctx, f, "f"), _dof(ctx, u_prev, "u_prev"),
                             _dof(ctx, u_prev2, "u_prev2"), float(extrap), float(pcg_rtol),
                             _dof(ctx, u_out, "u_out"), C.byref(info))
    if st not in (EP_OK, EP_ENOTCONV):
        _check(ctx, st)
    return st, {k: getattr(info, k) for k, _ in ep_warm_info._fields_}


class Mlp:
    """Owns an ep_mlp handle; torch tensors for inputs and outputs."""

    def __init__(self, prec=EP_FP32, max_batch=8192):
        import torch
        self.torch = torch
        self.prec = prec
        self.max_batch = max_batch
        self.h = ep_mlp_create(prec, max_batch)

    def close(self):
        if self.h is not None:
            ep_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        t = self.torch.as_tensor(np.ascontiguousarray(params, dtype=np.float32)).cuda() \
            if not isinstance(params, self.torch.Tensor) else params.contiguous()
        ep_mlp_set_params(self.h, t)
        self.torch.cuda.synchronize()

    def params(self):
        p = self.torch.empty(MLP_NPARAM, dtype=self.torch.float32, device="cuda")
        ep_mlp_get_params(self.h, p)
        return p

    def forward(self, X):
        n = X.shape[0]
        Y = self.torch.empty((n, MLP_YS), dtype=self.torch.float32, device="cuda")
        ep_mlp_forward(self.h, X, n, Y)
        return Y

    def loss_grad(self, X, T):
        g = self.torch.empty(MLP_NPARAM, dtype=self.torch.float32, device="cuda")
        loss = self.torch.empty(1, dtype=self.torch.float32, device="cuda")
        ep_mlp_loss_grad(self.h, X, T, X.shape[0], g, loss)
        return g, loss

    def adam_step(self, X, T, lr, loss=None):
        ep_mlp_adam_step(self.h, X, T, X.shape[0], lr, loss)
