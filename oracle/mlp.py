"""Plain FP64 CPU oracle of the learned warm start (not part of the paper's
method; the exact return map it is trained on is Sections 2.2 and 2.3).

TEST INFRASTRUCTURE ONLY: imported by tests/ and the smoke check, never by
the HIP product path.

The network is the per-point MLP 13 -> 128 -> 128 -> 7 with ReLU, written
out with numpy matrix products in float64:
    h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3,
its loss over a batch of n samples
    L = (1/n) sum_s [ (1/6) sum_{j<6} (y_j - t_j)^2 + log(1 + e^{y_6}) - t_6 y_6 ],
the gradient by the chain rule (backpropagation), and Adam (Kingma & Ba,
2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias correction.

Features and targets (the same encoding the library documents):
    x = [s_in (eps - eps_p), s_in eps_p, s_in kappa, 0, 0, 0],
    t = [s_out (sigma - sigma_tr), plastic flag, 0],   s_in = E/S, s_out = 1/S,
with S = sqrt(3/2) Y (von Mises) or c (Drucker-Prager) and sigma_tr =
C (eps - eps_p) the elastic trial stress: the network learns the plastic
correction of the stress, which is zero at elastic points.

The learned constitutive step and the warm start follow their definitions:
the network's flag selects the branch, the tangent is the consistent
tangent of the trial state on that branch (eq. DT_kinematic for von Mises
with the radius ratio capped at 1; the cone / apex tangents of Section 2.3
for Drucker-Prager with the multiplier max(CRIT1, 0)/h), the stress is the
trial stress plus the network's correction at predicted-plastic points and
the trial stress elsewhere; one direct solve with that tangent and residual
gives the candidate start, kept only if its exact residual is below the
plain start's.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O

NI, NH, NO, XS, YS = 13, 128, 7, 16, 8
SIZES = [("W1", (NH, NI)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
         ("W3", (NO, NH)), ("b3", (NO,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(params):
    """Parameter vector -> dict of float64 arrays (W[out][in])."""
    p = np.asarray(params, dtype=np.float64)
    out, k = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[k:k + n].reshape(shape)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def forward(params, X):
    """Outputs y (n, 7) and the activations needed by backward."""
    P = unpack(params)
    x = np.asarray(X, dtype=np.float64)[:, :NI]
    a1 = x @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ P["W3"].T + P["b3"]
    return y, (x, a1, h1, a2, h2)


def softplus(z):
    """log(1 + e^z) without overflow."""
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def loss(params, X, T):
    y, _ = forward(params, X)
    t = np.asarray(T, dtype=np.float64)
    n = y.shape[0]
    mse = ((y[:, :6] - t[:, :6]) ** 2).sum(axis=1) / 6.0
    bce = softplus(y[:, 6]) - t[:, 6] * y[:, 6]
    return float((mse + bce).sum() / n)


def loss_grad(params, X, T):
    """(L, dL/dparams) by backpropagation."""
    P = unpack(params)
    y, (x, a1, h1, a2, h2) = forward(params, X)
    t = np.asarray(T, dtype=np.float64)
    n = y.shape[0]
    L = loss(params, X, T)
    dy = np.zeros_like(y)
    dy[:, :6] = (2.0 / 6.0) * (y[:, :6] - t[:, :6]) / n
    dy[:, 6] = (1.0 / (1.0 + np.exp(-y[:, 6])) - t[:, 6]) / n
    g = {"W3": dy.T @ h2, "b3": dy.sum(axis=0)}
    dh2 = (dy @ P["W3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ P["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ x
    g["b1"] = dh1.sum(axis=0)
    return L, pack(g)


def adam_step(params, m, v, grad, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Encoding and sample generation
# ---------------------------------------------------------------------------

def scales(material):
    S = math.sqrt(1.5) * material.Y if material.model == "VM" else material.c
    return material.E / S, 1.0 / S


def back_stress(material, ep6):
    """beta = a eps_p as tensors (stress-type shears are halved)."""
    b = material.a * np.asarray(ep6, dtype=np.float64)
    b = b.copy()
    b[:, 3:] *= 0.5
    return b


def encode(material, eps6, ep6, kappa):
    """Features (n, 16) float32 of trial states (float64 in, one rounding)."""
    s_in, _ = scales(material)
    n = eps6.shape[0]
    X = np.zeros((n, XS))
    X[:, 0:6] = s_in * (eps6 - ep6)
    X[:, 6:12] = s_in * ep6
    X[:, 12] = s_in * kappa
    return X.astype(np.float32)


def datagen(material, idx, eps_pool, ep_pool, beta_pool, kappa_pool, deps):
    """Samples of the exact return map at pooled states plus increments.
    Pools are [6][n_pool] (kappa [n_pool]), deps [6][n]; returns (X, T)
    float32 with rows of out-of-range indices zero."""
    idx = np.asarray(idx)
    n_pool = eps_pool.shape[1]
    ok = (idx >= 0) & (idx < n_pool)
    i = np.where(ok, idx, 0)
    eps = (eps_pool[:, i] + deps).T
    ep6 = ep_pool[:, i].T
    beta6 = beta_pool[:, i].T if beta_pool is not None else back_stress(material, ep6)
    kappa = kappa_pool[i] if kappa_pool is not None else np.zeros(len(i))
    out = O.constitutive(material, eps, ep6, beta6, kappa)
    X = encode(material, eps, ep6, kappa)
    _, s_out = scales(material)
    C, _, _ = _elastic(material)
    T = np.zeros((len(i), YS))
    T[:, :6] = s_out * (out["sig"] - (eps - ep6) @ C.T)
    T[:, 6] = out["flag"] != 0
    T = T.astype(np.float32)
    X[~ok] = 0
    T[~ok] = 0
    return X, T


# ---------------------------------------------------------------------------
# Learned constitutive step and warm start
# ---------------------------------------------------------------------------

def _elastic(material):
    G, K = material.shear, material.bulk
    one = np.array([1.0, 1, 1, 0, 0, 0])
    dev = np.diag([1.0, 1, 1, 0.5, 0.5, 0.5]) - np.outer(one, one) / 3.0
    return 2.0 * G * dev + K * np.outer(one, one), dev, one


def predicted_tangent(material, eps6, ep6, beta6, kappa):
    """Consistent tangent (n, 6, 6) of each trial state taken as plastic."""
    G, K, a = material.shear, material.bulk, material.a
    C, dev, one = _elastic(material)
    n = eps6.shape[0]
    D = np.zeros((n, 6, 6))
    for k in range(n):
        e = eps6[k] - ep6[k]
        tr = e[:3].sum()
        dv = np.array([e[0] - tr / 3, e[1] - tr / 3, e[2] - tr / 3, e[3] / 2, e[4] / 2, e[5] / 2])
        if material.model == "VM":
            s = 2 * G * dv - beta6[k]
            ns = math.sqrt((s[:3] ** 2).sum() + 2 * (s[3:] ** 2).sum())
            nv = s / ns if ns > 0 else np.zeros(6)
            c1 = 4 * G * G / (2 * G + a)
            r = material.Y / ns if ns > material.Y else 1.0
            D[k] = C - c1 * dev + c1 * r * (dev - np.outer(nv, nv))
        else:
            eta, c = material.eta, material.c + a * kappa[k]
            p = K * tr
            rho = 2 * G * math.sqrt((dv[:3] ** 2).sum() + 2 * (dv[3:] ** 2).sum())
            crit1 = rho / math.sqrt(2) + eta * p - c
            crit2 = eta * p - c - (K * eta * eta + a) * rho / (math.sqrt(2) * G)
            if crit2 <= 0:
                h = G + K * eta * eta + a
                dl = max(crit1, 0.0) / h
                nv = 2 * G * dv / rho if rho > 0 else np.zeros(6)
                M = math.sqrt(2) * G * nv + K * eta * one
                c2 = 2 * math.sqrt(2) * G * G * dl / rho if rho > 0 else 0.0
                D[k] = C - c2 * (dev - np.outer(nv, nv)) - np.outer(M, M) / h
            else:
                D[k] = (K * a / (K * eta * eta + a)) * np.outer(one, one)
    return D


def learned_constitutive(material, eps6, ep6, beta6, kappa, Y):
    """Flag, stress and tangent of the learned step from network outputs Y."""
    C, _, _ = _elastic(material)
    S = 1.0 / scales(material)[1]
    flag = np.asarray(Y)[:, 6] > 0
    sig = (eps6 - ep6) @ C.T
    D = np.repeat(C[None], eps6.shape[0], axis=0)
    if flag.any():
        sig[flag] += S * np.asarray(Y, dtype=np.float64)[flag, :6]
        D[flag] = predicted_tangent(material, eps6[flag], ep6[flag], beta6[flag], kappa[flag])
    return flag, sig, D


def features(mesh, material, u, ep6, kappa, dphi=None):
    if dphi is None:
        dphi, _ = O.geometry(mesh)
    eps = O.strain(mesh, dphi, u)
    return encode(material, eps, ep6, kappa)


def warm_start(mesh, material, free, f, u_prev, u_prev2, extrap, ep6, beta6, kappa, network):
    """The learned start: network(features) -> Y at the extrapolated u, one
    direct solve with the learned tangent and residual, accepted if its exact
    residual is below the plain start's.  network maps float32 features to
    outputs Y.  Returns (u_out, info dict)."""
    import scipy.sparse.linalg as spla
    dphi, w = O.geometry(mesh)
    rp, ci = O.pattern(mesh)
    q = free.astype(bool)
    fq = np.linalg.norm(f[q])

    def exact_res(u):
        out = O.constitutive(material, O.strain(mesh, dphi, u), ep6, beta6, kappa)
        F = O.internal_force(mesh, dphi, w, out["sig"])
        return np.linalg.norm(((f - F) * free)[q]) / fq

    u_pred = u_prev.copy()
    if u_prev2 is not None:
        u_pred[q] = u_prev[q] + extrap * (u_prev[q] - u_prev2[q])
    X = features(mesh, material, u_pred, ep6, kappa, dphi)
    Y = network(X)
    eps = O.strain(mesh, dphi, u_pred)
    flag, sig, D = learned_constitutive(material, eps, ep6, beta6, kappa, Y)
    F = O.internal_force(mesh, dphi, w, sig)
    r = (f - F) * free
    _, _, val = O.assemble(mesh, dphi, w, D, rp, ci)
    K = O.csr_to_scipy(rp, ci, val, mesh.n_dof)[q][:, q]
    w_ = u_pred.copy()
    w_[q] += spla.spsolve(K.tocsc(), r[q])
    info = dict(res_rel_pred=np.linalg.norm(r[q]) / fq, res_rel_start=exact_res(u_prev),
                res_rel_warm=exact_res(w_), n_plastic_pred=int(flag.sum()))
    info["accepted"] = int(info["res_rel_warm"] < info["res_rel_start"])
    return (w_ if info["accepted"] else u_prev.copy()), info
