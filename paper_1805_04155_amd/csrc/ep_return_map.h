// Return maps of the two material models on single points (device code),
// shared by the constitutive kernels and the training-data generator.
#pragma once
#include "ep_internal.h"

namespace ep {

// ----------------------------------------------------------------------------
// Return maps on Voigt vectors.  eps, ep: strain-type (engineering shears);
// sig, beta, n: stress-type.  desc receives the tangent increment
//   D - C = alpha*DEV + b*n n^T + g*(n 1^T + 1 n^T) + d*1 1^T
// as [n(6), alpha, b, g, d] with DEV the deviatoric projector mapping
// strain-type to stress-type vectors and 1 = (1,1,1,0,0,0).
// ----------------------------------------------------------------------------
__device__ inline void trial(const MatC &m, const double eps[6], const double ep[6], double dv[6],
                             double &tr) {
  double e[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) e[i] = eps[i] - ep[i];
  tr = e[0] + e[1] + e[2];
  const double t3 = tr / 3.0;
  dv[0] = e[0] - t3;
  dv[1] = e[1] - t3;
  dv[2] = e[2] - t3;
  dv[3] = 0.5 * e[3];
  dv[4] = 0.5 * e[4];
  dv[5] = 0.5 * e[5];
}

// von Mises, linear kinematic hardening (eqs. T_kinematic, DT_kinematic, T_other)
__device__ inline int rm_vm(const MatC &m, const double eps[6], double ep[6], double beta[6],
                           double sig[6], double desc[10], bool commit) {
#pragma clang fp contract(off)
  double dv[6], tr;
  trial(m, eps, ep, dv, tr);
  const double G2 = 2.0 * m.G;
  double s[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    sig[i] = G2 * dv[i] + (i < 3 ? m.K * tr : 0.0);
    s[i] = G2 * dv[i] - beta[i];
  }
  const double ns = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] +
                         2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
  const double crit = ns - m.Y;
  if (!(crit > 0.0)) return 0;
  const double h = G2 + m.a;
  const double dl = crit / h;
  const double c1 = G2 * G2 / h;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const double n = s[i] / ns;
    desc[i] = n;
    sig[i] -= G2 * dl * n;
    if (commit) {
      ep[i] += (i < 3 ? 1.0 : 2.0) * dl * n;
      beta[i] += m.a * dl * n;
    }
  }
  desc[6] = c1 * (m.Y / ns - 1.0);
  desc[7] = -c1 * m.Y / ns;
  desc[8] = 0.0;
  desc[9] = 0.0;
  return 1;
}

// Drucker-Prager with yield function |s|/sqrt2 + eta p - (c + a kappa)
// (Section 2.3; a = 0 perfect plasticity).  1 = smooth cone, 2 = apex.
__device__ inline int rm_dp(const MatC &m, const double eps[6], double ep[6], double &kappa,
                           double sig[6], double desc[10], bool commit) {
#pragma clang fp contract(off)
  const double r2 = 1.4142135623730951;
  double dv[6], tr;
  trial(m, eps, ep, dv, tr);
  const double G2 = 2.0 * m.G;
  const double p = m.K * tr;
  const double dd = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2] +
                    2.0 * (dv[3] * dv[3] + dv[4] * dv[4] + dv[5] * dv[5]);
  const double rho = G2 * sqrt(dd);
#pragma unroll
  for (int i = 0; i < 6; ++i) sig[i] = G2 * dv[i] + (i < 3 ? p : 0.0);
  const double ck = m.c + m.a * kappa;
  const double Ke2 = m.K * m.eta * m.eta;
  const double crit1 = rho / r2 + m.eta * p - ck;
  const double crit2 = m.eta * p - ck - (Ke2 + m.a) * rho / (r2 * m.G);
  if (!(crit1 > 0.0)) return 0;
  if (crit2 <= 0.0) {
    const double h = m.G + Ke2 + m.a;
    const double dl = crit1 / h;
    const double c2 = 2.0 * r2 * m.G * m.G * dl / rho;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const double n = G2 * dv[i] / rho;
      desc[i] = n;
      sig[i] -= dl * (r2 * m.G * n + (i < 3 ? m.K * m.eta : 0.0));
      if (commit) ep[i] += i < 3 ? dl * (n / r2 + m.eta / 3.0) : 2.0 * dl * n / r2;
    }
    desc[6] = -c2;
    desc[7] = c2 - 2.0 * m.G * m.G / h;
    desc[8] = -r2 * m.G * m.K * m.eta / h;
    desc[9] = -Ke2 * m.K / h;
    if (commit) kappa += dl;
    return 1;
  }
  const double dl = (m.eta * p - ck) / (Ke2 + m.a);
  const double pk = p - m.K * m.eta * dl;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    sig[i] = i < 3 ? pk : 0.0;
    desc[i] = 0.0;
    if (commit) ep[i] = i < 3 ? eps[i] - pk / (3.0 * m.K) : eps[i];
  }
  desc[6] = -G2;
  desc[7] = 0.0;
  desc[8] = 0.0;
  desc[9] = -Ke2 * m.K / (Ke2 + m.a);
  if (commit) kappa += dl;
  return 2;
}

// Full Voigt tangent entry (I, J) = C + (D - C) from the descriptor.
__device__ inline double tangent_entry(const MatC &m, const double *desc, bool plastic, int I,
                                       int J) {
  const double one_I = I < 3 ? 1.0 : 0.0, one_J = J < 3 ? 1.0 : 0.0;
  const double dev = (I == J ? (I < 3 ? 1.0 : 0.5) : 0.0) - one_I * one_J / 3.0;
  double v = 2.0 * m.G * dev + m.K * one_I * one_J;
  if (plastic) {
    const double nI = desc[I], nJ = desc[J];
    v += desc[6] * dev + desc[7] * nI * nJ + desc[8] * (nI * one_J + one_I * nJ) +
         desc[9] * one_I * one_J;
  }
  return v;
}

// Tangent descriptor of the trial state on a branch given from outside (the
// learned warm start's predicted plastic flag) rather than by the yield
// test.  von Mises: the consistent tangent of eq. DT_kinematic with the
// radius ratio Y/|s_tr| capped at 1, so a point predicted plastic but inside
// the yield surface gets the continuum tangent C - c1 n n^T.  Drucker-Prager:
// the cone or apex branch by the same trial test as rm_dp, with the
// multiplier max(CRIT1, 0)/h.  Returns 1 (cone / von Mises) or 2 (apex).
__device__ inline int predicted_tangent(const MatC &m, const double eps[6], const double ep[6],
                                        const double beta[6], double kappa, double desc[10]) {
#pragma clang fp contract(off)
  double dv[6], tr;
  trial(m, eps, ep, dv, tr);
  const double G2 = 2.0 * m.G;
  if (m.model == EP_VM) {
    double s[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) s[i] = G2 * dv[i] - beta[i];
    const double ns = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] +
                           2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
    const double c1 = G2 * G2 / (G2 + m.a);
    const double r = ns > m.Y ? m.Y / ns : 1.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) desc[i] = ns > 0.0 ? s[i] / ns : 0.0;
    desc[6] = c1 * (r - 1.0);
    desc[7] = -c1 * r;
    desc[8] = 0.0;
    desc[9] = 0.0;
    return 1;
  }
  const double r2 = 1.4142135623730951;
  const double p = m.K * tr;
  const double dd = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2] +
                    2.0 * (dv[3] * dv[3] + dv[4] * dv[4] + dv[5] * dv[5]);
  const double rho = G2 * sqrt(dd);
  const double ck = m.c + m.a * kappa;
  const double Ke2 = m.K * m.eta * m.eta;
  const double crit1 = rho / r2 + m.eta * p - ck;
  const double crit2 = m.eta * p - ck - (Ke2 + m.a) * rho / (r2 * m.G);
  if (crit2 <= 0.0) {
    const double h = m.G + Ke2 + m.a;
    const double dl = crit1 > 0.0 ? crit1 / h : 0.0;
    const double c2 = rho > 0.0 ? 2.0 * r2 * m.G * m.G * dl / rho : 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) desc[i] = rho > 0.0 ? G2 * dv[i] / rho : 0.0;
    desc[6] = -c2;
    desc[7] = c2 - 2.0 * m.G * m.G / h;
    desc[8] = -r2 * m.G * m.K * m.eta / h;
    desc[9] = -Ke2 * m.K / h;
    return 1;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) desc[i] = 0.0;
  desc[6] = -G2;
  desc[7] = 0.0;
  desc[8] = 0.0;
  desc[9] = -Ke2 * m.K / (Ke2 + m.a);
  return 2;
}

}  // namespace ep
