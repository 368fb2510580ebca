// HIP kernels of the elastoplastic Newton hot path, written for CDNA4 (gfx950).
//
// Method: Cermak, Sysala, Valdman (arXiv 1805.04155).  Data layout: per-point
// arrays are structure-of-arrays [component][n_int]; the stiffness matrix is
// stored as node blocks (dim x dim values contiguous) in a CSR over nodes;
// element contributions reach it through an element position map of node
// pairs.  Geometry (Jacobian, inverse, gradients, weights) is recomputed from
// the element's node coordinates staged in LDS instead of storing B: this
// trades a few hundred FP64 operations per point for the bytes a stored B
// would cost, which is the right trade for these HBM-bound kernels.
//
// Determinism: every reduction has a fixed order; the scatter of element
// matrices uses colour rounds (elements of one colour share no node) and no
// floating-point atomics.
#include <cfloat>

#include "ep_internal.h"
#include "ep_return_map.h"

namespace ep {

#define RT(x)                                  \
  do {                                         \
    hipError_t e__ = (x);                      \
    if (e__ != hipSuccess) return e__;         \
  } while (0)

static inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Per-thread part of a one-block reduction of n partial results:
// sum over b = t, t + nt, t + 2 nt, ... < n of p[b * stride] in increasing
// b.  The loads of U strides are issued together, the last group masked
// (a reduction kernel that runs as a single block takes as long as its
// rounds of load latency; U = 16 where many blocks repeat the sum); the
// additions keep the stride order, so U does not change the result.
template <int U = 16>
__device__ inline double strided_sum(const double *p, int n, int stride, int t, int nt) {
  double v = 0.0;
  for (int b = t; b < n; b += U * nt) {
    double x[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int bj = b + j * nt;
      x[j] = bj < n ? p[(int64_t)bj * stride] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (b + j * nt < n) v += x[j];
  }
  return v;
}

// Both sums of interleaved pairs (p[2b], p[2b + 1]) in one pass, each as
// strided_sum would form it.
template <int U>
__device__ inline void strided_sum_pairs(const double *p, int n, int t, int nt, double &sa,
                                         double &sb) {
  double va = 0.0, vb = 0.0;
  for (int b = t; b < n; b += U * nt) {
    double x[U], y[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int bj = b + j * nt;
      x[j] = bj < n ? p[2 * (int64_t)bj] : 0.0;
      y[j] = bj < n ? p[2 * (int64_t)bj + 1] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (b + j * nt < n) {
        va += x[j];
        vb += y[j];
      }
  }
  sa = va;
  sb = vb;
}

// ----------------------------------------------------------------------------
// Geometry: J_ij = sum_p dphi_p/dxi_i x_{p,j} (eq. Jacobian); grad_x = J^{-1}
// grad_xi (eq. Jacobian2).  Returns det J.
// ----------------------------------------------------------------------------
template <int D, int NP>
__device__ inline double jac_inv(const double *xs, const double *dr, double Ji[D][D]) {
  double J[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) J[i][j] = 0.0;
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) J[i][j] += dr[p * D + i] * xs[p * D + j];
  double det;
  if constexpr (D == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double id = 1.0 / det;
    Ji[0][0] = J[1][1] * id;
    Ji[0][1] = -J[0][1] * id;
    Ji[1][0] = -J[1][0] * id;
    Ji[1][1] = J[0][0] * id;
  } else {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = 1.0 / det;
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  }
  return det;
}

template <int D>
__device__ inline void grad(const double Ji[D][D], const double *drp, double g[D]) {
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) s += Ji[i][k] * drp[k];
    g[i] = s;
  }
}

// ----------------------------------------------------------------------------
// Fused constitutive pass: strain, return map, tangent descriptor, element
// force vectors and plastic bitmask.  One thread per integration point; the
// EPB elements of a block stage their node coordinates and displacements in
// LDS.  Element e, point q -> ip = e*NQ + q.
// ----------------------------------------------------------------------------
struct KC {
  const double *coord;
  const int32_t *elem;
  const double *ref;
  int64_t n_n, n_e, n_int;
  const double *u;
  MatC m;
  double *ep, *beta, *kappa;
  uint8_t *flag;
  double *desc;
  double *Fe;
  const int32_t *fslot;
  uint32_t *emask;
  double *eps_out, *sig_out, *D_out;
  uint8_t *flag_out;
  int rm, commit, force;
  float *mlp_x;          // features out (LM = 1)
  const float *mlp_y;    // network outputs in (LM = 2)
  double s_in, S;        // feature scale E/S and stress scale S
};

constexpr int CT = 256;  // threads of the constitutive kernel

// LM = 0: exact return map.  LM = 1: per-point features of the learned warm
// start instead (trial elastic strain, plastic strain, kappa, scaled).
// LM = 2: plastic flag and stress from the network outputs; the tangent
// descriptor is that of the trial state on the predicted branch.
template <int ETID, int MODEL, int LM>
__global__ __launch_bounds__(CT) __attribute__((amdgpu_waves_per_eu(Et<ETID>::D == 2 ? 5 : 1, 8)))
void k_constitutive(KC a) {
  using T = Et<ETID>;
  constexpr int D = T::D, NP = T::NP, NQ = T::NQ;
  constexpr int EPB = CT / NQ;
  constexpr int NF = D * D;           // per point: A = w sigma J^{-T} (see the force phase)
  constexpr int NSC = D == 3 ? 6 : 4; // stored state components
  constexpr int NSTR = D == 3 ? 6 : 3;
  constexpr bool STASH = NP <= 8;
  __shared__ double s_ref[NQ * NP * D];
  __shared__ double s_wq[NQ];
  __shared__ double s_x[EPB * NP * D];
  __shared__ double s_u[EPB * NP * D];
  __shared__ double s_f[EPB * NQ * NF];
  __shared__ uint32_t s_mask[EPB];

  const int tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  for (int t = tid; t < NQ * NP * D; t += CT) s_ref[t] = a.ref[t];
  for (int t = tid; t < NQ; t += CT) s_wq[t] = a.ref[NQ * NP * D + t];
  for (int t = tid; t < EPB; t += CT) s_mask[t] = 0u;
  for (int t = tid; t < EPB * NP; t += CT) {
    const int64_t e = e0 + t / NP;
    if (e < a.n_e) {
      const int64_t node = a.elem[e * NP + t % NP];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        s_x[t * D + d] = a.coord[d * a.n_n + node];
        s_u[t * D + d] = a.u ? a.u[D * node + d] : 0.0;
      }
    }
  }
  __syncthreads();

  const int el = tid / NQ, q = tid - (tid / NQ) * NQ;
  const int64_t e = e0 + el;
  if (tid < EPB * NQ && e < a.n_e) {
    const int64_t ip = e * NQ + q;
    const int64_t N = a.n_int;
    const double *xs = s_x + el * NP * D, *us = s_u + el * NP * D, *dr = s_ref + q * NP * D;
    double Ji[D][D];
    const double det = jac_inv<D, NP>(xs, dr, Ji);
    const double w = fabs(det) * s_wq[q];
    // strain E = B u (eq. local_strain-displ), engineering Voigt.  The
    // gradients sum to zero, so E = sum_{p>=1} g_p (u_p - u_0): the
    // differences of nearby displacements are exact and the large common part
    // of u (rigid motion, gravity sag) does not enter the rounding.
    double eps[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int p = 1; p < NP; ++p) {
      double g[D];
      grad<D>(Ji, dr + p * D, g);
      double up[D];
#pragma unroll
      for (int d = 0; d < D; ++d) up[d] = us[p * D + d] - us[d];
      if constexpr (D == 3) {
        eps[0] += g[0] * up[0];
        eps[1] += g[1] * up[1];
        eps[2] += g[2] * up[2];
        eps[3] += g[1] * up[0] + g[0] * up[1];
        eps[4] += g[2] * up[1] + g[1] * up[2];
        eps[5] += g[2] * up[0] + g[0] * up[2];
      } else {
        eps[0] += g[0] * up[0];
        eps[1] += g[1] * up[1];
        eps[3] += g[1] * up[0] + g[0] * up[1];
      }
    }
    // elements of up to 8 nodes: w J^{-1} waits in this point's slot of the
    // force LDS while the return map runs (fewer registers live across it:
    // 8-node hexahedra 136 -> 125, 4 instead of 3 waves per SIMD; the larger
    // elements need more registers that way)
    if (STASH && a.force) {
      double *sf = s_f + tid * NF;
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) sf[i * D + j] = w * Ji[i][j];
    }
    if (a.eps_out) {
      if constexpr (D == 3) {
#pragma unroll
        for (int i = 0; i < 6; ++i) a.eps_out[i * N + ip] = eps[i];
      } else {
        a.eps_out[0 * N + ip] = eps[0];
        a.eps_out[1 * N + ip] = eps[1];
        a.eps_out[2 * N + ip] = eps[3];
      }
    }
    double sig[6] = {0, 0, 0, 0, 0, 0};
    if constexpr (LM == 1) {
      double ep[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int c = 0; c < NSC; ++c) ep[c] = a.ep[c * N + ip];
      const double kap = MODEL == EP_DP ? a.kappa[ip] : 0.0;
      float *x = a.mlp_x + ip * EP_MLP_XS;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        x[c] = (float)(a.s_in * (eps[c] - ep[c]));
        x[6 + c] = (float)(a.s_in * ep[c]);
      }
      x[12] = (float)(a.s_in * kap);
      x[13] = x[14] = x[15] = 0.f;
    } else if (a.rm) {
      double ep[6] = {0, 0, 0, 0, 0, 0}, bt[6] = {0, 0, 0, 0, 0, 0}, kap = 0.0;
#pragma unroll
      for (int c = 0; c < NSC; ++c) ep[c] = a.ep[c * N + ip];
      if (MODEL == EP_VM) {
#pragma unroll
        for (int c = 0; c < NSC; ++c) bt[c] = a.beta[c * N + ip];
      } else {
        kap = a.kappa[ip];
      }
      double desc[10];
      const bool commit = LM == 0 && a.commit != 0;
      int f;
      if constexpr (LM == 2) {
        // stress: elastic trial, plus the network's plastic correction at
        // points it predicts plastic
        const float *y = a.mlp_y + ip * EP_MLP_YS;
        f = y[6] > 0.f ? 1 : 0;
        double dv[6], tr;
        trial(a.m, eps, ep, dv, tr);
#pragma unroll
        for (int c = 0; c < 6; ++c) sig[c] = 2.0 * a.m.G * dv[c] + (c < 3 ? a.m.K * tr : 0.0);
        if (f) {
          f = predicted_tangent(a.m, eps, ep, bt, kap, desc);
#pragma unroll
          for (int c = 0; c < 6; ++c) sig[c] += a.S * (double)y[c];
        }
      } else {
        f = MODEL == EP_VM ? rm_vm(a.m, eps, ep, bt, sig, desc, commit)
                           : rm_dp(a.m, eps, ep, kap, sig, desc, commit);
      }
      a.flag[ip] = (uint8_t)f;
      if (a.flag_out) a.flag_out[ip] = (uint8_t)f;
      if (f) {
        if constexpr (D == 3) {
#pragma unroll
          for (int i = 0; i < 10; ++i) a.desc[i * N + ip] = desc[i];
        } else {
          a.desc[0 * N + ip] = desc[0];
          a.desc[1 * N + ip] = desc[1];
          a.desc[2 * N + ip] = desc[3];
#pragma unroll
          for (int i = 0; i < 4; ++i) a.desc[(3 + i) * N + ip] = desc[6 + i];
        }
        atomicOr(&s_mask[el], 1u << q);
      }
      if (a.sig_out) {
#pragma unroll
        for (int c = 0; c < NSC; ++c) a.sig_out[c * N + ip] = sig[c];
      }
      if (a.D_out) {
        constexpr int idx3[3] = {0, 1, 3};
#pragma unroll
        for (int I = 0; I < NSTR; ++I)
#pragma unroll
          for (int J = 0; J < NSTR; ++J) {
            const int vI = D == 3 ? I : idx3[I], vJ = D == 3 ? J : idx3[J];
            a.D_out[(I * NSTR + J) * N + ip] = tangent_entry(a.m, desc, f != 0, vI, vJ);
          }
      }
      if (commit && f) {
#pragma unroll
        for (int c = 0; c < NSC; ++c) a.ep[c * N + ip] = ep[c];
        if (MODEL == EP_VM) {
#pragma unroll
          for (int c = 0; c < NSC; ++c) a.beta[c * N + ip] = bt[c];
        } else {
          a.kappa[ip] = kap;
        }
      }
    }
    if (a.force) {
      // grad phi_p = J^{-1} dphi_p, so sigma grad phi_p = (sigma J^{-1}) dphi_p:
      // one D x D matrix per point instead of sigma and J^{-1}
      double sm[D][D];
      if constexpr (D == 3) {
        sm[0][0] = sig[0]; sm[1][1] = sig[1]; sm[2][2] = sig[2];
        sm[0][1] = sm[1][0] = sig[3];
        sm[1][2] = sm[2][1] = sig[4];
        sm[0][2] = sm[2][0] = sig[5];
      } else {
        sm[0][0] = sig[0]; sm[1][1] = sig[1];
        sm[0][1] = sm[1][0] = sig[3];
      }
      double *sf = s_f + tid * NF;
      if constexpr (STASH) {
        double wJ[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) wJ[i][j] = sf[i * D + j];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) v += sm[i][k] * wJ[k][j];
            sf[i * D + j] = v;
          }
      } else {
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) v += sm[i][k] * Ji[k][j];
            sf[i * D + j] = w * v;
          }
      }
    }
  }
  __syncthreads();
  if (!a.force) return;
  // F_e[p] = sum_q w_q sigma_q grad phi_p(q)  (B^T (WEIGHT .* S), Section 7)
  //        = sum_q A_q dphi_p(q) with A_q = w_q sigma_q J_q^{-1}
  for (int t = tid; t < EPB * NP; t += CT) {
    const int elx = t / NP, p = t - (t / NP) * NP;
    const int64_t ee = e0 + elx;
    if (ee >= a.n_e) continue;
    double f[D];
#pragma unroll
    for (int i = 0; i < D; ++i) f[i] = 0.0;
    for (int qq = 0; qq < NQ; ++qq) {
      const double *A = s_f + (elx * NQ + qq) * NF;
      const double *dr = s_ref + (qq * NP + p) * D;
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) f[i] += A[i * D + j] * dr[j];
    }
    const int64_t slot = a.fslot[ee * NP + p];
#pragma unroll
    for (int i = 0; i < D; ++i) a.Fe[slot * D + i] = f[i];
  }
  for (int t = tid; t < EPB; t += CT)
    if (e0 + t < a.n_e) a.emask[e0 + t] = s_mask[t];
}

// ----------------------------------------------------------------------------
// Geometry view (dphi, w) and the det J > 0 check.
// ----------------------------------------------------------------------------
template <int ETID>
__global__ void k_geometry(const double *coord, const int32_t *elem, const double *ref,
                           int64_t n_n, int64_t n_e, double *dphi, double *wout, int32_t *bad) {
  using T = Et<ETID>;
  constexpr int D = T::D, NP = T::NP, NQ = T::NQ;
  const int64_t ip = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ip >= n_e * NQ) return;
  const int64_t e = ip / NQ;
  const int q = (int)(ip - e * NQ);
  double xs[NP * D];
  for (int p = 0; p < NP; ++p) {
    const int64_t node = elem[e * NP + p];
    for (int d = 0; d < D; ++d) xs[p * D + d] = coord[d * n_n + node];
  }
  const double *dr = ref + q * NP * D;
  double Ji[D][D];
  const double det = jac_inv<D, NP>(xs, dr, Ji);
  if (!(det > 0.0)) atomicAdd(bad, 1);
  if (wout) wout[ip] = fabs(det) * ref[NQ * NP * D + q];
  if (dphi)
    for (int p = 0; p < NP; ++p) {
      double g[D];
      grad<D>(Ji, dr + p * D, g);
      for (int d = 0; d < D; ++d) dphi[(ip * NP + p) * D + d] = g[d];
    }
}

// ----------------------------------------------------------------------------
// Element-local tangent products scattered through the position map.
//   elastic = 1: K_elast, C at every point, accumulated into Ke (setup).
//   elastic = 0: for every element of the colour's work list (plastic now,
//                or plastic at the last assembly), Delta K_e = sum over its
//                plastic points of w_q B_q^T (D_q - C) B_q is added to the
//                base value of each node block: K_elast if the block was not
//                written yet in this assembly (stamp != cur), else K_tangent.
//                An element that left the plastic set contributes zero and
//                thereby restores K_elast on its untouched blocks.
// Per plastic point q the Voigt matrix M_q = w_q (D_q - C) (or w_q C) is
// formed from the tangent descriptor, then H_q = M_q B_q column by column
// (three non-zeros per column of B in 3D, two in 2D), and each node block is
// B_p^T H_p' summed over q.  The element matrix is symmetric (associative
// models), so one thread owns a node pair p <= p' and computes the block and
// its transpose.  A workgroup takes one element at a time and loops over the
// colour's elements with a software pipeline: the next element's list entry,
// mask, node ids and (sorted scatter) block positions load while the current
// one is processed; the stamps are read as an element starts, the base values
// in the scatter.  Quadrilaterals and 8-node hexahedra stage the element
// matrix in LDS and scatter it row by row in ascending column order (sorted
// scatter); the other elements write each pair's two blocks from registers.
// Points are processed in chunks of QC so that the per-point tables fit in
// LDS.
// ----------------------------------------------------------------------------
struct KA {
  const double *coord;
  const int32_t *elem;
  const double *ref;
  int64_t n_n, n_int;
  const double *desc;
  const uint32_t *emask;
  const int32_t *list;
  const int32_t *off;  // device segment bounds (work lists) or nullptr
  int colour;
  int64_t k0, k1;      // host segment bounds when off == nullptr
  const int32_t *bpos;
  const int32_t *bposs;  // position map in ascending-node column order (sorted scatter)
  const double *Ke;
  const float *Ke32;
  void *Kt;
  uint8_t *epoch;  // stamp of the last assembly that wrote each block
  int cur;         // this assembly's stamp, 1..255
  int elastic;
  double G, K;
  // element-matrix mode: the elements of work-list colours colour ..
  // colour_end - 1 with plastic points write Delta K_e (or K_e) to
  // emat[e][p][p'][r][c] (FP64: emat64, matrix cores: emat32) instead of
  // scattering it
  int colour_end;
  double *emat64;
  float *emat32;
  // with eslot: an element's matrix goes to the slot of its work-list
  // position (k - first position), recorded in eslot[e], so that the buffer
  // needs only as many slots as the list has entries; without: slot e
  int32_t *eslot;
};

template <int ETID>
struct AsmCfg {
  using T = Et<ETID>;
  static constexpr int NPAIR = T::NP * (T::NP + 1) / 2;
  static constexpr int BS = NPAIR <= 64 ? 64 : (NPAIR <= 128 ? 128 : 256);
  static constexpr int NBT = (NPAIR + BS - 1) / BS;
  // points per LDS chunk (4 for the 8-node hexahedron: LDS bounds its
  // occupancy; 6 for the 9-node quadrilateral: measured fastest of 3..9)
  static constexpr int QC =
      ETID == ET_Q1_3D ? 4 : (ETID == ET_Q2_2D ? 6 : (T::NQ <= 11 ? T::NQ : 9));
  static constexpr int WPE = T::D == 2 ? 6 : 4;       // occupancy target (waves/SIMD)
  // quadrilaterals and 8-node hexahedra stage the element matrix in LDS and
  // scatter it row by row in column order: on structured meshes an element's
  // blocks in a row form runs of consecutive nodes, so consecutive lanes write
  // consecutive blocks (simplices have no such runs)
  static constexpr bool SORTED =
      ETID == ET_Q1_2D || ETID == ET_Q2_2D || ETID == ET_Q2S_2D || ETID == ET_Q1_3D;
  static constexpr int NSLOT = SORTED ? (T::NP * T::NP + BS - 1) / BS : 1;
};

// dim x dim block loads / stores, 16-byte vectors where the block size allows
template <int D, typename VT>
__device__ inline void block_load(const VT *p, double *v) {
  if constexpr (D == 2 && sizeof(VT) == 8) {
    const double2 a = ((const double2 *)p)[0], b = ((const double2 *)p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  } else if constexpr (D == 2) {
    const float4 a = *(const float4 *)p;
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  } else {
#pragma unroll
    for (int i = 0; i < D * D; ++i) v[i] = (double)p[i];
  }
}
template <int D, typename VT>
__device__ inline void block_store(VT *p, const double *v) {
  if constexpr (D == 2 && sizeof(VT) == 8) {
    ((double2 *)p)[0] = double2{v[0], v[1]};
    ((double2 *)p)[1] = double2{v[2], v[3]};
  } else if constexpr (D == 2) {
    *(float4 *)p = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  } else {
#pragma unroll
    for (int i = 0; i < D * D; ++i) p[i] = (VT)v[i];
  }
}

// Voigt M = C + (alpha DEV + b n n^T + g (n 1^T + 1 n^T) + d 1 1^T) scaled by
// w, in the stored components (3D: 6, plane strain: 11, 22, 12).
template <int D>
__device__ inline void tangent_matrix(const double *desc, bool elastic, double G, double K,
                                      double w, double *M) {
  constexpr int NS = D == 3 ? 6 : 3;
  constexpr int NN = NS;
  double n[NS], al, be, ga, de;
  if (elastic) {
#pragma unroll
    for (int i = 0; i < NS; ++i) n[i] = 0.0;
    al = 2.0 * G;
    be = 0.0;
    ga = 0.0;
    de = K;
  } else {
#pragma unroll
    for (int i = 0; i < NS; ++i) n[i] = desc[i];
    al = desc[NN];
    be = desc[NN + 1];
    ga = desc[NN + 2];
    de = desc[NN + 3];
  }
#pragma unroll
  for (int I = 0; I < NS; ++I)
#pragma unroll
    for (int J = 0; J < NS; ++J) {
      const bool nI = D == 3 ? I < 3 : I < 2, nJ = D == 3 ? J < 3 : J < 2;  // normal rows
      const double oI = nI ? 1.0 : 0.0, oJ = nJ ? 1.0 : 0.0;
      const double dev = (I == J ? (nI ? 1.0 : 0.5) : 0.0) - oI * oJ / 3.0;
      M[I * NS + J] = w * (al * dev + be * n[I] * n[J] + ga * (n[I] * oJ + oI * n[J]) + de * oI * oJ);
    }
}

template <int ETID, typename VT, bool EMAT = false>
__global__ __launch_bounds__(AsmCfg<ETID>::BS)
__attribute__((amdgpu_waves_per_eu(AsmCfg<ETID>::WPE, 8))) void k_assemble(KA a) {
  using T = Et<ETID>;
  using Cfg = AsmCfg<ETID>;
  constexpr int D = T::D, NP = T::NP, NQ = T::NQ, BS = Cfg::BS, NBT = Cfg::NBT;
  constexpr int NPAIR = Cfg::NPAIR, QC = Cfg::QC, NB2 = NP * NP;
  constexpr int NS = D == 3 ? 6 : 3;
  constexpr int NDESC = D == 3 ? 10 : 7;
  constexpr bool SORTED = Cfg::SORTED;
  constexpr int NSLOT = Cfg::NSLOT;
  static_assert(NP * D <= BS && NQ <= BS, "one thread per coordinate and per point");
  __shared__ double s_x[NP * D];
  // per plastic point: n and the scalars c1..c4 of w (D_q - C) (see below)
  constexpr int PT = NS + 4;
  __shared__ double s_pt[NQ * PT];
  __shared__ double s_Ji[NQ * D * D];
  // per (point, node) of a chunk the vectors g, a, P, Q [q][4][d][p]; after
  // the local product the same LDS holds the element matrix [p][p'][r][c]
  // (sorted scatter)
  constexpr int NV_ = QC * 4 * D * NP, NK_ = SORTED ? NB2 * D * D : 0;
  __shared__ double s_HK[NV_ > NK_ ? NV_ : NK_];
  double *const s_V = s_HK;
  double *const s_K = s_HK;
  __shared__ int s_node[NP];
  __shared__ int s_ord[NP];                // local nodes by ascending global id
  __shared__ int s_q[NQ];                  // plastic points in order
  const int tid = threadIdx.x;
  int64_t k0 = a.k0, k1 = a.k1;
  if (a.off) {
    k0 = a.off[a.colour];
    k1 = a.off[EMAT ? a.colour_end : a.colour + 1];
  }
  VT *Kt = (VT *)a.Kt;
  const uint32_t qmask = NQ == 32 ? 0xffffffffu : ((1u << NQ) - 1u);
  // node pairs p <= p' of this thread (element-local product)
  int pp_[NBT], pq_[NBT];
  bool pon[NBT];
#pragma unroll
  for (int j = 0; j < NBT; ++j) {
    int t = tid + j * BS, p = 0;
    pon[j] = t < NPAIR;
    if (!pon[j]) t = 0;
    while (t >= NP - p) {
      t -= NP - p;
      ++p;
    }
    pp_[j] = p;
    pq_[j] = p + t;
  }
  // software pipeline over the elements of this block: the list entry, mask
  // and node ids of the next element are loaded while the current one is
  // processed
  // (sorted scatter: also the block positions of the next element, so that
  // the freshness stamps can be read as soon as an element starts)
  constexpr int NIP = SORTED ? NSLOT : 1;
  constexpr bool PREPOS = SORTED && !EMAT;  // positions prefetched for the sorted scatter
  int64_t k = k0 + blockIdx.x;
  int e_n = k < k1 ? a.list[k] : -1;
  uint32_t m_n = (e_n >= 0 && !a.elastic) ? a.emask[e_n] : 0xffffffffu;
  int node_n = (e_n >= 0 && tid < NP) ? a.elem[(int64_t)e_n * NP + tid] : 0;
  int32_t ip_n[NIP];
#pragma unroll
  for (int sl = 0; sl < NIP; ++sl) {
    const int t = tid + sl * BS;
    ip_n[sl] = (PREPOS && e_n >= 0 && t < NB2) ? a.bposs[(int64_t)e_n * NB2 + t] : 0;
  }
  for (; k < k1; k += gridDim.x) {
    const int e = e_n;
    const uint32_t mask = m_n & qmask;
    const int node_cur = node_n;
    int32_t ip_cur[NIP];
#pragma unroll
    for (int sl = 0; sl < NIP; ++sl) ip_cur[sl] = ip_n[sl];
    {
      const int64_t kn = k + gridDim.x;
      e_n = kn < k1 ? a.list[kn] : -1;
    }
    if (e < 0) {  // padding of the colour-major order (uniform)
      m_n = (e_n >= 0 && !a.elastic) ? a.emask[e_n] : 0xffffffffu;
      node_n = (e_n >= 0 && tid < NP) ? a.elem[(int64_t)e_n * NP + tid] : 0;
#pragma unroll
      for (int sl = 0; sl < NIP; ++sl) {
        const int t = tid + sl * BS;
        ip_n[sl] = (PREPOS && e_n >= 0 && t < NB2) ? a.bposs[(int64_t)e_n * NB2 + t] : 0;
      }
      continue;
    }
    if (EMAT && !mask) {  // no plastic point: no element term (uniform)
      m_n = (e_n >= 0 && !a.elastic) ? a.emask[e_n] : 0xffffffffu;
      node_n = (e_n >= 0 && tid < NP) ? a.elem[(int64_t)e_n * NP + tid] : 0;
      continue;
    }
    const int nq = __popc(mask);
    // scatter targets: sorted mode, slot t = p * NP + r is block (p, s_ord[r]);
    // pair mode, the blocks (p, p') and (p', p) of this thread's pairs
    int64_t i1[SORTED ? NSLOT : NBT], i2[SORTED ? 1 : NBT];
    bool f1[SORTED ? NSLOT : NBT], f2[SORTED ? 1 : NBT];
    if constexpr (EMAT) {
      if constexpr (SORTED) {
        __syncthreads();  // LDS of the previous element is no longer read
        if (tid < NP) s_node[tid] = node_cur;
        __syncthreads();
      }
    } else if constexpr (SORTED) {
      // slot t = p * NP + r: block (p, r-th node by global id), position
      // prefetched; its stamp is read at once
#pragma unroll
      for (int sl = 0; sl < NSLOT; ++sl) {
        const bool on = tid + sl * BS < NB2;
        i1[sl] = on ? (int64_t)ip_cur[sl] : 0;
        f1[sl] = (!a.elastic && on) ? (a.epoch[i1[sl]] != a.cur) : false;
      }
      __syncthreads();  // LDS of the previous element is no longer read
      if (tid < NP) s_node[tid] = node_cur;
      __syncthreads();
      if (tid < NP) {
        int r = 0;
        const int me = s_node[tid];
#pragma unroll
        for (int j = 0; j < NP; ++j) r += (s_node[j] < me) ? 1 : 0;
        s_ord[r] = tid;
      }
      __syncthreads();
    } else {
#pragma unroll
      for (int j = 0; j < NBT; ++j) {
        const bool on = pon[j];
        i1[j] = on ? (int64_t)a.bpos[(int64_t)e * NB2 + pp_[j] * NP + pq_[j]] : 0;
        i2[j] = on ? (int64_t)a.bpos[(int64_t)e * NB2 + pq_[j] * NP + pp_[j]] : 0;
      }
#pragma unroll
      for (int j = 0; j < NBT; ++j) {
        const bool on = pon[j];
        f1[j] = (!a.elastic && on) ? (a.epoch[i1[j]] != a.cur) : false;
        f2[j] = (!a.elastic && on) ? (a.epoch[i2[j]] != a.cur) : false;
      }
    }
    double acc[NBT][D * D];
#pragma unroll
    for (int j = 0; j < NBT; ++j)
#pragma unroll
      for (int i = 0; i < D * D; ++i) acc[j][i] = 0.0;
    if (mask) {
      if constexpr (!SORTED) __syncthreads();  // LDS of the previous element is no longer read
      if (tid < NP * D) {
        const int64_t node = SORTED ? s_node[tid / D] : a.elem[(int64_t)e * NP + tid / D];
        s_x[tid] = a.coord[(tid % D) * a.n_n + node];
      }
      if (tid < NQ) {
        const uint32_t below = mask & ((1u << tid) - 1u);
        if ((mask >> tid) & 1u) s_q[__popc(below)] = tid;
      }
      __syncthreads();
      if (tid < nq) {
        const int q = s_q[tid];
        double Ji[D][D];
        const double det = jac_inv<D, NP>(s_x, a.ref + q * NP * D, Ji);
        const double w = fabs(det) * a.ref[NQ * NP * D + q];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int jj = 0; jj < D; ++jj) s_Ji[tid * D * D + i * D + jj] = Ji[i][jj];
        // w (D_q - C) = w (alpha DEV + beta n n^T + gamma (n 1^T + 1 n^T) +
        // delta 1 1^T) in Voigt form; its node blocks B_p^T (.) B_p' reduce to
        // vectors of the nodes (below) with c1 = w (delta - alpha/3),
        // c2 = w gamma, c3 = w beta, c4 = w alpha / 2 (C itself: n = 0,
        // alpha = 2G, delta = K)
        double *pt = s_pt + tid * PT;
        double al, be, ga, de;
        if (!a.elastic) {
          const int64_t ip = (int64_t)e * NQ + q;
#pragma unroll
          for (int c = 0; c < NS; ++c) pt[c] = a.desc[c * a.n_int + ip];
          al = a.desc[NS * a.n_int + ip];
          be = a.desc[(NS + 1) * a.n_int + ip];
          ga = a.desc[(NS + 2) * a.n_int + ip];
          de = a.desc[(NS + 3) * a.n_int + ip];
        } else {
#pragma unroll
          for (int c = 0; c < NS; ++c) pt[c] = 0.0;
          al = 2.0 * a.G;
          be = 0.0;
          ga = 0.0;
          de = a.K;
        }
        pt[NS] = w * (de - al / 3.0);
        pt[NS + 1] = w * ga;
        pt[NS + 2] = w * be;
        pt[NS + 3] = 0.5 * w * al;
      }
      for (int q0 = 0; q0 < nq; q0 += QC) {
        const int nc = nq - q0 < QC ? nq - q0 : QC;
        __syncthreads();
        // per (point, node): g = grad phi_p, a = B_p^T n (the tensor of n
        // applied to g), P = c1 g + c2 a, Q = c3 a + c2 g
        for (int t = tid; t < nc * NP; t += BS) {
          const int ql = t / NP, p = t - (t / NP) * NP;
          const int qi = q0 + ql;
          double Ji[D][D];
#pragma unroll
          for (int i = 0; i < D; ++i)
#pragma unroll
            for (int jj = 0; jj < D; ++jj) Ji[i][jj] = s_Ji[qi * D * D + i * D + jj];
          double g[D], av[D];
          grad<D>(Ji, a.ref + (s_q[qi] * NP + p) * D, g);
          const double *pt = s_pt + qi * PT;
          if constexpr (D == 3) {
            av[0] = pt[0] * g[0] + pt[3] * g[1] + pt[5] * g[2];
            av[1] = pt[3] * g[0] + pt[1] * g[1] + pt[4] * g[2];
            av[2] = pt[5] * g[0] + pt[4] * g[1] + pt[2] * g[2];
          } else {
            av[0] = pt[0] * g[0] + pt[2] * g[1];
            av[1] = pt[2] * g[0] + pt[1] * g[1];
          }
          const double c1 = pt[NS], c2 = pt[NS + 1], c3 = pt[NS + 2];
          double *V = s_V + ql * 4 * D * NP + p;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            V[(0 * D + d) * NP] = g[d];
            V[(1 * D + d) * NP] = av[d];
            V[(2 * D + d) * NP] = c1 * g[d] + c2 * av[d];
            V[(3 * D + d) * NP] = c3 * av[d] + c2 * g[d];
          }
        }
        __syncthreads();
        // node blocks: (B_p^T w (D - C) B_p')_ij =
        //   g_i P'_j + a_i Q'_j + c4 (g'_i g_j + (g . g') delta_ij)
#pragma unroll
        for (int j = 0; j < NBT; ++j) {
          if (!pon[j]) continue;
          const int p = pp_[j], pq = pq_[j];
          for (int ql = 0; ql < nc; ++ql) {
            const double *V = s_V + ql * 4 * D * NP;
            const double c4 = s_pt[(q0 + ql) * PT + NS + 3];
            double gp[D], ap[D], gq[D], Pq[D], Qq[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
              gp[d] = V[(0 * D + d) * NP + p];
              ap[d] = V[(1 * D + d) * NP + p];
              gq[d] = V[(0 * D + d) * NP + pq];
              Pq[d] = V[(2 * D + d) * NP + pq];
              Qq[d] = V[(3 * D + d) * NP + pq];
            }
            double dot = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) dot += gp[d] * gq[d];
#pragma unroll
            for (int i = 0; i < D; ++i) {
              const double hq = c4 * gq[i];
#pragma unroll
              for (int jj = 0; jj < D; ++jj)
                acc[j][i * D + jj] += gp[i] * Pq[jj] + ap[i] * Qq[jj] + hq * gp[jj];
              acc[j][i * D + i] += c4 * dot;
            }
          }
        }
      }
      if constexpr (SORTED) {
        __syncthreads();  // H is no longer read
        // element matrix to LDS: block (p, p') and its transpose (p', p)
#pragma unroll
        for (int j = 0; j < NBT; ++j) {
          if (!pon[j]) continue;
          const int p = pp_[j], pq = pq_[j];
#pragma unroll
          for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
              s_K[(p * NP + pq) * D * D + r * D + c] = acc[j][r * D + c];
              s_K[(pq * NP + p) * D * D + c * D + r] = acc[j][r * D + c];
            }
        }
        __syncthreads();
      }
    }
    m_n = (e_n >= 0 && !a.elastic) ? a.emask[e_n] : 0xffffffffu;
    node_n = (e_n >= 0 && tid < NP) ? a.elem[(int64_t)e_n * NP + tid] : 0;
#pragma unroll
    for (int sl = 0; sl < NIP; ++sl) {
      const int t = tid + sl * BS;
      ip_n[sl] = (PREPOS && e_n >= 0 && t < NB2) ? a.bposs[(int64_t)e_n * NB2 + t] : 0;
    }
    if constexpr (EMAT) {
      // the element matrix, [p][p'][r][c], to its slot of the buffer
      const int64_t slot = a.eslot ? k - k0 : (int64_t)e;
      if (a.eslot && tid == 0) a.eslot[e] = (int32_t)slot;
      double *dst = a.emat64 + slot * NB2 * D * D;
      if constexpr (SORTED) {
        for (int t = tid; t < NB2 * D * D; t += BS) dst[t] = s_K[t];
      } else {
#pragma unroll
        for (int j = 0; j < NBT; ++j) {
          if (!pon[j]) continue;
          const int p = pp_[j], pq = pq_[j];
#pragma unroll
          for (int r = 0; r < D; ++r)
#pragma unroll
            for (int cc = 0; cc < D; ++cc) {
              dst[(p * NP + pq) * D * D + r * D + cc] = acc[j][r * D + cc];
              dst[(pq * NP + p) * D * D + cc * D + r] = acc[j][r * D + cc];
            }
        }
      }
      continue;
    }
    // base values (K_elast for blocks not yet written in this assembly, else
    // K_tangent) plus the element's contribution
    if constexpr (SORTED) {
#pragma unroll
      for (int sl = 0; sl < NSLOT; ++sl) {
        const int t = tid + sl * BS;
        if (t >= NB2) continue;
        const bool fresh = f1[sl];
        if (!mask && !fresh) continue;  // left the plastic set, block already rewritten
        const int64_t idx = i1[sl];
        double v[D * D];
        if (a.elastic || !fresh) block_load<D>(Kt + idx * D * D, v);
        else if constexpr (sizeof(VT) == 8) block_load<D>(a.Ke + idx * D * D, v);
        else block_load<D>(a.Ke32 + idx * D * D, v);
        if (mask) {
          const int p = t / NP, pc = s_ord[t - (t / NP) * NP];
          const double *kb = s_K + (p * NP + pc) * D * D;
#pragma unroll
          for (int i = 0; i < D * D; ++i) v[i] += kb[i];
        }
        block_store<D>(Kt + idx * D * D, v);
        if (!a.elastic) a.epoch[idx] = (uint8_t)a.cur;
      }
    } else {
#pragma unroll
      for (int j = 0; j < NBT; ++j) {
        if (!pon[j]) continue;
        const bool diag = pp_[j] == pq_[j];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          if (side == 1 && diag) continue;
          const int64_t idx = side == 0 ? i1[j] : i2[j];
          const bool fresh = side == 0 ? f1[j] : f2[j];
          if (!mask && !fresh) continue;  // left the plastic set, block already rewritten
          double base[D * D];
          if (a.elastic || !fresh) {
#pragma unroll
            for (int i = 0; i < D * D; ++i) base[i] = (double)Kt[idx * D * D + i];
          } else if constexpr (sizeof(VT) == 8) {
#pragma unroll
            for (int i = 0; i < D * D; ++i) base[i] = a.Ke[idx * D * D + i];
          } else {
#pragma unroll
            for (int i = 0; i < D * D; ++i) base[i] = (double)a.Ke32[idx * D * D + i];
          }
          VT *dst = Kt + idx * D * D;
#pragma unroll
          for (int r = 0; r < D; ++r)
#pragma unroll
            for (int cc = 0; cc < D; ++cc)
              dst[r * D + cc] = (VT)(base[r * D + cc] + (side == 0 ? acc[j][r * D + cc] : acc[j][cc * D + r]));
          if (!a.elastic) a.epoch[idx] = (uint8_t)a.cur;
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Element-local products on the matrix cores (27-node hexahedra, 10-node
// tetrahedra).  Delta K_e = B^T H with B the stacked B_q (6 n_q x 3 n_p) and
// H = blockdiag(M_q) B, M_q = w_q (D_q - C): a (3 n_p) x (3 n_p) x (6 n_q)
// product.  B and H are staged in LDS as BF16 (v_mfma_f32_16x16x32_bf16) or
// FP32 (v_mfma_f32_16x16x4_f32) tiles, a chunk of QC points at a time, and
// each wavefront accumulates upper-triangle 16x16 tiles of the (symmetric)
// element matrix in FP32 registers.  The element matrix then goes through
// LDS to the same stamped node-block scatter as the FP64 kernel.
// Lane layouts (checked on gfx950): lane l holds A[l%16][k-group l/16],
// B[k-group l/16][l%16], and the result rows 4(l/16)..4(l/16)+3 of column
// l%16.
// ----------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

template <int ETID, bool BF16>
struct MfmaCfg {
  using T = Et<ETID>;
  static constexpr int NL = 3 * T::NP;
  static constexpr int MP = ((NL + 15) / 16) * 16;
  static constexpr int TT = MP / 16;
  static constexpr int NT = TT * (TT + 1) / 2;
  static constexpr int QC = T::NQ <= 11 ? T::NQ : 9;
  static constexpr int KC = 6 * QC;
  static constexpr int KK = BF16 ? 32 : 4;
  static constexpr int KP = ((KC + KK - 1) / KK) * KK;
  static constexpr int LDK = BF16 ? KP + 8 : KP + 1;  // bank-conflict-free strides
  static constexpr int NPAIR = T::NP * (T::NP + 1) / 2;
  static constexpr int NBT = (NPAIR + 255) / 256;
  static constexpr int TPW = (NT + 3) / 4;
  // occupancy target (waves per SIMD): 3 (three workgroups per CU; the LDS
  // of the 27-node products fits that since the tangent is kept in its
  // vector form), except the P2 BF16 colour kernel, measured faster with
  // the compiler's own register budget
  static constexpr int wpe(bool emat) {
    return (emat || !(ETID == ET_P2_3D && BF16)) ? 3 : 1;
  }
};

template <bool BF16> struct MfmaElem { using type = float; };
template <> struct MfmaElem<true> { using type = __bf16; };

template <int ETID, typename VT, bool BF16, bool EMAT = false>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(MfmaCfg<ETID, BF16>::wpe(EMAT), 8))) void k_assemble_mfma(KA a) {
  using T = Et<ETID>;
  using C = MfmaCfg<ETID, BF16>;
  using ET = typename MfmaElem<BF16>::type;
  constexpr int NP = T::NP, NQ = T::NQ, NB2 = NP * NP;
  constexpr int NL = C::NL, MP = C::MP, TT = C::TT, NT = C::NT, QC = C::QC, KC = C::KC;
  constexpr int KK = C::KK, KP = C::KP, LDK = C::LDK, NPAIR = C::NPAIR, NBT = C::NBT;
  constexpr int TPW = C::TPW;
  static_assert(T::D == 3, "3D elements");
  // B and H tiles, and after the last chunk the element matrix: for the
  // large element matrices (20- and 27-node hexahedra) one shared LDS buffer
  // (a smaller footprint lets more workgroups share a CU; 27-node FP32
  // products 602 -> 463 us per pass on the block), separate buffers for the
  // small ones (whose padding would have to be cleared per element for
  // little LDS saved)
  constexpr bool ALIAS = NL >= 60;
  constexpr int NBH = (2 * MP * LDK * (int)sizeof(ET) + 3) / 4;
  __shared__ float s_BHK[ALIAS ? (NBH > NL * NL ? NBH : NL * NL) : NBH + NL * NL];
  ET *const s_B = (ET *)s_BHK;
  ET *const s_H = s_B + MP * LDK;
  float *const s_K = ALIAS ? s_BHK : s_BHK + NBH;
  __shared__ double s_x[NP * 3];
  // per plastic point: n and c1..c4 of w (D_q - C) (vector form, as in the
  // FP64 kernel)
  __shared__ double s_pt[NQ * 10];
  __shared__ double s_Ji[NQ * 9];
  __shared__ int s_q[NQ];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  // padding rows / columns of B and H are zero (with ALIAS, the part an
  // element matrix overwrites is cleared again per element)
  for (int t = tid; t < MP * LDK; t += 256) {
    const int m = t / LDK, kk = t - (t / LDK) * LDK;
    if (m >= NL || kk >= KC) {
      s_B[t] = (ET)0.0f;
      s_H[t] = (ET)0.0f;
    }
  }
  int pp_[NBT], pq_[NBT];
#pragma unroll
  for (int j = 0; j < NBT; ++j) {
    int t = tid + j * 256, p = 0;
    if (t >= NPAIR) t = 0;
    while (t >= NP - p) {
      t -= NP - p;
      ++p;
    }
    pp_[j] = p;
    pq_[j] = p + t;
  }
  int64_t k0 = a.k0, k1 = a.k1;
  if (a.off) {
    k0 = a.off[a.colour];
    k1 = a.off[EMAT ? a.colour_end : a.colour + 1];
  }
  VT *Kt = (VT *)a.Kt;
  const uint32_t qmask = (1u << NQ) - 1u;
  for (int64_t k = k0 + blockIdx.x; k < k1; k += gridDim.x) {
    const int e = a.list[k];
    if (e < 0) continue;
    const uint32_t mask = a.emask[e] & qmask;
    if (EMAT && !mask) continue;  // no plastic point: no element term (uniform)
    const int nq = __popc(mask);
    int64_t i1[NBT], i2[NBT];
    bool f1[NBT], f2[NBT];
    if constexpr (!EMAT) {
#pragma unroll
      for (int j = 0; j < NBT; ++j) {
        const bool on = tid + j * 256 < NPAIR;
        i1[j] = on ? (int64_t)a.bpos[(int64_t)e * NB2 + pp_[j] * NP + pq_[j]] : 0;
        i2[j] = on ? (int64_t)a.bpos[(int64_t)e * NB2 + pq_[j] * NP + pp_[j]] : 0;
      }
#pragma unroll
      for (int j = 0; j < NBT; ++j) {
        const bool on = tid + j * 256 < NPAIR;
        f1[j] = on ? (a.epoch[i1[j]] != a.cur) : false;
        f2[j] = on ? (a.epoch[i2[j]] != a.cur) : false;
      }
    }
    double acc[NBT][9];
#pragma unroll
    for (int j = 0; j < NBT; ++j)
#pragma unroll
      for (int i = 0; i < 9; ++i) acc[j][i] = 0.0;
    if (mask) {
      __syncthreads();  // LDS of the previous element is no longer read
      if constexpr (ALIAS) {
        // padding rows / columns of B and H are zero again where the
        // previous element matrix overwrote them (its first NL^2 floats)
        constexpr int OV = (4 * NL * NL + (int)sizeof(ET) - 1) / (int)sizeof(ET);
        for (int t = tid; t < (OV < 2 * MP * LDK ? OV : 2 * MP * LDK); t += 256) {
          const int tt = t < MP * LDK ? t : t - MP * LDK;
          const int m = tt / LDK, kk = tt - (tt / LDK) * LDK;
          if (m >= NL || kk >= KC) s_B[t] = (ET)0.0f;
        }
      }
      if (tid < NP * 3) {
        const int64_t node = a.elem[(int64_t)e * NP + tid / 3];
        s_x[tid] = a.coord[(tid % 3) * a.n_n + node];
      }
      if (tid < NQ && ((mask >> tid) & 1u)) s_q[__popc(mask & ((1u << tid) - 1u))] = tid;
      __syncthreads();
      if (tid < nq) {
        const int q = s_q[tid];
        double Ji[3][3];
        const double det = jac_inv<3, NP>(s_x, a.ref + q * NP * 3, Ji);
        const double w = fabs(det) * a.ref[NQ * NP * 3 + q];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int jj = 0; jj < 3; ++jj) s_Ji[tid * 9 + i * 3 + jj] = Ji[i][jj];
        const int64_t ip = (int64_t)e * NQ + q;
        double *pt = s_pt + tid * 10;
#pragma unroll
        for (int c = 0; c < 6; ++c) pt[c] = a.desc[c * a.n_int + ip];
        const double al = a.desc[6 * a.n_int + ip], be = a.desc[7 * a.n_int + ip];
        const double ga = a.desc[8 * a.n_int + ip], de = a.desc[9 * a.n_int + ip];
        pt[6] = w * (de - al / 3.0);
        pt[7] = w * ga;
        pt[8] = w * be;
        pt[9] = 0.5 * w * al;
      }
      f32x4_t tacc[TPW];
#pragma unroll
      for (int s = 0; s < TPW; ++s) tacc[s] = f32x4_t{0.f, 0.f, 0.f, 0.f};
      for (int c0 = 0; c0 < nq; c0 += QC) {
        const int nc = nq - c0 < QC ? nq - c0 : QC;
        __syncthreads();  // previous chunk consumed
        for (int t = tid; t < QC * NP; t += 256) {
          const int ql = t / NP, p = t - (t / NP) * NP;
          double bc[3][6], hc[3][6];
          if (ql < nc) {
            const int qi = c0 + ql;
            double Ji[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int jj = 0; jj < 3; ++jj) Ji[i][jj] = s_Ji[qi * 9 + i * 3 + jj];
            double g[3];
            grad<3>(Ji, a.ref + (s_q[qi] * NP + p) * 3, g);
            // columns (p, 0..2) of B_q, rows 11, 22, 33, 12, 23, 13
            const double z = 0.0;
            const double b0[6] = {g[0], z, z, g[1], z, g[2]};
            const double b1[6] = {z, g[1], z, g[0], g[2], z};
            const double b2[6] = {z, z, g[2], z, g[1], g[0]};
#pragma unroll
            for (int rr = 0; rr < 6; ++rr) {
              bc[0][rr] = b0[rr];
              bc[1][rr] = b1[rr];
              bc[2][rr] = b2[rr];
            }
            // H = w (D_q - C) B_q column by column: for the column of
            // (p, i), 2 c4 I_sym b + P_i 1 + Q_i n with a = N g,
            // P = c1 g + c2 a, Q = c3 a + c2 g (I_sym halves the shears)
            const double *pt = s_pt + qi * 10;
            double nv[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) nv[c] = pt[c];
            const double c1 = pt[6], c2 = pt[7], c3 = pt[8], c4 = pt[9];
            const double av[3] = {nv[0] * g[0] + nv[3] * g[1] + nv[5] * g[2],
                                  nv[3] * g[0] + nv[1] * g[1] + nv[4] * g[2],
                                  nv[5] * g[0] + nv[4] * g[1] + nv[2] * g[2]};
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              const double P = c1 * g[i] + c2 * av[i], Qv = c3 * av[i] + c2 * g[i];
#pragma unroll
              for (int rr = 0; rr < 6; ++rr)
                hc[i][rr] = (rr < 3 ? 2.0 * c4 : c4) * bc[i][rr] + (rr < 3 ? P : 0.0) + Qv * nv[rr];
            }
          } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int rr = 0; rr < 6; ++rr) {
                bc[i][rr] = 0.0;
                hc[i][rr] = 0.0;
              }
          }
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int rr = 0; rr < 6; ++rr) {
              s_B[(3 * p + i) * LDK + 6 * ql + rr] = (ET)(float)bc[i][rr];
              s_H[(3 * p + i) * LDK + 6 * ql + rr] = (ET)(float)hc[i][rr];
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
          int t = wv + 4 * s;
          if (t >= NT) break;
          int tm = 0;
          while (t >= TT - tm) {
            t -= TT - tm;
            ++tm;
          }
          const int tn = tm + t;
          const ET *ra = s_B + (16 * tm + r16) * LDK;
          const ET *rb = s_H + (16 * tn + r16) * LDK;
#pragma unroll
          for (int ks = 0; ks < KP / KK; ++ks) {
            if constexpr (BF16) {
              const bf16x8_t av = *(const bf16x8_t *)(ra + ks * 32 + kg * 8);
              const bf16x8_t bv = *(const bf16x8_t *)(rb + ks * 32 + kg * 8);
              tacc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, tacc[s], 0, 0, 0);
            } else {
              tacc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[ks * 4 + kg], rb[ks * 4 + kg],
                                                             tacc[s], 0, 0, 0);
            }
          }
        }
      }
      __syncthreads();  // every wave has read its last B and H tiles
      // tiles -> element matrix in LDS
#pragma unroll
      for (int s = 0; s < TPW; ++s) {
        int t = wv + 4 * s;
        if (t >= NT) break;
        int tm = 0;
        while (t >= TT - tm) {
          t -= TT - tm;
          ++tm;
        }
        const int tn = tm + t;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = 16 * tm + 4 * kg + i, n = 16 * tn + r16;
          if (m < NL && n < NL) s_K[m * NL + n] = tacc[s][i];
        }
      }
      __syncthreads();
      if constexpr (EMAT) {
        // the element matrix, [p][p'][r][c] (FP32 accumulators), to its slot
        const int64_t slot = a.eslot ? k - k0 : (int64_t)e;
        if (a.eslot && tid == 0) a.eslot[e] = (int32_t)slot;
        float *dst = a.emat32 + slot * NB2 * 9;
        for (int t = tid; t < NB2 * 9; t += 256) {
          const int pb = t / 9, rc = t - (t / 9) * 9;
          const int p = pb / NP, pq = pb - (pb / NP) * NP;
          const int m = 3 * p + rc / 3, n = 3 * pq + rc % 3;
          dst[t] = m <= n ? s_K[m * NL + n] : s_K[n * NL + m];
        }
        __syncthreads();  // s_K is read before the next element writes it
        continue;
      }
#pragma unroll
      for (int j = 0; j < NBT; ++j) {
        if (tid + j * 256 >= NPAIR) continue;
#pragma unroll
        for (int r3 = 0; r3 < 3; ++r3)
#pragma unroll
          for (int c3 = 0; c3 < 3; ++c3) {
            const int m = 3 * pp_[j] + r3, n = 3 * pq_[j] + c3;
            acc[j][r3 * 3 + c3] = (double)(m <= n ? s_K[m * NL + n] : s_K[n * NL + m]);
          }
      }
    }
#pragma unroll
    for (int j = 0; j < NBT; ++j) {
      if (tid + j * 256 >= NPAIR) continue;
      const bool diag = pp_[j] == pq_[j];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        if (side == 1 && diag) continue;
        const int64_t idx = side == 0 ? i1[j] : i2[j];
        const bool fresh = side == 0 ? f1[j] : f2[j];
        if (!mask && !fresh) continue;
        double base[9];
        if (!fresh) {
#pragma unroll
          for (int i = 0; i < 9; ++i) base[i] = (double)Kt[idx * 9 + i];
        } else if constexpr (sizeof(VT) == 8) {
#pragma unroll
          for (int i = 0; i < 9; ++i) base[i] = a.Ke[idx * 9 + i];
        } else {
#pragma unroll
          for (int i = 0; i < 9; ++i) base[i] = (double)a.Ke32[idx * 9 + i];
        }
        VT *dst = Kt + idx * 9;
#pragma unroll
        for (int r3 = 0; r3 < 3; ++r3)
#pragma unroll
          for (int c3 = 0; c3 < 3; ++c3)
            dst[r3 * 3 + c3] = (VT)(base[r3 * 3 + c3] + (side == 0 ? acc[j][r3 * 3 + c3] : acc[j][c3 * 3 + r3]));
        a.epoch[idx] = (uint8_t)a.cur;
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Node-row gather of the element matrices: K_tangent row block of node m =
// K_elast row + sum over the elements e containing m that have plastic
// points now (ascending e) of the node's rows of Delta K_e, taken from the
// element-matrix buffer.  One workgroup per active row (a row is active
// when an element containing the node has plastic points now or had them at
// the last assembly: every row the last assembly changed is rewritten, so
// inactive rows hold K_elast).  The row is accumulated in LDS, then written
// once, coalesced: no colours, no stamps, no float atomics; the sum order
// is fixed.  em_cur == nullptr: every row and element (K_elast from the
// element matrices of C, base nullptr = 0).
// ----------------------------------------------------------------------------
struct KR {
  int64_t n_n;
  const int32_t *bptr, *n2e_ptr, *n2e, *bpos;
  const uint32_t *em_cur, *em_prev;
  const void *emat;   // OT [n_e][n_p][n_p][dim][dim]
  const void *base;   // VT [nnzb][dim][dim] or nullptr
  void *out;          // VT [nnzb][dim][dim]
  int max_slots;      // largest node-to-element count (LDS after the row)
  // short work lists: the rows of the listed elements' nodes instead of a
  // scan of every row (list[n_list], elem[n_e][n_p]); a row shared by two
  // listed elements is computed twice, with the same values
  const int32_t *list, *elem;
  int64_t n_list;
  // element e's matrix at slot eslot[e] of emat (element matrices stored by
  // work-list position), or at slot e when null
  const int32_t *eslot;
};

template <int ETID>
struct RowCfg {
  using T = Et<ETID>;
  static constexpr int NV = T::NP * T::D * T::D;  // values of a node's rows
  static constexpr int BS = NV <= 96 ? 64 : (NV <= 192 ? 128 : 256);
  // node slots gathered per step (their loads issued together)
  static constexpr int CH = ETID == ET_P1_3D ? 16 : (T::D == 2 && ETID != ET_P1_2D ? 4 : 8);
  static constexpr int IPT = (CH * NV + BS - 1) / BS;
};

template <int ETID, typename OT, typename VT>
__global__ __launch_bounds__(RowCfg<ETID>::BS) void k_row_gather(KR a) {
  using T = Et<ETID>;
  using R = RowCfg<ETID>;
  constexpr int D = T::D, NP = T::NP, DD = D * D, NV = R::NV, BS = R::BS, CH = R::CH;
  constexpr int IPT = R::IPT;
  extern __shared__ double s_dyn[];
  const int tid = threadIdx.x;
  const bool all = a.em_cur == nullptr;
  const OT *emat = (const OT *)a.emat;
  const VT *base = (const VT *)a.base;
  VT *out = (VT *)a.out;
  const int64_t n_work = a.list ? a.n_list * NP : a.n_n;
  for (int64_t b = blockIdx.x; b < n_work; b += gridDim.x) {
    const int64_t m = a.list ? (int64_t)a.elem[(int64_t)a.list[b / NP] * NP + b % NP] : b;
    const int k0 = a.n2e_ptr[m], k1 = a.n2e_ptr[m + 1];
    const int64_t r0 = a.bptr[m];
    const int L = (int)(a.bptr[m + 1] - r0) * DD;
    double *s_acc = s_dyn;
    int *s_sv = (int *)(s_dyn + L);  // slot value e * n_p + p, or -1 (no term now)
    int *s_ev = s_sv + a.max_slots;  // its element matrix's rows: slot * n_p + p
    // slots of the row: element terms present now, and whether the row is
    // touched by an element listed now or at the last assembly
    bool act = all || a.list != nullptr;
    for (int k = k0 + tid; k < k1; k += BS) {
      const int sv = a.n2e[k];
      const int e = sv / NP;
      const uint32_t now = all ? 1u : a.em_cur[e];
      const uint32_t before = (all || !a.em_prev) ? 0u : a.em_prev[e];
      s_sv[k - k0] = now ? sv : -1;
      if (now) s_ev[k - k0] = a.eslot ? a.eslot[e] * NP + (sv - e * NP) : sv;
      act = act || ((now | before) != 0u);
    }
    act = __syncthreads_or(act) != 0;
    if (!act) continue;  // uniform
    for (int v = tid; v < L; v += BS) s_acc[v] = base ? (double)base[r0 * DD + v] : 0.0;
    __syncthreads();
    for (int kc = 0; kc < k1 - k0; kc += CH) {
      const int ns = (k1 - k0 - kc) < CH ? (k1 - k0 - kc) : CH;
      double val[IPT];
      int dst[IPT], sl[IPT];
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const int it = tid + i * BS;  // item: slot it / NV, value it % NV
        const int sj = it / NV, t = it - (it / NV) * NV;
        sl[i] = -1;
        dst[i] = 0;
        val[i] = 0.0;
        if (sj < ns) {
          const int sv = s_sv[kc + sj];
          if (sv >= 0) {
            const int pp = t / DD, ij = t - (t / DD) * DD;
            dst[i] = (a.bpos[(int64_t)sv * NP + pp] - (int32_t)r0) * DD + ij;
            val[i] = (double)emat[(int64_t)s_ev[kc + sj] * NV + t];
            sl[i] = sj;
          }
        }
      }
      // slots in order: the terms of one slot go to distinct values
      for (int sj = 0; sj < ns; ++sj) {
#pragma unroll
        for (int i = 0; i < IPT; ++i)
          if (sl[i] == sj) s_acc[dst[i]] += val[i];
        __syncthreads();
      }
    }
    for (int v = tid; v < L; v += BS) out[r0 * DD + v] = (VT)s_acc[v];
    __syncthreads();  // the LDS row is free for the next row
  }
}

// ----------------------------------------------------------------------------
// Fused node-row assembly of K_tangent: one wavefront per row of nodes forms
// the rows of the element terms w B_p^T (D_q - C) B_p' (eq. K-split) of the
// row's elements with plastic points now, in place, and writes the row once
// as its K_elast row plus those terms (ascending element).  No element
// matrices, colours or stamps; the geometry of an element at a plastic point
// is recomputed by each row that needs it.
//   (slot, point) items: J^-1, c1..c4 and n of w (D_q - C) (the vector form
//   of the element-local product), g and a = N g of the row's node;
//   (slot, column node, point part) items: the 3x3 (2x2) block of the term,
//   g_i P'_j + a_i Q'_j + c4 (g'_i g_j + (g . g') delta_ij), summed over the
//   element's plastic points; the parts are summed across adjacent lanes in
//   a fixed order.
// ----------------------------------------------------------------------------
struct KF {
  KR r;
  const double *coord;  // [dim][n_n]
  const double *ref;    // reference gradients [n_q][n_p][dim], then weights [n_q]
  const double *desc;   // tangent descriptors [n_desc][n_int]
  int64_t n_int;
};

template <int ETID>
struct FusedCfg {
  using T = Et<ETID>;
  static constexpr int BS = 64;               // one wavefront per row
  static constexpr int CHS = BS / T::NP;      // element slots per chunk
  static constexpr int NS = T::D == 3 ? 6 : 3;
  static constexpr int PW = T::D * T::D + 4 + NS + 2 * T::D;  // doubles per (slot, point)
  static size_t lds(int max_slots, int max_deg) {
    return sizeof(double) * ((size_t)CHS * T::NQ * PW + (size_t)CHS * T::NP * T::D +
                             (size_t)max_slots + (size_t)max_deg * T::D * T::D);
  }
};

template <int ETID, typename VT>
__global__ __launch_bounds__(64) void k_row_fused(KF f) {
  using T = Et<ETID>;
  using F = FusedCfg<ETID>;
  constexpr int D = T::D, NP = T::NP, NQ = T::NQ, DD = D * D, BS = F::BS, CHS = F::CHS;
  constexpr int NS = F::NS, PW = F::PW;
  constexpr int OC = DD, ON = DD + 4, OG = DD + 4 + NS, OA = OG + D;  // offsets in an item
  const KR &a = f.r;
  extern __shared__ double s_dyn[];
  double *const s_pq = s_dyn;                               // [CHS][NQ][PW]
  double *const s_x = s_pq + CHS * NQ * PW;                 // [CHS][NP][D]
  int *const s_sv = (int *)(s_x + CHS * NP * D);            // active slots e * n_p + p
  uint32_t *const s_sm = (uint32_t *)(s_sv + a.max_slots);  // their point masks
  double *const s_acc = s_x + CHS * NP * D + a.max_slots;   // the row
  const int tid = threadIdx.x;
  const VT *base = (const VT *)a.base;
  VT *out = (VT *)a.out;
  const uint32_t qmask = NQ == 32 ? 0xffffffffu : ((1u << NQ) - 1u);
  const int64_t n_work = a.list ? a.n_list * NP : a.n_n;
  for (int64_t b = blockIdx.x; b < n_work; b += gridDim.x) {
    const int64_t m = a.list ? (int64_t)a.elem[(int64_t)a.list[b / NP] * NP + b % NP] : b;
    const int k0 = a.n2e_ptr[m], k1 = a.n2e_ptr[m + 1];
    const int64_t r0 = a.bptr[m];
    const int L = (int)(a.bptr[m + 1] - r0) * DD;
    // the row's element slots with plastic points now, in slot order (a
    // row's slots fit in the wavefront)
    uint32_t now = 0u, before = 0u;
    int sv = 0;
    if (tid < k1 - k0) {
      sv = a.n2e[k0 + tid];
      now = a.em_cur[sv / NP] & qmask;
      before = a.em_prev ? a.em_prev[sv / NP] : 0u;
    }
    const unsigned long long bal = __ballot(now != 0u);
    if (now) {
      const int r = __popcll(bal & ((1ull << tid) - 1ull));
      s_sv[r] = sv;
      s_sm[r] = now;
    }
    const int nact = __popcll(bal);
    const bool act = __syncthreads_or(a.list != nullptr || (now | before) != 0u) != 0;
    if (!act) continue;  // uniform: neither now nor at the last assembly
    for (int v = tid; v < L; v += BS) s_acc[v] = (double)base[r0 * DD + v];
    for (int c0 = 0; c0 < nact; c0 += CHS) {
      const int nc = nact - c0 < CHS ? nact - c0 : CHS;
      for (int t = tid; t < nc * NP * D; t += BS) {
        const int j = t / (NP * D), r = t - j * (NP * D);
        const int64_t e = s_sv[c0 + j] / NP;
        s_x[t] = f.coord[(int64_t)(r % D) * a.n_n + a.elem[e * NP + r / D]];
      }
      __syncthreads();
      for (int t = tid; t < nc * NQ; t += BS) {
        const int j = t / NQ, q = t - j * NQ;
        if (!((s_sm[c0 + j] >> q) & 1u)) continue;
        const int svj = s_sv[c0 + j];
        const int64_t e = svj / NP;
        const int p = svj - (int)e * NP;
        double Ji[D][D];
        const double det = jac_inv<D, NP>(s_x + j * NP * D, f.ref + q * NP * D, Ji);
        const double w = fabs(det) * f.ref[NQ * NP * D + q];
        const int64_t ip = e * NQ + q;
        double nv[NS];
#pragma unroll
        for (int c = 0; c < NS; ++c) nv[c] = f.desc[c * f.n_int + ip];
        const double al = f.desc[NS * f.n_int + ip], be = f.desc[(NS + 1) * f.n_int + ip];
        const double ga = f.desc[(NS + 2) * f.n_int + ip], de = f.desc[(NS + 3) * f.n_int + ip];
        double g[D], av[D];
        grad<D>(Ji, f.ref + (q * NP + p) * D, g);
        if constexpr (D == 3) {
          av[0] = nv[0] * g[0] + nv[3] * g[1] + nv[5] * g[2];
          av[1] = nv[3] * g[0] + nv[1] * g[1] + nv[4] * g[2];
          av[2] = nv[5] * g[0] + nv[4] * g[1] + nv[2] * g[2];
        } else {
          av[0] = nv[0] * g[0] + nv[2] * g[1];
          av[1] = nv[2] * g[0] + nv[1] * g[1];
        }
        double *o = s_pq + t * PW;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int jj = 0; jj < D; ++jj) o[i * D + jj] = Ji[i][jj];
        o[OC + 0] = w * (de - al / 3.0);
        o[OC + 1] = w * ga;
        o[OC + 2] = w * be;
        o[OC + 3] = 0.5 * w * al;
#pragma unroll
        for (int c = 0; c < NS; ++c) o[ON + c] = nv[c];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          o[OG + d] = g[d];
          o[OA + d] = av[d];
        }
      }
      __syncthreads();
      // points split over 2^k adjacent lanes when the chunk leaves lanes free
      int split = 1;
      while (4 * split * nc * NP <= 2 * BS && 2 * split <= NQ) split *= 2;
      const bool on = tid < nc * NP * split;
      const int h = tid & (split - 1), jp = tid / split;
      const int j = on ? jp / NP : 0, pp = jp - j * NP;
      double acc[DD];
#pragma unroll
      for (int i = 0; i < DD; ++i) acc[i] = 0.0;
      int dst = 0;
      if (on) {
        const int svj = s_sv[c0 + j];
        dst = (a.bpos[(int64_t)svj * NP + pp] - (int32_t)r0) * DD;
        const uint32_t msk = s_sm[c0 + j];
        for (int q = h; q < NQ; q += split) {
          if (!((msk >> q) & 1u)) continue;
          const double *o = s_pq + (j * NQ + q) * PW;
          double Ji[D][D];
#pragma unroll
          for (int i = 0; i < D; ++i)
#pragma unroll
            for (int jj = 0; jj < D; ++jj) Ji[i][jj] = o[i * D + jj];
          double g2[D], a2[D], gp[D], ap[D];
          grad<D>(Ji, f.ref + (q * NP + pp) * D, g2);
          if constexpr (D == 3) {
            a2[0] = o[ON + 0] * g2[0] + o[ON + 3] * g2[1] + o[ON + 5] * g2[2];
            a2[1] = o[ON + 3] * g2[0] + o[ON + 1] * g2[1] + o[ON + 4] * g2[2];
            a2[2] = o[ON + 5] * g2[0] + o[ON + 4] * g2[1] + o[ON + 2] * g2[2];
          } else {
            a2[0] = o[ON + 0] * g2[0] + o[ON + 2] * g2[1];
            a2[1] = o[ON + 2] * g2[0] + o[ON + 1] * g2[1];
          }
          const double c1 = o[OC], c2 = o[OC + 1], c3 = o[OC + 2], c4 = o[OC + 3];
          double dot = 0.0;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            gp[d] = o[OG + d];
            ap[d] = o[OA + d];
            dot += gp[d] * g2[d];
          }
#pragma unroll
          for (int jj = 0; jj < D; ++jj) {
            const double P = c1 * g2[jj] + c2 * a2[jj], Qv = c3 * a2[jj] + c2 * g2[jj];
#pragma unroll
            for (int i = 0; i < D; ++i)
              acc[i * D + jj] += gp[i] * P + ap[i] * Qv + c4 * g2[i] * gp[jj];
          }
#pragma unroll
          for (int i = 0; i < D; ++i) acc[i * D + i] += c4 * dot;
        }
      }
      for (int o = split >> 1; o > 0; o >>= 1)
#pragma unroll
        for (int i = 0; i < DD; ++i) acc[i] += __shfl_xor(acc[i], o);
      // slots in order: the blocks of one slot go to distinct blocks of the row
      for (int jj = 0; jj < nc; ++jj) {
        if (on && h == 0 && j == jj)
#pragma unroll
          for (int i = 0; i < DD; ++i) s_acc[dst + i] += acc[i];
        __syncthreads();
      }
    }
    __syncthreads();
    for (int v = tid; v < L; v += BS) out[r0 * DD + v] = (VT)s_acc[v];
    __syncthreads();  // the LDS row is free for the next row
  }
}

// ----------------------------------------------------------------------------
// Deterministic node gather of the element force vectors, residual and
// partial norms |r|^2, |Q f|^2 and |(I - Q) F|^2 (reactions).
// ----------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_force_gather(int64_t n_n, const int32_t *n2e_ptr,
                                                      const double *Fe,
                                                      const double *f, const uint8_t *freem,
                                                      double *F_out, double *r_out,
                                                      double *partials) {
  __shared__ double s_a[256], s_b[256], s_c[256];
  const int tid = threadIdx.x;
  const int64_t m = (int64_t)blockIdx.x * 256 + tid;
  double rr = 0.0, ff = 0.0, rc = 0.0;
  if (m < n_n) {
    // the free mask and the load do not depend on the slots: issue them
    // with the slot range, then the slots four at a time (unconditional
    // loads from a clamped index, predicated additions in slot order)
    const int k0 = n2e_ptr[m], k1 = n2e_ptr[m + 1];
    bool fr[D];
    double fl[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      fr[i] = freem[D * m + i] != 0;
      fl[i] = f ? f[D * m + i] : 0.0;
    }
    double s[D];
#pragma unroll
    for (int i = 0; i < D; ++i) s[i] = 0.0;
    for (int k = k0; k < k1; k += 4) {
      double v[4][D];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t kk = k + j < k1 ? k + j : k0;
#pragma unroll
        for (int i = 0; i < D; ++i) v[j][i] = Fe[kk * D + i];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k + j < k1) {
#pragma unroll
          for (int i = 0; i < D; ++i) s[i] += v[j][i];
        }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const int64_t dof = D * m + i;
      if (F_out) F_out[dof] = s[i];
      const double fv = fr[i] ? fl[i] : 0.0;
      const double r = fr[i] ? fv - s[i] : 0.0;
      if (r_out) r_out[dof] = r;
      rr += r * r;
      ff += fv * fv;
      if (!fr[i]) rc += s[i] * s[i];  // reaction at a Dirichlet dof
    }
  }
  s_a[tid] = rr;
  s_b[tid] = ff;
  s_c[tid] = rc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      s_a[tid] += s_a[tid + s];
      s_b[tid] += s_b[tid + s];
      s_c[tid] += s_c[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    partials[3 * blockIdx.x] = s_a[0];
    partials[3 * blockIdx.x + 1] = s_b[0];
    partials[3 * blockIdx.x + 2] = s_c[0];
  }
}

// Sum of nblk partial vectors of `width` doubles, fixed order.
__global__ __launch_bounds__(256) void k_reduce(const double *partials, int nblk, int width,
                                                double *out) {
  __shared__ double s[256];
  const int tid = threadIdx.x;
  for (int c = 0; c < width; ++c) {
    s[tid] = strided_sum<32>(partials + c, nblk, width, tid, 256);
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) s[tid] += s[tid + h];
      __syncthreads();
    }
    if (tid == 0) out[c] = s[0];
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// Split form of the tangent, K_t = K_elast + sum over the plastic elements of
// Delta K_e (eq. K_elast-split), with the plastic part applied element by
// element instead of assembled.  For every element of the work list that has
// plastic points now, with M_q = w_q (D_q - C) from the tangent descriptor:
//   MODE 0: v_e = sum_q B_q^T M_q B_q x_e   (x gathered at the element nodes)
//   MODE 1: v_e = diagonal of Delta K_e     (Jacobi preconditioner)
// Sums over the plastic points run in point order.  The element vectors go
// to the node-ordered slots used by the internal force, and k_split_gather
// adds them per node, so no two threads write one value.
// ----------------------------------------------------------------------------
struct KS {
  const double *coord;
  const int32_t *elem;
  const double *ref;
  int64_t n_n, n_int;
  const double *desc;
  const uint32_t *emask;   // plastic points of each element, current
  const int32_t *list;     // work list of the last compaction
  const int32_t *list_n;   // device: its length
  const int32_t *fslot;
  const double *x;         // MODE 0
  double *Fp;              // element vectors in node-ordered slots
  const double *sc;        // PCG scalars (skip once converged) or nullptr
  double G, K;
};

template <int ETID, int MODE>
__global__ __launch_bounds__(CT) void k_split_apply(KS a) {
  using T = Et<ETID>;
  constexpr int D = T::D, NP = T::NP, NQ = T::NQ;
  constexpr int EPB = CT / NQ;
  constexpr int NS = D == 3 ? 6 : 3;
  constexpr int NDESC = D == 3 ? 10 : 7;
  constexpr int NMS = NS * (NS + 1) / 2;           // packed symmetric M
  constexpr int NA = MODE == 0 ? D * D : NMS + D * D;
  __shared__ double s_ref[NQ * NP * D];
  __shared__ double s_wq[NQ];
  __shared__ double s_x[EPB * NP * D];
  __shared__ double s_u[MODE == 0 ? EPB * NP * D : 1];
  __shared__ double s_A[EPB * NQ * NA];
  __shared__ int s_e[EPB];
  __shared__ uint32_t s_m[EPB];
  if (a.sc && a.sc[SC_DONE] != 0.0) return;
  const int tid = threadIdx.x;
  const int64_t n_list = *a.list_n;
  const int64_t k0 = (int64_t)blockIdx.x * EPB;
  if (k0 >= n_list) return;  // uniform
  for (int t = tid; t < NQ * NP * D; t += CT) s_ref[t] = a.ref[t];
  for (int t = tid; t < NQ; t += CT) s_wq[t] = a.ref[NQ * NP * D + t];
  for (int t = tid; t < EPB; t += CT) {
    const int64_t k = k0 + t;
    const int e = k < n_list ? a.list[k] : -1;
    const uint32_t m = e >= 0 ? a.emask[e] : 0u;
    s_e[t] = m ? e : -1;
    s_m[t] = m;
  }
  __syncthreads();
  for (int t = tid; t < EPB * NP; t += CT) {
    const int e = s_e[t / NP];
    if (e < 0) continue;
    const int64_t node = a.elem[(int64_t)e * NP + t % NP];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      s_x[t * D + d] = a.coord[d * a.n_n + node];
      if constexpr (MODE == 0) s_u[t * D + d] = a.x[D * node + d];
    }
  }
  __syncthreads();
  // per (element, plastic point)
  {
    const int el = tid / NQ, q = tid - (tid / NQ) * NQ;
    const int e = tid < EPB * NQ ? s_e[el] : -1;
    if (e >= 0 && ((s_m[el] >> q) & 1u)) {
      const double *xs = s_x + el * NP * D, *dr = s_ref + q * NP * D;
      double Ji[D][D];
      const double det = jac_inv<D, NP>(xs, dr, Ji);
      const double w = fabs(det) * s_wq[q];
      double dsc[NDESC];
      const int64_t ip = (int64_t)e * NQ + q;
#pragma unroll
      for (int c = 0; c < NDESC; ++c) dsc[c] = a.desc[c * a.n_int + ip];
      double *A = s_A + tid * NA;
      if constexpr (MODE == 0) {
        // engineering Voigt strain of x_e, then sigma' = M eps with
        // M = w (alpha DEV + beta n n^T + gamma (n 1^T + 1 n^T) + delta 1 1^T)
        // applied term by term (the matrix of tangent_matrix, not formed)
        double ev[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) ev[i] = 0.0;
        const double *us = s_u + el * NP * D;
#pragma unroll 3
        for (int p = 0; p < NP; ++p) {
          double g[D];
          grad<D>(Ji, dr + p * D, g);
          const double *up = us + p * D;
          if constexpr (D == 3) {
            ev[0] += g[0] * up[0];
            ev[1] += g[1] * up[1];
            ev[2] += g[2] * up[2];
            ev[3] += g[1] * up[0] + g[0] * up[1];
            ev[4] += g[2] * up[1] + g[1] * up[2];
            ev[5] += g[2] * up[0] + g[0] * up[2];
          } else {
            ev[0] += g[0] * up[0];
            ev[1] += g[1] * up[1];
            ev[2] += g[1] * up[0] + g[0] * up[1];
          }
        }
        constexpr int NN = D == 3 ? 3 : 2;  // normal components
        double tr = 0.0, ne = 0.0;
#pragma unroll
        for (int i = 0; i < NN; ++i) tr += ev[i];
#pragma unroll
        for (int i = 0; i < NS; ++i) ne += dsc[i] * ev[i];
        const double al = dsc[NS], be = dsc[NS + 1], ga = dsc[NS + 2], de = dsc[NS + 3];
        double sg[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const bool nI = i < NN;
          const double dev = nI ? ev[i] - tr / 3.0 : 0.5 * ev[i];
          sg[i] = w * (al * dev + be * dsc[i] * ne + ga * (dsc[i] * tr + (nI ? ne : 0.0)) +
                       (nI ? de * tr : 0.0));
        }
        // B_p^T sigma' = S g_p with S the symmetric tensor of sigma', and
        // g_p = J^{-1} dphi_p, so one D x D matrix A = S J^{-1} per point
        double sm[D][D];
        if constexpr (D == 3) {
          sm[0][0] = sg[0]; sm[1][1] = sg[1]; sm[2][2] = sg[2];
          sm[0][1] = sm[1][0] = sg[3];
          sm[1][2] = sm[2][1] = sg[4];
          sm[0][2] = sm[2][0] = sg[5];
        } else {
          sm[0][0] = sg[0]; sm[1][1] = sg[1];
          sm[0][1] = sm[1][0] = sg[2];
        }
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) v += sm[i][k] * Ji[k][j];
            A[i * D + j] = v;
          }
      } else {
        double M[NS * NS];
        tangent_matrix<D>(dsc, false, a.G, a.K, w, M);
        int o = 0;
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
          for (int j = i; j < NS; ++j) A[o++] = M[i * NS + j];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) A[NMS + i * D + j] = Ji[i][j];
      }
    }
  }
  __syncthreads();
  // per (element, node): sum over the plastic points in order
  for (int t = tid; t < EPB * NP; t += CT) {
    const int el = t / NP, p = t - (t / NP) * NP;
    const int e = s_e[el];
    if (e < 0) continue;
    const uint32_t mask = s_m[el];
    double f[D];
#pragma unroll
    for (int i = 0; i < D; ++i) f[i] = 0.0;
    for (int qq = 0; qq < NQ; ++qq) {
      if (!((mask >> qq) & 1u)) continue;
      const double *A = s_A + (el * NQ + qq) * NA;
      const double *dr = s_ref + (qq * NP + p) * D;
      if constexpr (MODE == 0) {
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) f[i] += A[i * D + j] * dr[j];
      } else {
        double Ji[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) Ji[i][j] = A[NMS + i * D + j];
        double g[D];
        grad<D>(Ji, dr, g);
        double Mf[NS][NS];
        {
          int o = 0;
#pragma unroll
          for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int j = i; j < NS; ++j) {
              Mf[i][j] = A[o];
              Mf[j][i] = A[o];
              ++o;
            }
        }
        // column of B for displacement component i of node p
#pragma unroll
        for (int i = 0; i < D; ++i) {
          double b[NS];
#pragma unroll
          for (int k = 0; k < NS; ++k) b[k] = 0.0;
          if constexpr (D == 3) {
            if (i == 0) { b[0] = g[0]; b[3] = g[1]; b[5] = g[2]; }
            if (i == 1) { b[1] = g[1]; b[3] = g[0]; b[4] = g[2]; }
            if (i == 2) { b[2] = g[2]; b[4] = g[1]; b[5] = g[0]; }
          } else {
            if (i == 0) { b[0] = g[0]; b[2] = g[1]; }
            if (i == 1) { b[1] = g[1]; b[2] = g[0]; }
          }
          double v = 0.0;
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            double mb = 0.0;
#pragma unroll
            for (int l = 0; l < NS; ++l) mb += Mf[k][l] * b[l];
            v += b[k] * mb;
          }
          f[i] += v;
        }
      }
    }
    const int64_t slot = a.fslot[(int64_t)e * NP + p];
#pragma unroll
    for (int i = 0; i < D; ++i) a.Fp[slot * D + i] = f[i];
  }
}

// Node sums of the split-form element vectors (elements plastic now only).
//   MODE 0: y += Q v; optional per-block partial p.y (fixed tree) for PCG.
//   MODE 1: dinv = Q / (diag K_elast + v).
template <int D, int MODE>
__global__ __launch_bounds__(256) void k_split_gather(int64_t n_n, const int32_t *n2e_ptr,
                                                      const int32_t *slot_elem,
                                                      const uint32_t *emask, const double *Fp,
                                                      const uint8_t *freem, double *y,
                                                      const double *p, double *partials,
                                                      const double *sc, const int32_t *bdiag,
                                                      const double *Ke, double *dinv) {
  __shared__ double s_a[256];
  if (sc && sc[SC_DONE] != 0.0) return;
  const int tid = threadIdx.x;
  const int64_t m = (int64_t)blockIdx.x * 256 + tid;
  double dot = 0.0;
  if (m < n_n) {
    double s[D];
#pragma unroll
    for (int i = 0; i < D; ++i) s[i] = 0.0;
    // four slots at a time: element ids, their masks, then the vectors
    // (unconditional loads from clamped indices, predicated additions in
    // slot order)
    const int k0 = n2e_ptr[m], k1 = n2e_ptr[m + 1];
    for (int k = k0; k < k1; k += 4) {
      int64_t kk[4];
      int el[4];
      uint32_t em[4];
      double v[4][D];
#pragma unroll
      for (int j = 0; j < 4; ++j) kk[j] = k + j < k1 ? k + j : k0;
#pragma unroll
      for (int j = 0; j < 4; ++j) el[j] = slot_elem[kk[j]];
#pragma unroll
      for (int j = 0; j < 4; ++j) em[j] = emask[el[j]];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < D; ++i) v[j][i] = Fp[kk[j] * D + i];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k + j < k1 && em[j] != 0u) {
#pragma unroll
          for (int i = 0; i < D; ++i) s[i] += v[j][i];
        }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const int64_t r = D * m + i;
      const bool fr = freem[r] != 0;
      if constexpr (MODE == 0) {
        const double yv = y[r] + (fr ? s[i] : 0.0);
        y[r] = yv;
        if (p) dot += p[r] * yv;
      } else {
        const double d = Ke[((int64_t)bdiag[m] * D + i) * D + i] + s[i];
        dinv[r] = fr ? 1.0 / d : 0.0;
      }
    }
  }
  if (MODE != 0 || !partials) return;
  s_a[tid] = dot;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) s_a[tid] += s_a[tid + h];
    __syncthreads();
  }
  if (tid == 0) partials[blockIdx.x] = s_a[0];
}

// ----------------------------------------------------------------------------
// Stable compaction (wavefront ballot + block scan).  Items i < n (optionally
// through a permutation, -1 = padding) with predicate (src | src2) != 0; kind
// 0: uint8 source, kind 1: uint32 source (bitmask), src2 uint32 or null.
// ----------------------------------------------------------------------------
// The CMP_ITEMS items of this thread (item k at base + k*CMP_THREADS + tid,
// through perm when given; -1 past n or for padding) and their predicate
// words (src: uint8 for KIND 0, uint32 for KIND 1; src2 uint32 or null).
// Every load is unconditional (out-of-range lanes read element 0, which
// every source array has, and discard it), and the index loads are issued
// before the value loads that depend on them: a thread waits for two memory
// round trips, not 2*CMP_ITEMS.
template <int KIND>
__device__ inline void cmp_load(const void *src, const uint32_t *src2, const int32_t *perm,
                                int64_t n, int64_t base, int tid, int64_t *item, uint32_t *v,
                                uint32_t *v2) {
  int64_t idx[CMP_ITEMS];
#pragma unroll
  for (int k = 0; k < CMP_ITEMS; ++k) {
    const int64_t i = base + (int64_t)k * CMP_THREADS + tid;
    idx[k] = i < n ? i : -1;
  }
  if (perm) {
    int32_t pv[CMP_ITEMS];
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k) pv[k] = perm[idx[k] >= 0 ? idx[k] : 0];
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k) item[k] = idx[k] >= 0 ? (int64_t)pv[k] : -1;
  } else {
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k) item[k] = idx[k];
  }
  uint32_t raw[CMP_ITEMS];
#pragma unroll
  for (int k = 0; k < CMP_ITEMS; ++k) {
    const int64_t j = item[k] >= 0 ? item[k] : 0;
    raw[k] = KIND == 0 ? (uint32_t)((const uint8_t *)src)[j] : ((const uint32_t *)src)[j];
  }
#pragma unroll
  for (int k = 0; k < CMP_ITEMS; ++k) v[k] = item[k] >= 0 ? raw[k] : 0u;
  if (src2) {
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k) raw[k] = src2[item[k] >= 0 ? item[k] : 0];
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k) v2[k] = item[k] >= 0 ? raw[k] : 0u;
  } else {
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k) v2[k] = 0u;
  }
}

template <int KIND>
__global__ __launch_bounds__(CMP_THREADS) void k_compact_count(const void *src,
                                                               const uint32_t *src2,
                                                               const int32_t *perm, int64_t n,
                                                               int32_t *counts, int32_t *counts2,
                                                               int32_t *counts3) {
  __shared__ int32_t s_c[CMP_THREADS / 64], s_b[CMP_THREADS / 64], s_z[CMP_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * CMP_CHUNK;
  int64_t item[CMP_ITEMS];
  uint32_t v[CMP_ITEMS], v2[CMP_ITEMS];
  cmp_load<KIND>(src, src2, perm, n, base, tid, item, v, v2);
  int32_t cnt = 0, bits = 0, nz = 0;
#pragma unroll
  for (int k = 0; k < CMP_ITEMS; ++k) {
    cnt += __popcll(__ballot((v[k] | v2[k]) != 0u));
    nz += __popcll(__ballot(v[k] != 0u));
    bits += __popc(v[k]);
  }
  for (int o = 32; o > 0; o >>= 1) bits += __shfl_down(bits, o, 64);
  if (lane == 0) {
    s_c[wv] = cnt;
    s_b[wv] = bits;
    s_z[wv] = nz;
  }
  __syncthreads();
  if (tid == 0) {
    int32_t c = 0, bb = 0, z = 0;
    for (int w = 0; w < CMP_THREADS / 64; ++w) {
      c += s_c[w];
      bb += s_b[w];
      z += s_z[w];
    }
    counts[blockIdx.x] = c;
    counts2[blockIdx.x] = bb;
    counts3[blockIdx.x] = z;
  }
}

// Scatter of the selected items.  Each block first sums the counts of the
// blocks before it (its output offset); block 0 also writes the totals
// [0] selected items, [1] set bits, [2] items with src != 0, and the output
// offset of every colour segment.  Integer sums: exact in any order.
template <int KIND>
__global__ __launch_bounds__(CMP_THREADS) void k_compact_scatter(
    const void *src, const uint32_t *src2, const int32_t *perm, int64_t n,
    const int32_t *counts, const int32_t *counts2, const int32_t *counts3, int nblk,
    const int32_t *colour_first_block, int n_col, int32_t *colour_off, int32_t *totals,
    int32_t *out) {
  __shared__ int32_t s_w[CMP_THREADS / 64];
  __shared__ int32_t s_r[3][CMP_THREADS];
  __shared__ int32_t s_cfb[CMP_MAX_COLOURS + 1], s_cc[CMP_MAX_COLOURS + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * CMP_CHUNK;
  // this thread's items first (their loads overlap the offset reduction)
  int64_t item[CMP_ITEMS];
  uint32_t vv[CMP_ITEMS], vv2[CMP_ITEMS];
  cmp_load<KIND>(src, src2, perm, n, base, tid, item, vv, vv2);
  // offset of this block; block 0: the three totals
  {
    int32_t a = 0, b2 = 0, b3 = 0;
    const int lim = blockIdx.x == 0 ? nblk : (int)blockIdx.x;
    for (int j = tid; j < lim; j += CMP_THREADS) {
      a += counts[j];
      if (blockIdx.x == 0) {
        b2 += counts2[j];
        b3 += counts3[j];
      }
    }
    s_r[0][tid] = a;
    s_r[1][tid] = b2;
    s_r[2][tid] = b3;
    __syncthreads();
    for (int o = CMP_THREADS / 2; o > 0; o >>= 1) {
      if (tid < o) {
        s_r[0][tid] += s_r[0][tid + o];
        s_r[1][tid] += s_r[1][tid + o];
        s_r[2][tid] += s_r[2][tid + o];
      }
      __syncthreads();
    }
  }
  int32_t run = blockIdx.x == 0 ? 0 : s_r[0][0];
  if (blockIdx.x == 0) {
    const int32_t total = s_r[0][0];
    if (tid == 0) {
      totals[0] = total;
      totals[1] = s_r[1][0];
      totals[2] = s_r[2][0];
    }
    if (colour_off) {
      // each block of the colour-major order lies in one colour (every
      // colour is padded to whole blocks): the selected counts summed per
      // colour (integer sums: exact in any order), then the offsets in
      // colour order
      for (int c = tid; c <= n_col; c += CMP_THREADS) {
        s_cfb[c] = colour_first_block[c];
        s_cc[c] = 0;
      }
      __syncthreads();
      for (int j = tid; j < nblk; j += CMP_THREADS) {
        int lo = 0, hi = n_col - 1;  // the last colour whose first block is <= j
        while (lo < hi) {
          const int mid = (lo + hi + 1) / 2;
          if (s_cfb[mid] <= j) lo = mid;
          else hi = mid - 1;
        }
        atomicAdd(&s_cc[lo], counts[j]);
      }
      __syncthreads();
      for (int c = tid; c <= n_col; c += CMP_THREADS) {
        int32_t off = 0;
        for (int k = 0; k < c; ++k) off += s_cc[k];
        colour_off[c] = off;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < CMP_ITEMS; ++k) {
    const uint32_t v = vv[k] | vv2[k];
    const uint64_t b = __ballot(v != 0u);
    const int rank = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) s_w[wv] = __popcll(b);
    __syncthreads();
    int32_t before = 0, tot = 0;
    for (int w = 0; w < CMP_THREADS / 64; ++w) {
      if (w < wv) before += s_w[w];
      tot += s_w[w];
    }
    if (v != 0u) out[run + before + rank] = (int32_t)item[k];
    run += tot;
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// Sparse matrix views, SpMV and PCG vectors
// ----------------------------------------------------------------------------
template <int D, typename VT>
__global__ void k_csr_expand(int64_t n_n, int64_t nnzb, const int32_t *bptr,
                             const int32_t *bcol, const VT *val, int32_t *row_ptr,
                             int32_t *col_idx, double *vout) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > D * n_n) return;
  if (r == D * n_n) {
    if (row_ptr) row_ptr[r] = (int32_t)(D * D * nnzb);
    return;
  }
  const int64_t m = r / D;
  const int i = (int)(r - m * D);
  const int64_t b0 = bptr[m], deg = bptr[m + 1] - b0;
  const int64_t rp = D * D * b0 + i * D * deg;
  if (row_ptr) row_ptr[r] = (int32_t)rp;
  for (int64_t t = 0; t < deg; ++t)
    for (int j = 0; j < D; ++j) {
      if (col_idx) col_idx[rp + D * t + j] = (int32_t)(D * bcol[b0 + t] + j);
      if (vout) vout[rp + D * t + j] = (double)val[((b0 + t) * D + i) * D + j];
    }
}

template <int ETID>
__global__ void k_pos_expand(int64_t n_e, const int32_t *elem, const int32_t *bptr,
                             const int32_t *bpos, int32_t *pos) {
  using T = Et<ETID>;
  constexpr int D = T::D, NP = T::NP;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_e * NP * NP) return;
  const int64_t e = t / (NP * NP);
  const int p = (int)((t / NP) % NP), pp = (int)(t % NP);
  const int64_t m = elem[e * NP + p];
  const int64_t b0 = bptr[m], deg = bptr[m + 1] - b0;
  const int64_t tt = bpos[t] - b0;
  constexpr int NL = D * NP;
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j)
      pos[(e * NL + D * p + i) * NL + D * pp + j] =
          (int32_t)(D * D * b0 + i * D * deg + D * tt + j);
}

template <int D, typename VT>
__global__ void k_diag_inv(int64_t n_n, const int32_t *bdiag, const VT *Kt, const uint8_t *freem,
                           double *dinv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D * n_n) return;
  const int64_t m = r / D;
  const int i = (int)(r - m * D);
  const double d = (double)Kt[((int64_t)bdiag[m] * D + i) * D + i];
  dinv[r] = freem[r] ? 1.0 / d : 0.0;
}


// y = Q K x with G lanes per node row: the lanes of a group read consecutive
// node blocks of the row (coalesced), each lane accumulates the dim rows of
// the block row, and a butterfly over the G lanes (fixed order, identical
// in every lane) reduces them.  freem == nullptr: y = K x on every row.
// Optional per-block partial x.y (fixed order); with sc, nothing is done
// once PCG has converged.
template <int D, typename VT, int G>
__global__ __launch_bounds__(256) void k_spmv(int64_t n_n, const int32_t *bptr,
                                              const int32_t *bcol, const VT *val,
                                              const double *x, const uint8_t *freem, double *y,
                                              double *partials, const double *sc,
                                              const double *x1, const double *x2) {
  __shared__ double s[256 / G];
  if (sc && sc[SC_DONE] != 0.0) return;
  const int tid = threadIdx.x;
  const int g = tid % G;
  const int64_t m = ((int64_t)blockIdx.x * 256 + tid) / G;
  double acc[D];
#pragma unroll
  for (int i = 0; i < D; ++i) acc[i] = 0.0;
  if (m < n_n) {
    const int b1 = bptr[m + 1];
    for (int b = bptr[m] + g; b < b1; b += G) {
      const int64_t c = bcol[b];
      double xv[D];
      if constexpr (D == 3) {
        // read through x1 = x + 1 and x2 = x + 2 so that the compiler keeps
        // three aligned 8-byte loads (merged, they become a 16-byte load at a
        // 24-byte stride, misaligned for every other node: measurably slower)
        xv[0] = x[3 * c];
        xv[1] = x1[3 * c];
        xv[2] = x2[3 * c];
      } else {
#pragma unroll
        for (int j = 0; j < D; ++j) xv[j] = x[D * c + j];
      }
      const VT *v = val + (int64_t)b * D * D;
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) acc[i] += (double)v[i * D + j] * xv[j];
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] += __shfl_xor(acc[i], o, G);
  double dot = 0.0;
  if (m < n_n && g == 0) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const int64_t r = D * m + i;
      const double yv = (!freem || freem[r]) ? acc[i] : 0.0;
      y[r] = yv;
      dot += x[r] * yv;
    }
  }
  if (!partials) return;  // uniform
  // block sum of the group leaders' dots, fixed order
  if (g == 0) s[tid / G] = dot;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < 256 / G; ++k) t += s[k];
    partials[blockIdx.x] = t;
  }
}

// alpha = rz / pq
__global__ __launch_bounds__(256) void k_pcg_alpha(const double *partials, int nblk, double *sc) {
  __shared__ double s[256];
  if (sc[SC_DONE] != 0.0) return;
  const int tid = threadIdx.x;
  s[tid] = strided_sum<32>(partials, nblk, 1, tid, 256);
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) s[tid] += s[tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    const double pq = s[0];
    sc[SC_PQ] = pq;
    // breakdown: the operator is not positive definite along p (possible
    // for a tangent near the Drucker-Prager apex) or a scalar is not finite;
    // stop with the last iterate
    if (!(pq > 0.0 && pq <= DBL_MAX) || !(fabs(sc[SC_RZ]) <= DBL_MAX)) {
      sc[SC_ALPHA] = 0.0;
      sc[SC_BREAK] = 1.0;
      sc[SC_DONE] = 1.0;
    } else {
      sc[SC_ALPHA] = sc[SC_RZ] / pq;
    }
  }
}

// new search direction p = z + beta p_old
__global__ __launch_bounds__(256) void k_pcg_direction(int64_t n, const double *z,
                                                       const double *pold, double *pnew,
                                                       const double *sc) {
  if (sc[SC_DONE] != 0.0) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) pnew[i] = z[i] + sc[SC_BETA] * pold[i];
}

// x += alpha p, r -= alpha q, z = dinv r, partial (r.z, r.r)
__global__ __launch_bounds__(256) void k_pcg_update(int64_t n, double *x, const double *p,
                                                    double *r, const double *q, double *z,
                                                    const double *dinv, const double *sc,
                                                    double *partials) {
  __shared__ double sa[256], sb[256];
  if (sc[SC_DONE] != 0.0) return;
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  double rz = 0.0, rr = 0.0;
  if (i < n) {
    const double al = sc[SC_ALPHA];
    x[i] += al * p[i];
    const double rv = r[i] - al * q[i];
    r[i] = rv;
    const double zv = dinv[i] * rv;
    z[i] = zv;
    rz = rv * zv;
    rr = rv * rv;
  }
  sa[tid] = rz;
  sb[tid] = rr;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      sa[tid] += sa[tid + h];
      sb[tid] += sb[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    partials[2 * blockIdx.x] = sa[0];
    partials[2 * blockIdx.x + 1] = sb[0];
  }
}

// beta = rz_new / rz, convergence flag
__global__ __launch_bounds__(256) void k_pcg_beta(const double *partials, int nblk, double *sc,
                                                  int init, double rtol) {
  __shared__ double sa[256], sb[256];
  if (!init && sc[SC_DONE] != 0.0) return;
  const int tid = threadIdx.x;
  strided_sum_pairs<32>(partials, nblk, tid, 256, sa[tid], sb[tid]);
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      sa[tid] += sa[tid + h];
      sb[tid] += sb[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const bool finite = fabs(sa[0]) <= DBL_MAX && sb[0] <= DBL_MAX;
    if (init) {
      sc[SC_RZ] = sa[0];
      sc[SC_RR] = sb[0];
      sc[SC_RR0] = sb[0];
      sc[SC_TOL] = rtol * rtol * sb[0];
      sc[SC_ITS] = 0.0;
      sc[SC_BETA] = 0.0;
      sc[SC_NEED] = 0.0;
      sc[SC_BREAK] = finite ? 0.0 : 1.0;
      sc[SC_DONE] = (!finite || sb[0] <= sc[SC_TOL]) ? 1.0 : 0.0;
    } else if (!finite) {
      // the update just made is not trusted beyond this point: stop
      sc[SC_BREAK] = 1.0;
      sc[SC_DONE] = 1.0;
    } else {
      sc[SC_BETA] = sa[0] / sc[SC_RZ];
      sc[SC_RZ] = sa[0];
      sc[SC_RR] = sb[0];
      sc[SC_ITS] += 1.0;
      if (sb[0] <= sc[SC_TOL]) sc[SC_DONE] = 1.0;
    }
  }
}

// PCG iteration in two kernels (systems of moderate size).  The scalar
// steps of the single-block kernels (alpha, beta) are repeated by every block
// of the kernel that follows them: each block sums the same partials in the
// same order (strided_sum, then the same tree), so all blocks hold the values
// the single-block kernel would have computed, and block 0 records them in
// the other scalar buffer (sc_in is only read inside a kernel).
//   k_pcg_spmv2: the beta step left by k_pcg_update2 (SC_NEED), then
//     q = Q K p with p = z + beta p_old formed at each use (the rows of the
//     block store their p) and the block's partial p.q;
//   k_pcg_update2: alpha with the breakdown test, then x, r, z and the
//     block's partials r.z, r.r (SC_NEED = 1);
//   k_pcg_finish2 (one block, after a chunk of iterations): the pending beta
//     step, so that the host sees the same scalars as after the five-kernel
//     iteration.
__device__ inline void pcg2_beta_step(double *st, double rz, double rr) {
  const bool finite = fabs(rz) <= DBL_MAX && rr <= DBL_MAX;
  if (!finite) {
    st[SC_BREAK] = 1.0;
    st[SC_DONE] = 1.0;
  } else {
    st[SC_BETA] = rz / st[SC_RZ];
    st[SC_RZ] = rz;
    st[SC_RR] = rr;
    st[SC_ITS] += 1.0;
    if (rr <= st[SC_TOL]) st[SC_DONE] = 1.0;
  }
  st[SC_NEED] = 0.0;
}

// the beta step's two sums over the update kernel's partials (every thread of
// the block calls it; the tree is that of k_pcg_beta)
__device__ inline void pcg2_sums(const double *pin, int nin, double *sa, double *sb) {
  const int tid = threadIdx.x;
  sa[tid] = strided_sum(pin, nin, 2, tid, 256);
  sb[tid] = strided_sum(pin + 1, nin, 2, tid, 256);
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      sa[tid] += sa[tid + h];
      sb[tid] += sb[tid + h];
    }
    __syncthreads();
  }
}

template <int D, typename VT, int G>
__global__ __launch_bounds__(256) void k_pcg_spmv2(int64_t n_n, const int32_t *bptr,
                                                   const int32_t *bcol, const VT *val,
                                                   const double *z, const double *pold,
                                                   double *pnew, const uint8_t *freem, double *q,
                                                   const double *pin, int nin,
                                                   const double *sc_in, double *sc_out,
                                                   double *pout) {
  __shared__ double sa[256], sb[256];
  __shared__ double s_st[SC_N];
  const int tid = threadIdx.x;
  if (tid < SC_N) s_st[tid] = sc_in[tid];
  __syncthreads();
  if (s_st[SC_NEED] != 0.0 && s_st[SC_DONE] == 0.0) {  // uniform
    pcg2_sums(pin, nin, sa, sb);
    if (tid == 0) pcg2_beta_step(s_st, sa[0], sb[0]);
    __syncthreads();
  }
  if (blockIdx.x == 0 && tid < SC_N) sc_out[tid] = s_st[tid];
  if (s_st[SC_DONE] != 0.0) return;  // uniform
  const double beta = s_st[SC_BETA];
  const int g = tid % G;
  const int64_t m = ((int64_t)blockIdx.x * 256 + tid) / G;
  double acc[D];
#pragma unroll
  for (int i = 0; i < D; ++i) acc[i] = 0.0;
  if (m < n_n) {
    const int b1 = bptr[m + 1];
    for (int b = bptr[m] + g; b < b1; b += G) {
      const int64_t cn = bcol[b];
      double xv[D];
#pragma unroll
      for (int j = 0; j < D; ++j) xv[j] = z[D * cn + j] + beta * pold[D * cn + j];
      const VT *v = val + (int64_t)b * D * D;
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) acc[i] += (double)v[i * D + j] * xv[j];
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] += __shfl_xor(acc[i], o, G);
  double dot = 0.0;
  if (m < n_n && g == 0) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const int64_t r = D * m + i;
      const double pv = z[r] + beta * pold[r];
      pnew[r] = pv;
      const double yv = freem[r] ? acc[i] : 0.0;
      q[r] = yv;
      dot += pv * yv;
    }
  }
  // block sum of the group leaders' dots, fixed order (as k_spmv)
  __shared__ double s[256 / G];
  if (g == 0) s[tid / G] = dot;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < 256 / G; ++k) t += s[k];
    pout[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(256) void k_pcg_update2(int64_t n, double *x, const double *p,
                                                     double *r, const double *q, double *z,
                                                     const double *dinv, const double *pin,
                                                     int nin, const double *sc_in,
                                                     double *sc_out, double *pout) {
  __shared__ double sa[256], sb[256];
  __shared__ double s_st[SC_N];
  const int tid = threadIdx.x;
  if (tid < SC_N) s_st[tid] = sc_in[tid];
  __syncthreads();
  if (s_st[SC_DONE] == 0.0) {  // uniform: alpha as k_pcg_alpha
    sa[tid] = strided_sum(pin, nin, 1, tid, 256);
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) sa[tid] += sa[tid + h];
      __syncthreads();
    }
    if (tid == 0) {
      const double pq = sa[0];
      s_st[SC_PQ] = pq;
      if (!(pq > 0.0 && pq <= DBL_MAX) || !(fabs(s_st[SC_RZ]) <= DBL_MAX)) {
        s_st[SC_ALPHA] = 0.0;
        s_st[SC_BREAK] = 1.0;
        s_st[SC_DONE] = 1.0;
      } else {
        s_st[SC_ALPHA] = s_st[SC_RZ] / pq;
        s_st[SC_NEED] = 1.0;
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && tid < SC_N) sc_out[tid] = s_st[tid];
  if (s_st[SC_DONE] != 0.0) return;  // uniform
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  double rz = 0.0, rr = 0.0;
  if (i < n) {
    const double al = s_st[SC_ALPHA];
    x[i] += al * p[i];
    const double rv = r[i] - al * q[i];
    r[i] = rv;
    const double zv = dinv[i] * rv;
    z[i] = zv;
    rz = rv * zv;
    rr = rv * rv;
  }
  sa[tid] = rz;
  sb[tid] = rr;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      sa[tid] += sa[tid + h];
      sb[tid] += sb[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    pout[2 * blockIdx.x] = sa[0];
    pout[2 * blockIdx.x + 1] = sb[0];
  }
}

__global__ __launch_bounds__(256) void k_pcg_finish2(const double *pin, int nin, double *sc) {
  __shared__ double sa[256], sb[256];
  if (sc[SC_NEED] == 0.0 || sc[SC_DONE] != 0.0) return;
  pcg2_sums(pin, nin, sa, sb);
  if (threadIdx.x == 0) pcg2_beta_step(sc, sa[0], sb[0]);
}

// PCG iterations of a small system in one workgroup: the same steps and
// scalars as the five-kernel iteration (p = z + beta p, q = Q K p with p.q,
// alpha with the breakdown test, x, r, z updates with r.z and r.r, beta and
// the stopping test), the direction updated in place, the reductions over
// the workgroup in a fixed tree, the scalars in LDS and written back at the
// end.  At most n_it iterations; stops early when done.
constexpr int PCGS_T = 1024;

// sums of a and b over the workgroup, fixed order: a butterfly inside each
// wavefront, then the wavefronts' sums in order (every thread gets both)
__device__ inline void pcgs_sum2(double *s, double &a, double &b) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if (lane == 0) {
    s[2 * w] = a;
    s[2 * w + 1] = b;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
#pragma unroll
  for (int k = 0; k < PCGS_T / 64; ++k) {
    ta += s[2 * k];
    tb += s[2 * k + 1];
  }
  __syncthreads();
  a = ta;
  b = tb;
}

template <int D, typename VT>
__global__ __launch_bounds__(PCGS_T) void k_pcg_small(int n_it, int64_t n_n, const int32_t *bptr,
                                                      const int32_t *bcol, const VT *val,
                                                      const uint8_t *freem, const double *dinv,
                                                      double *x, double *r, double *z, double *p,
                                                      double *q, double *sc) {
  __shared__ double s_red[2 * (PCGS_T / 64)];
  __shared__ double s_sc[SC_N];
  const int tid = threadIdx.x;
  const int64_t n_dof = D * n_n;
  if (tid < SC_N) s_sc[tid] = sc[tid];
  __syncthreads();
  for (int it = 0; it < n_it && s_sc[SC_DONE] == 0.0; ++it) {
    const double beta = s_sc[SC_BETA];
    for (int64_t i = tid; i < n_dof; i += PCGS_T) p[i] = z[i] + beta * p[i];
    __syncthreads();
    double dot = 0.0;
    for (int64_t m = tid; m < n_n; m += PCGS_T) {
      double acc[D];
#pragma unroll
      for (int i = 0; i < D; ++i) acc[i] = 0.0;
      const int b1 = bptr[m + 1];
      for (int b = bptr[m]; b < b1; ++b) {
        const int64_t cn = bcol[b];
        const VT *v = val + (int64_t)b * D * D;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) acc[i] += (double)v[i * D + j] * p[D * cn + j];
      }
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const int64_t rr = D * m + i;
        const double yv = freem[rr] ? acc[i] : 0.0;
        q[rr] = yv;
        dot += p[rr] * yv;
      }
    }
    double pq = dot, unused = 0.0;
    pcgs_sum2(s_red, pq, unused);
    if (tid == 0) {
      s_sc[SC_PQ] = pq;
      if (!(pq > 0.0 && pq <= DBL_MAX) || !(fabs(s_sc[SC_RZ]) <= DBL_MAX)) {
        s_sc[SC_ALPHA] = 0.0;
        s_sc[SC_BREAK] = 1.0;
        s_sc[SC_DONE] = 1.0;
      } else {
        s_sc[SC_ALPHA] = s_sc[SC_RZ] / pq;
      }
    }
    __syncthreads();
    if (s_sc[SC_DONE] != 0.0) break;
    const double al = s_sc[SC_ALPHA];
    double rz = 0.0, rsq = 0.0;
    for (int64_t i = tid; i < n_dof; i += PCGS_T) {
      x[i] += al * p[i];
      const double rv = r[i] - al * q[i];
      r[i] = rv;
      const double zv = dinv[i] * rv;
      z[i] = zv;
      rz += rv * zv;
      rsq += rv * rv;
    }
    double srz = rz, srr = rsq;
    pcgs_sum2(s_red, srz, srr);
    if (tid == 0) {
      if (!(fabs(srz) <= DBL_MAX && srr <= DBL_MAX)) {
        s_sc[SC_BREAK] = 1.0;
        s_sc[SC_DONE] = 1.0;
      } else {
        s_sc[SC_BETA] = srz / s_sc[SC_RZ];
        s_sc[SC_RZ] = srz;
        s_sc[SC_RR] = srr;
        s_sc[SC_ITS] += 1.0;
        if (srr <= s_sc[SC_TOL]) s_sc[SC_DONE] = 1.0;
      }
    }
    __syncthreads();
  }
  if (tid < SC_N) sc[tid] = s_sc[tid];
}

// r = Q b, x = 0, z = dinv r, p_old = 0, partial (r.z, r.r)
__global__ __launch_bounds__(256) void k_pcg_init(int64_t n, const double *b, const uint8_t *freem,
                                                  double *x, double *r, double *z, double *pold,
                                                  const double *dinv, double *partials) {
  __shared__ double sa[256], sb[256];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  double rz = 0.0, rr = 0.0;
  if (i < n) {
    const double rv = freem[i] ? b[i] : 0.0;
    x[i] = 0.0;
    r[i] = rv;
    const double zv = dinv[i] * rv;
    z[i] = zv;
    pold[i] = 0.0;
    rz = rv * zv;
    rr = rv * rv;
  }
  sa[tid] = rz;
  sb[tid] = rr;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      sa[tid] += sa[tid + h];
      sb[tid] += sb[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    partials[2 * blockIdx.x] = sa[0];
    partials[2 * blockIdx.x + 1] = sb[0];
  }
}

__global__ void k_axpy_free(int64_t n, const double *du, const uint8_t *freem, double a,
                            double *u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && freem[i]) u[i] += a * du[i];
}

// trial displacement of a line search: out = u + a du on free dofs
__global__ void k_trial(int64_t n, const double *u, const double *du, double a,
                        const uint8_t *freem, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = freem[i] ? u[i] + a * du[i] : u[i];
}

// per-block partial dot products x_k . y_k (up to 4 pairs), fixed-order
// tree in the block; k_reduce sums the blocks in order
struct DotPairs {
  const double *x[4];
  const double *y[4];
};
template <int NPAIR>
__global__ __launch_bounds__(256) void k_dots(int64_t n, DotPairs p, double *partials) {
  __shared__ double s[NPAIR][256];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
#pragma unroll
  for (int k = 0; k < NPAIR; ++k) s[k][tid] = i < n ? p.x[k][i] * p.y[k][i] : 0.0;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int k = 0; k < NPAIR; ++k) s[k][tid] += s[k][tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < NPAIR; ++k) partials[NPAIR * blockIdx.x + k] = s[k][0];
  }
}

__global__ void k_extrapolate(int64_t n, const double *u, const double *u2, double t,
                              const uint8_t *freem, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = u[i];
  out[i] = (u2 && freem[i]) ? v + t * (v - u2[i]) : v;
}

__global__ void k_to_float(const double *src, float *dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// ----------------------------------------------------------------------------
// Launch wrappers
// ----------------------------------------------------------------------------
template <int ETID>
static hipError_t constitutive_et(Ctx &c, const ConstArgs &ca) {
  using T = Et<ETID>;
  constexpr int EPB = CT / T::NQ;
  KC a;
  a.coord = c.coord;
  a.elem = c.elem;
  a.ref = c.ref;
  a.n_n = c.n_n;
  a.n_e = c.n_e;
  a.n_int = c.n_int;
  a.u = ca.u;
  a.m = c.mat;
  a.ep = c.ep_s;
  a.beta = c.beta_s;
  a.kappa = c.kappa_s;
  a.flag = c.flag;
  a.desc = c.desc;
  a.Fe = c.Fe;
  a.fslot = c.fslot;
  a.emask = c.em[c.em_cur];
  a.eps_out = ca.eps_out;
  a.sig_out = ca.sig_out;
  a.D_out = ca.D_out;
  a.flag_out = ca.flag_out;
  a.rm = ca.return_map;
  a.commit = ca.commit;
  a.force = ca.force;
  a.mlp_x = ca.mlp_x;
  a.mlp_y = ca.mlp_y;
  double s_out;
  mlp_scales(c.mat, c.E, a.s_in, s_out);
  a.S = 1.0 / s_out;
  const int grid = ceil_div(c.n_e, EPB);
  if (grid == 0) return hipSuccess;
#define CONST_LAUNCH(MODEL, LM) \
  EP_LAUNCH((k_constitutive<ETID, MODEL, LM>), dim3(grid), dim3(CT), 0, c, a)
  if (c.mat.model == EP_VM) {
    if (ca.learned == 1) CONST_LAUNCH(EP_VM, 1);
    else if (ca.learned == 2) CONST_LAUNCH(EP_VM, 2);
    else CONST_LAUNCH(EP_VM, 0);
  } else {
    if (ca.learned == 1) CONST_LAUNCH(EP_DP, 1);
    else if (ca.learned == 2) CONST_LAUNCH(EP_DP, 2);
    else CONST_LAUNCH(EP_DP, 0);
  }
#undef CONST_LAUNCH
  return hipGetLastError();
}

#define DISPATCH_ET(FN, ...)                                   \
  switch (c.et) {                                              \
    case ET_P1_2D: return FN<ET_P1_2D>(__VA_ARGS__);           \
    case ET_Q1_2D: return FN<ET_Q1_2D>(__VA_ARGS__);           \
    case ET_Q2_2D: return FN<ET_Q2_2D>(__VA_ARGS__);           \
    case ET_P1_3D: return FN<ET_P1_3D>(__VA_ARGS__);           \
    case ET_P2_3D: return FN<ET_P2_3D>(__VA_ARGS__);           \
    case ET_Q1_3D: return FN<ET_Q1_3D>(__VA_ARGS__);           \
    case ET_Q2_3D: return FN<ET_Q2_3D>(__VA_ARGS__);           \
    case ET_Q2S_2D: return FN<ET_Q2S_2D>(__VA_ARGS__);         \
    case ET_Q2S_3D: return FN<ET_Q2S_3D>(__VA_ARGS__);         \
  }                                                            \
  return hipErrorInvalidValue;

hipError_t launch_constitutive(Ctx &c, const ConstArgs &a) { DISPATCH_ET(constitutive_et, c, a) }

template <int ETID>
static hipError_t geometry_et(Ctx &c, double *dphi, double *w, int32_t *bad) {
  const int64_t n = c.n_int;
  if (n == 0) return hipSuccess;
  EP_LAUNCH((k_geometry<ETID>), dim3(ceil_div(n, 128)), dim3(128), 0, c, c.coord,
            c.elem, c.ref, c.n_n, c.n_e, dphi, w, bad);
  return hipGetLastError();
}
hipError_t launch_geometry(Ctx &c, double *dphi, double *w, int32_t *bad) {
  DISPATCH_ET(geometry_et, c, dphi, w, bad)
}

hipError_t launch_force_gather(Ctx &c, const double *f, double *F_out, double *r_out,
                               double *partials, int nblk) {
  if (nblk == 0) return hipSuccess;
  if (c.dim == 2)
    EP_LAUNCH((k_force_gather<2>), dim3(nblk), dim3(256), 0, c, c.n_n,
              c.n2e_ptr, c.Fe, f, c.freem, F_out, r_out, partials);
  else
    EP_LAUNCH((k_force_gather<3>), dim3(nblk), dim3(256), 0, c, c.n_n,
              c.n2e_ptr, c.Fe, f, c.freem, F_out, r_out, partials);
  return hipGetLastError();
}

hipError_t launch_reduce(Ctx &c, const double *partials, int nblk, int width, double *out) {
  EP_LAUNCH(k_reduce, dim3(1), dim3(256), 0, c, partials, nblk, width, out);
  return hipGetLastError();
}

hipError_t launch_compact(Ctx &c, int kind, const void *src, const uint32_t *src2,
                          const int32_t *perm, int64_t n, int32_t *out,
                          int32_t *colour_first_block, int n_col, int32_t *colour_off,
                          int32_t *totals) {
  const int nblk = ceil_div(n, CMP_CHUNK);
  if (nblk > c.cmp_cap) return hipErrorInvalidValue;
#define CMP_LAUNCH(K)                                                                      \
  if (nblk > 0)                                                                            \
    EP_LAUNCH((k_compact_count<K>), dim3(nblk), dim3(CMP_THREADS), 0, c, src, src2, perm, n, \
              c.cmp_counts, c.cmp_counts2, c.cmp_counts3);                                 \
  /* at least one block: block 0 writes the totals and colour offsets */                   \
  EP_LAUNCH((k_compact_scatter<K>), dim3(nblk > 0 ? nblk : 1), dim3(CMP_THREADS), 0, c, src, \
            src2, perm, n, c.cmp_counts, c.cmp_counts2, c.cmp_counts3, nblk,                \
            colour_first_block, n_col, colour_off, totals, out)
  if (kind == 0) {
    CMP_LAUNCH(0);
  } else {
    CMP_LAUNCH(1);
  }
#undef CMP_LAUNCH
  return hipGetLastError();
}

template <int ETID>
static hipError_t elastic_et(Ctx &c) {
  using Cfg = AsmCfg<ETID>;
  for (int col = 0; col < c.n_col; ++col) {
    KA a{};
    a.coord = c.coord;
    a.elem = c.elem;
    a.ref = c.ref;
    a.n_n = c.n_n;
    a.n_int = c.n_int;
    a.list = c.ecol_perm;
    a.off = nullptr;
    a.k0 = (int64_t)c.colour_first_block[col] * CMP_CHUNK;
    a.k1 = a.k0 + c.colour_size[col];
    a.bpos = c.bpos;
    a.bposs = c.bposs;
    a.Kt = c.Ke;
    a.elastic = 1;
    a.G = c.mat.G;
    a.K = c.mat.K;
    const int64_t cnt = a.k1 - a.k0;
    if (cnt == 0) continue;
    const int grid = (int)(cnt < 65536 ? cnt : 65536);
    EP_LAUNCH((k_assemble<ETID, double>), dim3(grid), dim3(Cfg::BS), 0, c, a);
    RT(hipGetLastError());
  }
  return hipSuccess;
}
hipError_t launch_emat(Ctx &c, bool elastic, int64_t listed);
hipError_t launch_elastic_assembly(Ctx &c) {
  if (c.opt.assembly == EP_ASSEMBLY_ROWS) {
    RT(launch_emat(c, true, -1));
    return launch_row_gather(c, true, -1);
  }
  DISPATCH_ET(elastic_et, c)
}

template <int ETID>
static hipError_t colour_et(Ctx &c, int colour, int epoch, int64_t listed) {
  using Cfg = AsmCfg<ETID>;
  KA a{};
  a.coord = c.coord;
  a.elem = c.elem;
  a.ref = c.ref;
  a.n_n = c.n_n;
  a.n_int = c.n_int;
  a.desc = c.desc;
  a.emask = c.em[c.em_cur];
  a.list = c.plist;
  a.off = c.coff;
  a.colour = colour;
  a.bpos = c.bpos;
  a.bposs = c.bposs;
  a.Ke = c.Ke;
  a.Ke32 = c.Ke32;
  a.Kt = c.Kt;
  a.epoch = c.epoch;
  a.cur = epoch;
  a.elastic = 0;
  a.G = c.mat.G;
  a.K = c.mat.K;
  const int64_t cnt = listed >= 0 ? listed : c.colour_size[colour];
  if (cnt == 0) return hipSuccess;
  const int grid = (int)(cnt < 65536 ? cnt : 65536);
  // the FP64/FP32 kernel loops over elements with a software pipeline: a grid
  // of about twice the resident blocks gives each block a few elements
  const int gcap = 48 * c.n_cu;
  const int gpipe = grid < gcap ? grid : gcap;
  const bool f32 = c.opt.tangent_prec == EP_FP32;
  if constexpr (ETID == ET_Q2_3D || ETID == ET_Q2S_3D || ETID == ET_P2_3D) {
    if (c.opt.local_prec == EP_BF16 || c.opt.local_prec == EP_FP32) {
      const bool bf = c.opt.local_prec == EP_BF16;
#define MF(VT, BF) \
  EP_LAUNCH((k_assemble_mfma<ETID, VT, BF>), dim3(grid), dim3(256), 0, c, a)
      if (f32) {
        if (bf) MF(float, true); else MF(float, false);
      } else {
        if (bf) MF(double, true); else MF(double, false);
      }
#undef MF
      return hipGetLastError();
    }
  }
  if (f32)
    EP_LAUNCH((k_assemble<ETID, float>), dim3(gpipe), dim3(Cfg::BS), 0, c, a);
  else
    EP_LAUNCH((k_assemble<ETID, double>), dim3(gpipe), dim3(Cfg::BS), 0, c, a);
  return hipGetLastError();
}
hipError_t launch_colour_assembly(Ctx &c, int colour, int epoch, int64_t listed) {
  DISPATCH_ET(colour_et, c, colour, epoch, listed)
}

// Element matrices of every element of the work list with plastic points
// now (elastic: of every element, C at every point) into the element-matrix
// buffer: one launch, no colours (each element writes its own slot).
template <int ETID>
static hipError_t emat_et(Ctx &c, bool elastic, int64_t listed) {
  using Cfg = AsmCfg<ETID>;
  KA a{};
  a.coord = c.coord;
  a.elem = c.elem;
  a.ref = c.ref;
  a.n_n = c.n_n;
  a.n_int = c.n_int;
  a.desc = c.desc;
  a.G = c.mat.G;
  a.K = c.mat.K;
  a.elastic = elastic ? 1 : 0;
  a.emat64 = (double *)c.emat;
  a.emat32 = (float *)c.emat;
  a.eslot = elastic ? nullptr : c.eslot;
  int64_t cnt;
  if (elastic) {
    a.list = c.ecol_perm;
    a.off = nullptr;
    a.k0 = 0;
    a.k1 = c.n_perm;
    cnt = c.n_perm;
  } else {
    a.emask = c.em[c.em_cur];
    a.list = c.plist;
    a.off = c.coff;
    a.colour = 0;
    a.colour_end = c.n_col;
    cnt = listed >= 0 ? listed : c.n_e;
  }
  if (cnt == 0) return hipSuccess;
  const int gcap = 48 * c.n_cu;
  if constexpr (ETID == ET_Q2_3D || ETID == ET_Q2S_3D || ETID == ET_P2_3D) {
    if (!elastic && (c.opt.local_prec == EP_BF16 || c.opt.local_prec == EP_FP32)) {
      const int grid = (int)(cnt < 65536 ? cnt : 65536);
      if (c.opt.local_prec == EP_BF16)
        EP_LAUNCH((k_assemble_mfma<ETID, double, true, true>), dim3(grid), dim3(256), 0, c, a);
      else
        EP_LAUNCH((k_assemble_mfma<ETID, double, false, true>), dim3(grid), dim3(256), 0, c, a);
      return hipGetLastError();
    }
  }
  const int grid = (int)(cnt < gcap ? cnt : gcap);
  EP_LAUNCH((k_assemble<ETID, double, true>), dim3(grid), dim3(Cfg::BS), 0, c, a);
  return hipGetLastError();
}
hipError_t launch_emat(Ctx &c, bool elastic, int64_t listed) {
  DISPATCH_ET(emat_et, c, elastic, listed)
}

// Node-row gather of the element matrices into K_tangent (elastic: into
// K_elast from zero).
template <int ETID>
static hipError_t row_gather_et(Ctx &c, bool elastic, int64_t listed) {
  using R = RowCfg<ETID>;
  KR a{};
  a.n_n = c.n_n;
  a.bptr = c.bptr;
  a.n2e_ptr = c.n2e_ptr;
  a.n2e = c.n2e;
  a.bpos = c.bpos;
  a.emat = c.emat;
  a.eslot = elastic ? nullptr : c.eslot;
  a.max_slots = c.max_slots;
  if (elastic) {
    a.em_cur = nullptr;
    a.em_prev = nullptr;
    a.base = nullptr;
    a.out = c.Ke;
  } else {
    a.em_cur = c.em[c.em_cur];
    a.em_prev = c.em_asm >= 0 ? c.em[c.em_asm] : nullptr;
    a.base = c.opt.tangent_prec == EP_FP32 ? (const void *)c.Ke32 : (const void *)c.Ke;
    a.out = c.Kt;
  }
  if (c.n_n == 0) return hipSuccess;
  const int D = c.dim;
  const size_t lds = sizeof(double) * (size_t)c.max_deg * D * D + 2 * sizeof(int) * c.max_slots;
  int64_t work = c.n_n;
  if (!elastic && listed >= 0 && listed * c.n_p < c.n_n / 2) {
    // short list (its length known on the host): the listed elements' rows
    a.list = c.plist;
    a.elem = c.elem;
    a.n_list = listed;
    work = listed * c.n_p;
    if (work == 0) return hipSuccess;
  }
  const int grid = (int)(work < (1 << 20) ? work : (1 << 20));
  const bool e32 = !elastic && c.opt.local_prec != EP_FP64;  // matrix-core element matrices
  const bool v32 = !elastic && c.opt.tangent_prec == EP_FP32;
#define RG(OT, VT) \
  EP_LAUNCH((k_row_gather<ETID, OT, VT>), dim3(grid), dim3(R::BS), lds, c, a)
  if (e32) {
    if (v32) RG(float, float); else RG(float, double);
  } else {
    if (v32) RG(double, float); else RG(double, double);
  }
#undef RG
  return hipGetLastError();
}
hipError_t launch_row_gather(Ctx &c, bool elastic, int64_t listed) {
  DISPATCH_ET(row_gather_et, c, elastic, listed)
}

// Fused node-row assembly of K_tangent (FP64 element-local products).
template <int ETID>
static hipError_t row_fused_et(Ctx &c, int64_t listed) {
  using F = FusedCfg<ETID>;
  KF f{};
  KR &a = f.r;
  a.n_n = c.n_n;
  a.bptr = c.bptr;
  a.n2e_ptr = c.n2e_ptr;
  a.n2e = c.n2e;
  a.bpos = c.bpos;
  a.max_slots = c.max_slots;
  a.em_cur = c.em[c.em_cur];
  a.em_prev = c.em_asm >= 0 ? c.em[c.em_asm] : nullptr;
  a.base = c.opt.tangent_prec == EP_FP32 ? (const void *)c.Ke32 : (const void *)c.Ke;
  a.out = c.Kt;
  a.elem = c.elem;
  f.coord = c.coord;
  f.ref = c.ref;
  f.desc = c.desc;
  f.n_int = c.n_int;
  if (c.n_n == 0) return hipSuccess;
  if (c.max_slots > F::BS) return hipErrorInvalidValue;  // refused at setup
  int64_t work = c.n_n;
  if (listed >= 0 && listed * c.n_p < c.n_n / 2) {
    a.list = c.plist;
    a.n_list = listed;
    work = listed * c.n_p;
    if (work == 0) return hipSuccess;
  }
  const int grid = (int)(work < (1 << 20) ? work : (1 << 20));
  const size_t lds = F::lds(c.max_slots, c.max_deg);
  if (c.opt.tangent_prec == EP_FP32)
    EP_LAUNCH((k_row_fused<ETID, float>), dim3(grid), dim3(F::BS), lds, c, f);
  else
    EP_LAUNCH((k_row_fused<ETID, double>), dim3(grid), dim3(F::BS), lds, c, f);
  return hipGetLastError();
}
hipError_t launch_row_fused(Ctx &c, int64_t listed) {
  DISPATCH_ET(row_fused_et, c, listed)
}
size_t row_fused_lds(const Ctx &c) {
  switch (c.et) {
    case ET_P1_2D: return FusedCfg<ET_P1_2D>::lds(c.max_slots, c.max_deg);
    case ET_Q1_2D: return FusedCfg<ET_Q1_2D>::lds(c.max_slots, c.max_deg);
    case ET_Q2_2D: return FusedCfg<ET_Q2_2D>::lds(c.max_slots, c.max_deg);
    case ET_P1_3D: return FusedCfg<ET_P1_3D>::lds(c.max_slots, c.max_deg);
    case ET_P2_3D: return FusedCfg<ET_P2_3D>::lds(c.max_slots, c.max_deg);
    case ET_Q1_3D: return FusedCfg<ET_Q1_3D>::lds(c.max_slots, c.max_deg);
    case ET_Q2_3D: return FusedCfg<ET_Q2_3D>::lds(c.max_slots, c.max_deg);
    case ET_Q2S_2D: return FusedCfg<ET_Q2S_2D>::lds(c.max_slots, c.max_deg);
    case ET_Q2S_3D: return FusedCfg<ET_Q2S_3D>::lds(c.max_slots, c.max_deg);
  }
  return (size_t)-1;
}

hipError_t launch_copy_ke_to_kt(Ctx &c) {
  const int64_t n = c.nnzb * c.dim * c.dim;
  if (c.opt.tangent_prec == EP_FP32)
    return hipMemcpyAsync(c.Kt, c.Ke32, n * sizeof(float), hipMemcpyDeviceToDevice, c.stream);
  return hipMemcpyAsync(c.Kt, c.Ke, n * sizeof(double), hipMemcpyDeviceToDevice, c.stream);
}

hipError_t launch_to_float(const double *src, float *dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_float, dim3(ceil_div(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_csr_expand(Ctx &c, int which, int32_t *row_ptr, int32_t *col_idx,
                             double *val) {
  const int64_t n = c.n_dof + 1;
  const int grid = ceil_div(n, 256);
  const bool f32 = which == 1 && c.opt.tangent_prec == EP_FP32;
  const void *v = which == 1 ? c.Kt : (const void *)c.Ke;
#define CSRX(D, VT)                                                                          \
  EP_LAUNCH((k_csr_expand<D, VT>), dim3(grid), dim3(256), 0, c, c.n_n, c.nnzb, \
            c.bptr, c.bcol, (const VT *)v, row_ptr, col_idx, val)
  if (c.dim == 2) {
    if (f32) CSRX(2, float); else CSRX(2, double);
  } else {
    if (f32) CSRX(3, float); else CSRX(3, double);
  }
#undef CSRX
  return hipGetLastError();
}

template <int ETID>
static hipError_t pos_et(Ctx &c, int32_t *pos) {
  using T = Et<ETID>;
  const int64_t n = c.n_e * T::NP * T::NP;
  if (n == 0) return hipSuccess;
  EP_LAUNCH((k_pos_expand<ETID>), dim3(ceil_div(n, 256)), dim3(256), 0, c, c.n_e,
            c.elem, c.bptr, c.bpos, pos);
  return hipGetLastError();
}
hipError_t launch_pos_expand(Ctx &c, int32_t *pos) { DISPATCH_ET(pos_et, c, pos) }

template <int ETID>
static hipError_t split_apply_et(Ctx &c, int mode, const double *x, const double *sc) {
  constexpr int EPB = CT / Et<ETID>::NQ;
  KS a{};
  a.coord = c.coord;
  a.elem = c.elem;
  a.ref = c.ref;
  a.n_n = c.n_n;
  a.n_int = c.n_int;
  a.desc = c.desc;
  a.emask = c.em[c.em_cur];
  a.list = c.plist;
  a.list_n = c.coff + c.n_col;
  a.fslot = c.fslot;
  a.x = x;
  a.Fp = c.Fp;
  a.sc = sc;
  a.G = c.mat.G;
  a.K = c.mat.K;
  // one block per EPB list entries; blocks past the list length (known on
  // the device only) return at once
  const int grid = ceil_div(c.n_e, EPB);
  if (grid == 0) return hipSuccess;
  if (mode == 0)
    EP_LAUNCH((k_split_apply<ETID, 0>), dim3(grid), dim3(CT), 0, c, a);
  else
    EP_LAUNCH((k_split_apply<ETID, 1>), dim3(grid), dim3(CT), 0, c, a);
  return hipGetLastError();
}
hipError_t launch_split_apply(Ctx &c, int mode, const double *x, const double *sc) {
  DISPATCH_ET(split_apply_et, c, mode, x, sc)
}

hipError_t launch_split_gather(Ctx &c, int mode, double *y, const double *p, double *partials,
                               const double *sc, int *nblk) {
  const int grid = ceil_div(c.n_n, 256);
  *nblk = grid;
  if (grid == 0) return hipSuccess;
#define SG(D, M)                                                                             \
  EP_LAUNCH((k_split_gather<D, M>), dim3(grid), dim3(256), 0, c, c.n_n,      \
            c.n2e_ptr, c.slot_elem, c.em[c.em_cur], c.Fp, c.freem, y, p, partials, \
            sc, c.bdiag, c.Ke, c.dinv)
  if (c.dim == 2) {
    if (mode == 0) SG(2, 0); else SG(2, 1);
  } else {
    if (mode == 0) SG(3, 0); else SG(3, 1);
  }
#undef SG
  return hipGetLastError();
}

hipError_t launch_diag_inv(Ctx &c) {
  if (c.opt.operator_form == EP_OPERATOR_SPLIT) {
    int nblk = 0;
    RT(launch_split_apply(c, 1, nullptr, nullptr));
    return launch_split_gather(c, 1, nullptr, nullptr, nullptr, nullptr, &nblk);
  }
  const int grid = ceil_div(c.n_dof, 256);
  const bool f32 = c.opt.tangent_prec == EP_FP32;
#define DG(D, VT)                                                                               \
  EP_LAUNCH((k_diag_inv<D, VT>), dim3(grid), dim3(256), 0, c, c.n_n, c.bdiag, \
            (const VT *)c.Kt, c.freem, c.dinv)
  if (c.dim == 2) {
    if (f32) DG(2, float); else DG(2, double);
  } else {
    if (f32) DG(3, float); else DG(3, double);
  }
#undef DG
  return hipGetLastError();
}

// lanes per node row, from the mean row length
static int spmv_lanes(const Ctx &c) {
  const double deg = c.n_n > 0 ? (double)c.nnzb / (double)c.n_n : 1.0;
  return deg <= 12 ? 4 : (deg <= 24 ? 8 : (deg <= 48 ? 16 : 32));
}

template <int D, typename VT>
static hipError_t spmv_launch(Ctx &c, const void *vals, const double *x, double *y,
                              double *partials, const double *sc, int *nblk,
                              bool masked = true) {
  const int G = spmv_lanes(c);
  const int grid = ceil_div(c.n_n * G, 256);
  *nblk = grid;
  if (grid == 0) return hipSuccess;
#define SPG(GG)                                                                              \
  EP_LAUNCH((k_spmv<D, VT, GG>), dim3(grid), dim3(256), 0, c, c.n_n, c.bptr, \
            c.bcol, (const VT *)vals, x, masked ? c.freem : nullptr, y, partials, sc, x + 1, \
            x + 2)
  switch (G) {
    case 4: SPG(4); break;
    case 8: SPG(8); break;
    case 16: SPG(16); break;
    default: SPG(32); break;
  }
#undef SPG
  return hipGetLastError();
}

// values: the assembled tangent, or K_elast for the split form (stored in
// the tangent's precision)
static hipError_t spmv_any(Ctx &c, bool elastic, const double *x, double *y, double *partials,
                           const double *sc, int *nblk) {
  const bool f32 = c.opt.tangent_prec == EP_FP32;
  const void *vals = !elastic ? c.Kt : (f32 ? (const void *)c.Ke32 : (const void *)c.Ke);
  if (c.dim == 2)
    return f32 ? spmv_launch<2, float>(c, vals, x, y, partials, sc, nblk)
               : spmv_launch<2, double>(c, vals, x, y, partials, sc, nblk);
  return f32 ? spmv_launch<3, float>(c, vals, x, y, partials, sc, nblk)
             : spmv_launch<3, double>(c, vals, x, y, partials, sc, nblk);
}

hipError_t launch_spmv(Ctx &c, const double *x, double *y) {
  int nblk = 0;
  return spmv_any(c, false, x, y, nullptr, nullptr, &nblk);
}

hipError_t launch_apply_split(Ctx &c, const double *x, double *y) {
  int nblk = 0;
  RT(spmv_any(c, true, x, y, nullptr, nullptr, &nblk));
  RT(launch_split_apply(c, 0, x, nullptr));
  return launch_split_gather(c, 0, y, nullptr, nullptr, nullptr, &nblk);
}

hipError_t launch_pcg_init(Ctx &c, const double *b, double *x) {
  const int grid = ceil_div(c.n_dof, 256);
  c.pcur = 0;
  EP_LAUNCH(k_pcg_init, dim3(grid), dim3(256), 0, c, c.n_dof, b, c.freem, x, c.r,
            c.pz, c.pp[0], c.dinv, c.partials);
  RT(hipGetLastError());
  return hipSuccess;
}

hipError_t launch_pcg_beta_init(Ctx &c, double rtol);

hipError_t launch_pcg_iteration(Ctx &c, double *x) {
  const int grid = ceil_div(c.n_dof, 256);
  double *pold = c.pp[c.pcur], *pnew = c.pp[1 - c.pcur];
  int nblk = 0;
  const bool split = c.opt.operator_form == EP_OPERATOR_SPLIT;
  {
    ProfScope ps(c, PROF_SPMV);
    // p = z + beta p_old as a vector pass, so that the product gathers one
    // vector (beta = 0 at the first iteration)
    EP_LAUNCH(k_pcg_direction, dim3(grid), dim3(256), 0, c, c.n_dof, c.pz, pold,
              pnew, c.sc);
    RT(hipGetLastError());
    RT(spmv_any(c, split, pnew, c.pq, split ? nullptr : c.partials, c.sc, &nblk));
  }
  if (split) {
    // q = Q K_elast p + Q sum_e Delta K_e p_e, then the partial p.q
    ProfScope ps(c, PROF_SPLIT);
    RT(launch_split_apply(c, 0, pnew, c.sc));
    RT(launch_split_gather(c, 0, c.pq, pnew, c.partials, c.sc, &nblk));
  }
  EP_LAUNCH(k_pcg_alpha, dim3(1), dim3(256), 0, c, c.partials, nblk, c.sc);
  RT(hipGetLastError());
  {
    ProfScope ps(c, PROF_PCGVEC);
    EP_LAUNCH(k_pcg_update, dim3(grid), dim3(256), 0, c, c.n_dof, x, pnew, c.r,
              c.pq, c.pz, c.dinv, c.sc, c.partials);
    RT(hipGetLastError());
  }
  EP_LAUNCH(k_pcg_beta, dim3(1), dim3(256), 0, c, c.partials, grid, c.sc, 0, 0.0);
  RT(hipGetLastError());
  c.pcur = 1 - c.pcur;
  return hipSuccess;
}

hipError_t launch_pcg_small(Ctx &c, double *x, int n_it) {
  ProfScope ps(c, PROF_PCGSMALL);
  if (ps.tok >= 0) c.pending[ps.tok].count = n_it;
  double *p = c.pp[c.pcur];
#define PS(DIM, VT)                                                                           \
  EP_LAUNCH((k_pcg_small<DIM, VT>), dim3(1), dim3(PCGS_T), 0, c, n_it, c.n_n, c.bptr, c.bcol, \
            (const VT *)c.Kt, c.freem, c.dinv, x, c.r, c.pz, p, c.pq, c.sc)
  const bool f32 = c.opt.tangent_prec == EP_FP32;
  if (c.dim == 2) {
    if (f32) PS(2, float); else PS(2, double);
  } else {
    if (f32) PS(3, float); else PS(3, double);
  }
#undef PS
  return hipGetLastError();
}

// Two-kernel PCG iteration: scalars sc -> sc2 (k_pcg_spmv2) -> sc
// (k_pcg_update2), partials partials2 -> partials -> partials2.
template <int D, typename VT>
static hipError_t pcg_spmv2_launch(Ctx &c, const double *pold, double *pnew, int nin,
                                   int *nblk) {
  const int G = spmv_lanes(c);
  const int grid = ceil_div(c.n_n * G, 256);
  *nblk = grid;
#define SP2(GG)                                                                               \
  EP_LAUNCH((k_pcg_spmv2<D, VT, GG>), dim3(grid), dim3(256), 0, c, c.n_n, c.bptr, c.bcol,   \
            (const VT *)c.Kt, c.pz, pold, pnew, c.freem, c.pq, c.partials2, nin, c.sc, c.sc2, \
            c.partials)
  switch (G) {
    case 4: SP2(4); break;
    case 8: SP2(8); break;
    case 16: SP2(16); break;
    default: SP2(32); break;
  }
#undef SP2
  return hipGetLastError();
}

hipError_t launch_pcg_iteration2(Ctx &c, double *x) {
  const int grid = ceil_div(c.n_dof, 256);
  double *pold = c.pp[c.pcur], *pnew = c.pp[1 - c.pcur];
  int nblk = 0;
  {
    ProfScope ps(c, PROF_SPMV);
    const bool f32 = c.opt.tangent_prec == EP_FP32;
    hipError_t e;
    if (c.dim == 2)
      e = f32 ? pcg_spmv2_launch<2, float>(c, pold, pnew, grid, &nblk)
              : pcg_spmv2_launch<2, double>(c, pold, pnew, grid, &nblk);
    else
      e = f32 ? pcg_spmv2_launch<3, float>(c, pold, pnew, grid, &nblk)
              : pcg_spmv2_launch<3, double>(c, pold, pnew, grid, &nblk);
    RT(e);
  }
  {
    ProfScope ps(c, PROF_PCGVEC);
    EP_LAUNCH(k_pcg_update2, dim3(grid), dim3(256), 0, c, c.n_dof, x, pnew, c.r, c.pq, c.pz,
              c.dinv, c.partials, nblk, c.sc2, c.sc, c.partials2);
    RT(hipGetLastError());
  }
  c.pcur = 1 - c.pcur;
  return hipSuccess;
}

hipError_t launch_pcg_finish2(Ctx &c) {
  const int grid = ceil_div(c.n_dof, 256);
  EP_LAUNCH(k_pcg_finish2, dim3(1), dim3(256), 0, c, c.partials2, grid, c.sc);
  return hipGetLastError();
}

hipError_t launch_pcg_beta_init(Ctx &c, double rtol) {
  const int grid = ceil_div(c.n_dof, 256);
  EP_LAUNCH(k_pcg_beta, dim3(1), dim3(256), 0, c, c.partials, grid, c.sc, 1, rtol);
  return hipGetLastError();
}

hipError_t launch_axpy_free(Ctx &c, const double *du, double *u, double a) {
  if (c.n_dof == 0) return hipSuccess;
  EP_LAUNCH(k_axpy_free, dim3(ceil_div(c.n_dof, 256)), dim3(256), 0, c, c.n_dof,
            du, c.freem, a, u);
  return hipGetLastError();
}

hipError_t launch_trial(Ctx &c, const double *u, const double *du, double a, double *out) {
  if (c.n_dof == 0) return hipSuccess;
  EP_LAUNCH(k_trial, dim3(ceil_div(c.n_dof, 256)), dim3(256), 0, c, c.n_dof, u, du, a,
            c.freem, out);
  return hipGetLastError();
}

hipError_t launch_spmv_elastic_full(Ctx &c, const double *x, double *y) {
  int nblk = 0;
  if (c.dim == 2) return spmv_launch<2, double>(c, c.Ke, x, y, nullptr, nullptr, &nblk, false);
  return spmv_launch<3, double>(c, c.Ke, x, y, nullptr, nullptr, &nblk, false);
}

hipError_t launch_dots(Ctx &c, int n_pairs, const double *const *x, const double *const *y,
                       double *out) {
  if (n_pairs < 1 || n_pairs > 4) return hipErrorInvalidValue;
  DotPairs p{};
  for (int k = 0; k < n_pairs; ++k) {
    p.x[k] = x[k];
    p.y[k] = y[k];
  }
  const int grid = std::max(1, ceil_div(c.n_dof, 256));
  if ((int64_t)grid * n_pairs > c.partials_cap) return hipErrorInvalidValue;
#define DT(NP_)                                                                          \
  EP_LAUNCH((k_dots<NP_>), dim3(grid), dim3(256), 0, c, c.n_dof, p, c.partials)
  switch (n_pairs) {
    case 1: DT(1); break;
    case 2: DT(2); break;
    case 3: DT(3); break;
    default: DT(4); break;
  }
#undef DT
  RT(hipGetLastError());
  return launch_reduce(c, c.partials, grid, n_pairs, out);
}

hipError_t launch_extrapolate(Ctx &c, const double *u, const double *u2, double t, double *out) {
  if (c.n_dof == 0) return hipSuccess;
  EP_LAUNCH(k_extrapolate, dim3(ceil_div(c.n_dof, 256)), dim3(256), 0, c, c.n_dof,
            u, u2, t, c.freem, out);
  return hipGetLastError();
}

}  // namespace ep
