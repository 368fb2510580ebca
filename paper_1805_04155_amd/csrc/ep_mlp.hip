// Per-point MLP of the learned Newton warm start: training-sample generator
// (exact return map), fused forward / loss / backward tiles on the matrix
// cores, deterministic gradient reduction and Adam.
//
// Network 13 -> 128 -> 128 -> 7 with ReLU; parameters in one FP32 array
// W1[128][13] b1 W2[128][128] b2 W3[7][128] b3.  A block takes 32 samples:
// the activations of all three layers stay in LDS, each wavefront computes
// 16x16 output tiles with v_mfma_f32_16x16x4f32 (FP32 operands) or
// v_mfma_f32_16x16x32_bf16 (operands rounded to BF16), FP32 accumulation.
// Weight gradients of a block go to a partial buffer, summed afterwards in
// block order (no atomics), so a gradient is bitwise reproducible.
#include <cmath>
#include <mutex>
#include <string>

#include "ep_internal.h"
#include "ep_return_map.h"

namespace ep {

namespace {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

constexpr int NI = EP_MLP_IN, NH = EP_MLP_HID, NO = EP_MLP_OUT;
constexpr int XS = EP_MLP_XS, YS = EP_MLP_YS, NPAR = EP_MLP_NPARAM;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NO * NH;
static_assert(OFF_B3 + NO == NPAR, "parameter layout");

constexpr int TB = 32;    // samples per block (LDS stays under 64 KB)
constexpr int LA = 132;   // LDS row stride of 128-wide activations
constexpr int LX = 17;    // LDS row stride of inputs (16 used)
constexpr int LY = 17;    // LDS row stride of outputs / output gradients

// One 16x16 tile C(m, n) = sum_{k < KP} A(m, k) B(n, k), with
//   A(m, k) = A[m*am + k*ak] for k < ka, else 0,
//   B(n, k) = B[n*bn + k*bk] for k < kb and n < nb, else 0.
// Lane l supplies A(l%16, k-group l/16) and B(l%16, k-group l/16) and
// receives C(4(l/16) + i, l%16) in element i.
template <bool BF16>
__device__ inline f32x4_t mma16(const float *A, int am, int ak, int ka, const float *B, int bn,
                                int bk, int kb, int nb, int KP, int lane) {
  const int r = lane & 15, g = lane >> 4;
  const bool nok = r < nb;
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  if constexpr (!BF16) {
    for (int k0 = 0; k0 < KP; k0 += 4) {
      const int k = k0 + g;
      const float av = k < ka ? A[r * am + k * ak] : 0.f;
      const float bv = (nok && k < kb) ? B[r * bn + k * bk] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < KP; k0 += 32) {
      bf16x8_t av, bv;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + 8 * g + j;
        av[j] = (__bf16)(k < ka ? A[r * am + k * ak] : 0.f);
        bv[j] = (__bf16)((nok && k < kb) ? B[r * bn + k * bk] : 0.f);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
  }
  return acc;
}

struct MlpArgs {
  const float *params;
  const float *X;   // [n][XS]
  const float *T;   // [n][YS] targets (training)
  float *Y;         // [n][YS] outputs (inference)
  float *part;      // [n_blocks][NPAR] partial gradients
  float *part_loss; // [n_blocks]
  int64_t n;
  float inv_n;
};

template <bool BF16, bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp_tile(MlpArgs a) {
  __shared__ float sX[TB * LX];
  __shared__ float sH1[TB * LA];
  __shared__ float sH2[TB * LA];  // H2, then dH1
  __shared__ float sG[TB * LA];   // dH2
  __shared__ float sY[TB * LY];   // outputs, then dL/dY
  __shared__ float sL[TB];
  constexpr int K1 = BF16 ? 32 : 16, K3 = BF16 ? 32 : 8;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int64_t s0 = (int64_t)blockIdx.x * TB;
  const int nv = (int)(a.n - s0 < TB ? a.n - s0 : TB);
  const float *P = a.params;
  for (int t = tid; t < TB * 16; t += 256) {
    const int s = t >> 4, i = t & 15;
    sX[s * LX + i] = (s < nv && i < NI) ? a.X[(s0 + s) * XS + i] : 0.f;
  }
  __syncthreads();
  // layer 1: H1 = relu(X W1^T + b1), 2 x 8 tiles
  for (int t = wv; t < 16; t += 4) {
    const int tm = t >> 3, tn = t & 7;
    const f32x4_t c = mma16<BF16>(sX + 16 * tm * LX, LX, 1, NI, P + OFF_W1 + 16 * tn * NI, NI, 1,
                                  NI, 16, K1, lane);
    const int n = 16 * tn + r16;
    const float b = P[OFF_B1 + n];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * tm + 4 * g4 + i;
      const float h = c[i] + b;
      sH1[m * LA + n] = (m < nv && h > 0.f) ? h : 0.f;
    }
  }
  __syncthreads();
  // layer 2: H2 = relu(H1 W2^T + b2)
  for (int t = wv; t < 16; t += 4) {
    const int tm = t >> 3, tn = t & 7;
    const f32x4_t c = mma16<BF16>(sH1 + 16 * tm * LA, LA, 1, NH, P + OFF_W2 + 16 * tn * NH, NH, 1,
                                  NH, 16, NH, lane);
    const int n = 16 * tn + r16;
    const float b = P[OFF_B2 + n];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * tm + 4 * g4 + i;
      const float h = c[i] + b;
      sH2[m * LA + n] = (m < nv && h > 0.f) ? h : 0.f;
    }
  }
  __syncthreads();
  // layer 3: Y = H2 W3^T + b3, one tile per wavefront 0, 1
  if (wv < TB / 16) {
    const int tm = wv;
    const f32x4_t c = mma16<BF16>(sH2 + 16 * tm * LA, LA, 1, NH, P + OFF_W3, NH, 1, NH, NO, NH,
                                  lane);
    const int n = r16;
    const float b = n < NO ? P[OFF_B3 + n] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * tm + 4 * g4 + i;
      sY[m * LY + n] = n < NO ? c[i] + b : 0.f;
    }
  }
  __syncthreads();
  if constexpr (!TRAIN) {
    for (int t = tid; t < TB * YS; t += 256) {
      const int s = t / YS, j = t - (t / YS) * YS;
      if (s < nv) a.Y[(s0 + s) * YS + j] = j < NO ? sY[s * LY + j] : 0.f;
    }
    return;
  } else {
    // loss and dL/dY (rows past the batch end are zero)
    if (tid < TB) {
      const int s = tid;
      float l = 0.f;
      float *y = sY + s * LY;
      if (s < nv) {
        const float *t = a.T + (s0 + s) * YS;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          const float d = y[j] - t[j];
          l += d * d * (1.0f / 6.0f);
          y[j] = d * (2.0f / 6.0f) * a.inv_n;
        }
        const float z = y[6], f = t[6];
        l += fmaxf(z, 0.f) - f * z + log1pf(expf(-fabsf(z)));
        const float sg = 1.0f / (1.0f + expf(-z));
        y[6] = (sg - f) * a.inv_n;
      } else {
#pragma unroll
        for (int j = 0; j < NO; ++j) y[j] = 0.f;
      }
      sL[s] = l;
    }
    __syncthreads();
    float *part = a.part + (int64_t)blockIdx.x * NPAR;
    if (tid == 0) {
      float l = 0.f;
      for (int s = 0; s < TB; ++s) l += sL[s];
      a.part_loss[blockIdx.x] = l;
    }
    // dW3[o][i] = sum_s dY[s][o] H2[s][i]   (o < 7: one tile row)
    for (int tn = wv; tn < 8; tn += 4) {
      const f32x4_t c = mma16<BF16>(sY, 1, LY, TB, sH2 + 16 * tn, 1, LA, TB, 16, TB, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = 4 * g4 + i;
        if (o < NO) part[OFF_W3 + o * NH + 16 * tn + r16] = c[i];
      }
    }
    if (tid < NO) {
      float s = 0.f;
      for (int k = 0; k < TB; ++k) s += sY[k * LY + tid];
      part[OFF_B3 + tid] = s;
    }
    // dH2 = (dY W3) .* (H2 > 0)
    for (int t = wv; t < 16; t += 4) {
      const int tm = t >> 3, tn = t & 7;
      const f32x4_t c = mma16<BF16>(sY + 16 * tm * LY, LY, 1, NO, P + OFF_W3 + 16 * tn, 1, NH, NO,
                                    16, K3, lane);
      const int n = 16 * tn + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 16 * tm + 4 * g4 + i;
        sG[m * LA + n] = sH2[m * LA + n] > 0.f ? c[i] : 0.f;
      }
    }
    __syncthreads();
    // dW2[o][i] = sum_s dH2[s][o] H1[s][i]
    for (int t = wv; t < 64; t += 4) {
      const int tm = t >> 3, tn = t & 7;
      const f32x4_t c = mma16<BF16>(sG + 16 * tm, 1, LA, TB, sH1 + 16 * tn, 1, LA, TB, 16, TB, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        part[OFF_W2 + (16 * tm + 4 * g4 + i) * NH + 16 * tn + r16] = c[i];
    }
    if (tid < NH) {
      float s = 0.f;
      for (int k = 0; k < TB; ++k) s += sG[k * LA + tid];
      part[OFF_B2 + tid] = s;
    }
    // dH1 = (dH2 W2) .* (H1 > 0), into the H2 buffer (H2 is no longer read)
    for (int t = wv; t < 16; t += 4) {
      const int tm = t >> 3, tn = t & 7;
      const f32x4_t c = mma16<BF16>(sG + 16 * tm * LA, LA, 1, NH, P + OFF_W2 + 16 * tn, 1, NH, NH,
                                    16, NH, lane);
      const int n = 16 * tn + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 16 * tm + 4 * g4 + i;
        sH2[m * LA + n] = sH1[m * LA + n] > 0.f ? c[i] : 0.f;
      }
    }
    __syncthreads();
    // dW1[o][i] = sum_s dH1[s][o] X[s][i]   (i < 13: one tile column)
    for (int tm = wv; tm < 8; tm += 4) {
      const f32x4_t c = mma16<BF16>(sH2 + 16 * tm, 1, LA, TB, sX, 1, LX, TB, NI, TB, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (r16 < NI) part[OFF_W1 + (16 * tm + 4 * g4 + i) * NI + r16] = c[i];
    }
    if (tid < NH) {
      float s = 0.f;
      for (int k = 0; k < TB; ++k) s += sH2[k * LA + tid];
      part[OFF_B1 + tid] = s;
    }
  }
}

// grad = sum of the block partials in a fixed order (4 interleaved partial
// sums per parameter, combined in LDS); optionally one Adam step (bias
// corrections bc1 = 1 - beta1^t, bc2 = 1 - beta2^t from the host).
constexpr int RED_P = 64;  // parameters per block of the reduction
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *part, const float *part_loss,
                                                     int nblk, float inv_n, float *grad,
                                                     float *loss, float *params, float *m1,
                                                     float *m2, float lr, float bc1, float bc2,
                                                     int adam) {
  __shared__ float s[4][RED_P];
  const int lane = threadIdx.x & (RED_P - 1), grp = threadIdx.x / RED_P;
  const int p = blockIdx.x * RED_P + lane;
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
    float l = 0.f;
    for (int b = 0; b < nblk; ++b) l += part_loss[b];
    loss[0] = l * inv_n;
  }
  float g = 0.f;
  if (p < NPAR)
    for (int b = grp; b < nblk; b += 4) g += part[(int64_t)b * NPAR + p];
  s[grp][lane] = g;
  __syncthreads();
  if (grp != 0 || p >= NPAR) return;
  g = (s[0][lane] + s[1][lane]) + (s[2][lane] + s[3][lane]);
  if (grad) grad[p] = g;
  if (adam) {
    const float a1 = 0.9f * m1[p] + 0.1f * g;
    const float a2 = 0.999f * m2[p] + 0.001f * g * g;
    m1[p] = a1;
    m2[p] = a2;
    params[p] -= lr * (a1 / bc1) / (sqrtf(a2 / bc2) + 1e-8f);
  }
}

// Training samples: exact return map at pooled states plus an increment.
__global__ __launch_bounds__(256) void k_mlp_datagen(MatC m, int64_t n, const int64_t *idx,
                                                      int64_t n_pool, const double *eps_pool,
                                                      const double *ep_pool,
                                                      const double *beta_pool,
                                                      const double *kappa_pool,
                                                      const double *deps, float *X, float *T,
                                                      double s_in, double s_out) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const int64_t i = idx[j];
  float *x = X + j * XS, *t = T + j * YS;
  if (i < 0 || i >= n_pool) {
    for (int c = 0; c < XS; ++c) x[c] = 0.f;
    for (int c = 0; c < YS; ++c) t[c] = 0.f;
    return;
  }
  double eps[6], ep[6], bt[6], sig[6], desc[10];
  double kap = kappa_pool ? kappa_pool[i] : 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    eps[c] = eps_pool[c * n_pool + i] + deps[c * n + j];
    ep[c] = ep_pool[c * n_pool + i];
    bt[c] = beta_pool ? beta_pool[c * n_pool + i] : m.a * ep[c] * (c < 3 ? 1.0 : 0.5);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    x[c] = (float)(s_in * (eps[c] - ep[c]));
    x[6 + c] = (float)(s_in * ep[c]);
  }
  x[12] = (float)(s_in * kap);
  x[13] = x[14] = x[15] = 0.f;
  const int f = m.model == EP_VM ? rm_vm(m, eps, ep, bt, sig, desc, false)
                                 : rm_dp(m, eps, ep, kap, sig, desc, false);
  // target: the plastic correction sigma - sigma_tr (zero at elastic points)
  double dv[6], tr;
  trial(m, eps, ep, dv, tr);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const double str = 2.0 * m.G * dv[c] + (c < 3 ? m.K * tr : 0.0);
    t[c] = (float)(s_out * (sig[c] - str));
  }
  t[6] = f ? 1.f : 0.f;
  t[7] = 0.f;
}

inline int blocks_of(int64_t n, int64_t b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t launch_mlp_forward(const MlpImpl &m, const float *X, int64_t n, float *Y,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  MlpArgs a{};
  a.params = m.params;
  a.X = X;
  a.Y = Y;
  a.n = n;
  if (m.prec == EP_BF16)
    hipLaunchKernelGGL((k_mlp_tile<true, false>), dim3(blocks_of(n, TB)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_mlp_tile<false, false>), dim3(blocks_of(n, TB)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Loss gradient (and optionally one Adam step) of a batch with the
// per-tile partials in part[n_tiles][NPAR] and part_loss[n_tiles]
hipError_t mlp_grad(int prec, const float *params, float *part, float *part_loss,
                           hipStream_t s, const float *X, const float *T, int64_t n, float *grad,
                           float *loss, float *adam_params, float *m1, float *m2, float lr,
                           float bc1, float bc2) {
  MlpArgs a{};
  a.params = params;
  a.X = X;
  a.T = T;
  a.part = part;
  a.part_loss = part_loss;
  a.n = n;
  a.inv_n = 1.0f / (float)n;
  const int nblk = blocks_of(n, TB);
  if (prec == EP_BF16)
    hipLaunchKernelGGL((k_mlp_tile<true, true>), dim3(nblk), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_mlp_tile<false, true>), dim3(nblk), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks_of(NPAR, RED_P)), dim3(256), 0, s, part,
                     part_loss, nblk, a.inv_n, grad, loss, adam_params, m1, m2, lr, bc1, bc2,
                     adam_params ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_mlp_train(MlpImpl &m, const float *X, const float *T, int64_t n, float *grad,
                            float *loss, bool adam, float lr, float bc1, float bc2) {
  return mlp_grad(m.prec, m.params, m.part, m.part_loss, m.stream, X, T, n, grad, loss,
                  adam ? m.params : nullptr, m.m1, m.m2, lr, bc1, bc2);
}

hipError_t launch_mlp_datagen(const MatC &mat, int64_t n, const int64_t *idx, int64_t n_pool,
                              const double *eps_pool, const double *ep_pool,
                              const double *beta_pool, const double *kappa_pool,
                              const double *deps, float *X, float *T, double s_in, double s_out,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_datagen, dim3(blocks_of(n, 256)), dim3(256), 0, s, mat, n, idx, n_pool,
                     eps_pool, ep_pool, beta_pool, kappa_pool, deps, X, T, s_in, s_out);
  return hipGetLastError();
}

int64_t mlp_tile_samples() { return TB; }

}  // namespace ep

// ---------------------------------------------------------------------------
// Device scratch of ep_mlp_loss_grad_noalloc: per-tile partial gradients
// [EP_MLP_NOALLOC_MAX_BATCH / 32][NPAR] followed by the per-tile losses.  One
// copy per device, alive until the process ends; host code uses only the
// address hipGetSymbolAddress returns for the current device (the symbol
// itself is a host-side stand-in).
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t NOALLOC_TILES = EP_MLP_NOALLOC_MAX_BATCH / 32;
static_assert(EP_MLP_NOALLOC_MAX_BATCH % 32 == 0, "whole tiles of 32 samples");
__device__ __align__(256) float scratch[NOALLOC_TILES * (EP_MLP_NPARAM + 1)];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[MAX_DEVICES] = {};
thread_local std::string g_noalloc_err;

// address of this device's scratch (looked up once per device, with the
// device current)
hipError_t scratch_address(int dev, float **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<float *>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI of the network (include/ep.h)
// ---------------------------------------------------------------------------
using ep::MlpImpl;

namespace {
ep_status mlp_fail(MlpImpl *m, const char *what, hipError_t e) {
  m->err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? EP_ENOMEM : EP_EDEVICE;
}
#define MLPC(m, x)                                      \
  do {                                                  \
    hipError_t e__ = (x);                               \
    if (e__ != hipSuccess) return mlp_fail(m, #x, e__); \
  } while (0)
}  // namespace

extern "C" {

ep_status ep_mlp_create(int32_t prec, int64_t max_batch, void *hip_stream, ep_mlp **out) {
  if (!out || (prec != EP_FP32 && prec != EP_BF16) || max_batch < 1) return EP_EINVAL;
  *out = nullptr;
  MlpImpl *m = new MlpImpl();
  m->prec = prec;
  m->max_batch = max_batch;
  m->stream = (hipStream_t)hip_stream;
  const int64_t nblk = (max_batch + ep::mlp_tile_samples() - 1) / ep::mlp_tile_samples();
  hipError_t e = hipSuccess;
  for (float **p : {&m->params, &m->m1, &m->m2})
    if (e == hipSuccess) e = hipMalloc(p, EP_MLP_NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->part, nblk * EP_MLP_NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->part_loss, nblk * sizeof(float));
  for (float *p : {m->params, m->m1, m->m2})
    if (e == hipSuccess) e = hipMemsetAsync(p, 0, EP_MLP_NPARAM * sizeof(float), m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    ep_mlp_destroy(reinterpret_cast<ep_mlp *>(m));
    return e == hipErrorOutOfMemory ? EP_ENOMEM : EP_EDEVICE;
  }
  *out = reinterpret_cast<ep_mlp *>(m);
  return EP_OK;
}

void ep_mlp_destroy(ep_mlp *mlp) {
  if (!mlp) return;
  MlpImpl *m = reinterpret_cast<MlpImpl *>(mlp);
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  else (void)hipDeviceSynchronize();
  for (float *p : {m->params, m->m1, m->m2, m->part, m->part_loss})
    if (p) (void)hipFree(p);
  delete m;
}

const char *ep_mlp_last_error(const ep_mlp *mlp) {
  return mlp ? reinterpret_cast<const MlpImpl *>(mlp)->err.c_str() : "NULL network";
}

ep_status ep_mlp_set_params(ep_mlp *mlp, const float *params) {
  if (!mlp || !params) return EP_EINVAL;
  MlpImpl *m = reinterpret_cast<MlpImpl *>(mlp);
  MLPC(m, hipMemcpyAsync(m->params, params, EP_MLP_NPARAM * sizeof(float),
                         hipMemcpyDeviceToDevice, m->stream));
  MLPC(m, hipMemsetAsync(m->m1, 0, EP_MLP_NPARAM * sizeof(float), m->stream));
  MLPC(m, hipMemsetAsync(m->m2, 0, EP_MLP_NPARAM * sizeof(float), m->stream));
  m->step = 0;
  return EP_OK;
}

ep_status ep_mlp_get_params(ep_mlp *mlp, float *params) {
  if (!mlp || !params) return EP_EINVAL;
  MlpImpl *m = reinterpret_cast<MlpImpl *>(mlp);
  MLPC(m, hipMemcpyAsync(params, m->params, EP_MLP_NPARAM * sizeof(float),
                         hipMemcpyDeviceToDevice, m->stream));
  return EP_OK;
}

ep_status ep_mlp_forward(ep_mlp *mlp, const float *X, int64_t n, float *Y) {
  if (!mlp || n < 0 || (n > 0 && (!X || !Y))) return EP_EINVAL;
  MlpImpl *m = reinterpret_cast<MlpImpl *>(mlp);
  MLPC(m, ep::launch_mlp_forward(*m, X, n, Y, m->stream));
  return EP_OK;
}

ep_status ep_mlp_loss_grad(ep_mlp *mlp, const float *X, const float *T, int64_t n, float *grad,
                           float *loss) {
  if (!mlp || !X || !T) return EP_EINVAL;
  MlpImpl *m = reinterpret_cast<MlpImpl *>(mlp);
  if (n < 1 || n > m->max_batch) {
    m->err = "ep_mlp_loss_grad: need 1 <= n <= max_batch";
    return EP_EINVAL;
  }
  MLPC(m, ep::launch_mlp_train(*m, X, T, n, grad, loss, false, 0.f, 1.f, 1.f));
  return EP_OK;
}

ep_status ep_mlp_adam_step(ep_mlp *mlp, const float *X, const float *T, int64_t n, float lr,
                           float *loss) {
  if (!mlp || !X || !T || !(lr >= 0.f)) return EP_EINVAL;
  MlpImpl *m = reinterpret_cast<MlpImpl *>(mlp);
  if (n < 1 || n > m->max_batch) {
    m->err = "ep_mlp_adam_step: need 1 <= n <= max_batch";
    return EP_EINVAL;
  }
  m->step += 1;
  const float bc1 = (float)(1.0 - std::pow(0.9, (double)m->step));
  const float bc2 = (float)(1.0 - std::pow(0.999, (double)m->step));
  MLPC(m, ep::launch_mlp_train(*m, X, T, n, nullptr, loss, true, lr, bc1, bc2));
  return EP_OK;
}

ep_status ep_mlp_loss_grad_noalloc(int32_t prec, const float *params, const float *X,
                                   const float *T, int64_t n, float *grad, float *loss,
                                   void *hip_stream) {
  auto fail = [](const std::string &m, ep_status st) {
    g_noalloc_err = m;
    return st;
  };
  if (prec != EP_FP32 && prec != EP_BF16)
    return fail("ep_mlp_loss_grad_noalloc: prec must be EP_FP32 or EP_BF16", EP_EINVAL);
  if (!params || !X || !T)
    return fail("ep_mlp_loss_grad_noalloc: NULL params, X or T", EP_EINVAL);
  if (n < 1 || n > EP_MLP_NOALLOC_MAX_BATCH)
    return fail("ep_mlp_loss_grad_noalloc: need 1 <= n <= EP_MLP_NOALLOC_MAX_BATCH (" +
                    std::to_string(EP_MLP_NOALLOC_MAX_BATCH) + "), got " + std::to_string(n),
                EP_EINVAL);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
    return fail(std::string("ep_mlp_loss_grad_noalloc: no usable current device: ") +
                    hipGetErrorString(e), EP_EDEVICE);
  float *scr = nullptr;
  e = scratch_address(dev, &scr);
  if (e != hipSuccess)
    return fail(std::string("ep_mlp_loss_grad_noalloc: hipGetSymbolAddress: ") +
                    hipGetErrorString(e), EP_EDEVICE);
  // every tile writes all of its partials: nothing needs clearing
  e = ep::mlp_grad(prec, params, scr, scr + NOALLOC_TILES * EP_MLP_NPARAM,
                   (hipStream_t)hip_stream, X, T, n, grad, loss, nullptr, nullptr, nullptr, 0.f,
                   1.f, 1.f);
  if (e != hipSuccess)
    return fail(std::string("ep_mlp_loss_grad_noalloc: launch: ") + hipGetErrorString(e),
                EP_EDEVICE);
  return EP_OK;
}

const char *ep_mlp_noalloc_last_error(void) { return g_noalloc_err.c_str(); }

ep_status ep_mlp_datagen(const ep_material *material, int64_t n, const int64_t *idx,
                         int64_t n_pool, const double *eps_pool, const double *ep_pool,
                         const double *beta_pool, const double *kappa_pool, const double *deps,
                         float *X, float *T, void *hip_stream) {
  if (!material || n < 0 || n_pool < 1 || ep::material_error(material)) return EP_EINVAL;
  if (n > 0 && (!idx || !eps_pool || !ep_pool || !deps || !X || !T)) return EP_EINVAL;
  const ep::MatC mc = ep::make_matc(*material);
  double s_in, s_out;
  ep::mlp_scales(mc, material->E, s_in, s_out);
  const hipError_t e = ep::launch_mlp_datagen(mc, n, idx, n_pool, eps_pool, ep_pool, beta_pool,
                                              kappa_pool, deps, X, T, s_in, s_out,
                                              (hipStream_t)hip_stream);
  return e == hipSuccess ? EP_OK : EP_EDEVICE;
}

}  // extern "C"
