// Internal declarations shared by the host part of the library and its
// HIP kernels.  Not part of the C ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ep.h"

namespace ep {

// Element kinds the kernels are specialised on.
enum EtId { ET_P1_2D = 0, ET_Q1_2D, ET_Q2_2D, ET_P1_3D, ET_P2_3D, ET_Q1_3D, ET_Q2_3D, ET_Q2S_2D,
            ET_Q2S_3D, ET_COUNT };

template <int ID> struct Et;
template <> struct Et<ET_P1_2D> { static constexpr int D = 2, NP = 3, NQ = 1; };
template <> struct Et<ET_Q1_2D> { static constexpr int D = 2, NP = 4, NQ = 4; };
template <> struct Et<ET_Q2_2D> { static constexpr int D = 2, NP = 9, NQ = 9; };
template <> struct Et<ET_P1_3D> { static constexpr int D = 3, NP = 4, NQ = 1; };
template <> struct Et<ET_P2_3D> { static constexpr int D = 3, NP = 10, NQ = 11; };
template <> struct Et<ET_Q1_3D> { static constexpr int D = 3, NP = 8, NQ = 8; };
template <> struct Et<ET_Q2_3D> { static constexpr int D = 3, NP = 27, NQ = 27; };
template <> struct Et<ET_Q2S_2D> { static constexpr int D = 2, NP = 8, NQ = 9; };
template <> struct Et<ET_Q2S_3D> { static constexpr int D = 3, NP = 20, NQ = 27; };

// Material constants used on the device.
struct MatC {
  int model;       // EP_VM / EP_DP
  double G, K, a, Y, eta, c;
};

// Items per block of the compaction kernels (256 threads x 8 items).
constexpr int CMP_THREADS = 256;
constexpr int CMP_ITEMS = 8;
constexpr int CMP_CHUNK = CMP_THREADS * CMP_ITEMS;
// most element colours a mesh may need (the compaction keeps a count per
// colour in LDS)
constexpr int CMP_MAX_COLOURS = 512;
// colour-round assembly: work lists of at most this many (element, node,
// point) triples (listed elements x n_p x n_q) go through the fused row pass
constexpr int64_t SHORT_LIST_WORK = 4096;
// colour-round assembly: longer work lists of at most this many elements,
// and element-matrix entries, per compute unit go through the element
// matrices and the node-row gather
constexpr int64_t ROW_ROUTE_PER_CU = 16;
constexpr int64_t ROW_ROUTE_ENTRIES_PER_CU = 24576;

// PCG scalars on the device (sc[SC_N]); SC_BREAK = 1 when PCG stopped on
// p.q <= 0 or a non-finite scalar; SC_NEED = 1 when the two-kernel iteration
// has left its beta step to the next kernel.
enum { SC_RZ = 0, SC_PQ, SC_RR, SC_TOL, SC_DONE, SC_ITS, SC_ALPHA, SC_BETA, SC_RR0, SC_BREAK,
       SC_NEED, SC_N };

// Kernel ids for ep_profile.
enum ProfId { PROF_CONST = 0, PROF_COMPACT, PROF_SPLIT, PROF_ASSEMBLE, PROF_FORCE, PROF_SPMV,
              PROF_PCGVEC, PROF_ELASTIC, PROF_PCGSMALL, PROF_COUNT };
// PCG of systems of at most this many dofs runs in one workgroup (a launch
// per chunk of iterations instead of five per iteration)
constexpr int64_t SMALL_PCG_DOFS = 12288;
// up to this many dofs (assembled operator) a PCG iteration is two kernels:
// each repeats the single-block scalar step of the one before it
constexpr int64_t MEDIUM_PCG_DOFS = 131072;

struct Ctx;

// ---- launch wrappers (ep_kernels.hip) ----
struct ConstArgs {
  const double *u;       // [n_dof] or nullptr (= zero displacement)
  double *eps_out;       // [n_str][n_int] or nullptr
  bool return_map;       // false: strain only
  double *sig_out;       // [n_sc][n_int] or nullptr
  double *D_out;         // [n_str^2][n_int] or nullptr
  uint8_t *flag_out;     // [n_int] or nullptr (internal flag always written)
  bool commit;           // write the updated state
  bool force;            // element force vectors + plastic mask
  // learned warm start: 1 = write MLP features to mlp_x instead of the
  // return map; 2 = take the plastic flag and stress from the MLP outputs
  // mlp_y (tangent of the trial state on the predicted branch)
  int learned = 0;
  float *mlp_x = nullptr;       // [n_int][EP_MLP_XS]
  const float *mlp_y = nullptr; // [n_int][EP_MLP_YS]
};
hipError_t launch_constitutive(Ctx &c, const ConstArgs &a);
hipError_t launch_geometry(Ctx &c, double *dphi, double *w, int32_t *bad_count);
hipError_t launch_force_gather(Ctx &c, const double *f, double *F_out, double *r_out,
                               double *partials, int nblk);
hipError_t launch_reduce(Ctx &c, const double *partials, int nblk, int width, double *out);
// Stable compaction of items i < n (through perm when given, -1 = padding)
// with predicate (src[item] | src2[item]) != 0; kind 0: uint8 src, kind 1:
// uint32 src (src2 optional, uint32).  totals[0] = selected items,
// totals[1] = set bits of src, totals[2] = items with src != 0.
hipError_t launch_compact(Ctx &c, int kind, const void *src, const uint32_t *src2,
                          const int32_t *perm, int64_t n, int32_t *out,
                          int32_t *colour_first_block, int n_col, int32_t *colour_off,
                          int32_t *totals);
hipError_t launch_elastic_assembly(Ctx &c);
// listed: the colour's work-list length when the host knows it (-1: not
// known; the grid then covers the colour)
hipError_t launch_colour_assembly(Ctx &c, int colour, int epoch, int64_t listed);
hipError_t launch_copy_ke_to_kt(Ctx &c);
hipError_t launch_to_float(const double *src, float *dst, int64_t n, hipStream_t s);
hipError_t launch_csr_expand(Ctx &c, int which, int32_t *row_ptr, int32_t *col_idx, double *val);
hipError_t launch_pos_expand(Ctx &c, int32_t *pos);
// element matrices of the listed elements with plastic points now (elastic:
// of every element) into c.emat; listed = work-list length if known (< 0:
// unknown)
hipError_t launch_emat(Ctx &c, bool elastic, int64_t listed);
// node-row gather of c.emat into K_tangent (elastic: into K_elast); listed:
// work-list length if known on the host (< 0: unknown)
hipError_t launch_row_gather(Ctx &c, bool elastic, int64_t listed);
hipError_t launch_row_fused(Ctx &c, int64_t listed);
hipError_t launch_pcg_small(Ctx &c, double *x, int n_it);
hipError_t launch_pcg_iteration2(Ctx &c, double *x);
hipError_t launch_pcg_finish2(Ctx &c);
size_t row_fused_lds(const Ctx &c);  // dynamic LDS of the fused row pass
hipError_t launch_diag_inv(Ctx &c);
hipError_t launch_spmv(Ctx &c, const double *x, double *y);
// split form of the tangent: y = Q K_elast x + Q sum over plastic elements of
// Delta K_e x_e (element by element, no assembly)
hipError_t launch_apply_split(Ctx &c, const double *x, double *y);
hipError_t launch_pcg_init(Ctx &c, const double *b, double *x);
hipError_t launch_pcg_iteration(Ctx &c, double *x);
// u += a du on free dofs
hipError_t launch_axpy_free(Ctx &c, const double *du, double *u, double a = 1.0);
// out = u + a du on free dofs, u on Dirichlet dofs
hipError_t launch_trial(Ctx &c, const double *u, const double *du, double a, double *out);
// y = K_elast x (FP64 values, every row: no Dirichlet mask)
hipError_t launch_spmv_elastic_full(Ctx &c, const double *x, double *y);
// out[k] = x_k . y_k for the n_pairs (<= 4) pairs, fixed-order sums
hipError_t launch_dots(Ctx &c, int n_pairs, const double *const *x, const double *const *y,
                       double *out);
// u_out = u + t (u - u2) on free dofs, u on Dirichlet dofs (u2 == nullptr: copy)
hipError_t launch_extrapolate(Ctx &c, const double *u, const double *u2, double t, double *u_out);

// ---- MLP (ep_mlp.hip) ----
struct MlpImpl {
  std::string err;
  int prec = EP_FP32;
  int64_t max_batch = 0;
  hipStream_t stream = nullptr;
  float *params = nullptr, *m1 = nullptr, *m2 = nullptr;
  float *part = nullptr, *part_loss = nullptr;  // per-tile partial gradients
  int64_t step = 0;                             // Adam steps taken
};
hipError_t launch_mlp_forward(const MlpImpl &m, const float *X, int64_t n, float *Y,
                              hipStream_t s);
hipError_t launch_mlp_train(MlpImpl &m, const float *X, const float *T, int64_t n, float *grad,
                            float *loss, bool adam, float lr, float bc1, float bc2);
hipError_t launch_mlp_datagen(const MatC &mat, int64_t n, const int64_t *idx, int64_t n_pool,
                              const double *eps_pool, const double *ep_pool,
                              const double *beta_pool, const double *kappa_pool,
                              const double *deps, float *X, float *T, double s_in, double s_out,
                              hipStream_t s);
int64_t mlp_tile_samples();
// loss gradient of a batch (and, with adam_params, one Adam step on them)
// with the per-tile partials in part[n_tiles][EP_MLP_NPARAM] and
// part_loss[n_tiles] (n_tiles = ceil(n / 32))
hipError_t mlp_grad(int prec, const float *params, float *part, float *part_loss, hipStream_t s,
                    const float *X, const float *T, int64_t n, float *grad, float *loss,
                    float *adam_params, float *m1, float *m2, float lr, float bc1, float bc2);
// feature / output scales of a material: s_in = E/S, s_out = 1/S
void mlp_scales(const MatC &m, double E, double &s_in, double &s_out);
// material checks shared by ep_setup and the sample generator (ep_host.cpp)
const char *material_error(const ep_material *mat);  // nullptr if valid
MatC make_matc(const ep_material &mat);

// ---- context ----
struct Ctx {
  std::string err;
  hipStream_t stream = nullptr;
  int dev = 0;
  int n_cu = 256;          // compute units of the device

  // sizes
  int et = 0;            // EtId
  int dim = 0, n_p = 0, n_q = 0, n_str = 0, n_sc = 0, n_desc = 0;
  int64_t n_n = 0, n_e = 0, n_int = 0, n_dof = 0, nnzb = 0;
  int n_col = 0;
  MatC mat{};
  ep_options opt{};

  // mesh (device)
  double *coord = nullptr;     // [dim][n_n]
  int32_t *elem = nullptr;     // [n_e][n_p]
  uint8_t *freem = nullptr;    // [n_dof]
  double *ref = nullptr;       // [n_q][n_p][dim] reference gradients, then [n_q] weights

  // node-block CSR of K (device)
  int32_t *bptr = nullptr;     // [n_n+1]
  int32_t *bcol = nullptr;     // [nnzb]
  int32_t *bdiag = nullptr;    // [n_n] block index of (m, m)
  int32_t *bpos = nullptr;     // [n_e][n_p][n_p] block index of (node p, node p')
  // the same with the columns in ascending global node order (quadrilaterals
  // and 8-node hexahedra: the sorted scatter), else unused
  int32_t *bposs = nullptr;
  double *Ke = nullptr;        // [nnzb][dim][dim]
  float *Ke32 = nullptr;
  void *Kt = nullptr;          // double or float, [nnzb][dim][dim]
  uint8_t *epoch = nullptr;    // [nnzb] assembly stamp of each block (1..255, 0 = none)
  int epoch_counter = 0;

  // element force vectors are stored node by node: the entries of node m
  // (one per incident element, ascending element) are n2e_ptr[m] ..
  // n2e_ptr[m+1]-1, and element e's local node p writes entry fslot[e*n_p+p]
  int32_t *n2e_ptr = nullptr;  // [n_n+1]
  int32_t *n2e = nullptr;      // [n_e*n_p] slot -> e * n_p + p
  bool fused_ok = false;       // the fused row pass fits (FP64 products, slots, LDS)
  // element matrices [slot][n_p][n_p][dim][dim] (double, or float for
  // matrix-core local products) of the row-gather assembly: emat_cap slots
  // (rows mode: n_e; colour mode: the work lists it routes to the gather);
  // a tangent assembly stores element e at its work-list position,
  // eslot[e] (K_elast, rows mode only: at slot e)
  void *emat = nullptr;
  int64_t emat_cap = 0;
  int32_t *eslot = nullptr;    // [n_e]
  int max_deg = 0, max_slots = 0;  // largest node row (blocks) and node-to-element count
  int32_t *fslot = nullptr;    // [n_e*n_p]

  // colouring
  std::vector<int64_t> colour_size;        // host
  std::vector<int32_t> colour_first_block; // host, per colour + end
  int32_t *ecol_perm = nullptr;            // [n_perm] colour-major, padded with -1
  int64_t n_perm = 0;
  int32_t *d_colour_first_block = nullptr; // [n_col+1]

  // state and per-iteration data (device)
  double *ep_s = nullptr;      // [n_sc][n_int]
  double *beta_s = nullptr;    // [n_sc][n_int]
  double *kappa_s = nullptr;   // [n_int]
  uint8_t *flag = nullptr;     // [n_int]
  double *desc = nullptr;      // [n_desc][n_int]
  double *Fe = nullptr;        // [n_e*n_p][dim], in node order (fslot)
  // plastic-point bitmask per element, two buffers: the one written by the
  // last constitutive pass and the one the last assembly used
  uint32_t *em[2] = {nullptr, nullptr};   // [n_e] each
  int em_cur = 0;
  int em_asm = -1;                        // -1: no assembly yet
  bool have_const = false;

  // work list of the assembly (colour-major): elements plastic now or at
  // the last assembly; coff[c] .. coff[c+1] is colour c's segment
  int32_t *plist = nullptr;
  std::vector<int32_t> coff_h;  // host copy of the colour offsets of the work list
  bool coff_known = false;     // coff_h matches the device offsets
  int32_t *coff = nullptr;                 // [n_col+1]
  int32_t *ptotals = nullptr;              // [8]: list length, plastic points,
                                           // plastic elements, scratch
  int32_t *iscratch = nullptr;  // [max(n_int, n_e)] ascending plastic lists

  // compaction scratch
  int32_t *cmp_counts = nullptr, *cmp_counts2 = nullptr, *cmp_counts3 = nullptr;
  int64_t cmp_cap = 0;  // blocks

  // vectors
  double *F = nullptr, *r = nullptr;
  // split form: element vectors of the plastic part (node-ordered slots) and
  // the element of each slot
  double *Fp = nullptr;
  int32_t *slot_elem = nullptr;
  double *partials = nullptr;  // reduction scratch
  double *partials2 = nullptr, *sc2 = nullptr;  // two-kernel PCG iteration
  int64_t partials_cap = 0;
  double *norms = nullptr;     // [8] device
  double *norms_h = nullptr;   // pinned host [8]

  // energy norms of a Newton correction: K_elast u, K_elast dx; line search:
  // trial displacement and the Newton residual kept through PCG (allocated
  // at the first damped step)
  double *ky[2] = {nullptr, nullptr};
  double *ut = nullptr, *rn = nullptr;

  // PCG
  double *pz = nullptr, *pp[2] = {nullptr, nullptr}, *pq = nullptr, *px = nullptr,
         *dinv = nullptr, *sc = nullptr, *sc_h = nullptr;
  int pcur = 0;

  // PCG iterations replayed as a HIP graph: captured on gstream (a stream of
  // the context, default priority) for a chunk of pcg_graph_n iterations
  // updating pcg_graph_x
  hipStream_t gstream = nullptr;
  hipGraphExec_t pcg_graph = nullptr;
  const double *pcg_graph_x = nullptr;
  int pcg_graph_n = 0;
  int pcg_graph_em = -1;

  // learned warm start (allocated at first use)
  float *mlp_x = nullptr, *mlp_y = nullptr;  // [n_int][16], [n_int][8]
  double *wu_pred = nullptr, *wu_warm = nullptr;  // [n_dof]
  double E = 0.0;

  // profiling: a profiled section hands its two events to the kernel
  // launches inside it (EP_LAUNCH); the first launch records the start
  // time, every launch the stop time
  uint32_t prof_mask = 0;  // bit k: time kernel id k
  struct Pending { int id; hipEvent_t a, b; int count; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  hipEvent_t launch_start = nullptr, launch_stop = nullptr;
  double prof_ms[PROF_COUNT] = {0};
  int64_t prof_n[PROF_COUNT] = {0};
  int prof_begin(int id);
  void prof_end(int token);
  void prof_collect();
  hipEvent_t take_start() {
    hipEvent_t e = launch_start;
    launch_start = nullptr;
    return e;
  }
};

// A profiled section that ends with its scope, also on an early error
// return (no later launch then carries the section's events).
struct ProfScope {
  Ctx &c;
  const int tok;
  ProfScope(Ctx &ctx, int id) : c(ctx), tok(ctx.prof_begin(id)) {}
  ~ProfScope() { c.prof_end(tok); }
  ProfScope(const ProfScope &) = delete;
  ProfScope &operator=(const ProfScope &) = delete;
};

// Kernel launch on the context's stream (hipLaunchKernelGGL's arguments with
// the context in place of the stream).  Inside a profiled section the
// section's events travel with the dispatch itself, so timing adds no marker
// command between kernels.
#define EP_LAUNCH(K, G, B, SHM, C, ...)                                                   \
  hipExtLaunchKernelGGL(K, G, B, SHM, (C).stream, (C).take_start(), (C).launch_stop, 0, \
                        __VA_ARGS__)

}  // namespace ep
