// Host part of the MI355X elastoplastic hot-path library: reference tables,
// sparsity structures, element colouring, device memory, and the C ABI of
// include/ep.h.
//
// Method: Cermak, Sysala, Valdman (arXiv 1805.04155).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "ep_internal.h"
#include "ep_mesh_graph.h"

using namespace ep;

namespace ep {
hipError_t launch_pcg_beta_init(Ctx &c, double rtol);

const char *material_error(const ep_material *mat) {
  if (!(mat->E > 0) || !(mat->nu >= 0 && mat->nu < 0.5)) return "need E > 0 and 0 <= nu < 0.5";
  if (mat->model == EP_VM) {
    if (!(mat->Y > 0) || !(mat->a >= 0)) return "von Mises needs Y > 0, a >= 0";
  } else if (mat->model == EP_DP) {
    if (!(mat->eta > 0) || !(mat->c > 0) || !(mat->a >= 0))
      return "Drucker-Prager needs eta > 0, c > 0, a >= 0";
  } else {
    return "unknown model";
  }
  return nullptr;
}

// shear and bulk moduli from E and nu (Section 2.1)
MatC make_matc(const ep_material &mat) {
  MatC m{};
  m.model = mat.model;
  m.G = mat.E / (2.0 * (1.0 + mat.nu));
  m.K = mat.E / (3.0 * (1.0 - 2.0 * mat.nu));
  m.a = mat.a;
  m.Y = mat.Y;
  m.eta = mat.eta;
  m.c = mat.c;
  return m;
}

void mlp_scales(const MatC &m, double E, double &s_in, double &s_out) {
  const double S = m.model == EP_VM ? std::sqrt(1.5) * m.Y : m.c;
  s_in = E / S;
  s_out = 1.0 / S;
}
}  // namespace ep

namespace {

thread_local std::string g_setup_err;

#define HIPC(x)                                                               \
  do {                                                                        \
    hipError_t e__ = (x);                                                     \
    if (e__ != hipSuccess) {                                                  \
      c->err = std::string(#x) + " failed: " + hipGetErrorString(e__);       \
      return EP_EDEVICE;                                                      \
    }                                                                         \
  } while (0)

#define CHECK_CTX(c)                        \
  do {                                      \
    if (!(c)) return EP_EINVAL;             \
  } while (0)

// ---------------------------------------------------------------------------
// Reference elements (Appendix) and quadrature
// ---------------------------------------------------------------------------
struct ElemDef {
  int id, dim, n_p, n_q;
};

bool elem_def(int dim, int type, ElemDef &d) {
  if (dim == 2 && type == EP_P1) d = {ET_P1_2D, 2, 3, 1};
  else if (dim == 2 && type == EP_Q1) d = {ET_Q1_2D, 2, 4, 4};
  else if (dim == 2 && type == EP_Q2) d = {ET_Q2_2D, 2, 9, 9};
  else if (dim == 3 && type == EP_P1) d = {ET_P1_3D, 3, 4, 1};
  else if (dim == 3 && type == EP_P2) d = {ET_P2_3D, 3, 10, 11};
  else if (dim == 3 && type == EP_Q1) d = {ET_Q1_3D, 3, 8, 8};
  else if (dim == 3 && type == EP_Q2) d = {ET_Q2_3D, 3, 27, 27};
  else if (dim == 2 && type == EP_Q2S) d = {ET_Q2S_2D, 2, 8, 9};
  else if (dim == 3 && type == EP_Q2S) d = {ET_Q2S_3D, 3, 20, 27};
  else return false;
  return true;
}

// Local coordinates of tensor-product nodes: value in {-1, 0, 1} per axis.
const int kQuad4[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
const int kQuad9[9][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}, {0, -1},
                          {1, 0},   {0, 1},  {-1, 0}, {0, 0}};
const int kHex27[27][3] = {
    {-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {1, 1, 1},
    {-1, 1, 1},   {0, -1, -1}, {1, 0, -1}, {0, 1, -1},  {-1, 0, -1}, {0, -1, 1}, {1, 0, 1},
    {0, 1, 1},    {-1, 0, 1},  {-1, -1, 0}, {1, -1, 0}, {1, 1, 0},   {-1, 1, 0}, {0, 0, -1},
    {0, 0, 1},    {0, -1, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0},  {0, 0, 0}};
// P2 tetrahedron edges (paper's nodes 5..10)
const int kTetEdge[6][2] = {{0, 1}, {1, 2}, {0, 2}, {1, 3}, {2, 3}, {0, 3}};

// 1D Lagrange basis and derivative: linear on {-1, 1}, quadratic on {-1, 0, 1}.
void lag1d(int order, int node, double t, double &v, double &dv) {
  if (order == 1) {
    v = 0.5 * (1.0 + node * t);
    dv = 0.5 * node;
    return;
  }
  switch (node) {
    case -1: v = 0.5 * t * (t - 1.0); dv = t - 0.5; break;
    case 0: v = (1.0 - t) * (1.0 + t); dv = -2.0 * t; break;
    default: v = 0.5 * t * (t + 1.0); dv = t + 0.5; break;
  }
}

// Reference gradients g[p*dim + i] = d phi_p / d xi_i at xi.
void ref_gradients(int id, const double *xi, double *g) {
  switch (id) {
    case ET_P1_2D: {
      const double G[6] = {-1, -1, 1, 0, 0, 1};
      std::copy(G, G + 6, g);
      return;
    }
    case ET_P1_3D: {
      const double G[12] = {-1, -1, -1, 1, 0, 0, 0, 1, 0, 0, 0, 1};
      std::copy(G, G + 12, g);
      return;
    }
    case ET_P2_3D: {
      const double lam[4] = {1.0 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]};
      const double dl[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
      for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) g[3 * k + i] = (4.0 * lam[k] - 1.0) * dl[k][i];
      for (int k = 0; k < 6; ++k) {
        const int a = kTetEdge[k][0], b = kTetEdge[k][1];
        for (int i = 0; i < 3; ++i) g[3 * (4 + k) + i] = 4.0 * (dl[a][i] * lam[b] + lam[a] * dl[b][i]);
      }
      return;
    }
    case ET_Q2S_2D:
    case ET_Q2S_3D: {
      // Serendipity element (Appendix): an edge-midpoint function is the
      // quadratic bubble 1 - t^2 along its edge times the linear factors
      // (1 + s x) of the other axes; a vertex function is the multilinear
      // vertex function minus half of the three (2D: two) edge functions
      // of the edges meeting at the vertex.
      const int dim = id == ET_Q2S_2D ? 2 : 3;
      const int n_p = dim == 2 ? 8 : 20, n_v = dim == 2 ? 4 : 8;
      auto node = [&](int p, int a) {
        return dim == 2 ? kQuad9[p][a] : kHex27[p][a];
      };
      // value and gradient of the edge function of node p
      auto edge = [&](int p, double &v, double *dv) {
        double f[3], df[3];
        for (int a = 0; a < dim; ++a) {
          const int s = node(p, a);
          if (s == 0) { f[a] = 1.0 - xi[a] * xi[a]; df[a] = -2.0 * xi[a]; }
          else { f[a] = 0.5 * (1.0 + s * xi[a]); df[a] = 0.5 * s; }
        }
        v = 1.0;
        for (int a = 0; a < dim; ++a) v *= f[a];
        for (int i = 0; i < dim; ++i) {
          double t = df[i];
          for (int a = 0; a < dim; ++a)
            if (a != i) t *= f[a];
          dv[i] = t;
        }
      };
      for (int p = n_v; p < n_p; ++p) {
        double v, dv[3];
        edge(p, v, dv);
        for (int i = 0; i < dim; ++i) g[p * dim + i] = dv[i];
      }
      for (int p = 0; p < n_v; ++p) {
        double f[3], df[3];
        for (int a = 0; a < dim; ++a) {
          f[a] = 0.5 * (1.0 + node(p, a) * xi[a]);
          df[a] = 0.5 * node(p, a);
        }
        for (int i = 0; i < dim; ++i) {
          double t = df[i];
          for (int a = 0; a < dim; ++a)
            if (a != i) t *= f[a];
          g[p * dim + i] = t;
        }
        // edges at vertex p: the midpoints that differ from it in one axis
        for (int q = n_v; q < n_p; ++q) {
          int diff = 0;
          for (int a = 0; a < dim; ++a) diff += node(q, a) != node(p, a) ? 1 : 0;
          if (diff != 1) continue;
          double v, dv[3];
          edge(q, v, dv);
          for (int i = 0; i < dim; ++i) g[p * dim + i] -= 0.5 * dv[i];
        }
      }
      return;
    }
    default: break;
  }
  // tensor-product elements
  int dim, n_p, order;
  const int *nodes;
  if (id == ET_Q1_2D) { dim = 2; n_p = 4; order = 1; nodes = &kQuad4[0][0]; }
  else if (id == ET_Q2_2D) { dim = 2; n_p = 9; order = 2; nodes = &kQuad9[0][0]; }
  else if (id == ET_Q1_3D) { dim = 3; n_p = 8; order = 1; nodes = &kHex27[0][0]; }
  else { dim = 3; n_p = 27; order = 2; nodes = &kHex27[0][0]; }
  for (int p = 0; p < n_p; ++p) {
    double v[3], dv[3];
    for (int a = 0; a < dim; ++a) lag1d(order, nodes[p * dim + a], xi[a], v[a], dv[a]);
    for (int i = 0; i < dim; ++i) {
      double s = 1.0;
      for (int a = 0; a < dim; ++a) s *= (a == i) ? dv[a] : v[a];
      g[p * dim + i] = s;
    }
  }
}

void builtin_rule(int id, int dim, std::vector<double> &xi, std::vector<double> &w) {
  xi.clear();
  w.clear();
  if (id == ET_P1_2D) { xi = {1.0 / 3, 1.0 / 3}; w = {0.5}; return; }
  if (id == ET_P1_3D) { xi = {0.25, 0.25, 0.25}; w = {1.0 / 6}; return; }
  if (id == ET_P2_3D) {
    // Keast's 11-point rule (degree 4) with the exact values of the table
    const double a = 1.0 / 14, b = 11.0 / 14, s = std::sqrt(5.0 / 14);
    const double c = 0.25 * (1 + s), d = 0.25 * (1 - s);
    xi = {0.25, 0.25, 0.25, a, a, a, b, a, a, a, b, a, a, a, b,
          c, d, d, d, c, d, d, d, c, c, c, d, c, d, c, d, c, c};
    w = {-74.0 / 5625};
    for (int k = 0; k < 4; ++k) w.push_back(343.0 / 45000);
    for (int k = 0; k < 6; ++k) w.push_back(56.0 / 2250);
    return;
  }
  const bool two = (id == ET_Q1_2D || id == ET_Q1_3D);
  std::vector<double> x1, w1;
  if (two) { x1 = {-1 / std::sqrt(3.0), 1 / std::sqrt(3.0)}; w1 = {1, 1}; }
  else { x1 = {-std::sqrt(0.6), 0.0, std::sqrt(0.6)}; w1 = {5.0 / 9, 8.0 / 9, 5.0 / 9}; }
  const int m = (int)x1.size();
  const int nz = dim == 3 ? m : 1;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        xi.push_back(x1[i]);
        xi.push_back(x1[j]);
        if (dim == 3) xi.push_back(x1[k]);
        w.push_back(w1[i] * w1[j] * (dim == 3 ? w1[k] : 1.0));
      }
}


template <class T>
hipError_t dalloc(T **p, int64_t n) {
  *p = nullptr;
  if (n <= 0) n = 1;
  return hipMalloc((void **)p, sizeof(T) * (size_t)n);
}

template <class T>
hipError_t upload(T *d, const std::vector<T> &h, hipStream_t s) {
  if (h.empty()) return hipSuccess;
  return hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s);
}

void free_ctx(Ctx *c) {
  if (!c) return;
  void *ptrs[] = {c->coord, c->elem, c->freem, c->ref, c->bptr, c->bcol, c->bdiag, c->bpos,
                  c->Ke, c->Ke32, c->Kt, c->epoch, c->bposs, c->n2e_ptr, c->n2e, c->emat, c->eslot, c->fslot, c->slot_elem, c->Fp, c->ecol_perm,
                  c->d_colour_first_block, c->ep_s, c->beta_s, c->kappa_s, c->flag, c->desc,
                  c->Fe, c->em[0], c->em[1], c->plist, c->coff, c->ptotals, c->cmp_counts,
                  c->cmp_counts2, c->cmp_counts3, c->F, c->r, c->partials,
                  c->norms, c->pz, c->pp[0], c->pp[1], c->pq, c->px, c->dinv, c->sc,
                  c->iscratch, c->mlp_x, c->mlp_y, c->wu_pred, c->wu_warm, c->ky[0],
                  c->ky[1], c->ut, c->rn, c->partials2, c->sc2};
  if (c->pcg_graph) (void)hipGraphExecDestroy(c->pcg_graph);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (c->norms_h) (void)hipHostFree(c->norms_h);
  if (c->sc_h) (void)hipHostFree(c->sc_h);
  for (auto &pd : c->pending) {
    (void)hipEventDestroy(pd.a);
    (void)hipEventDestroy(pd.b);
  }
  for (auto ev : c->event_pool) (void)hipEventDestroy(ev);
  delete c;
}

}  // namespace

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
int Ctx::prof_begin(int id) {
  if (!((prof_mask >> id) & 1u)) return -1;
  hipEvent_t a, b;
  if (event_pool.size() >= 2) {
    a = event_pool.back();
    event_pool.pop_back();
    b = event_pool.back();
    event_pool.pop_back();
  } else {
    // no system-scope fence: the times are read after a stream
    // synchronisation, which makes every result visible anyway
    if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess) return -1;
    if (hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
      (void)hipEventDestroy(a);
      return -1;
    }
  }
  pending.push_back({id, a, b, 1});
  launch_start = a;
  launch_stop = b;
  return (int)pending.size() - 1;
}

void Ctx::prof_end(int token) {
  if (token < 0) return;
  if (launch_start) {
    // no kernel was launched in the section: nothing to time
    event_pool.push_back(pending[token].a);
    event_pool.push_back(pending[token].b);
    pending.erase(pending.begin() + token);
  }
  launch_start = launch_stop = nullptr;
}

void Ctx::prof_collect() {
  if (pending.empty()) return;
  (void)hipStreamSynchronize(stream);
  for (auto &pd : pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pd.a, pd.b) == hipSuccess) {
      prof_ms[pd.id] += ms;
      prof_n[pd.id] += pd.count;
    }
    event_pool.push_back(pd.a);
    event_pool.push_back(pd.b);
  }
  pending.clear();
}

// ---------------------------------------------------------------------------
// internal steps
// ---------------------------------------------------------------------------
namespace {

ep_status do_constitutive(Ctx *c, const double *u, double *sig, double *D, uint8_t *flag,
                          const float *learned_y = nullptr) {
  ConstArgs a{};
  a.u = u;
  if (learned_y) {
    a.learned = 2;
    a.mlp_y = learned_y;
  }
  a.return_map = true;
  a.sig_out = sig;
  a.D_out = D;
  a.flag_out = flag;
  a.commit = false;
  a.force = true;
  // the plastic masks go to the buffer the last assembly did not use
  c->em_cur = c->em_asm == 0 ? 1 : 0;
  {
    ProfScope ps(*c, PROF_CONST);
    HIPC(launch_constitutive(*c, a));
  }
  // assembly work list, grouped by colour: elements plastic now or at the
  // last assembly
  {
    ProfScope ps(*c, PROF_COMPACT);
    HIPC(launch_compact(*c, 1, c->em[c->em_cur], c->em_asm >= 0 ? c->em[c->em_asm] : nullptr,
                        c->ecol_perm, c->n_perm, c->plist, c->d_colour_first_block, c->n_col,
                        c->coff, c->ptotals));
  }
  c->coff_known = false;  // new offsets on the device
  c->have_const = true;
  return EP_OK;
}

ep_status do_assemble(Ctx *c) {
  if (!c->have_const) {
    c->err = "ep_assemble_tangent: no constitutive evaluation since setup or commit";
    return EP_ESTATE;
  }
  if (c->opt.assembly == EP_ASSEMBLY_ROWS) {
    // element matrices of the listed elements with plastic points now, then
    // the node-row gather of every row they or the last assembly touched
    const int64_t listed = c->coff_known ? (int64_t)(c->coff_h[c->n_col] - c->coff_h[0]) : -1;
    if (listed != 0) {
      ProfScope ps(*c, PROF_ASSEMBLE);
      if (ps.tok >= 0) c->pending[ps.tok].count = 2;
      HIPC(launch_emat(*c, false, listed));
      HIPC(launch_row_gather(*c, false, listed));
    }
    c->em_asm = c->em_cur;
    c->coff_known = false;
    return EP_OK;
  }
  if (c->opt.assembly == EP_ASSEMBLY_FUSED) {
    // one pass over the rows touched now or at the last assembly, the
    // element terms formed in place
    const int64_t listed = c->coff_known ? (int64_t)(c->coff_h[c->n_col] - c->coff_h[0]) : -1;
    if (listed != 0) {
      ProfScope ps(*c, PROF_ASSEMBLE);
      HIPC(launch_row_fused(*c, listed));
    }
    c->em_asm = c->em_cur;
    c->coff_known = false;
    return EP_OK;
  }
  // a short work list whose length the host holds (inside a Newton step):
  // one fused row pass instead of a launch per colour, which the launch
  // latency of the colour rounds would dominate.  Both leave every block of a
  // listed element at K_elast plus the terms of the elements plastic now and
  // every other block at K_elast, so the next assembly may take either path
  // (blocks without this assembly's stamp start from K_elast).
  if (c->coff_known && c->fused_ok) {
    const int64_t listed = (int64_t)(c->coff_h[c->n_col] - c->coff_h[0]);
    if (listed > 0 && listed * c->n_p * c->n_q <= SHORT_LIST_WORK) {
      {
        ProfScope ps(*c, PROF_ASSEMBLE);
        HIPC(launch_row_fused(*c, listed));
      }
      c->em_asm = c->em_cur;
      c->coff_known = false;
      return EP_OK;
    }
  }
  // a longer list that fits the element-matrix buffer (a few elements per
  // compute unit): the colour rounds would hold about one element per
  // compute unit each and last one element's latency chain apiece; the
  // element matrices (one launch over the whole list) and the node-row
  // gather fill the device instead.  The gather also leaves K_elast plus the
  // present terms in every block of a listed element.
  if (c->coff_known && c->emat_cap > 0) {
    const int64_t listed = (int64_t)(c->coff_h[c->n_col] - c->coff_h[0]);
    if (listed > 0 && listed <= c->emat_cap) {
      {
        ProfScope ps(*c, PROF_ASSEMBLE);
        if (ps.tok >= 0) c->pending[ps.tok].count = 2;
        HIPC(launch_emat(*c, false, listed));
        HIPC(launch_row_gather(*c, false, listed));
      }
      c->em_asm = c->em_cur;
      c->coff_known = false;
      return EP_OK;
    }
  }
  // colour rounds with one-byte stamps: before the counter passes 255 every
  // stamp is cleared (a block without this assembly's stamp starts from
  // K_elast, so clearing is always safe)
  if (c->epoch_counter == 255) {
    HIPC(hipMemsetAsync(c->epoch, 0, std::max<int64_t>(c->nnzb, 1), c->stream));
    c->epoch_counter = 0;
  }
  const int epoch = ++c->epoch_counter;
  // colours with an empty work list are skipped when the host holds the
  // list's colour offsets (after a Newton step's synchronisation)
  auto listed = [&](int col) -> int64_t {
    return c->coff_known ? (int64_t)(c->coff_h[col + 1] - c->coff_h[col]) : -1;
  };
  int last = -1, n_launch = 0;
  for (int col = 0; col < c->n_col; ++col)
    if (c->colour_size[col] > 0 && listed(col) != 0) {
      last = col;
      ++n_launch;
    }
  // one timed section over the colour launches: the start event travels with
  // the first launch and the stop event with the last, and the section
  // counts one per launch
  {
    ProfScope ps(*c, PROF_ASSEMBLE);
    const hipEvent_t stop = c->launch_stop;
    if (ps.tok >= 0) c->pending[ps.tok].count = n_launch;
    for (int col = 0; col < c->n_col; ++col) {
      c->launch_stop = col == last ? stop : nullptr;
      HIPC(launch_colour_assembly(*c, col, epoch, listed(col)));
    }
  }
  c->em_asm = c->em_cur;
  c->coff_known = false;
  return EP_OK;
}

// residual r = Q(f - F), norms -> c->norms[0] = |r|^2, [1] = |Qf|^2,
// [2] = |(I - Q) F|^2 (reactions at the Dirichlet dofs); residual = false:
// F only (into F_out)
ep_status do_residual(Ctx *c, const double *f, double *F_out, bool residual = true) {
  const int nblk = (int)((c->n_n + 255) / 256);
  {
    ProfScope ps(*c, PROF_FORCE);
    HIPC(launch_force_gather(*c, f, F_out, residual ? c->r : nullptr, c->partials, nblk));
  }
  if (residual) HIPC(launch_reduce(*c, c->partials, nblk, 3, c->norms));
  return EP_OK;
}

// |Q(f - F)| relative to |Q f|; under pure displacement control (Q f = 0)
// relative to the reactions |(I - Q) F|; absolute if both vanish
double relative_residual(const double *norms_h) {
  const double rn = std::sqrt(norms_h[0]), fn = std::sqrt(norms_h[1]);
  const double scale = fn > 0 ? fn : std::sqrt(norms_h[2]);
  return scale > 0 ? rn / scale : rn;
}

// n PCG iterations.  Even chunks without profiling replay a HIP graph of
// the chunk (captured once per solution vector, chunk length and plastic
// mask buffer, which the split form's kernels read; the iterations
// alternate two search-direction buffers, so an even chunk ends where it
// started); otherwise the kernels are launched one by one.
ep_status pcg_chunk(Ctx *c, double *x, int n) {
  const bool assembled = c->opt.operator_form == EP_OPERATOR_ASSEMBLED;
  // small assembled systems: the chunk in one single-workgroup launch
  if (assembled && c->n_dof <= SMALL_PCG_DOFS) {
    HIPC(launch_pcg_small(*c, x, n));
    return EP_OK;
  }
  // moderate sizes: two kernels per iteration, the last beta step after the
  // chunk; otherwise five kernels per iteration
  const bool two = assembled && c->n_dof <= MEDIUM_PCG_DOFS;
  auto enqueue = [&](int m) -> hipError_t {
    hipError_t e = hipSuccess;
    for (int k = 0; k < m && e == hipSuccess; ++k)
      e = two ? launch_pcg_iteration2(*c, x) : launch_pcg_iteration(*c, x);
    if (two && e == hipSuccess) e = launch_pcg_finish2(*c);
    return e;
  };
  if (c->prof_mask || n < 2 || n % 2 != 0) {
    HIPC(enqueue(n));
    return EP_OK;
  }
  if (!c->pcg_graph || c->pcg_graph_x != x || c->pcg_graph_n != n ||
      c->pcg_graph_em != c->em_cur) {
    if (c->pcg_graph) {
      HIPC(hipGraphExecDestroy(c->pcg_graph));
      c->pcg_graph = nullptr;
    }
    if (!c->gstream) HIPC(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    const int pcur = c->pcur;
    c->stream = c->gstream;
    hipError_t e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = enqueue(n);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->gstream, &g);
    c->stream = user;
    c->pcur = pcur;
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&c->pcg_graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->pcg_graph = nullptr;
      c->err = std::string("PCG graph capture: ") + hipGetErrorString(e);
      return EP_EDEVICE;
    }
    c->pcg_graph_x = x;
    c->pcg_graph_n = n;
    c->pcg_graph_em = c->em_cur;
  }
  HIPC(hipGraphLaunch(c->pcg_graph, c->stream));
  return EP_OK;
}

ep_status do_pcg(Ctx *c, const double *b, double *x, double rtol, int max_it, int *its,
                 double *relres, bool *breakdown = nullptr) {
  HIPC(launch_diag_inv(*c));
  HIPC(launch_pcg_init(*c, b, x));
  HIPC(launch_pcg_beta_init(*c, rtol));
  const int chunk = std::max(1, c->opt.pcg_check_every);
  int done_its = 0;
  bool done = false;
  while (!done) {
    const int n = std::min(chunk, max_it - done_its);
    if (n <= 0) break;
    const ep_status st = pcg_chunk(c, x, n);
    if (st) return st;
    done_its += n;
    HIPC(hipMemcpyAsync(c->sc_h, c->sc, 16 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPC(hipStreamSynchronize(c->stream));
    done = c->sc_h[SC_DONE] != 0.0;
  }
  *its = (int)c->sc_h[SC_ITS];
  *relres = c->sc_h[SC_RR0] > 0 ? std::sqrt(c->sc_h[SC_RR] / c->sc_h[SC_RR0]) : 0.0;
  const bool brk = c->sc_h[SC_BREAK] != 0.0;
  if (breakdown) *breakdown = brk;
  if (brk) {
    c->err = "PCG breakdown after " + std::to_string(*its) +
             " iterations (p.q <= 0 or a non-finite scalar); x is the last finite iterate";
    return EP_ENOTCONV;
  }
  if (!done) {
    c->err = "PCG reached its iteration limit";
    return EP_ENOTCONV;
  }
  return EP_OK;
}

// exact residual |Q(f - F(u))| / |Q f| (constitutive pass + force gather);
// synchronises
ep_status exact_residual(Ctx *c, const double *f, const double *u, double *res_rel) {
  ep_status st = do_constitutive(c, u, nullptr, nullptr, nullptr);
  if (st) return st;
  st = do_residual(c, f, nullptr);
  if (st) return st;
  HIPC(hipMemcpyAsync(c->norms_h, c->norms, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPC(hipStreamSynchronize(c->stream));
  *res_rel = relative_residual(c->norms_h);
  return EP_OK;
}

// Energy products of the correction dx = c->px at u (whole vectors, no
// Dirichlet mask): y0 = K_elast u, y1 = K_elast dx, then
// norms[4..7] = dx.y1, u.y0, dx.y0, dx.dx (fixed-order sums).  Enqueued.
ep_status energy_dots(Ctx *c, const double *u) {
  HIPC(launch_spmv_elastic_full(*c, u, c->ky[0]));
  HIPC(launch_spmv_elastic_full(*c, c->px, c->ky[1]));
  const double *x[4] = {c->px, u, c->px, c->px};
  const double *y[4] = {c->ky[1], c->ky[0], c->ky[0], c->px};
  HIPC(launch_dots(*c, 4, x, y, c->norms + 4));
  return EP_OK;
}

// g(a) = dx . Q(f - F(u + a dx)), the negative derivative of the incremental
// energy along the Newton correction dx = c->px: constitutive pass and
// residual at the trial displacement, fixed-order dot.  Synchronises.
ep_status ls_g(Ctx *c, const double *f, const double *u, double a, double *g) {
  HIPC(launch_trial(*c, u, c->px, a, c->ut));
  ep_status st = do_constitutive(c, c->ut, nullptr, nullptr, nullptr);
  if (st) return st;
  st = do_residual(c, f, nullptr);
  if (st) return st;
  const double *x[1] = {c->px};
  const double *y[1] = {c->r};
  HIPC(launch_dots(*c, 1, x, y, c->norms + 8));
  HIPC(hipMemcpyAsync(c->norms_h + 8, c->norms + 8, sizeof(double), hipMemcpyDeviceToHost,
                      c->stream));
  HIPC(hipStreamSynchronize(c->stream));
  *g = c->norms_h[8];
  if (!std::isfinite(*g)) {
    c->err = "ep_newton_step: line-search residual not finite at step length " +
             std::to_string(a);
    return EP_ENONFINITE;
  }
  return EP_OK;
}

// Step length of the damped Newton method.  The models are associative, so
// the incremental energy J(u + a dx) is convex in a and g = -J' decreases;
// g(0) = dx . r > 0 when dx is a descent direction.  The full step is kept
// if g(1) >= -theta g(0) (the minimiser is at or close before a = 1);
// otherwise the root of g in (0, 1) is bracketed by [0, 1] and approached by
// regula falsi with the Illinois modification (the end point kept twice in
// a row has its value halved), stopping at |g| <= theta g(0) or after
// ls_max_evals evaluations (the last point is taken).
ep_status line_search(Ctx *c, const double *f, const double *u, double g0, double *alpha,
                      int *evals) {
  const double theta = c->opt.newton_damping;
  double g1 = 0.0;
  ep_status st = ls_g(c, f, u, 1.0, &g1);
  if (st) return st;
  *evals = 1;
  *alpha = 1.0;
  if (!(g0 > 0.0) || g1 >= -theta * g0) return EP_OK;
  double lo = 0.0, g_lo = g0, hi = 1.0, g_hi = g1, x = 1.0;
  int kept = 0;  // +1: the upper end was kept last time, -1: the lower end
  while (*evals < c->opt.ls_max_evals) {
    x = (lo * g_hi - hi * g_lo) / (g_hi - g_lo);
    double gx = 0.0;
    st = ls_g(c, f, u, x, &gx);
    if (st) return st;
    ++*evals;
    if (std::fabs(gx) <= theta * g0) break;
    if (gx > 0.0) {
      lo = x;
      g_lo = gx;
      if (kept == 1) g_hi *= 0.5;
      kept = 1;
    } else {
      hi = x;
      g_hi = gx;
      if (kept == -1) g_lo *= 0.5;
      kept = -1;
    }
  }
  *alpha = x;
  return EP_OK;
}

ep_status ensure_warm_buffers(Ctx *c) {
  if (c->mlp_x) return EP_OK;
  HIPC(dalloc(&c->mlp_x, c->n_int * EP_MLP_XS));
  HIPC(dalloc(&c->mlp_y, c->n_int * EP_MLP_YS));
  HIPC(dalloc(&c->wu_pred, c->n_dof));
  HIPC(dalloc(&c->wu_warm, c->n_dof));
  return EP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *ep_last_error(const ep_ctx *ctx) {
  if (!ctx) return g_setup_err.c_str();
  return reinterpret_cast<const Ctx *>(ctx)->err.c_str();
}

void ep_destroy(ep_ctx *ctx) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (c && c->stream) (void)hipStreamSynchronize(c->stream);
  free_ctx(c);
}

ep_status ep_setup(const ep_mesh *mesh, const ep_quadrature *quad, const ep_material *mat,
                   const ep_options *opt_in, void *hip_stream, ep_ctx **out) {
  if (out) *out = nullptr;
  auto fail = [](const std::string &m, ep_status s) {
    g_setup_err = m;
    return s;
  };
  if (!mesh || !mat || !out) return fail("ep_setup: NULL argument", EP_EINVAL);
  ElemDef ed;
  if (!elem_def(mesh->dim, mesh->type, ed)) return fail("ep_setup: unsupported element", EP_EINVAL);
  if (mesh->n_nodes <= 0 || mesh->n_elems < 0 || !mesh->coord || !mesh->elem || !mesh->free_mask)
    return fail("ep_setup: invalid mesh arrays", EP_EINVAL);
  if ((int64_t)mesh->dim * mesh->n_nodes >= (int64_t)1 << 31 ||
      mesh->n_elems * ed.n_p * ed.n_p >= (int64_t)1 << 31)
    return fail("ep_setup: mesh too large for 32-bit indices", EP_EINVAL);
  if (const char *bad = material_error(mat)) return fail(std::string("ep_setup: ") + bad, EP_EINVAL);
  const int64_t n_n = mesh->n_nodes, n_e = mesh->n_elems;
  const int dim = ed.dim, n_p = ed.n_p, n_q = ed.n_q;

  ep_options opt{EP_FP64, EP_FP64, 20000, 50, 1e-10, 1e-2, EP_OPERATOR_ASSEMBLED, 0.0, 12,
                 EP_ASSEMBLY_COLOURS};
  if (opt_in) opt = *opt_in;
  if (opt.assembly != EP_ASSEMBLY_COLOURS && opt.assembly != EP_ASSEMBLY_ROWS &&
      opt.assembly != EP_ASSEMBLY_FUSED)
    return fail("ep_setup: assembly must be EP_ASSEMBLY_COLOURS, EP_ASSEMBLY_ROWS or "
                "EP_ASSEMBLY_FUSED", EP_EINVAL);
  if (opt.assembly == EP_ASSEMBLY_FUSED && opt.local_prec != EP_FP64)
    return fail("ep_setup: the fused row assembly forms its element terms in FP64 "
                "(local_prec must be EP_FP64)", EP_EINVAL);
  if (!(opt.newton_damping >= 0.0 && opt.newton_damping < 1.0))
    return fail("ep_setup: newton_damping must lie in [0, 1)", EP_EINVAL);
  if (opt.ls_max_evals <= 0) opt.ls_max_evals = 12;
  if (opt.operator_form != EP_OPERATOR_ASSEMBLED && opt.operator_form != EP_OPERATOR_SPLIT)
    return fail("ep_setup: operator_form must be EP_OPERATOR_ASSEMBLED or EP_OPERATOR_SPLIT",
                EP_EINVAL);
  if (opt.operator_form == EP_OPERATOR_SPLIT && opt.local_prec != EP_FP64)
    return fail("ep_setup: the split operator form applies its element terms in FP64 "
                "(local_prec must be EP_FP64)", EP_EINVAL);
  if (opt.tangent_prec != EP_FP64 && opt.tangent_prec != EP_FP32)
    return fail("ep_setup: tangent_prec must be EP_FP64 or EP_FP32", EP_EINVAL);
  if (opt.local_prec != EP_FP64 && !(opt.local_prec == EP_FP32 || opt.local_prec == EP_BF16))
    return fail("ep_setup: local_prec must be EP_FP64, EP_FP32 or EP_BF16", EP_EINVAL);
  if (opt.local_prec != EP_FP64 &&
      !(ed.id == ET_Q2_3D || ed.id == ET_Q2S_3D || ed.id == ET_P2_3D))
    return fail("ep_setup: matrix-core local products (EP_FP32 / EP_BF16) are built for the "
                "27- and 20-node hexahedra and the 10-node tetrahedron only", EP_EINVAL);
  if (opt.pcg_max_it <= 0) opt.pcg_max_it = 20000;
  if (opt.pcg_check_every <= 0) opt.pcg_check_every = 50;

  // reference tables
  std::vector<double> xi, wq;
  if (quad) {
    if (quad->n_q != n_q || !quad->xi || !quad->w)
      return fail("ep_setup: quadrature must have the element's number of points", EP_EINVAL);
    xi.assign(quad->xi, quad->xi + n_q * dim);
    wq.assign(quad->w, quad->w + n_q);
  } else {
    builtin_rule(ed.id, dim, xi, wq);
  }
  std::vector<double> ref((size_t)n_q * n_p * dim + n_q);
  for (int q = 0; q < n_q; ++q) ref_gradients(ed.id, &xi[q * dim], &ref[(size_t)q * n_p * dim]);
  for (int q = 0; q < n_q; ++q) ref[(size_t)n_q * n_p * dim + q] = wq[q];

  // mesh graph: node-block pattern, position maps, colouring (host)
  const bool sorted_scatter = ed.id == ET_Q1_2D || ed.id == ET_Q2_2D || ed.id == ET_Q2S_2D ||
                              ed.id == ET_Q1_3D;
  MeshGraph gr;
  {
    const std::string why = build_mesh_graph(n_n, n_e, n_p, dim, mesh->elem, sorted_scatter,
                                             CMP_CHUNK, CMP_MAX_COLOURS, gr);
    if (!why.empty()) return fail("ep_setup: " + why, EP_EINVAL);
  }

  Ctx *c = new Ctx();
  c->stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&c->dev);
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->dev) !=
          hipSuccess || c->n_cu < 1)
    c->n_cu = 256;
  c->et = ed.id;
  c->dim = dim;
  c->n_p = n_p;
  c->n_q = n_q;
  c->n_str = dim == 3 ? 6 : 3;
  c->n_sc = dim == 3 ? 6 : 4;
  c->n_desc = dim == 3 ? 10 : 7;
  c->n_n = n_n;
  c->n_e = n_e;
  c->n_int = n_e * n_q;
  c->n_dof = dim * n_n;
  c->opt = opt;
  c->mat = make_matc(*mat);
  c->E = mat->E;

  auto bail = [&](ep_status s) {
    g_setup_err = c->err;
    free_ctx(c);
    return s;
  };
#define SETUP_HIP(x)                                                         \
  do {                                                                       \
    hipError_t e__ = (x);                                                    \
    if (e__ != hipSuccess) {                                                 \
      c->err = std::string("ep_setup: ") + #x + ": " + hipGetErrorString(e__); \
      return bail(e__ == hipErrorOutOfMemory ? EP_ENOMEM : EP_EDEVICE);      \
    }                                                                        \
  } while (0)

  const int32_t *E = mesh->elem;
  const int64_t nnzb = gr.nnzb;
  c->nnzb = nnzb;
  const int n_col = gr.n_col;
  c->n_col = n_col;
  c->colour_size.assign(gr.colour_size.begin(), gr.colour_size.end());
  c->colour_first_block = gr.colour_first_chunk;
  c->n_perm = (int64_t)c->colour_first_block[n_col] * CMP_CHUNK;
  for (int64_t m = 0; m < n_n; ++m) {
    c->max_deg = std::max(c->max_deg, gr.bptr[m + 1] - gr.bptr[m]);
    c->max_slots = std::max(c->max_slots, gr.n2e_ptr[m + 1] - gr.n2e_ptr[m]);
  }
  if (sizeof(double) * (size_t)c->max_deg * dim * dim + 2 * sizeof(int) * (size_t)c->max_slots >
      65536) {
    c->err = "ep_setup: a node row does not fit the 64 KB of LDS of the row gather";
    return bail(EP_EINVAL);
  }
  c->fused_ok = opt.local_prec == EP_FP64 && c->max_slots <= 64 && row_fused_lds(*c) <= 65536;
  if (opt.assembly == EP_ASSEMBLY_FUSED && !c->fused_ok) {
    c->err = "ep_setup: the fused row assembly takes at most 64 elements per node and a node "
             "row that fits 64 KB of LDS with its element data";
    return bail(EP_EINVAL);
  }
  const std::vector<int32_t> &n2e_ptr = gr.n2e_ptr, &fslot = gr.fslot, &slot_elem = gr.slot_elem,
                             &bptr = gr.bptr, &bcol = gr.bcol, &bdiag = gr.bdiag,
                             &bpos = gr.bpos, &bposs = gr.bposs, &perm = gr.perm;

  // device memory
  hipStream_t s = c->stream;
  const int64_t n_int = c->n_int, n_dof = c->n_dof;
  SETUP_HIP(dalloc(&c->coord, dim * n_n));
  SETUP_HIP(dalloc(&c->elem, n_e * n_p));
  SETUP_HIP(dalloc(&c->freem, n_dof));
  SETUP_HIP(dalloc(&c->ref, (int64_t)ref.size()));
  SETUP_HIP(dalloc(&c->bptr, n_n + 1));
  SETUP_HIP(dalloc(&c->bcol, nnzb));
  SETUP_HIP(dalloc(&c->bdiag, n_n));
  SETUP_HIP(dalloc(&c->bpos, n_e * n_p * n_p));
  if (sorted_scatter) SETUP_HIP(dalloc(&c->bposs, n_e * n_p * n_p));
  SETUP_HIP(dalloc(&c->Ke, nnzb * dim * dim));
  if (opt.tangent_prec == EP_FP32) {
    SETUP_HIP(dalloc(&c->Ke32, nnzb * dim * dim));
    SETUP_HIP(hipMalloc(&c->Kt, sizeof(float) * std::max<int64_t>(1, nnzb * dim * dim)));
  } else {
    SETUP_HIP(hipMalloc(&c->Kt, sizeof(double) * std::max<int64_t>(1, nnzb * dim * dim)));
  }
  SETUP_HIP(dalloc(&c->epoch, nnzb));
  SETUP_HIP(dalloc(&c->n2e_ptr, n_n + 1));
  SETUP_HIP(dalloc(&c->n2e, n_e * n_p));
  // element matrices of the row-gather assembly, FP64 size (matrix-core
  // products store FP32 in it): every element in rows mode; in colour mode
  // the work lists of at most ROW_ROUTE_PER_CU elements and
  // ROW_ROUTE_ENTRIES_PER_CU element-matrix entries per compute unit (about
  // 50 MB on 256 compute units)
  if (opt.assembly == EP_ASSEMBLY_ROWS) {
    c->emat_cap = n_e;
  } else if (opt.assembly == EP_ASSEMBLY_COLOURS) {
    const int64_t entries = (int64_t)n_p * n_p * dim * dim;
    c->emat_cap = std::min<int64_t>({n_e, ROW_ROUTE_PER_CU * c->n_cu,
                                     ROW_ROUTE_ENTRIES_PER_CU * c->n_cu / entries});
  }
  if (c->emat_cap > 0) {
    SETUP_HIP(hipMalloc(&c->emat, sizeof(double) * c->emat_cap * n_p * n_p * dim * dim));
    SETUP_HIP(dalloc(&c->eslot, n_e));
  }
  SETUP_HIP(dalloc(&c->fslot, n_e * n_p));
  SETUP_HIP(dalloc(&c->slot_elem, n_e * n_p));
  SETUP_HIP(dalloc(&c->Fp, n_e * n_p * dim));
  SETUP_HIP(dalloc(&c->ecol_perm, (int64_t)perm.size()));
  SETUP_HIP(dalloc(&c->d_colour_first_block, n_col + 1));
  SETUP_HIP(dalloc(&c->ep_s, c->n_sc * n_int));
  if (mat->model == EP_VM) SETUP_HIP(dalloc(&c->beta_s, c->n_sc * n_int));
  SETUP_HIP(dalloc(&c->kappa_s, n_int));
  SETUP_HIP(dalloc(&c->flag, n_int));
  SETUP_HIP(dalloc(&c->desc, c->n_desc * n_int));
  SETUP_HIP(dalloc(&c->Fe, n_e * n_p * dim));
  SETUP_HIP(dalloc(&c->em[0], n_e));
  SETUP_HIP(dalloc(&c->em[1], n_e));
  SETUP_HIP(dalloc(&c->plist, n_e));
  SETUP_HIP(dalloc(&c->coff, n_col + 1));
  SETUP_HIP(dalloc(&c->ptotals, 8));
  SETUP_HIP(dalloc(&c->iscratch, std::max(n_int, n_e)));
  c->cmp_cap = std::max<int64_t>((n_int + CMP_CHUNK - 1) / CMP_CHUNK, c->n_perm / CMP_CHUNK) + 2;
  c->cmp_cap = std::max<int64_t>(c->cmp_cap, (n_e + CMP_CHUNK - 1) / CMP_CHUNK + 2);
  SETUP_HIP(dalloc(&c->cmp_counts, c->cmp_cap));
  SETUP_HIP(dalloc(&c->cmp_counts2, c->cmp_cap));
  SETUP_HIP(dalloc(&c->cmp_counts3, c->cmp_cap));
  SETUP_HIP(dalloc(&c->F, n_dof));
  SETUP_HIP(dalloc(&c->r, n_dof));
  SETUP_HIP(dalloc(&c->ky[0], n_dof));
  SETUP_HIP(dalloc(&c->ky[1], n_dof));
  // reductions: 2 per 256 dofs (PCG vectors, force gather) or 1 per SpMV
  // block of up to 32 lanes per node
  c->partials_cap = std::max<int64_t>(2 * ((n_dof + 255) / 256), (n_n * 32 + 255) / 256) + 64;
  SETUP_HIP(dalloc(&c->partials, c->partials_cap));
  SETUP_HIP(dalloc(&c->partials2, c->partials_cap));
  SETUP_HIP(dalloc(&c->sc2, 16));
  SETUP_HIP(dalloc(&c->norms, 16));
  SETUP_HIP(hipHostMalloc((void **)&c->norms_h, 16 * sizeof(double), hipHostMallocDefault));
  SETUP_HIP(dalloc(&c->pz, n_dof));
  SETUP_HIP(dalloc(&c->pp[0], n_dof));
  SETUP_HIP(dalloc(&c->pp[1], n_dof));
  SETUP_HIP(dalloc(&c->pq, n_dof));
  SETUP_HIP(dalloc(&c->px, n_dof));
  SETUP_HIP(dalloc(&c->dinv, n_dof));
  SETUP_HIP(dalloc(&c->sc, 16));
  SETUP_HIP(hipHostMalloc((void **)&c->sc_h, 16 * sizeof(double), hipHostMallocDefault));

  SETUP_HIP(hipMemcpyAsync(c->coord, mesh->coord, sizeof(double) * dim * n_n, hipMemcpyHostToDevice, s));
  if (n_e > 0)
    SETUP_HIP(hipMemcpyAsync(c->elem, E, sizeof(int32_t) * n_e * n_p, hipMemcpyHostToDevice, s));
  SETUP_HIP(hipMemcpyAsync(c->freem, mesh->free_mask, n_dof, hipMemcpyHostToDevice, s));
  SETUP_HIP(upload(c->ref, ref, s));
  SETUP_HIP(upload(c->bptr, bptr, s));
  SETUP_HIP(upload(c->bcol, bcol, s));
  SETUP_HIP(upload(c->bdiag, bdiag, s));
  SETUP_HIP(upload(c->bpos, bpos, s));
  if (sorted_scatter) SETUP_HIP(upload(c->bposs, bposs, s));
  SETUP_HIP(upload(c->n2e_ptr, n2e_ptr, s));
  SETUP_HIP(upload(c->n2e, gr.n2e, s));
  SETUP_HIP(upload(c->fslot, fslot, s));
  SETUP_HIP(upload(c->slot_elem, slot_elem, s));
  SETUP_HIP(upload(c->ecol_perm, perm, s));
  SETUP_HIP(upload(c->d_colour_first_block, c->colour_first_block, s));
  SETUP_HIP(hipMemsetAsync(c->ep_s, 0, sizeof(double) * c->n_sc * n_int, s));
  if (c->beta_s) SETUP_HIP(hipMemsetAsync(c->beta_s, 0, sizeof(double) * c->n_sc * n_int, s));
  SETUP_HIP(hipMemsetAsync(c->kappa_s, 0, sizeof(double) * n_int, s));
  for (int k = 0; k < 2; ++k)
    SETUP_HIP(hipMemsetAsync(c->em[k], 0, sizeof(uint32_t) * std::max<int64_t>(n_e, 1), s));
  SETUP_HIP(hipMemsetAsync(c->epoch, 0, std::max<int64_t>(nnzb, 1), s));
  SETUP_HIP(hipMemsetAsync(c->Ke, 0, sizeof(double) * std::max<int64_t>(1, nnzb * dim * dim), s));
  SETUP_HIP(hipMemsetAsync(c->ptotals, 0, sizeof(int32_t) * 8, s));
  SETUP_HIP(hipMemsetAsync(c->coff, 0, sizeof(int32_t) * (n_col + 1), s));

  // geometry check: det J > 0 at every point
  int32_t *bad = c->ptotals + 7;
  SETUP_HIP(launch_geometry(*c, nullptr, nullptr, bad));
  int32_t bad_h = 0;
  SETUP_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SETUP_HIP(hipStreamSynchronize(s));
  if (bad_h > 0) {
    c->err = "ep_setup: " + std::to_string(bad_h) + " integration points with det J <= 0";
    return bail(EP_EINVAL);
  }
  // K_elast = B^T D_elast B (eq. K_elast-split), colour rounds
  SETUP_HIP(launch_elastic_assembly(*c));
  if (opt.tangent_prec == EP_FP32) SETUP_HIP(launch_to_float(c->Ke, c->Ke32, nnzb * dim * dim, s));
  SETUP_HIP(launch_copy_ke_to_kt(*c));
  SETUP_HIP(hipStreamSynchronize(s));
  c->epoch_counter = 0;
  c->em_cur = 0;
  c->em_asm = -1;
  c->have_const = false;
  *out = reinterpret_cast<ep_ctx *>(c);
  return EP_OK;
#undef SETUP_HIP
}

ep_status ep_set_stream(ep_ctx *ctx, void *hip_stream) {
  CHECK_CTX(ctx);
  reinterpret_cast<Ctx *>(ctx)->stream = (hipStream_t)hip_stream;
  return EP_OK;
}

ep_status ep_get_sizes(const ep_ctx *ctx, ep_sizes *o) {
  CHECK_CTX(ctx);
  if (!o) return EP_EINVAL;
  const Ctx *c = reinterpret_cast<const Ctx *>(ctx);
  o->dim = c->dim;
  o->n_p = c->n_p;
  o->n_q = c->n_q;
  o->n_str = c->n_str;
  o->n_sc = c->n_sc;
  o->n_colours = c->n_col;
  o->n_nodes = c->n_n;
  o->n_elems = c->n_e;
  o->n_int = c->n_int;
  o->n_dof = c->n_dof;
  o->nnz = c->nnzb * c->dim * c->dim;
  o->nnz_blocks = c->nnzb;
  return EP_OK;
}

ep_status ep_set_state(ep_ctx *ctx, const double *ep, const double *beta, const double *kappa) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  const size_t nb = sizeof(double) * c->n_sc * c->n_int;
  if (ep) HIPC(hipMemcpyAsync(c->ep_s, ep, nb, hipMemcpyDeviceToDevice, c->stream));
  else HIPC(hipMemsetAsync(c->ep_s, 0, nb, c->stream));
  if (c->beta_s) {
    if (beta) HIPC(hipMemcpyAsync(c->beta_s, beta, nb, hipMemcpyDeviceToDevice, c->stream));
    else HIPC(hipMemsetAsync(c->beta_s, 0, nb, c->stream));
  }
  if (kappa) HIPC(hipMemcpyAsync(c->kappa_s, kappa, sizeof(double) * c->n_int, hipMemcpyDeviceToDevice, c->stream));
  else HIPC(hipMemsetAsync(c->kappa_s, 0, sizeof(double) * c->n_int, c->stream));
  c->have_const = false;
  return EP_OK;
}

ep_status ep_get_state(ep_ctx *ctx, double *ep, double *beta, double *kappa) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  const size_t nb = sizeof(double) * c->n_sc * c->n_int;
  if (ep) HIPC(hipMemcpyAsync(ep, c->ep_s, nb, hipMemcpyDeviceToDevice, c->stream));
  if (beta) {
    if (c->beta_s) HIPC(hipMemcpyAsync(beta, c->beta_s, nb, hipMemcpyDeviceToDevice, c->stream));
    else HIPC(hipMemsetAsync(beta, 0, nb, c->stream));
  }
  if (kappa) HIPC(hipMemcpyAsync(kappa, c->kappa_s, sizeof(double) * c->n_int, hipMemcpyDeviceToDevice, c->stream));
  return EP_OK;
}

ep_status ep_geometry(ep_ctx *ctx, double *dphi, double *w) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  int32_t *bad = c->ptotals + 7;
  HIPC(launch_geometry(*c, dphi, w, bad));
  return EP_OK;
}

ep_status ep_strain(ep_ctx *ctx, const double *u, double *eps) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!eps) return EP_EINVAL;
  ConstArgs a{};
  a.u = u;
  a.eps_out = eps;
  a.return_map = false;
  a.force = false;
  HIPC(launch_constitutive(*c, a));
  return EP_OK;
}

ep_status ep_constitutive(ep_ctx *ctx, const double *u, double *sig, double *D, uint8_t *flag) {
  CHECK_CTX(ctx);
  return do_constitutive(reinterpret_cast<Ctx *>(ctx), u, sig, D, flag);
}

ep_status ep_assemble_tangent(ep_ctx *ctx) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (c->opt.operator_form == EP_OPERATOR_SPLIT) {
    // the split form's PCG applies K_elast and the element terms of the
    // current plastic masks; an assembly would also move the mask buffer the
    // next evaluation writes
    c->err = "ep_assemble_tangent: the context applies the split operator form "
             "(operator_form SPLIT); K_tangent is not assembled";
    return EP_EINVAL;
  }
  return do_assemble(c);
}

ep_status ep_internal_force(ep_ctx *ctx, double *F) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c->have_const) {
    c->err = "ep_internal_force: no constitutive evaluation since setup or commit";
    return EP_ESTATE;
  }
  return do_residual(c, nullptr, F, false);
}

ep_status ep_newton_step(ep_ctx *ctx, const double *f, double *u, ep_newton_info *info) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!f || !u || !info) return EP_EINVAL;
  std::memset(info, 0, sizeof(*info));
  ep_status st = do_constitutive(c, u, nullptr, nullptr, nullptr);
  if (st) return st;
  st = do_residual(c, f, nullptr);
  if (st) return st;
  HIPC(hipMemcpyAsync(c->norms_h, c->norms, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  int32_t tot[3];
  HIPC(hipMemcpyAsync(tot, c->ptotals, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  c->coff_h.resize(c->n_col + 1);
  HIPC(hipMemcpyAsync(c->coff_h.data(), c->coff, sizeof(int32_t) * (c->n_col + 1),
                      hipMemcpyDeviceToHost, c->stream));
  HIPC(hipStreamSynchronize(c->stream));
  c->coff_known = true;
  info->res_norm = std::sqrt(c->norms_h[0]);
  info->f_norm = std::sqrt(c->norms_h[1]);
  info->res_rel = relative_residual(c->norms_h);
  info->n_plastic_elem = tot[2];
  info->n_plastic_ip = tot[1];
  if (!std::isfinite(info->res_rel)) {
    c->err = "ep_newton_step: the residual at u is not finite (NaN or Inf in u, f or the state)";
    return EP_ENONFINITE;
  }
  if (info->res_rel <= c->opt.newton_rtol) {
    info->converged = 1;
    return EP_OK;
  }
  const bool damped = c->opt.newton_damping > 0.0;
  if (damped) {
    if (!c->ut) HIPC(dalloc(&c->ut, c->n_dof));
    if (!c->rn) HIPC(dalloc(&c->rn, c->n_dof));
    // PCG works in place on r: keep the Newton residual for g(0) = dx . r
    HIPC(hipMemcpyAsync(c->rn, c->r, sizeof(double) * c->n_dof, hipMemcpyDeviceToDevice,
                        c->stream));
  }
  if (c->opt.operator_form == EP_OPERATOR_ASSEMBLED) {
    st = do_assemble(c);
    if (st) return st;
  }
  // forcing term min(max, |r|/|f|), but no tighter than needed to reach the
  // Newton tolerance in this step
  const double rtol = std::min(c->opt.pcg_forcing_max,
                               std::max(info->res_rel, 0.5 * c->opt.newton_rtol / info->res_rel));
  int its = 0;
  double rel = 0;
  bool brk = false;
  const ep_status ps = do_pcg(c, c->r, c->px, rtol, c->opt.pcg_max_it, &its, &rel, &brk);
  if (ps != EP_OK && ps != EP_ENOTCONV) return ps;
  const std::string pcg_err = c->err;
  info->pcg_its = its;
  info->pcg_relres = rel;
  info->pcg_breakdown = brk ? 1 : 0;
  // energy norms of ALG-NEWTON's stopping test at u (before the update)
  st = energy_dots(c, u);
  if (st) return st;
  if (damped) {
    const double *x[1] = {c->px};
    const double *y[1] = {c->rn};
    HIPC(launch_dots(*c, 1, x, y, c->norms + 8));
  }
  HIPC(hipMemcpyAsync(c->norms_h + 4, c->norms + 4, 5 * sizeof(double), hipMemcpyDeviceToHost,
                      c->stream));
  HIPC(hipStreamSynchronize(c->stream));
  const double dKd = c->norms_h[4], uKu = c->norms_h[5], dKu = c->norms_h[6],
               dd = c->norms_h[7];
  if (!std::isfinite(dd) || !std::isfinite(dKd) || !std::isfinite(dKu) || !std::isfinite(uKu)) {
    c->err = "ep_newton_step: the Newton correction is not finite; u left unchanged";
    return EP_ENONFINITE;
  }
  double alpha = 1.0;
  int evals = 0;
  if (damped) {
    st = line_search(c, f, u, c->norms_h[8], &alpha, &evals);
    if (st) return st;
  }
  info->step = alpha;
  info->ls_evals = evals;
  // |du|_e / (|u|_e + |u + du|_e) for du = alpha dx, the norms expanded in
  // the products above
  const double e_du = alpha * alpha * dKd;
  const double e_new = uKu + 2.0 * alpha * dKu + alpha * alpha * dKd;
  const double den = std::sqrt(std::max(uKu, 0.0)) + std::sqrt(std::max(e_new, 0.0));
  info->energy_incr = den > 0.0 ? std::sqrt(std::max(e_du, 0.0)) / den : 0.0;
  HIPC(launch_axpy_free(*c, c->px, u, alpha));
  if (ps != EP_OK) c->err = pcg_err;
  return ps;
}

ep_status ep_commit_step(ep_ctx *ctx, const double *u) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  ConstArgs a{};
  a.u = u;
  a.return_map = true;
  a.commit = true;
  a.force = false;
  HIPC(launch_constitutive(*c, a));
  c->have_const = false;
  return EP_OK;
}

ep_status ep_get_plastic(ep_ctx *ctx, int32_t *ip, int64_t *n_ip, int32_t *elem, int64_t *n_elem) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c->have_const) {
    c->err = "ep_get_plastic: no constitutive evaluation";
    return EP_ESTATE;
  }
  int32_t *tot = c->ptotals + 4;  // scratch totals
  int32_t th[3] = {0, 0, 0};
  // plastic elements (ascending) and the plastic-point count
  HIPC(launch_compact(*c, 1, c->em[c->em_cur], nullptr, nullptr, c->n_e, elem ? elem : c->iscratch,
                      nullptr, 0, nullptr, tot));
  HIPC(hipMemcpyAsync(th, tot, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPC(hipStreamSynchronize(c->stream));
  if (n_elem) *n_elem = th[0];
  if (n_ip) *n_ip = th[1];
  if (ip) {
    HIPC(launch_compact(*c, 0, c->flag, nullptr, nullptr, c->n_int, ip, nullptr, 0, nullptr, tot));
    HIPC(hipMemcpyAsync(th, tot, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPC(hipStreamSynchronize(c->stream));
    if (n_ip) *n_ip = th[0];
  }
  return EP_OK;
}

ep_status ep_get_csr(ep_ctx *ctx, int32_t which, int32_t *row_ptr, int32_t *col_idx, double *val) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (which != 0 && which != 1) return EP_EINVAL;
  HIPC(launch_csr_expand(*c, which, row_ptr, col_idx, val));
  return EP_OK;
}

ep_status ep_get_position_map(ep_ctx *ctx, int32_t *pos) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!pos) return EP_EINVAL;
  HIPC(launch_pos_expand(*c, pos));
  return EP_OK;
}

ep_status ep_spmv(ep_ctx *ctx, const double *x, double *y) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!x || !y) return EP_EINVAL;
  HIPC(launch_spmv(*c, x, y));
  return EP_OK;
}

ep_status ep_assemble_elastic(ep_ctx *ctx) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  const int64_t n = c->nnzb * c->dim * c->dim;
  HIPC(hipMemsetAsync(c->Ke, 0, sizeof(double) * std::max<int64_t>(1, n), c->stream));
  {
    ProfScope ps(*c, PROF_ELASTIC);
    HIPC(launch_elastic_assembly(*c));
  }
  if (c->opt.tangent_prec == EP_FP32) HIPC(launch_to_float(c->Ke, c->Ke32, n, c->stream));
  HIPC(launch_copy_ke_to_kt(*c));
  c->em_asm = -1;  // K_tangent = K_elast: no element terms to restore
  return EP_OK;
}

ep_status ep_apply_tangent(ep_ctx *ctx, const double *x, double *y) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!x || !y) return EP_EINVAL;
  if (!c->have_const) {
    c->err = "ep_apply_tangent: no constitutive evaluation since setup or commit";
    return EP_ESTATE;
  }
  HIPC(launch_apply_split(*c, x, y));
  return EP_OK;
}

ep_status ep_pcg(ep_ctx *ctx, const double *b, double *x, double rtol, int32_t max_it, int32_t *its,
                 double *relres) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!b || !x || max_it <= 0) return EP_EINVAL;
  if (c->opt.operator_form == EP_OPERATOR_SPLIT && !c->have_const) {
    c->err = "ep_pcg: the split operator needs a constitutive evaluation since setup or commit";
    return EP_ESTATE;
  }
  int it = 0;
  double rel = 0;
  const ep_status st = do_pcg(c, b, x, rtol, max_it, &it, &rel);
  if (its) *its = it;
  if (relres) *relres = rel;
  return st;
}

ep_status ep_profile(ep_ctx *ctx, int32_t mask) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  c->prof_collect();
  c->prof_mask = (uint32_t)mask & EP_PROFILE_ALL;
  return EP_OK;
}

ep_status ep_profile_read(ep_ctx *ctx, int32_t k, double *ms, int64_t *count) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (k < 0 || k >= PROF_COUNT) return EP_EINVAL;
  c->prof_collect();
  if (ms) *ms = c->prof_ms[k];
  if (count) *count = c->prof_n[k];
  c->prof_ms[k] = 0;
  c->prof_n[k] = 0;
  return EP_OK;
}


ep_status ep_mlp_features(ep_ctx *ctx, const double *u, float *X) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!u || !X) return EP_EINVAL;
  ConstArgs a{};
  a.u = u;
  a.learned = 1;
  a.mlp_x = X;
  HIPC(launch_constitutive(*c, a));
  return EP_OK;
}

ep_status ep_predictor(ep_ctx *ctx, const double *u_prev, const double *u_prev2, double extrap,
                       double *u_out) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!u_prev || !u_out || !std::isfinite(extrap)) return EP_EINVAL;
  HIPC(launch_extrapolate(*c, u_prev, u_prev2, extrap, u_out));
  return EP_OK;
}

ep_status ep_warm_start(ep_ctx *ctx, ep_mlp *mlp, const double *f, const double *u_prev,
                        const double *u_prev2, double extrap, double pcg_rtol, double *u_out,
                        ep_warm_info *info) {
  CHECK_CTX(ctx);
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!mlp || !f || !u_prev || !u_out || !info || !(pcg_rtol > 0) || !std::isfinite(extrap)) {
    c->err = "ep_warm_start: invalid argument";
    return EP_EINVAL;
  }
  std::memset(info, 0, sizeof(*info));
  const MlpImpl *m = reinterpret_cast<const MlpImpl *>(mlp);
  if (m->stream != c->stream) HIPC(hipStreamSynchronize(m->stream));
  ep_status st = ensure_warm_buffers(c);
  if (st) return st;
  // exact residual of the plain start
  st = exact_residual(c, f, u_prev, &info->res_rel_start);
  if (st) return st;
  // prediction at the extrapolated displacement
  HIPC(launch_extrapolate(*c, u_prev, u_prev2, extrap, c->wu_pred));
  ConstArgs fa{};
  fa.u = c->wu_pred;
  fa.learned = 1;
  fa.mlp_x = c->mlp_x;
  HIPC(launch_constitutive(*c, fa));
  HIPC(launch_mlp_forward(*m, c->mlp_x, c->n_int, c->mlp_y, c->stream));
  st = do_constitutive(c, c->wu_pred, nullptr, nullptr, nullptr, c->mlp_y);
  if (st) return st;
  st = do_residual(c, f, nullptr);
  if (st) return st;
  int32_t tot[3];
  HIPC(hipMemcpyAsync(c->norms_h, c->norms, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPC(hipMemcpyAsync(tot, c->ptotals, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPC(hipStreamSynchronize(c->stream));
  {
    info->res_rel_pred = relative_residual(c->norms_h);
  }
  info->n_plastic_pred = tot[1];
  // one solve with the predicted tangent and residual
  if (c->opt.operator_form == EP_OPERATOR_ASSEMBLED) {
    st = do_assemble(c);
    if (st) return st;
  }
  int its = 0;
  double rel = 0;
  const ep_status ps = do_pcg(c, c->r, c->px, pcg_rtol, c->opt.pcg_max_it, &its, &rel);
  if (ps != EP_OK && ps != EP_ENOTCONV) return ps;
  info->pcg_its = its;
  HIPC(hipMemcpyAsync(c->wu_warm, c->wu_pred, c->n_dof * sizeof(double), hipMemcpyDeviceToDevice,
                      c->stream));
  HIPC(launch_axpy_free(*c, c->px, c->wu_warm));
  // the exact residual decides
  st = exact_residual(c, f, c->wu_warm, &info->res_rel_warm);
  if (st) return st;
  info->accepted = std::isfinite(info->res_rel_warm) && info->res_rel_warm < info->res_rel_start;
  const double *src = info->accepted ? c->wu_warm : u_prev;
  if (src != u_out)
    HIPC(hipMemcpyAsync(u_out, src, c->n_dof * sizeof(double), hipMemcpyDeviceToDevice,
                        c->stream));
  HIPC(hipStreamSynchronize(c->stream));
  return EP_OK;
}

}  // extern "C"
