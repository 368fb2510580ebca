/*
 * ep.h - C ABI of the MI355X elastoplastic Newton hot path.
 *
 * Method: Cermak, Sysala, Valdman, "Efficient and flexible MATLAB
 * implementation of 2D and 3D elastoplastic problems" (arXiv 1805.04155).
 * One Newton iteration of its semismooth Newton method (Section 4,
 * ALG-NEWTON) consists of
 *   - the strain E = B u at every integration point (Section 6.2),
 *   - the return map T_k and consistent tangent T_k^o (Sections 2.2, 2.3),
 *   - the compaction of the plastic integration points,
 *   - the tangent K = K_elast + B^T (D_tangent - D_elast) B (eq. K-split),
 *     assembled, or applied element by element in its split form,
 *   - the internal force F = B^T (WEIGHT .* S) (Section 7),
 *   - a linear solve for the Newton correction (here Jacobi-PCG).
 * Load paths (force- or displacement-controlled, Section 8) are driven by
 * the caller: one ep_newton_step per iteration, ep_commit_step per step.
 *
 * Conventions
 *   - Pointers are DEVICE pointers unless the comment says host.  Device
 *     buffers passed in are owned by the caller; the library never frees
 *     them and never keeps them past the call.  Host arrays are copied
 *     during the call.
 *   - Indices are 0-based.  dof = dim*node + component (Section 5).
 *   - Integration point ip = e*n_q + q (element-major, Section 6.1).
 *   - Per-point arrays are structure-of-arrays: [component][n_int].
 *   - Voigt order 11,22,33,12,23,13.  Strain-type vectors carry doubled
 *     shears (engineering strain), stress-type vectors do not (Section 5).
 *     In plane strain (dim = 2) the strain has the 3 in-plane components
 *     (11, 22, 12), the stress, plastic strain and back stress have the 4
 *     components (11, 22, 33, 12), and the tangent is the in-plane 3x3 block.
 *   - n_str = 6 (3D) or 3 (2D) strain components; n_sc = 6 or 4 stress /
 *     state components.
 *   - All device work of a context is enqueued on its stream (the
 *     hip_stream given to ep_setup or ep_set_stream).  Calls return once the
 *     work is enqueued, except where a host-visible result is documented.
 *   - Errors are status codes; ep_last_error gives the context's message.
 *     A context is not thread-safe.
 */
#ifndef EP_H
#define EP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ep_ctx ep_ctx;

typedef enum {
  EP_OK = 0,
  EP_EINVAL = -1,    /* invalid argument or mesh                           */
  EP_ENOMEM = -2,    /* device or host allocation failed                   */
  EP_EDEVICE = -3,   /* a HIP runtime call failed                          */
  EP_ENOTCONV = -4,  /* PCG reached its iteration limit                    */
  EP_ESTATE = -5,    /* call out of order (e.g. assembly before constitutive) */
  EP_ENONFINITE = -6 /* a residual, PCG scalar or correction is NaN or Inf   */
} ep_status;

/* Lagrange elements of the paper's Appendix.  EP_P1: 3-node triangle /
 * 4-node tetrahedron, 1 point.  EP_P2: 10-node tetrahedron, 11-point rule
 * (3D only).  EP_Q1: 4-node quadrilateral (2x2 Gauss) / 8-node hexahedron
 * (2x2x2).  EP_Q2: 9-node quadrilateral (3x3) / 27-node hexahedron (3x3x3),
 * tensor-product Lagrange with the paper's 20 hexahedron nodes first, then
 * the face centres (-xi3,+xi3,-xi2,+xi1,+xi2,-xi1) and the centre; the
 * 9-node quadrilateral lists vertices counter-clockwise, edge midpoints
 * (bottom, right, top, left) and the centre.  EP_Q2S: the serendipity
 * elements of the Appendix's Q2 definition, the 8-node quadrilateral (3x3)
 * and the 20-node hexahedron (3x3x3), nodes as the first 8 / 20 of EP_Q2. */
typedef enum { EP_P1 = 1, EP_P2 = 2, EP_Q1 = 3, EP_Q2 = 4, EP_Q2S = 5 } ep_elem;

/* EP_VM: von Mises with linear kinematic hardening (Section 2.2; a = 0 is
 *        perfect plasticity).  State: plastic strain, back stress.
 * EP_DP: Drucker-Prager (Section 2.3) with yield function
 *        |dev s|/sqrt(2) + eta*p - (c + a*kappa), p = tr(sigma)/3 and
 *        associated flow; a = 0 is the paper's perfect plasticity, a > 0
 *        linear hardening of the cohesion in the accumulated multiplier
 *        kappa.  State: plastic strain, kappa. */
typedef enum { EP_VM = 1, EP_DP = 2 } ep_model;

typedef enum { EP_FP64 = 0, EP_FP32 = 1, EP_BF16 = 2 } ep_prec;

/* How the Newton step applies the tangent (eq. K-split):
 * ASSEMBLED: K_tangent is assembled into the CSR values and PCG multiplies
 *            by it (ep_assemble_tangent);
 * SPLIT:     nothing is assembled; PCG applies K_elast (CSR) plus, element
 *            by element, B^T (D_tangent - D_elast) B over the elements with
 *            plastic points (ep_apply_tangent), and its Jacobi diagonal is
 *            diag K_elast plus the diagonals of those element terms. */
typedef enum { EP_OPERATOR_ASSEMBLED = 0, EP_OPERATOR_SPLIT = 1 } ep_operator;

/* How an assembled K_tangent (and K_elast) is formed from the element terms
 * of eq. K-split; both give the same K up to the order of the sums.
 * COLOURS: one launch per element colour (elements of a colour share no
 *          node); each element adds its node blocks to K in place, a
 *          one-byte stamp per block telling whether the block still holds
 *          the previous assembly's values (then it starts from K_elast).
 *          A work list whose length the host holds (inside ep_newton_step)
 *          is routed by its length: at most 4096 (element, node, point)
 *          triples (FP64 local products) take the single launch of FUSED;
 *          at most 16 elements and 24576 element-matrix entries per compute
 *          unit the two launches of ROWS, in a buffer of that many
 *          element slots; longer lists the colour rounds.
 * ROWS:    two launches: the element matrices of the elements with plastic
 *          points go to a buffer (slot: the element's work-list position),
 *          then every node
 *          row touched by an element plastic now or at the last assembly
 *          is rewritten once as its K_elast row plus those elements' rows
 *          (ascending element), accumulated in LDS.
 * FUSED:   one launch, ROWS without the buffer: each touched node row forms
 *          its part of the element terms in place (the element geometry at
 *          a plastic point is recomputed by each row of the element), no
 *          colours or stamps.  FP64 element-local products only
 *          (local_prec EP_FP64), at most 64 elements per node; K_elast is
 *          assembled by colour rounds. */
typedef enum {
  EP_ASSEMBLY_COLOURS = 0,
  EP_ASSEMBLY_ROWS = 1,
  EP_ASSEMBLY_FUSED = 2
} ep_assembly;

typedef struct {
  int32_t dim;               /* 2 (plane strain) or 3                        */
  int32_t type;              /* ep_elem                                      */
  int64_t n_nodes, n_elems;
  const double *coord;       /* host [dim][n_nodes]                          */
  const int32_t *elem;       /* host [n_elems][n_p], local order of ep_elem  */
  const uint8_t *free_mask;  /* host [dim*n_nodes], 1 = free, 0 = Dirichlet  */
} ep_mesh;

/* Optional quadrature override: same number of points as the built-in rule
 * of the element (the kernels are specialised on it). */
typedef struct {
  int32_t n_q;
  const double *xi;          /* host [n_q][dim] reference coordinates        */
  const double *w;           /* host [n_q] weights (sign kept, Section 6.3)  */
} ep_quadrature;

typedef struct {
  int32_t model;             /* ep_model                                     */
  double E, nu;              /* K = E/(3(1-2nu)), G = E/(2(1+nu)) (Sec. 8.1) */
  double Y;                  /* VM yield level on |dev(sigma) - beta|        */
  double a;                  /* hardening modulus (VM kinematic, DP cohesion) */
  double eta, c;             /* DP friction and cohesion parameters          */
} ep_material;

typedef struct {
  int32_t tangent_prec;      /* EP_FP64 or EP_FP32: storage of the K values  */
  int32_t local_prec;        /* EP_FP64 (default) or EP_FP32: element-local
                                B^T (D - D_e) B products                      */
  int32_t pcg_max_it;        /* PCG iteration limit per Newton step          */
  int32_t pcg_check_every;   /* PCG iterations between host checks           */
  double newton_rtol;        /* |Q(f - F)| <= newton_rtol |Q f|              */
  double pcg_forcing_max;    /* PCG stops at min(this, res_rel) relative     */
  int32_t operator_form;     /* ep_operator (default EP_OPERATOR_ASSEMBLED); SPLIT
                                requires local_prec = EP_FP64                 */
  double newton_damping;     /* theta of the damped Newton method (Section 4
                                remark after eq. lin_syst); 0 = full steps    */
  int32_t ls_max_evals;      /* residual evaluations per line search (<= 0:
                                12)                                          */
  int32_t assembly;          /* ep_assembly (default EP_ASSEMBLY_COLOURS)    */
} ep_options;

typedef struct {
  int32_t dim, n_p, n_q, n_str, n_sc, n_colours;
  int64_t n_nodes, n_elems, n_int, n_dof;
  int64_t nnz;               /* scalar CSR entries of K                      */
  int64_t nnz_blocks;        /* dim x dim node blocks of K                   */
} ep_sizes;

typedef struct {
  double res_rel;            /* |Q(f - F(u))| / |Q f| at the u passed in;
                                with Q f = 0 (pure displacement control)
                                relative to the reactions |(I - Q) F(u)|,
                                absolute if both vanish                       */
  double res_norm, f_norm;
  double pcg_relres;         /* final relative PCG residual (if solved)      */
  int32_t pcg_its;
  int32_t converged;         /* 1: res_rel <= newton_rtol; u left unchanged  */
  int64_t n_plastic_ip, n_plastic_elem;
  double energy_incr;        /* stopping quantity of ALG-NEWTON for the
                                correction made: |du|_e / (|u_old|_e +
                                |u_old + du|_e), |v|_e^2 = v^T K_elast v
                                (whole vectors, Dirichlet dofs included)    */
  double step;               /* step length a of the correction du = a dx
                                (1 without damping)                         */
  int32_t ls_evals;          /* residual evaluations of the line search     */
  int32_t pcg_breakdown;     /* 1: PCG stopped on p.q <= 0 or a non-finite
                                scalar                                       */
} ep_newton_info;

/* Builds everything that depends only on the mesh (Sections 6.1-6.3):
 * reference tables, the node-block CSR pattern of K, the element position
 * map, an element colouring (no two elements of one colour share a node),
 * the node-to-element map, the geometry check (det J > 0 at every point)
 * and K_elast = B^T D_elast B.  The plastic state starts at zero.
 * quadrature and options may be NULL (built-in rule, default options).
 * Size limits (32-bit indices): dim * n_nodes, n_elems * n_p^2 and the
 * scalar non-zeros of K (dim^2 per node block) below 2^31; larger meshes,
 * invalid arrays or materials, a non-positive det J or more than 512
 * colours give EP_EINVAL, a failed allocation EP_ENOMEM.
 * On error *out is NULL and ep_last_error(NULL) holds the message.
 * Synchronises the stream. */
ep_status ep_setup(const ep_mesh *mesh, const ep_quadrature *quadrature,
                   const ep_material *material, const ep_options *options,
                   void *hip_stream, ep_ctx **out);

/* Releases every allocation of the context.  NULL is accepted. */
void ep_destroy(ep_ctx *ctx);

/* Message of the last failed call on ctx (ctx = NULL: of the last failed
 * ep_setup of this thread).  Never NULL. */
const char *ep_last_error(const ep_ctx *ctx);

ep_status ep_set_stream(ep_ctx *ctx, void *hip_stream);
ep_status ep_get_sizes(const ep_ctx *ctx, ep_sizes *out /* host */);

/* State from the previous load step (eps^p_{k-1}, beta_{k-1}, kappa_{k-1}),
 * [n_sc][n_int] and [n_int].  beta is used by EP_VM, kappa by EP_DP; a NULL
 * pointer sets that array to zero.  ep_get_state copies the state out
 * (NULL outputs are skipped). */
ep_status ep_set_state(ep_ctx *ctx, const double *ep, const double *beta,
                       const double *kappa);
ep_status ep_get_state(ep_ctx *ctx, double *ep, double *beta, double *kappa);

/* Gradients of the basis functions at every point, dphi[n_int][n_p][dim],
 * and WEIGHT = |det J| * omega_q, w[n_int] (Section 6.1, eq.
 * basis_derivative).  The hot kernels recompute these on the fly; this
 * entry point exposes them for checking.  Either output may be NULL. */
ep_status ep_geometry(ep_ctx *ctx, double *dphi, double *w);

/* E = B u (Section 6.2): eps[n_str][n_int], engineering strain. */
ep_status ep_strain(ep_ctx *ctx, const double *u, double *eps);

/* Strain, return map and consistent tangent at every point for the
 * displacement u[n_dof], against the stored state (eqs. T_kinematic,
 * DT_kinematic; Section 2.3), followed by the element force vectors used by
 * ep_internal_force and the plastic-element bitmask used by
 * ep_assemble_tangent.  Optional outputs (NULL = skipped): sig[n_sc][n_int],
 * D[n_str*n_str][n_int] (row-major Voigt tangent, strain-type to
 * stress-type), flag[n_int] (0 elastic, 1 plastic / smooth cone, 2 apex). */
ep_status ep_constitutive(ep_ctx *ctx, const double *u, double *sig, double *D,
                          uint8_t *flag);

/* K_tangent = K_elast + B^T (D_tangent - D_elast) B (eq. K-split) for the
 * last ep_constitutive.  The work list (built by ep_constitutive) holds the
 * elements plastic now or at the previous assembly, grouped by colour; for
 * each, the element-local products over its plastic points are added to
 * K_elast (blocks not yet written in this assembly) or to K_tangent through
 * the position map, one colour at a time (deterministic, no float atomics);
 * elements that left the plastic set restore K_elast on their blocks.  Cost
 * is proportional to that list, not to the mesh.  The ROWS and FUSED modes
 * (options.assembly) rewrite instead every node row touched by a listed
 * element once, as its K_elast row plus the terms of the elements plastic
 * now; every mode gives the same K up to the order of the sums.
 * Returns EP_ESTATE if ep_constitutive has not run since setup or commit,
 * EP_EINVAL for a context with operator_form SPLIT (nothing is assembled
 * there). */
ep_status ep_assemble_tangent(ep_ctx *ctx);

/* Recomputes K_elast = B^T D_elast B (eq. K_elast-split, the setup step)
 * from scratch, colour round by colour round, and resets K_tangent to it
 * (the next ep_assemble_tangent adds the element terms of the elements
 * plastic at that time only).  Timed under profile id 7, so that the cost
 * of the incremental tangent can be set against it (Section 8.2). */
ep_status ep_assemble_elastic(ep_ctx *ctx);

/* F = B^T (WEIGHT .* S) (Section 7) for the last ep_constitutive,
 * F[n_dof].  Deterministic node gather of the element vectors. */
ep_status ep_internal_force(ep_ctx *ctx, double *F);

/* One iteration of ALG-NEWTON for the load vector f[n_dof] on the
 * displacement u[n_dof] (updated in place on free dofs; Dirichlet values of
 * u are kept).  Computes the residual r = Q(f - F(u)); if |r| <= newton_rtol
 * |Q f| it sets info->converged = 1 and leaves u unchanged; otherwise it
 * assembles K_tangent (operator_form ASSEMBLED; SPLIT assembles nothing),
 * solves K dx = r on the free dofs by Jacobi-PCG to the relative tolerance
 * min(pcg_forcing_max, max(res_rel, newton_rtol / (2 res_rel))) (no tighter
 * than the step needs to reach newton_rtol) and adds du = a dx to u.
 * a = 1 unless newton_damping = theta > 0 (the damped Newton method the
 * paper mentions after eq. lin_syst): then a minimises the incremental
 * energy along dx, whose derivative is -g(a), g(a) = dx . Q(f - F(u + a dx))
 * (each evaluation is a constitutive pass and a residual); a = 1 is kept if
 * g(1) >= -theta g(0), otherwise a is the root of g in (0, 1) by regula
 * falsi with the Illinois modification, stopped at |g(a)| <= theta g(0) or
 * after ls_max_evals evaluations.  info->energy_incr is the paper's
 * stopping quantity of the correction made (logged; the stopping test stays
 * the residual test).
 * Writes info (host).  Synchronises the stream.
 * Errors: EP_ENOTCONV if PCG hits its limit or breaks down (p.q <= 0;
 * info->pcg_breakdown = 1): u is still updated with the last finite
 * iterate.  EP_ENONFINITE if the residual at u, the correction or a
 * line-search residual is NaN or Inf: u is left unchanged. */
ep_status ep_newton_step(ep_ctx *ctx, const double *f, double *u,
                         ep_newton_info *info);

/* Accepts the load step: recomputes the return map at u and stores the
 * updated plastic strain, back stress and kappa (eq. T_other; Section 2.3)
 * as the state of the next step. */
ep_status ep_commit_step(ep_ctx *ctx, const double *u);

/* Plastic points of the last ep_constitutive, ascending:
 * ip[n_int] (capacity), elem[n_elems] (capacity); counts written to the
 * host pointers.  Any output may be NULL.  Synchronises the stream. */
ep_status ep_get_plastic(ep_ctx *ctx, int32_t *ip, int64_t *n_ip, int32_t *elem,
                         int64_t *n_elem);

/* Scalar CSR view of K (which = 0: K_elast, 1: K_tangent):
 * row_ptr[n_dof+1], col_idx[nnz] (ascending in each row), val[nnz]
 * (converted to double).  Any output may be NULL. */
ep_status ep_get_csr(ep_ctx *ctx, int32_t which, int32_t *row_ptr, int32_t *col_idx,
                     double *val);

/* Scalar position map pos[n_elems][dim*n_p][dim*n_p]: index in col_idx of
 * the entry (dof(e,a), dof(e,b)), local dof a = dim*p + i. */
ep_status ep_get_position_map(ep_ctx *ctx, int32_t *pos);

/* y = Q (K_tangent x): the product on free dofs, y = 0 on Dirichlet dofs
 * (x is used as given, also on Dirichlet dofs). */
ep_status ep_spmv(ep_ctx *ctx, const double *x, double *y);

/* y = Q (K_elast x + sum over the elements with plastic points of
 * B_e^T (D_tangent - D_elast) B_e x_e) for the last ep_constitutive: the
 * split form of K_tangent x (eq. K-split) without assembly, equal to
 * ep_spmv after ep_assemble_tangent up to rounding.  The element terms are
 * summed per node in a fixed order (deterministic).  x[n_dof], y[n_dof]
 * device; x is used as given, also on Dirichlet dofs.
 * Returns EP_ESTATE if ep_constitutive has not run since setup or commit. */
ep_status ep_apply_tangent(ep_ctx *ctx, const double *x, double *y);

/* Solves Q K_tangent Q x = Q b by Jacobi-PCG from x = 0 to
 * |r| <= rtol |Q b|, with the assembled K_tangent or, for operator_form
 * SPLIT, with the split form of ep_apply_tangent.  its and relres are host
 * outputs.  Synchronises. */
ep_status ep_pcg(ep_ctx *ctx, const double *b, double *x, double rtol, int32_t max_it,
                 int32_t *its, double *relres);

/* Per-kernel timing with HIP events on the context's stream: the events
 * travel with the kernel dispatches (start of the first kernel, end of the
 * last kernel of each timed call), so no marker command separates the
 * kernels.  mask selects the kernel ids to time (bit k for id k; 0 = off,
 * EP_PROFILE_ALL = every id): 0 constitutive, 1 compaction, 2 split-form
 * element terms and their node sum inside PCG, 3 colour assembly (one
 * count per colour launch), 4 force gather, 5 SpMV, 6 PCG vector update,
 * 7 K_elast assembly of ep_assemble_elastic, 8 single-workgroup PCG of small
 * systems (at most 12288 dofs, assembled operator: one launch runs a chunk
 * of iterations, counted once per iteration; ids 5 and 6 stay empty there).
 * While any id is timed, PCG launches its kernels one by one instead of
 * replaying a graph.  ep_profile_read returns the summed duration (ms) and
 * the count of kernel id k and resets both.  Both calls wait for the kernels
 * timed so far. */
#define EP_PROFILE_ALL 0x1ff
ep_status ep_profile(ep_ctx *ctx, int32_t mask);
ep_status ep_profile_read(ep_ctx *ctx, int32_t k, double *ms, int64_t *count);

/* ------------------------------------------------------------------------
 * Learned warm start (not part of the paper's method).  A per-point MLP
 * 13 -> 128 -> 128 -> 7 (ReLU) is trained on samples of the exact return
 * map (Sections 2.2, 2.3) and predicts, for a trial state, the stress and
 * whether the point is plastic.  ep_warm_start turns the prediction at an
 * extrapolated displacement into a Newton start: the predicted plastic set
 * selects the tangent branch, the predicted stress gives the residual, and
 * one linear solve gives the start; the exact residual decides whether it
 * is kept.  The converged solution is that of the exact return map.
 *
 * Features (one row of EP_MLP_XS floats per point):
 *   x[0:6]  = s_in (eps - eps_p)   trial elastic strain, 3D Voigt
 *                                  (engineering shears; plane strain: the
 *                                  embedded strain, 23 = 13 = 0)
 *   x[6:12] = s_in eps_p           plastic strain
 *   x[12]   = s_in kappa           Drucker-Prager hardening variable
 *   x[13:16] = 0
 * Targets / outputs (one row of EP_MLP_YS floats):
 *   y[0:6] = s_out (sigma - sigma_tr), the plastic correction of the 3D
 *   Voigt stress (sigma_tr = C (eps - eps_p), the elastic trial stress; the
 *   correction is 0 at elastic points), y[6] = plastic flag (targets: 0 or
 *   1; outputs: logit), y[7] = 0.  The predicted stress is
 *   sigma_tr + S y[0:6].
 * with s_in = E/S and s_out = 1/S, S = sqrt(3/2) Y (von Mises) or c
 * (Drucker-Prager).  The von Mises back stress is not a feature: the
 * generator and the warm start use beta = a eps_p (as tensors), which
 * linear kinematic hardening keeps from a state with beta_0 = a eps_p0.
 *
 * Parameters: one float array of EP_MLP_NPARAM values, in the order
 *   W1[128][13], b1[128], W2[128][128], b2[128], W3[7][128], b3[7]
 * (W[out][in]).  Loss of a batch of n samples:
 *   L = (1/n) sum_s [ (1/6) sum_{j<6} (y_j - t_j)^2
 *                     + log(1 + exp(y_6)) - t_6 y_6 ].
 * ------------------------------------------------------------------------ */
#define EP_MLP_IN 13
#define EP_MLP_HID 128
#define EP_MLP_OUT 7
#define EP_MLP_XS 16
#define EP_MLP_YS 8
#define EP_MLP_NPARAM 19207

typedef struct ep_mlp ep_mlp;

typedef struct {
  double res_rel_pred;       /* |Q(f - B^T W sigma_hat)| / |Q f| at u_pred  */
  double res_rel_start;      /* exact res_rel at u_prev (plain start)       */
  double res_rel_warm;       /* exact res_rel at the warm start             */
  int32_t pcg_its;           /* iterations of the warm-start solve          */
  int32_t accepted;          /* 1: u_out = warm start, 0: u_out = u_prev    */
  int64_t n_plastic_pred;    /* points predicted plastic                    */
} ep_warm_info;

/* Creates a network whose products use prec = EP_FP32 or EP_BF16 operands
 * (FP32 accumulation, FP32 parameters and Adam moments), with all
 * parameters 0; batches up to max_batch samples.  Work goes to hip_stream
 * (NULL: the default stream).  EP_EINVAL for another prec or
 * max_batch < 1; EP_ENOMEM. */
ep_status ep_mlp_create(int32_t prec, int64_t max_batch, void *hip_stream, ep_mlp **out);
void ep_mlp_destroy(ep_mlp *mlp);
const char *ep_mlp_last_error(const ep_mlp *mlp);

/* Copies params[EP_MLP_NPARAM] (device) in / out; set also clears the Adam
 * moments and step count. */
ep_status ep_mlp_set_params(ep_mlp *mlp, const float *params);
ep_status ep_mlp_get_params(ep_mlp *mlp, float *params);

/* Y[n][EP_MLP_YS] = network(X[n][EP_MLP_XS]) (any n >= 0). */
ep_status ep_mlp_forward(ep_mlp *mlp, const float *X, int64_t n, float *Y);

/* Gradient of L over the batch (X, T), 1 <= n <= max_batch: grad
 * [EP_MLP_NPARAM] and loss (one float) may be NULL.  Deterministic: fixed
 * tiles of 32 samples, summed in tile order. */
ep_status ep_mlp_loss_grad(ep_mlp *mlp, const float *X, const float *T, int64_t n,
                           float *grad, float *loss);

/* One Adam step (beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected)
 * with learning rate lr on the batch gradient; loss as above. */
ep_status ep_mlp_adam_step(ep_mlp *mlp, const float *X, const float *T, int64_t n, float lr,
                           float *loss);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): the loss gradient of ep_mlp_loss_grad for a network given
 * by its parameters alone, params[EP_MLP_NPARAM] (device, the layout of
 * ep_mlp_set_params), with products in prec = EP_FP32 or EP_BF16 (FP32
 * accumulation); X, T, grad, loss as in ep_mlp_loss_grad (grad and loss
 * may be NULL).  Allocates nothing: the per-tile partial gradients live in
 * a static device array of ceil(EP_MLP_NOALLOC_MAX_BATCH / 32) x
 * (EP_MLP_NPARAM + 1) floats (4.9 MB), one per device, kept until the
 * process ends.  Runs on the current device; hip_stream (NULL: the default
 * stream) must belong to it.  Enqueued; no synchronisation.  The result
 * equals ep_mlp_loss_grad's bit for bit (same kernels, same fixed-order
 * reduction).  Calls that overlap in time on one device share the array
 * and race: order them on one stream.  Errors (no context, so the message
 * is thread-local, from ep_mlp_noalloc_last_error): EP_EINVAL for another
 * prec, NULL inputs or n outside 1..EP_MLP_NOALLOC_MAX_BATCH; EP_EDEVICE if
 * the device array cannot be located or a launch fails. */
#define EP_MLP_NOALLOC_MAX_BATCH 2048
ep_status ep_mlp_loss_grad_noalloc(int32_t prec, const float *params, const float *X,
                                   const float *T, int64_t n, float *grad, float *loss,
                                   void *hip_stream);
const char *ep_mlp_noalloc_last_error(void);

/* Training samples from the exact return map (Sections 2.2, 2.3): sample j
 * takes the pooled state i = idx[j] (0 <= i < n_pool) - strain
 * eps_pool[6][n_pool], plastic strain ep_pool[6][n_pool], back stress
 * beta_pool[6][n_pool] (von Mises; NULL = a*ep) or kappa_pool[n_pool]
 * (Drucker-Prager; NULL = 0) - adds the strain increment deps[6][n], and
 * writes the features X[n][EP_MLP_XS] and targets T[n][EP_MLP_YS] of the
 * trial state eps_pool + deps.  3D Voigt throughout.  Enqueued on
 * hip_stream.  A sample whose index lies outside the pool gets all-zero
 * rows (checked on the device; no error is reported). */
ep_status ep_mlp_datagen(const ep_material *material, int64_t n, const int64_t *idx,
                         int64_t n_pool, const double *eps_pool, const double *ep_pool,
                         const double *beta_pool, const double *kappa_pool,
                         const double *deps, float *X, float *T, void *hip_stream);

/* Per-point features of the context's mesh at displacement u with the
 * committed state: X[n_int][EP_MLP_XS]. */
ep_status ep_mlp_features(ep_ctx *ctx, const double *u, float *X);

/* Secant predictor of a load step's start (no network): u_out = u_prev +
 * extrap * (u_prev - u_prev2) on free dofs, u_prev on Dirichlet dofs
 * (u_prev2 NULL: u_out = u_prev).  u_out may alias u_prev. */
ep_status ep_predictor(ep_ctx *ctx, const double *u_prev, const double *u_prev2, double extrap,
                       double *u_out);

/* Learned Newton start for load vector f.  u_pred = u_prev + extrap *
 * (u_prev - u_prev2) (u_prev2 NULL: u_pred = u_prev).  At u_pred the
 * network gives sigma_hat and the plastic set; the tangent is K_elast +
 * B^T (D_hat - D_e) B with D_hat the consistent tangent of the trial state
 * on the predicted branch (radius ratio capped at 1 where the exact test
 * says elastic), the residual is Q(f - B^T W sigma_hat) with
 * sigma_hat = sigma_tr + S y[0:6] at predicted-plastic points and the
 * elastic trial stress elsewhere, and Jacobi-PCG to relative tolerance pcg_rtol
 * gives w = u_pred + du.  The exact residuals at w and at u_prev then
 * decide: u_out = w if res(w) < res(u_prev), else u_prev.  u_out may alias
 * u_prev.  Writes info (host).  Synchronises. */
ep_status ep_warm_start(ep_ctx *ctx, ep_mlp *mlp, const double *f, const double *u_prev,
                        const double *u_prev2, double extrap, double pcg_rtol, double *u_out,
                        ep_warm_info *info);

#ifdef __cplusplus
}
#endif
#endif /* EP_H */
