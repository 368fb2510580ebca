/*
 * Plain FP64 CPU oracle for the elastoplastic Newton hot path of
 * Cermak, Sysala, Valdman, "Efficient and flexible MATLAB implementation of
 * 2D and 3D elastoplastic problems" (arXiv 1805.04155).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this code.  It shares no code,
 * header, table or constant with the HIP library: it has its own reference
 * elements, quadrature, geometry, return maps and assembly.  It is written to
 * be read against the paper, not to be fast:
 *   - stresses, strains and tangents are handled as full 3x3 tensors and
 *     3x3x3x3 arrays, converted to Voigt vectors only at the interface;
 *   - element matrices are formed with the explicit dense B matrix;
 *   - the stiffness matrix is the plain form  K = sum_e sum_q w B^T D B
 *     (the "Byczanski" form of the paper's Section 9), assembled from COO
 *     triplets sorted by (row, col, insertion order) and summed in that order.
 * Compile with -ffp-contract=off so that no fused multiply-add changes a
 * yield decision.
 *
 * Threads (OpenMP, or_set_threads): only loops whose iterations write
 * disjoint outputs run in parallel (strain and return map per point,
 * element force vectors and element matrices per element); every sum keeps
 * its serial order (the node sums of the internal force and the sorted COO
 * sums of K run on one thread), so the results do not depend on the thread
 * count.
 *
 * Array layouts at this interface (all 0-based, C order):
 *   coord [dim][n_n], elem [n_e][n_p], dphi [n_int][n_p][dim], w [n_int],
 *   eps/sig/ep/beta [n_int][6] Voigt (11,22,33,12,23,13; strain-type vectors
 *   carry doubled shears), D [n_int][6][6] mapping strain-type to stress-type
 *   Voigt, dof = dim*node + comp.  Plane strain (dim = 2) keeps 6-component
 *   tensors with eps_33 = gamma_23 = gamma_13 = 0 and uses the in-plane rows
 *   and columns (11, 22, 12).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads used by the parallel loops (n <= 0: keep the current setting);
   returns the count in effect (1 without OpenMP). */
int or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Element types (oracle-own codes)                                          */
/* ------------------------------------------------------------------------ */
enum {
  OR_P1_2D = 1, OR_Q1_2D = 2, OR_Q2_2D = 3,
  OR_P1_3D = 4, OR_P2_3D = 5, OR_Q1_3D = 6, OR_Q2_3D = 7,
  OR_Q2S_2D = 8, OR_Q2S_3D = 9  /* serendipity: 8-node quadrilateral, 20-node hexahedron */
};

int or_elem_info(int et, int *dim, int *n_p, int *n_q) {
  switch (et) {
    case OR_P1_2D: *dim = 2; *n_p = 3;  *n_q = 1;  return 0;
    case OR_Q1_2D: *dim = 2; *n_p = 4;  *n_q = 4;  return 0;
    case OR_Q2_2D: *dim = 2; *n_p = 9;  *n_q = 9;  return 0;
    case OR_P1_3D: *dim = 3; *n_p = 4;  *n_q = 1;  return 0;
    case OR_P2_3D: *dim = 3; *n_p = 10; *n_q = 11; return 0;
    case OR_Q1_3D: *dim = 3; *n_p = 8;  *n_q = 8;  return 0;
    case OR_Q2_3D: *dim = 3; *n_p = 27; *n_q = 27; return 0;
    case OR_Q2S_2D: *dim = 2; *n_p = 8;  *n_q = 9;  return 0;
    case OR_Q2S_3D: *dim = 3; *n_p = 20; *n_q = 27; return 0;
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Reference elements (Appendix; tensor Lagrange for 9- and 27-node cells)   */
/* ------------------------------------------------------------------------ */

/* 1D quadratic Lagrange polynomials on nodes -1, 0, 1 and their derivatives */
static double lag2(int node, double t) {
  if (node < 0) return 0.5 * t * (t - 1.0);
  if (node == 0) return 1.0 - t * t;
  return 0.5 * t * (t + 1.0);
}
static double lag2d(int node, double t) {
  if (node < 0) return t - 0.5;
  if (node == 0) return -2.0 * t;
  return t + 0.5;
}

/* node coordinates of the 9-node quadrilateral and 27-node hexahedron */
static const int QUAD9[9][2] = {
  {-1,-1},{1,-1},{1,1},{-1,1},{0,-1},{1,0},{0,1},{-1,0},{0,0}};
static const int HEX27[27][3] = {
  {-1,-1,-1},{1,-1,-1},{1,1,-1},{-1,1,-1},{-1,-1,1},{1,-1,1},{1,1,1},{-1,1,1},
  {0,-1,-1},{1,0,-1},{0,1,-1},{-1,0,-1},{0,-1,1},{1,0,1},{0,1,1},{-1,0,1},
  {-1,-1,0},{1,-1,0},{1,1,0},{-1,1,0},
  {0,0,-1},{0,0,1},{0,-1,0},{1,0,0},{0,1,0},{-1,0,0},{0,0,0}};
static const int HEX8[8][3] = {
  {-1,-1,-1},{1,-1,-1},{1,1,-1},{-1,1,-1},{-1,-1,1},{1,-1,1},{1,1,1},{-1,1,1}};
static const int QUAD4[4][2] = {{-1,-1},{1,-1},{1,1},{-1,1}};

/* Basis values phi[n_p] and reference gradients dphi[n_p][dim] at xi. */
void or_basis(int et, const double *xi, double *phi, double *dphi) {
  int p;
  switch (et) {
    case OR_P1_2D: {
      phi[0] = 1.0 - xi[0] - xi[1]; phi[1] = xi[0]; phi[2] = xi[1];
      dphi[0] = -1; dphi[1] = -1; dphi[2] = 1; dphi[3] = 0; dphi[4] = 0; dphi[5] = 1;
      return;
    }
    case OR_Q1_2D:
      for (p = 0; p < 4; ++p) {
        double a = QUAD4[p][0], b = QUAD4[p][1];
        phi[p] = 0.25 * (1 + a * xi[0]) * (1 + b * xi[1]);
        dphi[2 * p + 0] = 0.25 * a * (1 + b * xi[1]);
        dphi[2 * p + 1] = 0.25 * b * (1 + a * xi[0]);
      }
      return;
    case OR_Q2_2D:
      for (p = 0; p < 9; ++p) {
        int a = QUAD9[p][0], b = QUAD9[p][1];
        phi[p] = lag2(a, xi[0]) * lag2(b, xi[1]);
        dphi[2 * p + 0] = lag2d(a, xi[0]) * lag2(b, xi[1]);
        dphi[2 * p + 1] = lag2(a, xi[0]) * lag2d(b, xi[1]);
      }
      return;
    case OR_P1_3D:
      phi[0] = 1.0 - xi[0] - xi[1] - xi[2]; phi[1] = xi[0]; phi[2] = xi[1]; phi[3] = xi[2];
      { double g[12] = {-1,-1,-1, 1,0,0, 0,1,0, 0,0,1}; memcpy(dphi, g, sizeof g); }
      return;
    case OR_P2_3D: {
      /* barycentric l0 = 1 - x1 - x2 - x3, l1 = x1, l2 = x2, l3 = x3;
         vertices l(2l-1); edges 4 la lb for (0,1),(1,2),(0,2),(1,3),(2,3),(0,3) */
      double l[4] = {1.0 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]};
      double dl[4][3] = {{-1,-1,-1},{1,0,0},{0,1,0},{0,0,1}};
      static const int E[6][2] = {{0,1},{1,2},{0,2},{1,3},{2,3},{0,3}};
      int k, d;
      for (k = 0; k < 4; ++k) {
        phi[k] = l[k] * (2.0 * l[k] - 1.0);
        for (d = 0; d < 3; ++d) dphi[3 * k + d] = (4.0 * l[k] - 1.0) * dl[k][d];
      }
      for (k = 0; k < 6; ++k) {
        int a = E[k][0], b = E[k][1];
        phi[4 + k] = 4.0 * l[a] * l[b];
        for (d = 0; d < 3; ++d) dphi[3 * (4 + k) + d] = 4.0 * (dl[a][d] * l[b] + l[a] * dl[b][d]);
      }
      return;
    }
    case OR_Q1_3D:
      for (p = 0; p < 8; ++p) {
        double a = HEX8[p][0], b = HEX8[p][1], c = HEX8[p][2];
        double fa = 1 + a * xi[0], fb = 1 + b * xi[1], fc = 1 + c * xi[2];
        phi[p] = 0.125 * fa * fb * fc;
        dphi[3 * p + 0] = 0.125 * a * fb * fc;
        dphi[3 * p + 1] = 0.125 * fa * b * fc;
        dphi[3 * p + 2] = 0.125 * fa * fb * c;
      }
      return;
    case OR_Q2S_2D:
      /* 8-node serendipity quadrilateral (the 2D counterpart of the
         Appendix's 20-node element): vertices 1/4 (1+a x)(1+b y)(a x+b y-1),
         edge midpoints 1/2 (1-x^2)(1+b y) or 1/2 (1+a x)(1-y^2) */
      for (p = 0; p < 8; ++p) {
        int a = QUAD9[p][0], b = QUAD9[p][1];
        double x = xi[0], y = xi[1];
        if (a != 0 && b != 0) {
          double fa = 1 + a * x, fb = 1 + b * y, t = a * x + b * y - 1;
          phi[p] = 0.25 * fa * fb * t;
          dphi[2 * p + 0] = 0.25 * (a * fb * t + fa * fb * a);
          dphi[2 * p + 1] = 0.25 * (fa * b * t + fa * fb * b);
        } else if (a == 0) {
          phi[p] = 0.5 * (1 - x * x) * (1 + b * y);
          dphi[2 * p + 0] = 0.5 * (-2 * x) * (1 + b * y);
          dphi[2 * p + 1] = 0.5 * (1 - x * x) * b;
        } else {
          phi[p] = 0.5 * (1 + a * x) * (1 - y * y);
          dphi[2 * p + 0] = 0.5 * a * (1 - y * y);
          dphi[2 * p + 1] = 0.5 * (1 + a * x) * (-2 * y);
        }
      }
      return;
    case OR_Q2S_3D:
      /* 20-node serendipity hexahedron of the Appendix: vertices
         1/8 (1+a x1)(1+b x2)(1+c x3)(a x1+b x2+c x3-2), edge midpoints
         1/4 (1-x_k^2) times the two linear factors of the other axes */
      for (p = 0; p < 20; ++p) {
        int a = HEX27[p][0], b = HEX27[p][1], c = HEX27[p][2];
        double x = xi[0], y = xi[1], z = xi[2];
        if (a != 0 && b != 0 && c != 0) {
          double fa = 1 + a * x, fb = 1 + b * y, fc = 1 + c * z;
          double t = a * x + b * y + c * z - 2;
          phi[p] = 0.125 * fa * fb * fc * t;
          dphi[3 * p + 0] = 0.125 * (a * fb * fc * t + fa * fb * fc * a);
          dphi[3 * p + 1] = 0.125 * (fa * b * fc * t + fa * fb * fc * b);
          dphi[3 * p + 2] = 0.125 * (fa * fb * c * t + fa * fb * fc * c);
        } else if (a == 0) {
          double fb = 1 + b * y, fc = 1 + c * z;
          phi[p] = 0.25 * (1 - x * x) * fb * fc;
          dphi[3 * p + 0] = 0.25 * (-2 * x) * fb * fc;
          dphi[3 * p + 1] = 0.25 * (1 - x * x) * b * fc;
          dphi[3 * p + 2] = 0.25 * (1 - x * x) * fb * c;
        } else if (b == 0) {
          double fa = 1 + a * x, fc = 1 + c * z;
          phi[p] = 0.25 * fa * (1 - y * y) * fc;
          dphi[3 * p + 0] = 0.25 * a * (1 - y * y) * fc;
          dphi[3 * p + 1] = 0.25 * fa * (-2 * y) * fc;
          dphi[3 * p + 2] = 0.25 * fa * (1 - y * y) * c;
        } else {
          double fa = 1 + a * x, fb = 1 + b * y;
          phi[p] = 0.25 * fa * fb * (1 - z * z);
          dphi[3 * p + 0] = 0.25 * a * fb * (1 - z * z);
          dphi[3 * p + 1] = 0.25 * fa * b * (1 - z * z);
          dphi[3 * p + 2] = 0.25 * fa * fb * (-2 * z);
        }
      }
      return;
    case OR_Q2_3D:
      for (p = 0; p < 27; ++p) {
        int a = HEX27[p][0], b = HEX27[p][1], c = HEX27[p][2];
        double la = lag2(a, xi[0]), lb = lag2(b, xi[1]), lc = lag2(c, xi[2]);
        phi[p] = la * lb * lc;
        dphi[3 * p + 0] = lag2d(a, xi[0]) * lb * lc;
        dphi[3 * p + 1] = la * lag2d(b, xi[1]) * lc;
        dphi[3 * p + 2] = la * lb * lag2d(c, xi[2]);
      }
      return;
  }
}

/* Quadrature points xi[n_q][dim] and weights w[n_q]. */
int or_quadrature(int et, double *xi, double *w) {
  int dim, n_p, n_q, i, j, k, q = 0;
  if (or_elem_info(et, &dim, &n_p, &n_q)) return -1;
  if (et == OR_P1_2D) { xi[0] = xi[1] = 1.0 / 3.0; w[0] = 0.5; return 0; }
  if (et == OR_P1_3D) { xi[0] = xi[1] = xi[2] = 0.25; w[0] = 1.0 / 6.0; return 0; }
  if (et == OR_P2_3D) {
    /* Keast 11-point rule, exact rational / surd values of the tabulated one */
    double a1 = 1.0 / 14.0, b1 = 11.0 / 14.0;
    double s = sqrt(5.0 / 14.0);
    double a2 = (1.0 + s) / 4.0, b2 = (1.0 - s) / 4.0;
    double P[11][3] = {
      {0.25, 0.25, 0.25},
      {a1, a1, a1}, {b1, a1, a1}, {a1, b1, a1}, {a1, a1, b1},
      {a2, b2, b2}, {b2, a2, b2}, {b2, b2, a2}, {a2, a2, b2}, {a2, b2, a2}, {b2, a2, a2}};
    double W[11] = {-74.0 / 5625.0,
                    343.0 / 45000.0, 343.0 / 45000.0, 343.0 / 45000.0, 343.0 / 45000.0,
                    56.0 / 2250.0, 56.0 / 2250.0, 56.0 / 2250.0, 56.0 / 2250.0, 56.0 / 2250.0,
                    56.0 / 2250.0};
    memcpy(xi, P, sizeof P); memcpy(w, W, sizeof W); return 0;
  }
  {
    /* tensor Gauss rules, xi_1 fastest */
    double g2[2] = {-1.0 / sqrt(3.0), 1.0 / sqrt(3.0)}, w2[2] = {1.0, 1.0};
    double g3[3] = {-sqrt(0.6), 0.0, sqrt(0.6)}, w3[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    int m = (et == OR_Q1_2D || et == OR_Q1_3D) ? 2 : 3;
    double *g = m == 2 ? g2 : g3, *ww = m == 2 ? w2 : w3;
    if (dim == 2) {
      for (j = 0; j < m; ++j) for (i = 0; i < m; ++i, ++q) {
        xi[2 * q] = g[i]; xi[2 * q + 1] = g[j]; w[q] = ww[i] * ww[j];
      }
    } else {
      for (k = 0; k < m; ++k) for (j = 0; j < m; ++j) for (i = 0; i < m; ++i, ++q) {
        xi[3 * q] = g[i]; xi[3 * q + 1] = g[j]; xi[3 * q + 2] = g[k];
        w[q] = ww[i] * ww[j] * ww[k];
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Geometry: Jacobian, determinant, inverse, transformed gradients           */
/* (eq. Jacobian, Jacobian2, basis_derivative; WEIGHT = |det J| * omega)     */
/* ------------------------------------------------------------------------ */

/* Returns the number of integration points with det J <= 0 (0 = valid). */
int64_t or_geometry(int et, int64_t n_n, int64_t n_e, const double *coord,
                    const int32_t *elem, double *dphi, double *w) {
  int dim, n_p, n_q, q, p, i, j, k;
  int64_t e, bad = 0;
  double xi[27 * 3], wq[27], phi[27], dref[27][27 * 3];
  or_elem_info(et, &dim, &n_p, &n_q);
  or_quadrature(et, xi, wq);
  for (q = 0; q < n_q; ++q) or_basis(et, xi + dim * q, phi, dref[q]);
  for (e = 0; e < n_e; ++e) {
    for (q = 0; q < n_q; ++q) {
      double J[3][3] = {{0}}, Ji[3][3] = {{0}}, det;
      /* J_ij = d x_j / d xi_i = sum_p dphi_p/dxi_i * x_{p,j} */
      for (p = 0; p < n_p; ++p) {
        int64_t node = elem[e * n_p + p];
        for (i = 0; i < dim; ++i)
          for (j = 0; j < dim; ++j)
            J[i][j] += dref[q][dim * p + i] * coord[j * n_n + node];
      }
      if (dim == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        Ji[0][0] = J[1][1] / det;  Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
      } else {
        /* inverse by cofactors */
        det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
            - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
            + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        for (i = 0; i < 3; ++i)
          for (j = 0; j < 3; ++j) {
            int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
            Ji[i][j] = (J[r0][c0] * J[r1][c1] - J[r0][c1] * J[r1][c0]) / det;
          }
      }
      if (!(det > 0)) ++bad;
      w[e * n_q + q] = fabs(det) * wq[q];
      /* grad_x phi = J^{-1} grad_xi phi */
      for (p = 0; p < n_p; ++p)
        for (i = 0; i < dim; ++i) {
          double s = 0;
          for (k = 0; k < dim; ++k) s += Ji[i][k] * dref[q][dim * p + k];
          dphi[((e * n_q + q) * n_p + p) * dim + i] = s;
        }
    }
  }
  return bad;
}

/* ------------------------------------------------------------------------ */
/* Strain-displacement matrix B at one integration point (eq.               */
/* local_strain-displ).  3D: 6 x 3n_p, rows 11,22,33,12,23,13 (engineering  */
/* shears).  2D: 3 x 2n_p, rows 11,22,12.                                    */
/* ------------------------------------------------------------------------ */
static void build_B(int dim, int n_p, const double *g /*[n_p][dim]*/, double *B) {
  int p, ncol = dim * n_p;
  if (dim == 3) {
    memset(B, 0, sizeof(double) * 6 * ncol);
    for (p = 0; p < n_p; ++p) {
      double d1 = g[3 * p], d2 = g[3 * p + 1], d3 = g[3 * p + 2];
      int c = 3 * p;
      B[0 * ncol + c + 0] = d1;
      B[1 * ncol + c + 1] = d2;
      B[2 * ncol + c + 2] = d3;
      B[3 * ncol + c + 0] = d2; B[3 * ncol + c + 1] = d1;
      B[4 * ncol + c + 1] = d3; B[4 * ncol + c + 2] = d2;
      B[5 * ncol + c + 0] = d3; B[5 * ncol + c + 2] = d1;
    }
  } else {
    memset(B, 0, sizeof(double) * 3 * ncol);
    for (p = 0; p < n_p; ++p) {
      double d1 = g[2 * p], d2 = g[2 * p + 1];
      int c = 2 * p;
      B[0 * ncol + c + 0] = d1;
      B[1 * ncol + c + 1] = d2;
      B[2 * ncol + c + 0] = d2; B[2 * ncol + c + 1] = d1;
    }
  }
}

/* in-plane Voigt rows of the 6-vector for plane strain */
static const int PLANE[3] = {0, 1, 3};

/* E = B u at every integration point; eps [n_int][6]. */
void or_strain(int et, int64_t n_e, const int32_t *elem, const double *dphi,
               const double *u, double *eps) {
  int dim, n_p, n_q;
  int64_t e;
  or_elem_info(et, &dim, &n_p, &n_q);
#pragma omp parallel for schedule(static)
  for (e = 0; e < n_e; ++e) {
    int q, p, r, c;
    double B[6 * 81], ue[81];
    for (p = 0; p < n_p; ++p)
      for (c = 0; c < dim; ++c) ue[dim * p + c] = u[(int64_t)dim * elem[e * n_p + p] + c];
    for (q = 0; q < n_q; ++q) {
      int64_t ip = e * n_q + q;
      int nrow = dim == 3 ? 6 : 3;
      build_B(dim, n_p, dphi + ip * n_p * dim, B);
      for (r = 0; r < 6; ++r) eps[ip * 6 + r] = 0.0;
      for (r = 0; r < nrow; ++r) {
        double s = 0;
        for (c = 0; c < dim * n_p; ++c) s += B[r * dim * n_p + c] * ue[c];
        eps[ip * 6 + (dim == 3 ? r : PLANE[r])] = s;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Tensor helpers                                                            */
/* ------------------------------------------------------------------------ */
typedef double T2[3][3];
typedef double T4[3][3][3][3];
static const int VI[6] = {0, 1, 2, 0, 1, 0}, VJ[6] = {0, 1, 2, 1, 2, 2};

static void strain_voigt_to_tensor(const double *v, T2 t) {
  t[0][0] = v[0]; t[1][1] = v[1]; t[2][2] = v[2];
  t[0][1] = t[1][0] = 0.5 * v[3];
  t[1][2] = t[2][1] = 0.5 * v[4];
  t[0][2] = t[2][0] = 0.5 * v[5];
}
static void stress_voigt_to_tensor(const double *v, T2 t) {
  t[0][0] = v[0]; t[1][1] = v[1]; t[2][2] = v[2];
  t[0][1] = t[1][0] = v[3];
  t[1][2] = t[2][1] = v[4];
  t[0][2] = t[2][0] = v[5];
}
static void tensor_to_stress_voigt(T2 t, double *v) {
  int I;
  for (I = 0; I < 6; ++I) v[I] = t[VI[I]][VJ[I]];
}
static void tensor_to_strain_voigt(T2 t, double *v) {
  int I;
  for (I = 0; I < 6; ++I) v[I] = (I < 3 ? 1.0 : 2.0) * t[VI[I]][VJ[I]];
}
static double trace(T2 t) { return t[0][0] + t[1][1] + t[2][2]; }
static void deviator(T2 t, T2 d) {
  int i, j; double m = trace(t) / 3.0;
  for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) d[i][j] = t[i][j] - (i == j ? m : 0.0);
}
static double fnorm(T2 t) {
  int i, j; double s = 0;
  for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) s += t[i][j] * t[i][j];
  return sqrt(s);
}
static double kd(int i, int j) { return i == j ? 1.0 : 0.0; }
/* symmetric fourth-order identity, volumetric projector I (x) I, deviatoric */
static double Isym(int i, int j, int k, int l) { return 0.5 * (kd(i, k) * kd(j, l) + kd(i, l) * kd(j, k)); }
static double IIv(int i, int j, int k, int l) { return kd(i, j) * kd(k, l); }
static double IDev(int i, int j, int k, int l) { return Isym(i, j, k, l) - IIv(i, j, k, l) / 3.0; }

static void elastic_T4(double G, double K, T4 C) {
  int i, j, k, l;
  for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) for (k = 0; k < 3; ++k) for (l = 0; l < 3; ++l)
    C[i][j][k][l] = K * IIv(i, j, k, l) + 2.0 * G * IDev(i, j, k, l);
}
/* sigma = C eps = K tr(eps) I + 2G dev(eps)  (eq. elastic_law) */
static void elastic_stress(double G, double K, T2 e, T2 s) {
  int i, j; T2 d; double tr = trace(e);
  deviator(e, d);
  for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) s[i][j] = K * tr * kd(i, j) + 2.0 * G * d[i][j];
}
static void T4_to_voigt(T4 C, double *D) {
  int I, J;
  for (I = 0; I < 6; ++I) for (J = 0; J < 6; ++J) D[6 * I + J] = C[VI[I]][VJ[I]][VI[J]][VJ[J]];
}

/* ------------------------------------------------------------------------ */
/* Return maps (Section 2.2, 2.3; hardening extension of 2.3 below)          */
/* ------------------------------------------------------------------------ */

/* Von Mises yield criterion with linear kinematic hardening (eqs.
   T_kinematic, DT_kinematic, T_other).  Inputs per point: strain eps (strain
   Voigt), previous plastic strain ep (strain Voigt), previous back stress
   beta (stress Voigt).  Outputs: sigma (stress Voigt), D (6x6), flag
   (1 = plastic), updated ep and beta. */
static void rm_vm(double G, double K, double a, double Y,
                  const double *eps_v, const double *ep_v, const double *beta_v,
                  double *sig_v, double *D, uint8_t *flag, double *ep_out, double *beta_out,
                  double *crit_out) {
  T2 eps, ep, beta, etr, str, sdev, s, sig, n;
  T4 C;
  double ns, crit;
  int i, j, k, l;
  strain_voigt_to_tensor(eps_v, eps);
  strain_voigt_to_tensor(ep_v, ep);
  stress_voigt_to_tensor(beta_v, beta);
  for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) etr[i][j] = eps[i][j] - ep[i][j];
  elastic_stress(G, K, etr, str);            /* sigma_tr = C (eps - ep_prev) */
  deviator(str, sdev);
  for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) s[i][j] = sdev[i][j] - beta[i][j];
  ns = fnorm(s);
  crit = ns - Y;
  if (crit_out) { crit_out[0] = crit; crit_out[1] = 0.0; }
  elastic_T4(G, K, C);
  memcpy(sig, str, sizeof(T2));
  memcpy(ep_out, ep_v, 6 * sizeof(double));
  memcpy(beta_out, beta_v, 6 * sizeof(double));
  *flag = 0;
  if (crit > 0) {
    double dl = crit / (2.0 * G + a);
    double c1 = 4.0 * G * G / (2.0 * G + a);
    T2 epn, betan;
    for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) n[i][j] = s[i][j] / ns;
    for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) {
      sig[i][j] = str[i][j] - 2.0 * G * dl * n[i][j];
      epn[i][j] = ep[i][j] + dl * n[i][j];
      betan[i][j] = beta[i][j] + a * dl * n[i][j];
    }
    for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) for (k = 0; k < 3; ++k) for (l = 0; l < 3; ++l)
      C[i][j][k][l] += -c1 * IDev(i, j, k, l)
                       + c1 * (Y / ns) * (IDev(i, j, k, l) - n[i][j] * n[k][l]);
    tensor_to_strain_voigt(epn, ep_out);
    tensor_to_stress_voigt(betan, beta_out);
    *flag = 1;
  }
  tensor_to_stress_voigt(sig, sig_v);
  T4_to_voigt(C, D);
}

/* Drucker-Prager yield criterion (Section 2.3) with yield function
   Psi = |dev sigma|/sqrt(2) + eta*p - (c + a*kappa), p = tr(sigma)/3, and
   associated flow; a = 0 is the paper's perfect plasticity.  For a > 0 the
   cohesion hardens linearly with the accumulated multiplier kappa (the
   paper's framework with W = R and H(chi) = a*chi).  flag: 0 elastic,
   1 return to the smooth cone, 2 return to the apex.  At the tie the smooth
   branch is taken (smooth iff CRIT2 <= 0), as the paper's implementation of
   Section 2.3 decides; the text's inequalities leave the tie open. */
static void rm_dp(double G, double K, double a, double eta, double c,
                  const double *eps_v, const double *ep_v, double kappa,
                  double *sig_v, double *D, uint8_t *flag, double *ep_out, double *kappa_out,
                  double *crit_out) {
  T2 eps, ep, etr, str, s, sig, n, M, epn;
  T4 C;
  double ptr, rho, ck, crit1, crit2;
  int i, j, k, l;
  const double r2 = sqrt(2.0);
  strain_voigt_to_tensor(eps_v, eps);
  strain_voigt_to_tensor(ep_v, ep);
  for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) etr[i][j] = eps[i][j] - ep[i][j];
  elastic_stress(G, K, etr, str);
  ptr = trace(str) / 3.0;
  deviator(str, s);
  rho = fnorm(s);
  ck = c + a * kappa;
  crit1 = rho / r2 + eta * ptr - ck;
  crit2 = eta * ptr - ck - (K * eta * eta + a) * rho / (r2 * G);
  if (crit_out) { crit_out[0] = crit1; crit_out[1] = crit2; }
  elastic_T4(G, K, C);
  memcpy(sig, str, sizeof(T2));
  memcpy(ep_out, ep_v, 6 * sizeof(double));
  *kappa_out = kappa;
  *flag = 0;
  if (crit1 > 0 && crit2 <= 0) {
    double h = G + K * eta * eta + a;
    double dl = crit1 / h;
    for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) {
      n[i][j] = s[i][j] / rho;
      M[i][j] = r2 * G * n[i][j] + K * eta * kd(i, j);
    }
    for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) {
      sig[i][j] = str[i][j] - dl * M[i][j];
      epn[i][j] = ep[i][j] + dl * (n[i][j] / r2 + eta / 3.0 * kd(i, j));
    }
    for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) for (k = 0; k < 3; ++k) for (l = 0; l < 3; ++l)
      C[i][j][k][l] -= (2.0 * r2 * G * G * dl / rho) * (IDev(i, j, k, l) - n[i][j] * n[k][l])
                       + M[i][j] * M[k][l] / h;
    tensor_to_strain_voigt(epn, ep_out);
    *kappa_out = kappa + dl;
    *flag = 1;
  } else if (crit1 > 0 && crit2 > 0) {
    double dl = (eta * ptr - ck) / (K * eta * eta + a);
    double pk = ptr - K * eta * dl;
    for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) {
      sig[i][j] = pk * kd(i, j);
      epn[i][j] = eps[i][j] - pk / (3.0 * K) * kd(i, j);
    }
    for (i = 0; i < 3; ++i) for (j = 0; j < 3; ++j) for (k = 0; k < 3; ++k) for (l = 0; l < 3; ++l)
      C[i][j][k][l] = K * a / (K * eta * eta + a) * IIv(i, j, k, l);
    tensor_to_strain_voigt(epn, ep_out);
    *kappa_out = kappa + dl;
    *flag = 2;
  }
  tensor_to_stress_voigt(sig, sig_v);
  T4_to_voigt(C, D);
}

/* model: 1 = von Mises kinematic, 2 = Drucker-Prager (a >= 0).
   Any of the output pointers may be NULL.  crit[n][2] receives the yield
   tests the branch decisions are taken on: von Mises |s_tr| - Y (and 0);
   Drucker-Prager CRIT1 (trial yield function) and CRIT2 (the smooth / apex
   test). */
void or_constitutive_crit(int model, int64_t n, const double *eps, const double *ep,
                          const double *beta, const double *kappa,
                          double G, double K, double a, double Y, double eta, double c,
                          double *sig, double *D, uint8_t *flag,
                          double *ep_new, double *beta_new, double *kappa_new, double *crit) {
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < n; ++i) {
    double s[6], d[36], epn[6], bn[6], kn = 0;
    uint8_t f;
    double *cr = crit ? crit + 2 * i : NULL;
    if (model == 1) {
      rm_vm(G, K, a, Y, eps + 6 * i, ep + 6 * i, beta + 6 * i, s, d, &f, epn, bn, cr);
    } else {
      rm_dp(G, K, a, eta, c, eps + 6 * i, ep + 6 * i, kappa ? kappa[i] : 0.0, s, d, &f, epn, &kn,
            cr);
      memset(bn, 0, sizeof bn);
    }
    if (sig) memcpy(sig + 6 * i, s, sizeof s);
    if (D) memcpy(D + 36 * i, d, sizeof d);
    if (flag) flag[i] = f;
    if (ep_new) memcpy(ep_new + 6 * i, epn, sizeof epn);
    if (beta_new) memcpy(beta_new + 6 * i, bn, sizeof bn);
    if (kappa_new) kappa_new[i] = kn;
  }
}

void or_constitutive(int model, int64_t n, const double *eps, const double *ep,
                     const double *beta, const double *kappa,
                     double G, double K, double a, double Y, double eta, double c,
                     double *sig, double *D, uint8_t *flag,
                     double *ep_new, double *beta_new, double *kappa_new) {
  or_constitutive_crit(model, n, eps, ep, beta, kappa, G, K, a, Y, eta, c, sig, D, flag, ep_new,
                       beta_new, kappa_new, NULL);
}

/* ------------------------------------------------------------------------ */
/* Internal force  F = B^T (WEIGHT .* S)                                     */
/* ------------------------------------------------------------------------ */
void or_internal_force(int et, int64_t n_n, int64_t n_e, const int32_t *elem,
                       const double *dphi, const double *w, const double *sig, double *F) {
  int dim, n_p, n_q, nrow, nl;
  int64_t e, t;
  double *v;
  or_elem_info(et, &dim, &n_p, &n_q);
  nrow = dim == 3 ? 6 : 3;
  nl = dim * n_p;
  /* v[e][q][c] = w (B^T sigma)_c at point q of element e */
  v = (double *)malloc(sizeof(double) * (size_t)(n_e * n_q * nl > 0 ? n_e * n_q * nl : 1));
#pragma omp parallel for schedule(static)
  for (e = 0; e < n_e; ++e) {
    int q, r, c;
    double B[6 * 81];
    for (q = 0; q < n_q; ++q) {
      int64_t ip = e * n_q + q;
      build_B(dim, n_p, dphi + ip * n_p * dim, B);
      for (c = 0; c < nl; ++c) {
        double s = 0;
        for (r = 0; r < nrow; ++r)
          s += B[r * nl + c] * sig[ip * 6 + (dim == 3 ? r : PLANE[r])];
        v[ip * nl + c] = w[ip] * s;
      }
    }
  }
  /* node sums in element, point, local-dof order */
  memset(F, 0, sizeof(double) * dim * n_n);
  for (t = 0; t < n_e * n_q * nl; ++t) {
    int64_t ee = t / ((int64_t)n_q * nl);
    int c = (int)(t % nl);
    F[(int64_t)dim * elem[ee * n_p + c / dim] + c % dim] += v[t];
  }
  free(v);
}

/* ------------------------------------------------------------------------ */
/* Sparse pattern, position map, COO assembly                                */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t r, c, seq; double v; } trip;

static int cmp_rc(const void *A, const void *B) {
  const trip *a = A, *b = B;
  if (a->r != b->r) return a->r < b->r ? -1 : 1;
  if (a->c != b->c) return a->c < b->c ? -1 : 1;
  if (a->seq != b->seq) return a->seq < b->seq ? -1 : 1;
  return 0;
}

/* Pattern of sum_e (element dof pairs): the sorted set of (row, col) over
   every pair of dofs of a common element.  First call with col_idx == NULL
   returns nnz; second call fills row_ptr[n_dof+1] and col_idx[nnz]. */
int64_t or_pattern(int et, int64_t n_n, int64_t n_e, const int32_t *elem,
                   int32_t *row_ptr, int32_t *col_idx) {
  int dim, n_p, n_q, a, b, nl;
  int64_t e, m = 0, t, nnz = 0, n_dof;
  trip *T;
  or_elem_info(et, &dim, &n_p, &n_q);
  nl = dim * n_p;
  n_dof = dim * n_n;
  T = (trip *)malloc(sizeof(trip) * (size_t)(n_e * nl * nl));
  for (e = 0; e < n_e; ++e)
    for (a = 0; a < nl; ++a)
      for (b = 0; b < nl; ++b, ++m) {
        T[m].r = (int64_t)dim * elem[e * n_p + a / dim] + a % dim;
        T[m].c = (int64_t)dim * elem[e * n_p + b / dim] + b % dim;
        T[m].seq = 0; T[m].v = 0;
      }
  qsort(T, (size_t)m, sizeof(trip), cmp_rc);
  if (row_ptr) for (t = 0; t <= n_dof; ++t) row_ptr[t] = 0;
  for (t = 0; t < m; ++t) {
    if (t > 0 && T[t].r == T[t - 1].r && T[t].c == T[t - 1].c) continue;
    if (col_idx) { col_idx[nnz] = (int32_t)T[t].c; row_ptr[T[t].r + 1]++; }
    ++nnz;
  }
  if (row_ptr && col_idx) for (t = 0; t < n_dof; ++t) row_ptr[t + 1] += row_ptr[t];
  free(T);
  return nnz;
}

/* pos[e][a][b] = index of (dof(e,a), dof(e,b)) in col_idx, by binary search
   of the row. */
void or_position_map(int et, int64_t n_e, const int32_t *elem, const int32_t *row_ptr,
                     const int32_t *col_idx, int32_t *pos) {
  int dim, n_p, n_q, a, b, nl;
  int64_t e;
  or_elem_info(et, &dim, &n_p, &n_q);
  nl = dim * n_p;
  for (e = 0; e < n_e; ++e)
    for (a = 0; a < nl; ++a)
      for (b = 0; b < nl; ++b) {
        int64_t r = (int64_t)dim * elem[e * n_p + a / dim] + a % dim;
        int64_t c = (int64_t)dim * elem[e * n_p + b / dim] + b % dim;
        int64_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1, mid = -1;
        while (lo <= hi) {
          mid = (lo + hi) / 2;
          if (col_idx[mid] == c) break;
          if (col_idx[mid] < c) lo = mid + 1; else hi = mid - 1;
        }
        pos[(e * nl + a) * nl + b] = (col_idx[mid] == c) ? (int32_t)mid : -1;
      }
}

/* Element matrix  K_e = sum_q w_q B_q^T D_q B_q  with the dense B matrix.
   D is the 6x6 Voigt tangent per point; plane strain uses its in-plane
   rows/columns. */
static void element_matrix(int dim, int n_p, int n_q, const double *dphi_e,
                           const double *w_e, const double *D_e, double *Ke) {
  int q, r, s, a, b, nl = dim * n_p, nrow = dim == 3 ? 6 : 3;
  double B[6 * 81], DB[6 * 81];
  memset(Ke, 0, sizeof(double) * nl * nl);
  for (q = 0; q < n_q; ++q) {
    const double *Dq = D_e + 36 * q;
    build_B(dim, n_p, dphi_e + q * n_p * dim, B);
    for (r = 0; r < nrow; ++r)
      for (b = 0; b < nl; ++b) {
        double t = 0;
        for (s = 0; s < nrow; ++s) {
          int R = dim == 3 ? r : PLANE[r], S = dim == 3 ? s : PLANE[s];
          t += Dq[6 * R + S] * B[s * nl + b];
        }
        DB[r * nl + b] = t;
      }
    for (a = 0; a < nl; ++a)
      for (b = 0; b < nl; ++b) {
        double t = 0;
        for (r = 0; r < nrow; ++r) t += B[r * nl + a] * DB[r * nl + b];
        Ke[a * nl + b] += w_e[q] * t;
      }
  }
}

/* K = sum_e sum_q w B^T D B as COO triplets sorted by (row, col, order of
   generation) and summed in that order into the given pattern.  Returns 0,
   or -1 if a triplet falls outside the pattern. */
int or_assemble(int et, int64_t n_e, const int32_t *elem, const double *dphi,
                const double *w, const double *D, const int32_t *row_ptr,
                const int32_t *col_idx, double *val) {
  int dim, n_p, n_q, nl;
  int64_t e, m, t, k;
  trip *T;
  or_elem_info(et, &dim, &n_p, &n_q);
  nl = dim * n_p;
  T = (trip *)malloc(sizeof(trip) * (size_t)(n_e * nl * nl > 0 ? n_e * nl * nl : 1));
#pragma omp parallel for schedule(static)
  for (e = 0; e < n_e; ++e) {
    double Ke[81 * 81];
    int64_t mm = e * nl * nl;
    int a, b;
    element_matrix(dim, n_p, n_q, dphi + e * n_q * n_p * dim, w + e * n_q, D + e * n_q * 36, Ke);
    for (a = 0; a < nl; ++a)
      for (b = 0; b < nl; ++b, ++mm) {
        T[mm].r = (int64_t)dim * elem[e * n_p + a / dim] + a % dim;
        T[mm].c = (int64_t)dim * elem[e * n_p + b / dim] + b % dim;
        T[mm].seq = mm;
        T[mm].v = Ke[a * nl + b];
      }
  }
  m = n_e * nl * nl;
  qsort(T, (size_t)m, sizeof(trip), cmp_rc);
  k = -1;
  for (t = 0; t < m; ++t) {
    if (t == 0 || T[t].r != T[t - 1].r || T[t].c != T[t - 1].c) {
      /* next pattern entry of row r */
      int64_t r = T[t].r;
      if (k < row_ptr[r]) k = row_ptr[r]; else ++k;
      if (k >= row_ptr[r + 1] || col_idx[k] != T[t].c) { free(T); return -1; }
      val[k] = 0.0;
    }
    val[k] += T[t].v;
  }
  free(T);
  return 0;
}

/* Rows of K = sum w B^T D B, one at a time, for sampled checks on large
   meshes.  For each requested row r, the columns (sorted) and values are
   written at out_cols/out_vals + r_index*max_cols; out_n[r_index] holds the
   count.  Elements are found by scanning the connectivity. */
int or_K_rows(int et, int64_t n_e, const int32_t *elem, const double *dphi,
              const double *w, const double *D, int64_t n_rows, const int64_t *rows,
              int max_cols, int32_t *out_cols, double *out_vals, int32_t *out_n) {
  int dim, n_p, n_q, a, b, nl;
  int64_t e, ir;
  double *Ke;
  or_elem_info(et, &dim, &n_p, &n_q);
  nl = dim * n_p;
  Ke = (double *)malloc(sizeof(double) * nl * nl);
  for (ir = 0; ir < n_rows; ++ir) {
    int64_t r = rows[ir], node = r / dim;
    int comp = (int)(r % dim), n = 0, i, j;
    int32_t *cols = out_cols + ir * max_cols;
    double *vals = out_vals + ir * max_cols;
    for (e = 0; e < n_e; ++e) {
      int hit = -1;
      for (a = 0; a < n_p; ++a) if (elem[e * n_p + a] == node) hit = a;
      if (hit < 0) continue;
      element_matrix(dim, n_p, n_q, dphi + e * n_q * n_p * dim, w + e * n_q, D + e * n_q * 36, Ke);
      a = dim * hit + comp;
      for (b = 0; b < nl; ++b) {
        int32_t c = dim * elem[e * n_p + b / dim] + b % dim;
        /* insert into the sorted column list */
        for (i = 0; i < n && cols[i] < c; ++i) {}
        if (i < n && cols[i] == c) { vals[i] += Ke[a * nl + b]; continue; }
        if (n >= max_cols) { free(Ke); return -1; }
        for (j = n; j > i; --j) { cols[j] = cols[j - 1]; vals[j] = vals[j - 1]; }
        cols[i] = c; vals[i] = Ke[a * nl + b]; ++n;
      }
    }
    out_n[ir] = n;
  }
  free(Ke);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Jacobi-preconditioned CG on the free dofs (Dirichlet rows and columns     */
/* eliminated by the mask), x starts at 0.  Stops when |r| <= rtol*|b|.      */
/* Returns the iteration count, or -1 if max_it was reached.                 */
/* ------------------------------------------------------------------------ */
int or_pcg(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
           const uint8_t *free_dof, const double *b, double *x, double rtol, int max_it,
           double *relres) {
  double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
  double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
  double *dinv = malloc(sizeof(double) * n);
  double rz, bb = 0, rr;
  int64_t i, k;
  int it = 0;
  for (i = 0; i < n; ++i) {
    double d = 0;
    for (k = row_ptr[i]; k < row_ptr[i + 1]; ++k) if (col_idx[k] == i) d = val[k];
    dinv[i] = free_dof[i] ? 1.0 / d : 0.0;
    x[i] = 0; r[i] = free_dof[i] ? b[i] : 0.0;
    bb += r[i] * r[i];
  }
  bb = sqrt(bb);
  rz = 0; rr = 0;
  for (i = 0; i < n; ++i) { z[i] = dinv[i] * r[i]; p[i] = z[i]; rz += r[i] * z[i]; rr += r[i] * r[i]; }
  while (sqrt(rr) > rtol * bb && it < max_it) {
    double pq = 0, alpha, rzn = 0;
    for (i = 0; i < n; ++i) {
      double s = 0;
      if (free_dof[i])
        for (k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val[k] * p[col_idx[k]];
      q[i] = s; pq += p[i] * s;
    }
    alpha = rz / pq;
    rr = 0;
    for (i = 0; i < n; ++i) {
      x[i] += alpha * p[i]; r[i] -= alpha * q[i]; z[i] = dinv[i] * r[i];
      rzn += r[i] * z[i]; rr += r[i] * r[i];
    }
    for (i = 0; i < n; ++i) p[i] = z[i] + (rzn / rz) * p[i];
    rz = rzn;
    ++it;
  }
  if (relres) *relres = bb > 0 ? sqrt(rr) / bb : 0.0;
  free(r); free(z); free(p); free(q); free(dinv);
  return sqrt(rr) > rtol * bb ? -1 : it;
}
