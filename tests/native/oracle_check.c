/*
 * Runs every entry point of the C oracle once on the inputs of one binary
 * file and writes every output to another, so that a build with
 * AddressSanitizer / UndefinedBehaviorSanitizer can be driven from a test
 * and its outputs compared with the regular build's.
 *   usage: oracle_check IN OUT
 * IN:  int32 et, model; int64 n_n, n_e, n_rows; double G, K, a, Y, eta, c;
 *      double coord[dim][n_n]; int32 elem[n_e][n_p]; double u[dim n_n];
 *      uint8 free[dim n_n]; double ep[n_int][6], beta[n_int][6],
 *      kappa[n_int]; int64 rows[n_rows]
 * OUT: the outputs in the order of the calls below.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_elem_info(int et, int *dim, int *n_p, int *n_q);
int64_t or_geometry(int et, int64_t n_n, int64_t n_e, const double *coord, const int32_t *elem,
                    double *dphi, double *w);
void or_strain(int et, int64_t n_e, const int32_t *elem, const double *dphi, const double *u,
               double *eps);
void or_constitutive_crit(int model, int64_t n, const double *eps, const double *ep,
                          const double *beta, const double *kappa, double G, double K, double a,
                          double Y, double eta, double c, double *sig, double *D, uint8_t *flag,
                          double *ep_new, double *beta_new, double *kappa_new, double *crit);
void or_internal_force(int et, int64_t n_n, int64_t n_e, const int32_t *elem,
                       const double *dphi, const double *w, const double *sig, double *F);
int64_t or_pattern(int et, int64_t n_n, int64_t n_e, const int32_t *elem, int32_t *row_ptr,
                   int32_t *col_idx);
void or_position_map(int et, int64_t n_e, const int32_t *elem, const int32_t *row_ptr,
                     const int32_t *col_idx, int32_t *pos);
int or_assemble(int et, int64_t n_e, const int32_t *elem, const double *dphi, const double *w,
                const double *D, const int32_t *row_ptr, const int32_t *col_idx, double *val);
int or_K_rows(int et, int64_t n_e, const int32_t *elem, const double *dphi, const double *w,
              const double *D, int64_t n_rows, const int64_t *rows, int max_cols,
              int32_t *out_cols, double *out_vals, int32_t *out_n);
int or_pcg(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
           const uint8_t *free_dof, const double *b, double *x, double rtol, int max_it,
           double *relres);

static FILE *fin, *fout;
static void *rd(size_t size, size_t n) {
  void *p = malloc(size * (n ? n : 1));
  if (!p || fread(p, size, n, fin) != n) { fprintf(stderr, "short input\n"); exit(3); }
  return p;
}
static void *zalloc(size_t size, size_t n) { return calloc(n ? n : 1, size); }
static void wr(const void *p, size_t size, size_t n) {
  if (fwrite(p, size, n, fout) != n) { fprintf(stderr, "write failed\n"); exit(3); }
}

int main(int argc, char **argv) {
  int32_t *hdr, *elem, *row_ptr, *col_idx, *pos, *out_cols, *out_n, rc;
  int64_t *sizes, *rows, n_n, n_e, n_rows, n_int, n_dof, nnz, bad;
  double *par, *coord, *u, *ep, *beta, *kappa, *dphi, *w, *eps, *sig, *D, *epn, *bn, *kn, *crit;
  double *F, *val, *out_vals, *x, relres;
  uint8_t *free_dof, *flag;
  int dim, n_p, n_q, max_cols = 3 * 125 * 2, it;
  if (argc != 3 || !(fin = fopen(argv[1], "rb")) || !(fout = fopen(argv[2], "wb"))) return 2;
  hdr = rd(4, 2);
  sizes = rd(8, 3);
  n_n = sizes[0]; n_e = sizes[1]; n_rows = sizes[2];
  par = rd(8, 6);
  if (or_elem_info(hdr[0], &dim, &n_p, &n_q) != 0) {
    fprintf(stderr, "unknown element type %d\n", hdr[0]);
    free(hdr); free(sizes); free(par);
    return 2;
  }
  n_int = n_e * n_q;
  n_dof = dim * n_n;
  coord = rd(8, dim * n_n);
  elem = rd(4, n_e * n_p);
  u = rd(8, n_dof);
  free_dof = rd(1, n_dof);
  ep = rd(8, 6 * n_int);
  beta = rd(8, 6 * n_int);
  kappa = rd(8, n_int);
  rows = rd(8, n_rows);

  dphi = zalloc(8, n_int * n_p * dim);
  w = zalloc(8, n_int);
  bad = or_geometry(hdr[0], n_n, n_e, coord, elem, dphi, w);
  wr(&bad, 8, 1); wr(dphi, 8, n_int * n_p * dim); wr(w, 8, n_int);

  eps = zalloc(8, 6 * n_int);
  or_strain(hdr[0], n_e, elem, dphi, u, eps);
  wr(eps, 8, 6 * n_int);

  sig = zalloc(8, 6 * n_int); D = zalloc(8, 36 * n_int); flag = zalloc(1, n_int);
  epn = zalloc(8, 6 * n_int); bn = zalloc(8, 6 * n_int); kn = zalloc(8, n_int);
  crit = zalloc(8, 2 * n_int);
  or_constitutive_crit(hdr[1], n_int, eps, ep, beta, kappa, par[0], par[1], par[2], par[3],
                       par[4], par[5], sig, D, flag, epn, bn, kn, crit);
  wr(sig, 8, 6 * n_int); wr(D, 8, 36 * n_int); wr(flag, 1, n_int);
  wr(epn, 8, 6 * n_int); wr(bn, 8, 6 * n_int); wr(kn, 8, n_int); wr(crit, 8, 2 * n_int);

  F = zalloc(8, n_dof);
  or_internal_force(hdr[0], n_n, n_e, elem, dphi, w, sig, F);
  wr(F, 8, n_dof);

  nnz = or_pattern(hdr[0], n_n, n_e, elem, NULL, NULL);
  row_ptr = zalloc(4, n_dof + 1);
  col_idx = zalloc(4, nnz);
  or_pattern(hdr[0], n_n, n_e, elem, row_ptr, col_idx);
  wr(&nnz, 8, 1); wr(row_ptr, 4, n_dof + 1); wr(col_idx, 4, nnz);

  pos = zalloc(4, n_e * (dim * n_p) * (dim * n_p));
  or_position_map(hdr[0], n_e, elem, row_ptr, col_idx, pos);
  wr(pos, 4, n_e * (dim * n_p) * (dim * n_p));

  val = zalloc(8, nnz);
  rc = or_assemble(hdr[0], n_e, elem, dphi, w, D, row_ptr, col_idx, val);
  wr(&rc, 4, 1); wr(val, 8, nnz);

  out_cols = zalloc(4, n_rows * max_cols);
  out_vals = zalloc(8, n_rows * max_cols);
  out_n = zalloc(4, n_rows);
  rc = or_K_rows(hdr[0], n_e, elem, dphi, w, D, n_rows, rows, max_cols, out_cols, out_vals, out_n);
  wr(&rc, 4, 1); wr(out_n, 4, n_rows); wr(out_cols, 4, n_rows * max_cols);
  wr(out_vals, 8, n_rows * max_cols);

  x = zalloc(8, n_dof);
  it = or_pcg(n_dof, row_ptr, col_idx, val, free_dof, F, x, 1e-10, 100000, &relres);
  wr(&it, 4, 1); wr(&relres, 8, 1); wr(x, 8, n_dof);

  free(hdr); free(sizes); free(par); free(coord); free(elem); free(u); free(free_dof);
  free(ep); free(beta); free(kappa); free(rows); free(dphi); free(w); free(eps); free(sig);
  free(D); free(flag); free(epn); free(bn); free(kn); free(crit); free(F); free(row_ptr);
  free(col_idx); free(pos); free(val); free(out_cols); free(out_vals); free(out_n); free(x);
  fclose(fin);
  fclose(fout);
  return 0;
}
