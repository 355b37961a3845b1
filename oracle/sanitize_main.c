/*
 * Driver that runs every entry point of the oracle (sstep_oracle.c) on small
 * problems, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py compiles and runs it on the CPU).
 *
 * TEST INFRASTRUCTURE ONLY, like the oracle itself.  Exit status 0 when every
 * call returns the expected status; the sanitizers abort on a memory or
 * undefined-behaviour error.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int kind;
  int nx, ny, nz;
  int64_t n;
  const int32_t *rowptr;
  const int32_t *colind;
  const double *val;
  const double *k;
  double diag, off;
} orc_op;

typedef struct {
  int status, outer, cg_equiv;
  double true_rel;
  double *hist;
  int hist_cap, hist_len;
} orc_result;

typedef struct {
  int cap, len;
  double *vm, *alpha, *beta, *W, *P;
} orc_trace;

int64_t orc_stencil_nnz(int kind, int nx, int ny, int nz);
int64_t orc_csr_from_stencil(int kind, int nx, int ny, int nz, double diag, double off,
                             const double *k, int32_t *rowptr, int32_t *colind, double *val);
void orc_apply(const orc_op *A, const double *x, double *y);
void orc_diag(const orc_op *A, double *d);
int orc_pcg(const orc_op *A, int prec, const double *b, double *x, double rtol, int maxit,
            orc_result *res);
int orc_pfcg(const orc_op *A, int prec, const double *b, double *x, double rtol, int maxit,
             orc_result *res);
int orc_sstep(const orc_op *A, int prec, const double *b, double *x, int s, double rtol,
              int maxit, int fixed_outer, orc_result *res, orc_trace *tr);
int orc_sstep_cheb(const orc_op *A, int prec, const double *b, double *x, int s, double lo,
                   double hi, double rtol, int maxit, int fixed_outer, orc_result *res,
                   orc_trace *tr);
int orc_cheb_basis(const orc_op *A, int prec, const double *r, int s, double lo, double hi,
                   double *P);
int orc_mpk_cvm(const orc_op *A, int prec, const double *r, int s, double *P, double *vm);
int orc_sw(int s, const double *vm, const double *alpha_prev, const double *Wprev,
           double *beta, double *W, double *alpha);
int orc_spd_solve(int s, const double *W, double *c);
double orc_max_diag(const orc_op *A);
double orc_dot(int64_t n, const double *a, const double *b);

static int failures = 0;

static void expect(int cond, const char *what) {
  if (!cond) {
    fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

static void run_solvers(const orc_op *A, const char *name) {
  const int64_t n = A->n;
  double *b = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * n);
  double hist[4096];
  char what[160];
  for (int64_t i = 0; i < n; ++i) b[i] = sin(0.37 * (double)i) + 0.1;
  for (int prec = 0; prec <= 1; ++prec) {
    orc_result res = {0, 0, 0, 0.0, hist, 4096, 0};
    memset(x, 0, sizeof(double) * n);
    snprintf(what, sizeof what, "%s pcg prec %d", name, prec);
    expect(orc_pcg(A, prec, b, x, 1e-9, 4000, &res) == 0 && res.true_rel < 1e-8, what);
    memset(x, 0, sizeof(double) * n);
    snprintf(what, sizeof what, "%s pfcg prec %d", name, prec);
    expect(orc_pfcg(A, prec, b, x, 1e-9, 4000, &res) == 0 && res.true_rel < 1e-8, what);
    /* a block size the Krylov space allows converges on the larger grids */
    if (n >= 60) {
      memset(x, 0, sizeof(double) * n);
      snprintf(what, sizeof what, "%s sstep_cheb s 3 converges, prec %d", name, prec);
      const double hi3 = prec ? 2.0 : 2.0 * orc_max_diag(A);
      expect(orc_sstep_cheb(A, prec, b, x, 3, 0.0, hi3, 1e-8, 4000, 0, &res, NULL) == 0 &&
                 res.true_rel < 1e-7,
             what);
    }
    for (int s = 1; s <= 6; ++s) {
      double vm[32], tvm[4 * 32], tal[4 * 16], tbe[4 * 256], tW[4 * 256];
      orc_trace tr = {4, 0, tvm, tal, tbe, tW, NULL};
      /* tiny operators: a block larger than the Krylov space breaks down
       * (status 2) or stops at the iteration limit; s > n is rejected */
      memset(x, 0, sizeof(double) * n);
      snprintf(what, sizeof what, "%s sstep s %d prec %d", name, s, prec);
      const int st = orc_sstep(A, prec, b, x, s, 1e-8, 4000, 0, &res, &tr);
      expect(s > n ? st < 0 : (st >= 0 && st <= 2), what);
      memset(x, 0, sizeof(double) * n);
      snprintf(what, sizeof what, "%s sstep_cheb s %d prec %d", name, s, prec);
      const double hi = prec ? 2.0 : 2.0 * orc_max_diag(A);
      const int sc = orc_sstep_cheb(A, prec, b, x, s, 0.0, hi, 1e-8, 4000, 0, &res, &tr);
      expect(s > n ? sc < 0 : (sc >= 0 && sc <= 2), what);
      double *P = malloc(sizeof(double) * n * 2 * s);
      snprintf(what, sizeof what, "%s mpk_cvm / cheb_basis s %d", name, s);
      expect(orc_mpk_cvm(A, prec, b, s, P, vm) == 0 &&
                 orc_cheb_basis(A, prec, b, s, 0.0, hi, P) == 0,
             what);
      free(P);
    }
  }
  /* degenerate inputs: zero right-hand side, s > n, bad interval */
  orc_result res = {0, 0, 0, 0.0, hist, 4096, 0};
  memset(b, 0, sizeof(double) * n);
  memset(x, 0, sizeof(double) * n);
  snprintf(what, sizeof what, "%s zero rhs", name);
  expect(orc_sstep(A, 1, b, x, 2, 1e-8, 100, 0, &res, NULL) == 0 && x[0] == 0.0, what);
  snprintf(what, sizeof what, "%s s > n rejected", name);
  expect(n >= 16 || orc_sstep(A, 1, b, x, 16, 1e-8, 100, 0, &res, NULL) < 0, what);
  snprintf(what, sizeof what, "%s empty interval rejected", name);
  expect(orc_sstep_cheb(A, 1, b, x, 2, 1.0, 1.0, 1e-8, 100, 0, &res, NULL) < 0, what);
  free(b);
  free(x);
}

int main(void) {
  /* matrix-free stencils, including degenerate grid shapes */
  const int shapes[][4] = {{1, 9, 7, 1}, {2, 13, 11, 1}, {2, 1, 1, 5}, {3, 7, 6, 5}, {3, 1, 1, 3}};
  for (size_t t = 0; t < sizeof shapes / sizeof shapes[0]; ++t) {
    const int kind = shapes[t][0], nx = shapes[t][1], ny = shapes[t][2], nz = shapes[t][3];
    const double diag = kind == 1 ? 4.0 : kind == 2 ? 6.0 : 26.0;
    orc_op A = {kind, nx, ny, nz, (int64_t)nx * ny * nz, NULL, NULL, NULL, NULL, diag, -1.0};
    run_solvers(&A, "stencil");
    /* the same operator in CSR form */
    const int64_t nnz = orc_stencil_nnz(kind, nx, ny, nz);
    int32_t *rp = malloc(sizeof(int32_t) * (A.n + 1)), *ci = malloc(sizeof(int32_t) * nnz);
    double *va = malloc(sizeof(double) * nnz);
    expect(orc_csr_from_stencil(kind, nx, ny, nz, diag, -1.0, NULL, rp, ci, va) == nnz,
           "csr from stencil");
    orc_op C = {0, nx, ny, nz, A.n, rp, ci, va, NULL, 0.0, 0.0};
    run_solvers(&C, "csr");
    free(rp);
    free(ci);
    free(va);
  }
  /* variable coefficient */
  const int nx = 6, ny = 5, nz = 4;
  const int64_t n = nx * ny * nz;
  double *k = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n);
  for (int64_t i = 0; i < n; ++i) k[i] = exp(sin(0.7 * (double)i));
  orc_op V = {4, nx, ny, nz, n, NULL, NULL, NULL, k, 0.0, 0.0};
  orc_diag(&V, d);
  expect(d[0] > 0.0, "vark diagonal");
  run_solvers(&V, "vark");
  /* small dense algebra edge cases */
  double Wsing[4] = {1.0, 1.0, 1.0, 1.0}, c2[2] = {1.0, 2.0};
  expect(orc_spd_solve(2, Wsing, c2) == 1, "singular W is a breakdown");
  expect(orc_spd_solve(17, Wsing, c2) < 0, "s beyond the limit rejected");
  free(k);
  free(d);
  if (failures) {
    fprintf(stderr, "%d failure(s)\n", failures);
    return 1;
  }
  printf("oracle sanitizer run: all entry points ok\n");
  return 0;
}
