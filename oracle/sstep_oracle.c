/*
 * Plain FP64 CPU oracle for the preconditioned s-step (Chronopoulos-Gear)
 * conjugate gradient method and its standard-CG comparator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or helper with the
 * HIP library.
 *
 * Everything is IEEE double, round to nearest, built without -ffast-math and
 * with -ffp-contract=off.  Inner products use fixed 4096-row chunks summed in
 * row order, and the chunk partials are combined pairwise in a fixed order, so
 * results do not depend on the OpenMP thread count.
 *
 * Paper: Bernaschi, Carrozzo, Celestini, Piperno, D'Ambra, "Communication-
 * reduced Conjugate Gradient Variants for GPU-accelerated Clusters",
 * Euromicro PDP 2025 (arXiv 2501.03743).
 *   Alg. 1  PCG-HS                      -> orc_pcg
 *   Alg. 2  PFCG (one reduction a step) -> orc_pfcg
 *   Alg. 3  PCGs (outer loop)           -> orc_sstep
 *   Alg. 4  pMPK (matrix powers)        -> mpk()
 *   Alg. 5  cvm (2s moments)            -> cvm()
 *   Alg. 6  SW (alpha, beta, W)         -> sw()
 *   Sec. II-A, eq. (3)  W alpha = m     -> chol_solve()
 *
 * Readings taken where the paper is silent or garbled (each is listed with
 * its reason in the design notes of the repository):
 *   - stop when ||r||_2 <= rtol ||b||_2, on the recursive residual, tested
 *     once per outer iteration (Alg. 3 tests ||r|| < rtol; Sec. V says the
 *     relative residual is used);
 *   - maxit counts CG-equivalent steps, the outer limit is ceil(maxit/s);
 *   - the loop that fills b1 in Alg. 6 runs over the full s x s index range
 *     (the printed bound j=1:i-1 would drop entries of the symmetric matrix
 *     P_{i-1}^T A Z_i and lose conjugacy);
 *   - the "2s x 2s" moment matrix of Sec. II-A is the s x s Hankel matrix
 *     W(i,j) = vm(i+j) that Alg. 3 and Alg. 6 build;
 *   - the s x s SPD systems are solved by an unpivoted Cholesky factorisation
 *     of the lower triangle; the factor of W_{i-1} is reused for beta;
 *     a pivot (before the square root) <= s * 2^-52 * |W_jj| or a non-finite
 *     value is a breakdown, and so is |alpha_{i-1}(s)| <= 1e-300;
 *   - with P1 = 0 at k = 0 (Alg. 3) the P_{i-1} beta terms are skipped;
 *   - Alg. 2 returns the newest iterate x_{k+1} (the one whose residual passed
 *     the test), counts every step including the one before its loop against
 *     maxit, and reports a breakdown when rho_k is not positive or a step
 *     length is not finite.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_CHUNK 4096
#define ORC_SMAX 16

/* Operator kinds. */
#define ORC_OP_CSR 0
#define ORC_OP_2D5 1
#define ORC_OP_3D7 2
#define ORC_OP_3D27 3
#define ORC_OP_3D7_VARK 4

/* Status codes (same meaning as the library's, defined independently). */
#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_BREAKDOWN 2
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* Preconditioners. */
#define ORC_PREC_NONE 0
#define ORC_PREC_JACOBI 1

typedef struct {
  int kind;
  int nx, ny, nz;          /* grid sizes (stencils); nz = 1 for 2D */
  int64_t n;               /* number of unknowns */
  const int32_t *rowptr;   /* CSR: n+1 entries */
  const int32_t *colind;   /* CSR: nnz entries, ascending within a row */
  const double *val;       /* CSR: nnz entries */
  const double *k;         /* 3D7_VARK: cell coefficient, n entries */
  double diag, off;        /* constant stencils: diagonal and off-diagonal */
} orc_op;

typedef struct {
  int status;
  int outer;               /* outer iterations done (PCG: iterations) */
  int cg_equiv;            /* s * outer */
  double true_rel;         /* ||b - A x||_2 / ||b||_2 at exit */
  double *hist;            /* ||r_i||_2/||b||_2, entry 0 = initial residual */
  int hist_cap;
  int hist_len;
} orc_result;

typedef struct {
  int cap;                 /* outer iterations that fit in the buffers */
  int len;                 /* outer iterations recorded */
  double *vm;              /* cap x 2s   moments vm(1..2s) */
  double *alpha;           /* cap x s */
  double *beta;            /* cap x s*s  beta(l,j) at [l*s+j] (zero at k=0) */
  double *W;               /* cap x s*s  W_i used for alpha_i */
  double *P;               /* NULL or cap x 2s x n: [P_i | A P_i] after update,
                              column-major (column c at offset c*n) */
} orc_trace;

/* ------------------------------------------------------------------------ */
/* Deterministic inner products                                              */
/* ------------------------------------------------------------------------ */

static double pairwise_sum(const double *p, int64_t m) {
  if (m == 1) return p[0];
  int64_t h = m / 2;
  double a = pairwise_sum(p, h);
  double b = pairwise_sum(p + h, m - h);
  return a + b;
}

double orc_dot(int64_t n, const double *a, const double *b) {
  if (n <= 0) return 0.0;
  int64_t nch = (n + ORC_CHUNK - 1) / ORC_CHUNK;
  double *part = (double *)malloc((size_t)nch * sizeof(double));
  if (!part) return NAN;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nch; ++c) {
    int64_t lo = c * ORC_CHUNK, hi = lo + ORC_CHUNK;
    if (hi > n) hi = n;
    double acc = 0.0;
    for (int64_t i = lo; i < hi; ++i) acc += a[i] * b[i];
    part[c] = acc;
  }
  double r = pairwise_sum(part, nch);
  free(part);
  return r;
}

static double nrm2(int64_t n, const double *a) { return sqrt(orc_dot(n, a, a)); }

/* ------------------------------------------------------------------------ */
/* Operators                                                                 */
/* ------------------------------------------------------------------------ */

/* Harmonic mean of two cell coefficients: the face weight of the
 * variable-coefficient 7-point operator for -div(k grad u). */
static double face_w(double kp, double kq) { return 2.0 * kp * kq / (kp + kq); }

/* Number of stored entries of the stencil operator in CSR form. */
int64_t orc_stencil_nnz(int kind, int nx, int ny, int nz) {
  int64_t cnt = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        if (kind == ORC_OP_2D5 || kind == ORC_OP_3D7 || kind == ORC_OP_3D7_VARK) {
          cnt += 1 + (x > 0) + (x < nx - 1) + (y > 0) + (y < ny - 1);
          if (kind != ORC_OP_2D5) cnt += (z > 0) + (z < nz - 1);
        } else if (kind == ORC_OP_3D27) {
          int cx = 1 + (x > 0) + (x < nx - 1);
          int cy = 1 + (y > 0) + (y < ny - 1);
          int cz = 1 + (z > 0) + (z < nz - 1);
          cnt += (int64_t)cx * cy * cz;
        }
      }
  return cnt;
}

/* Builds the stencil operator in CSR form with ascending column indices in
 * each row; lexicographic unknown index x + nx*(y + ny*z); Dirichlet zero
 * outside the grid (neighbours outside are dropped).  Returns nnz or -1. */
int64_t orc_csr_from_stencil(int kind, int nx, int ny, int nz, double diag,
                             double off, const double *k, int32_t *rowptr,
                             int32_t *colind, double *val) {
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  if (kind == ORC_OP_2D5 && nz != 1) return -1;
  int64_t e = 0, row = 0;
  rowptr[0] = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x, ++row) {
        int64_t p = row;
        if (kind == ORC_OP_3D27) {
          for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx) {
                int qx = x + dx, qy = y + dy, qz = z + dz;
                if (qx < 0 || qx >= nx || qy < 0 || qy >= ny || qz < 0 || qz >= nz) continue;
                colind[e] = (int32_t)(qx + (int64_t)nx * (qy + (int64_t)ny * qz));
                val[e] = (dx == 0 && dy == 0 && dz == 0) ? diag : off;
                ++e;
              }
        } else {
          /* 5/7-point: neighbours in ascending index order: -z, -y, -x, self, +x, +y, +z */
          int is3d = (kind != ORC_OP_2D5);
          int64_t sy = nx, sz = (int64_t)nx * ny;
          int64_t nb[7];
          int ok[7];
          nb[0] = p - sz; ok[0] = is3d && z > 0;
          nb[1] = p - sy; ok[1] = y > 0;
          nb[2] = p - 1;  ok[2] = x > 0;
          nb[3] = p;      ok[3] = 1;
          nb[4] = p + 1;  ok[4] = x < nx - 1;
          nb[5] = p + sy; ok[5] = y < ny - 1;
          nb[6] = p + sz; ok[6] = is3d && z < nz - 1;
          if (kind == ORC_OP_3D7_VARK) {
            /* six faces; a face to the boundary has weight k_p */
            double kp = k[p];
            double dsum = 0.0;
            int inside[6] = {z > 0, y > 0, x > 0, x < nx - 1, y < ny - 1, z < nz - 1};
            int64_t q[6] = {p - sz, p - sy, p - 1, p + 1, p + sy, p + sz};
            double w[6];
            for (int f = 0; f < 6; ++f) {
              w[f] = inside[f] ? face_w(kp, k[q[f]]) : kp;
              dsum += w[f];
            }
            /* emit in ascending order: faces 0..2, diagonal, faces 3..5 */
            for (int f = 0; f < 3; ++f)
              if (inside[f]) { colind[e] = (int32_t)q[f]; val[e] = -w[f]; ++e; }
            colind[e] = (int32_t)p; val[e] = dsum; ++e;
            for (int f = 3; f < 6; ++f)
              if (inside[f]) { colind[e] = (int32_t)q[f]; val[e] = -w[f]; ++e; }
          } else {
            for (int t = 0; t < 7; ++t) {
              if (!ok[t]) continue;
              colind[e] = (int32_t)nb[t];
              val[e] = (t == 3) ? diag : off;
              ++e;
            }
          }
        }
        rowptr[row + 1] = (int32_t)e;
      }
  return e;
}

/* y = A x for any operator kind.  Matrix-free for the stencil kinds. */
void orc_apply(const orc_op *A, const double *x, double *y) {
  int64_t n = A->n;
  if (A->kind == ORC_OP_CSR) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int32_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e)
        acc += A->val[e] * x[A->colind[e]];
      y[i] = acc;
    }
    return;
  }
  int nx = A->nx, ny = A->ny, nz = A->nz;
  int64_t sy = nx, sz = (int64_t)nx * ny;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < n; ++p) {
    int x0 = (int)(p % nx);
    int y0 = (int)((p / nx) % ny);
    int z0 = (int)(p / sz);
    double acc;
    if (A->kind == ORC_OP_3D27) {
      double nbsum = 0.0;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0 && dz == 0) continue;
            int qx = x0 + dx, qy = y0 + dy, qz = z0 + dz;
            if (qx < 0 || qx >= nx || qy < 0 || qy >= ny || qz < 0 || qz >= nz) continue;
            nbsum += x[qx + sy * qy + sz * qz];
          }
      acc = A->diag * x[p] + A->off * nbsum;
    } else if (A->kind == ORC_OP_3D7_VARK) {
      double kp = A->k[p];
      int inside[6] = {z0 > 0, y0 > 0, x0 > 0, x0 < nx - 1, y0 < ny - 1, z0 < nz - 1};
      int64_t q[6] = {p - sz, p - sy, p - 1, p + 1, p + sy, p + sz};
      double dsum = 0.0, nbsum = 0.0;
      for (int f = 0; f < 6; ++f) {
        if (inside[f]) {
          double w = face_w(kp, A->k[q[f]]);
          dsum += w;
          nbsum += w * x[q[f]];
        } else {
          dsum += kp;
        }
      }
      acc = dsum * x[p] - nbsum;
    } else {
      int is3d = (A->kind == ORC_OP_3D7);
      double nbsum = 0.0;
      if (x0 > 0) nbsum += x[p - 1];
      if (x0 < nx - 1) nbsum += x[p + 1];
      if (y0 > 0) nbsum += x[p - sy];
      if (y0 < ny - 1) nbsum += x[p + sy];
      if (is3d && z0 > 0) nbsum += x[p - sz];
      if (is3d && z0 < nz - 1) nbsum += x[p + sz];
      acc = A->diag * x[p] + A->off * nbsum;
    }
    y[p] = acc;
  }
}

/* Diagonal of the operator (for the Jacobi preconditioner B = diag(A)). */
static void op_diag(const orc_op *A, double *d) {
  int64_t n = A->n;
  if (A->kind == ORC_OP_CSR) {
    for (int64_t i = 0; i < n; ++i) {
      d[i] = 0.0;
      for (int32_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e)
        if (A->colind[e] == i) d[i] += A->val[e];
    }
  } else if (A->kind == ORC_OP_3D7_VARK) {
    int nx = A->nx, ny = A->ny, nz = A->nz;
    int64_t sy = nx, sz = (int64_t)nx * ny;
    for (int64_t p = 0; p < n; ++p) {
      int x0 = (int)(p % nx), y0 = (int)((p / nx) % ny), z0 = (int)(p / sz);
      int inside[6] = {z0 > 0, y0 > 0, x0 > 0, x0 < nx - 1, y0 < ny - 1, z0 < nz - 1};
      int64_t q[6] = {p - sz, p - sy, p - 1, p + 1, p + sy, p + sz};
      double kp = A->k[p], dsum = 0.0;
      for (int f = 0; f < 6; ++f) dsum += inside[f] ? face_w(kp, A->k[q[f]]) : kp;
      d[p] = dsum;
    }
  } else {
    for (int64_t i = 0; i < n; ++i) d[i] = A->diag;
  }
}

void orc_diag(const orc_op *A, double *d) { op_diag(A, d); }

/* u = B^{-1} v.  B = I (no preconditioner) or B = diag(A) (Jacobi). */
static void prec_apply(int prec, int64_t n, const double *dinv, const double *v, double *u) {
  if (prec == ORC_PREC_JACOBI) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) u[i] = dinv[i] * v[i];
  } else {
    if (u != v) memcpy(u, v, (size_t)n * sizeof(double));
  }
}

static void residual(const orc_op *A, const double *b, const double *x, double *r, double *tmp) {
  orc_apply(A, x, tmp);
  for (int64_t i = 0; i < A->n; ++i) r[i] = b[i] - tmp[i];
}

static void hist_push(orc_result *res, double v) {
  if (res->hist && res->hist_len < res->hist_cap) res->hist[res->hist_len] = v;
  res->hist_len++;
}

static int op_check(const orc_op *A) {
  if (!A || A->n < 0) return 0;
  if (A->kind == ORC_OP_CSR) return A->rowptr && A->colind && A->val;
  if (A->kind == ORC_OP_3D7_VARK) return A->k != NULL;
  return A->kind >= ORC_OP_2D5 && A->kind <= ORC_OP_3D27;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1: preconditioned CG (Hestenes-Stiefel form)                        */
/* ------------------------------------------------------------------------ */

int orc_pcg(const orc_op *A, int prec, const double *b, double *x, double rtol,
            int maxit, orc_result *res) {
  res->status = ORC_EINVAL;
  res->outer = res->cg_equiv = 0;
  res->hist_len = 0;
  res->true_rel = NAN;
  if (!op_check(A) || maxit < 0) return ORC_EINVAL;
  int64_t n = A->n;
  double *r = malloc((size_t)n * sizeof(double));
  double *u = malloc((size_t)n * sizeof(double));
  double *p = malloc((size_t)n * sizeof(double));
  double *sv = malloc((size_t)n * sizeof(double));
  double *dinv = malloc((size_t)n * sizeof(double));
  if (!r || !u || !p || !sv || !dinv) {
    free(r); free(u); free(p); free(sv); free(dinv);
    res->status = ORC_ENOMEM;
    return ORC_ENOMEM;
  }
  op_diag(A, dinv);
  for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / dinv[i];

  double bn = nrm2(n, b);
  int status = ORC_NOT_CONVERGED;
  if (bn == 0.0) {
    memset(x, 0, (size_t)n * sizeof(double));
    hist_push(res, 0.0);
    res->status = ORC_OK;
    res->true_rel = 0.0;
    free(r); free(u); free(p); free(sv); free(dinv);
    return ORC_OK;
  }
  residual(A, b, x, r, sv);                 /* r0 = b - A x0 */
  double rn = nrm2(n, r);
  hist_push(res, rn / bn);
  int it = 0;
  if (rn <= rtol * bn) {
    status = ORC_OK;
  } else {
    prec_apply(prec, n, dinv, r, u);        /* u0 = B^{-1} r0 */
    memcpy(p, u, (size_t)n * sizeof(double)); /* p0 = u0 */
    double ur = orc_dot(n, u, r);
    for (int k = 0; k < maxit; ++k) {
      orc_apply(A, p, sv);                  /* s_k = A p_k */
      double ps = orc_dot(n, p, sv);
      double alpha = ur / ps;               /* alpha_k = u_k^T r_k / p_k^T s_k */
      if (!(ps > 0.0) || !isfinite(alpha)) { status = ORC_BREAKDOWN; break; }
      for (int64_t i = 0; i < n; ++i) x[i] += alpha * p[i];
      for (int64_t i = 0; i < n; ++i) r[i] -= alpha * sv[i];
      prec_apply(prec, n, dinv, r, u);      /* u_{k+1} = B^{-1} r_{k+1} */
      double ur_new = orc_dot(n, u, r);
      double beta = ur_new / ur;            /* beta_k */
      for (int64_t i = 0; i < n; ++i) p[i] = u[i] + beta * p[i];
      ur = ur_new;
      it = k + 1;
      rn = nrm2(n, r);
      hist_push(res, rn / bn);
      if (rn <= rtol * bn) { status = ORC_OK; break; }
    }
  }
  residual(A, b, x, r, sv);
  res->true_rel = nrm2(n, r) / bn;
  res->outer = it;
  res->cg_equiv = it;
  res->status = status;
  free(r); free(u); free(p); free(sv); free(dinv);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2: flexible PCG with one global reduction per step (PFCG)            */
/* ------------------------------------------------------------------------ */

int orc_pfcg(const orc_op *A, int prec, const double *b, double *x, double rtol,
             int maxit, orc_result *res) {
  res->status = ORC_EINVAL;
  res->outer = res->cg_equiv = 0;
  res->hist_len = 0;
  res->true_rel = NAN;
  if (!op_check(A) || maxit < 0) return ORC_EINVAL;
  int64_t n = A->n;
  double *r = malloc((size_t)n * sizeof(double));
  double *u = malloc((size_t)n * sizeof(double));
  double *p = malloc((size_t)n * sizeof(double));
  double *w = malloc((size_t)n * sizeof(double));
  double *sv = malloc((size_t)n * sizeof(double));
  double *dinv = malloc((size_t)n * sizeof(double));
  if (!r || !u || !p || !w || !sv || !dinv) {
    free(r); free(u); free(p); free(w); free(sv); free(dinv);
    res->status = ORC_ENOMEM;
    return ORC_ENOMEM;
  }
  op_diag(A, dinv);
  for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / dinv[i];

  double bn = nrm2(n, b);
  if (bn == 0.0) {
    memset(x, 0, (size_t)n * sizeof(double));
    hist_push(res, 0.0);
    res->status = ORC_OK;
    res->true_rel = 0.0;
    free(r); free(u); free(p); free(w); free(sv); free(dinv);
    return ORC_OK;
  }
  int status = ORC_NOT_CONVERGED;
  residual(A, b, x, r, w);                  /* r_0 = b - A x_0 */
  double rn = nrm2(n, r);
  hist_push(res, rn / bn);
  int it = 0;
  if (rn <= rtol * bn) {
    status = ORC_OK;
  } else if (maxit > 0) {
    /* the step before the loop */
    prec_apply(prec, n, dinv, r, u);        /* u_0 = p_0 = B^{-1} r_0 */
    memcpy(p, u, (size_t)n * sizeof(double));
    orc_apply(A, u, w);                     /* w_0 = s_0 = A u_0 */
    memcpy(sv, w, (size_t)n * sizeof(double));
    double alpha = orc_dot(n, u, r);        /* alpha_0 = u_0^T r_0 */
    double rho = orc_dot(n, p, sv);         /* beta_0 = rho_0 = p_0^T s_0 */
    double step = alpha / rho;
    if (!(rho > 0.0) || !isfinite(step)) {
      status = ORC_BREAKDOWN;
    } else {
      for (int64_t i = 0; i < n; ++i) x[i] += step * p[i];    /* x_1 */
      for (int64_t i = 0; i < n; ++i) r[i] -= step * sv[i];   /* r_1 */
      it = 1;
      rn = nrm2(n, r);
      hist_push(res, rn / bn);
      if (rn <= rtol * bn) status = ORC_OK;
      for (int k = 1; k < maxit && status == ORC_NOT_CONVERGED; ++k) {
        prec_apply(prec, n, dinv, r, u);    /* u_k = B^{-1} r_k */
        orc_apply(A, u, w);                 /* w_k = A u_k */
        alpha = orc_dot(n, u, r);           /* alpha_k = u_k^T r_k */
        double beta = orc_dot(n, u, w);     /* beta_k = u_k^T w_k */
        double gamma = orc_dot(n, u, sv);   /* gamma_k = u_k^T s_{k-1} */
        double rho_k = beta - gamma * gamma / rho;
        double g = gamma / rho;             /* gamma_k / rho_{k-1} */
        step = alpha / rho_k;               /* alpha_k / rho_k */
        if (!(rho_k > 0.0) || !isfinite(step) || !isfinite(g)) {
          status = ORC_BREAKDOWN;
          break;
        }
        for (int64_t i = 0; i < n; ++i) p[i] = u[i] - g * p[i];     /* p_k */
        for (int64_t i = 0; i < n; ++i) x[i] += step * p[i];        /* x_{k+1} */
        for (int64_t i = 0; i < n; ++i) sv[i] = w[i] - g * sv[i];   /* s_k */
        for (int64_t i = 0; i < n; ++i) r[i] -= step * sv[i];       /* r_{k+1} */
        rho = rho_k;
        it = k + 1;
        rn = nrm2(n, r);
        hist_push(res, rn / bn);
        if (rn <= rtol * bn) status = ORC_OK;
      }
    }
  }
  residual(A, b, x, r, w);
  res->true_rel = nrm2(n, r) / bn;
  res->outer = it;
  res->cg_equiv = it;
  res->status = status;
  free(r); free(u); free(p); free(w); free(sv); free(dinv);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Small dense SPD algebra (s x s, row-major)                                */
/* ------------------------------------------------------------------------ */

/* Lower Cholesky factor L of the lower triangle of W.  Returns 0, or 1 on a
 * pivot <= s*eps*|W_jj| (before the square root) or a non-finite value. */
static int chol(int s, const double *W, double *L) {
  const double eps = 2.220446049250313e-16; /* 2^-52 */
  for (int i = 0; i < s * s; ++i) L[i] = 0.0;
  for (int j = 0; j < s; ++j) {
    double d = W[j * s + j];
    for (int q = 0; q < j; ++q) d -= L[j * s + q] * L[j * s + q];
    if (!isfinite(d) || d <= (double)s * eps * fabs(W[j * s + j])) return 1;
    double ljj = sqrt(d);
    L[j * s + j] = ljj;
    for (int i = j + 1; i < s; ++i) {
      double v = W[i * s + j];
      for (int q = 0; q < j; ++q) v -= L[i * s + q] * L[j * s + q];
      L[i * s + j] = v / ljj;
      if (!isfinite(L[i * s + j])) return 1;
    }
  }
  return 0;
}

/* Solves L L^T y = c in place. */
static void chol_solve(int s, const double *L, double *c) {
  for (int i = 0; i < s; ++i) {
    double v = c[i];
    for (int q = 0; q < i; ++q) v -= L[i * s + q] * c[q];
    c[i] = v / L[i * s + i];
  }
  for (int i = s - 1; i >= 0; --i) {
    double v = c[i];
    for (int q = i + 1; q < s; ++q) v -= L[q * s + i] * c[q];
    c[i] = v / L[i * s + i];
  }
}

/* ------------------------------------------------------------------------ */
/* Alg. 4: preconditioned matrix-powers kernel                              */
/* ------------------------------------------------------------------------ */

/* Fills the n x 2s column-major block P with P(:,1) = B^{-1} v and the
 * alternation of A and B^{-1} that Alg. 4 prescribes: the A-products land in
 * columns s+1..2s and the B^{-1}-products in columns 2..s, so that
 * P(:,1:s) = [z, Kz, ..., K^{s-1}z] and P(:,s+1:2s) = A P(:,1:s), K = B^{-1}A. */
static void mpk(const orc_op *A, int prec, const double *dinv, const double *v,
                int s, double *P) {
  int64_t n = A->n;
  prec_apply(prec, n, dinv, v, P);           /* P(:,1) = B^{-1} v */
  int pin = 1, pout = s + 1;                 /* 1-based column numbers */
  for (int j = 2; j <= 2 * s; ++j) {
    double *in = P + (int64_t)(pin - 1) * n;
    double *out = P + (int64_t)(pout - 1) * n;
    if (j % 2 == 0)
      orc_apply(A, in, out);                 /* A-product */
    else
      prec_apply(prec, n, dinv, in, out);    /* B^{-1}-product */
    int ptemp = pin;
    pin = pout;
    pout = ptemp + 1;
  }
}

/* ------------------------------------------------------------------------ */
/* Alg. 5: the 2s moments in one pass                                        */
/* ------------------------------------------------------------------------ */

static void cvm(int64_t n, int s, const double *P, const double *r, double *vm) {
  const double *last = P + (int64_t)(2 * s - 1) * n;   /* P(:,2s) */
  for (int c = 0; c < s; ++c) vm[c] = orc_dot(n, P + (int64_t)c * n, r);
  for (int c = 0; c < s; ++c) vm[s + c] = orc_dot(n, P + (int64_t)c * n, last);
}

/* ------------------------------------------------------------------------ */
/* Alg. 6: beta, W and alpha from the moments (k > 0)                        */
/* ------------------------------------------------------------------------ */

/* Inputs: vm(1..2s) of r_i, alpha_{i-1}, and the Cholesky factor Lprev of
 * W_{i-1}.  Outputs beta (s x s), W_i and its factor L, alpha_i.  Returns 0
 * or 1 on breakdown.  1-based names in comments follow Alg. 6. */
static int sw(int s, const double *vm, const double *alpha_prev, const double *Lprev,
              double *beta, double *W, double *L, double *alpha) {
  double rhs[2 * ORC_SMAX];
  double b1[ORC_SMAX * ORC_SMAX];
  const double as = alpha_prev[s - 1];                /* alpha(s) */
  if (!(fabs(as) > 1e-300) || !isfinite(as)) return 1;
  for (int m = 0; m < 2 * s - 1; ++m) rhs[m] = 0.0;   /* rhs = zeros(2s-1,1) */
  /* for i = 1..s:  rhs(s-1+i) = -(vm(i) + sum_{j<i} rhs(s-1+j) alpha(s-i+j)) / alpha(s) */
  for (int i = 1; i <= s; ++i) {
    double t = vm[i - 1];
    for (int j = 1; j <= i - 1; ++j) t += rhs[s - 1 + j - 1] * alpha_prev[s - i + j - 1];
    rhs[s - 1 + i - 1] = -t / as;
    if (!isfinite(rhs[s - 1 + i - 1])) return 1;
  }
  /* b1(i,j) = -rhs(i+j-1), full s x s range */
  for (int i = 1; i <= s; ++i)
    for (int j = 1; j <= s; ++j) b1[(i - 1) * s + (j - 1)] = -rhs[i + j - 2];
  /* solve W_{i-1} beta = b1, one column at a time */
  for (int j = 0; j < s; ++j) {
    double col[ORC_SMAX];
    for (int i = 0; i < s; ++i) col[i] = b1[i * s + j];
    chol_solve(s, Lprev, col);
    for (int i = 0; i < s; ++i) beta[i * s + j] = col[i];
  }
  /* W(i,j) = vm(i+j), then W = W - b1 beta */
  for (int i = 1; i <= s; ++i)
    for (int j = 1; j <= s; ++j) W[(i - 1) * s + (j - 1)] = vm[i + j - 1];
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      double acc = 0.0;
      for (int q = 0; q < s; ++q) acc += b1[i * s + q] * beta[q * s + j];
      W[i * s + j] -= acc;
    }
  if (chol(s, W, L)) return 1;
  for (int i = 0; i < s; ++i) alpha[i] = vm[i];      /* W alpha = vm(1:s) */
  chol_solve(s, L, alpha);
  for (int i = 0; i < s; ++i) if (!isfinite(alpha[i])) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 3: preconditioned s-step CG                                          */
/* ------------------------------------------------------------------------ */

/* The four update lines of Alg. 3, in their order:
 *   P(:,1:s) += Pold(:,1:s) beta;   x += P(:,1:s) alpha;
 *   P(:,s+1:2s) += Pold(:,s+1:2s) beta;   r -= P(:,s+1:2s) alpha
 * (the Pold terms are skipped at k = 0, where Pold = 0). */
static void block_update(int64_t n, int s, int k, const double *beta, const double *alpha,
                         double *Pcur, const double *Pold, double *x, double *r) {
  for (int half = 0; half < 2; ++half) {
    double *Pc = Pcur + (int64_t)half * s * n;
    const double *Po = Pold + (int64_t)half * s * n;
    if (k > 0) {
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        double old[ORC_SMAX];
        for (int l = 0; l < s; ++l) old[l] = Po[(int64_t)l * n + i];
        for (int j = 0; j < s; ++j) {
          double acc = Pc[(int64_t)j * n + i];
          for (int l = 0; l < s; ++l) acc += old[l] * beta[l * s + j];
          Pc[(int64_t)j * n + i] = acc;
        }
      }
    }
    double *tgt = half == 0 ? x : r;
    double sgn = half == 0 ? 1.0 : -1.0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int j = 0; j < s; ++j) acc += Pc[(int64_t)j * n + i] * alpha[j];
      tgt[i] += sgn * acc;
    }
  }
}

/* fixed_outer > 0 runs exactly that many outer iterations (no stopping test)
 * unless a breakdown occurs; the final status then says whether the residual
 * test holds at the end.  tr may be NULL. */
int orc_sstep(const orc_op *A, int prec, const double *b, double *x, int s,
              double rtol, int maxit, int fixed_outer, orc_result *res,
              orc_trace *tr) {
  res->status = ORC_EINVAL;
  res->outer = res->cg_equiv = 0;
  res->hist_len = 0;
  res->true_rel = NAN;
  if (tr) tr->len = 0;
  if (!op_check(A) || s < 1 || s > ORC_SMAX || maxit < 0 || (A->n > 0 && s > A->n))
    return ORC_EINVAL;
  int64_t n = A->n;
  double *r = malloc((size_t)n * sizeof(double));
  double *tmp = malloc((size_t)n * sizeof(double));
  double *dinv = malloc((size_t)n * sizeof(double));
  double *P1 = calloc((size_t)n * 2 * s, sizeof(double));
  double *P2 = calloc((size_t)n * 2 * s, sizeof(double));
  if (!r || !tmp || !dinv || !P1 || !P2) {
    free(r); free(tmp); free(dinv); free(P1); free(P2);
    res->status = ORC_ENOMEM;
    return ORC_ENOMEM;
  }
  op_diag(A, dinv);
  for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / dinv[i];

  double bn = nrm2(n, b);
  int status = ORC_NOT_CONVERGED;
  if (bn == 0.0) {
    memset(x, 0, (size_t)n * sizeof(double));
    hist_push(res, 0.0);
    res->status = ORC_OK;
    res->true_rel = 0.0;
    free(r); free(tmp); free(dinv); free(P1); free(P2);
    return ORC_OK;
  }
  residual(A, b, x, r, tmp);                 /* r = b - A x0 */
  double rn = nrm2(n, r);
  hist_push(res, rn / bn);
  int outer_max = fixed_outer > 0 ? fixed_outer : (maxit + s - 1) / s;
  int done = 0;
  if (fixed_outer <= 0 && rn <= rtol * bn) { status = ORC_OK; outer_max = 0; }

  double vm[2 * ORC_SMAX], alpha[ORC_SMAX], alpha_prev[ORC_SMAX];
  double beta[ORC_SMAX * ORC_SMAX], W[ORC_SMAX * ORC_SMAX];
  double L[ORC_SMAX * ORC_SMAX], Lprev[ORC_SMAX * ORC_SMAX];
  double *Pcur = P2, *Pold = P1;             /* k even writes P2, k odd P1 */
  for (int k = 0; k < outer_max; ++k) {
    mpk(A, prec, dinv, r, s, Pcur);
    cvm(n, s, Pcur, r, vm);
    int bad;
    if (k == 0) {
      /* W(i,j) = vm(i+j), beta = 0, W alpha = vm(1:s) */
      for (int i = 1; i <= s; ++i)
        for (int j = 1; j <= s; ++j) W[(i - 1) * s + (j - 1)] = vm[i + j - 1];
      for (int i = 0; i < s * s; ++i) beta[i] = 0.0;
      bad = chol(s, W, L);
      if (!bad) {
        for (int i = 0; i < s; ++i) alpha[i] = vm[i];
        chol_solve(s, L, alpha);
        for (int i = 0; i < s; ++i) if (!isfinite(alpha[i])) bad = 1;
      }
    } else {
      bad = sw(s, vm, alpha_prev, Lprev, beta, W, L, alpha);
    }
    if (bad) { status = ORC_BREAKDOWN; break; }
    block_update(n, s, k, beta, alpha, Pcur, Pold, x, r);
    if (tr && k < tr->cap) {
      memcpy(tr->vm + (size_t)k * 2 * s, vm, sizeof(double) * 2 * s);
      memcpy(tr->alpha + (size_t)k * s, alpha, sizeof(double) * s);
      memcpy(tr->beta + (size_t)k * s * s, beta, sizeof(double) * s * s);
      memcpy(tr->W + (size_t)k * s * s, W, sizeof(double) * s * s);
      if (tr->P) memcpy(tr->P + (size_t)k * 2 * s * n, Pcur, sizeof(double) * 2 * s * n);
      tr->len = k + 1;
    }
    memcpy(alpha_prev, alpha, sizeof(alpha));
    memcpy(Lprev, L, sizeof(L));
    double *t = Pcur; Pcur = Pold; Pold = t;
    res->outer = k + 1;
    rn = nrm2(n, r);
    hist_push(res, rn / bn);
    if (fixed_outer <= 0 && rn <= rtol * bn) { status = ORC_OK; done = 1; break; }
  }
  if (fixed_outer > 0 && status != ORC_BREAKDOWN)
    status = (rn <= rtol * bn) ? ORC_OK : ORC_NOT_CONVERGED;
  (void)done;
  residual(A, b, x, r, tmp);
  res->true_rel = nrm2(n, r) / bn;
  res->cg_equiv = res->outer * s;
  res->status = status;
  free(r); free(tmp); free(dinv); free(P1); free(P2);
  return status;
}

/* ------------------------------------------------------------------------ */
/* s-step PCG on a Chebyshev basis with an explicit block Gram product       */
/* ------------------------------------------------------------------------ */
/*
 * The stabilised-basis variant (related work, Sec. IV: Newton and Chebyshev
 * bases; Sec. II-A: the monomial basis loses independence as s grows).  Alg. 3
 * is kept: directions P_i = Z_i + P_{i-1} beta_{i-1} with beta chosen so that
 * P_i is A-conjugate to P_{i-1}, W_i = P_i^T A P_i, alpha_i = W_i^{-1} Z_i^T r_i,
 * and the same four update lines.  Only the basis and the way the s x s
 * matrices are obtained change:
 *
 *   basis (K = B^{-1} A, interval [lo, hi] enclosing the spectrum of K,
 *   c = (hi + lo)/2, h = (hi - lo)/2, T_j the Chebyshev polynomials):
 *     z_1 = B^{-1} r,   z_{j+1} = T_j((K - c I)/h) z_1, i.e.
 *     z_2 = (K z_1 - c z_1)/h,   z_{j+1} = 2 (K z_j - c z_j)/h - z_{j-1};
 *     AZ(:,j) = A z_j, and K z_j = B^{-1} AZ(:,j) reuses that product.
 *
 *   Gram (the moments of Alg. 5 do not describe a non-monomial basis, so the
 *   inner products are taken directly):
 *     ZAZ(a,b) = z_a^T AZ(:,b),  ZAP(a,l) = z_a^T AP_{i-1}(:,l),  m(a) = z_a^T r.
 *
 *   s x s part (k > 0), with C = P_{i-1}^T A Z_i, i.e. C(l,j) = ZAP(j,l):
 *     W_{i-1} beta = -C          (A-conjugacy of P_i and P_{i-1}),
 *     W_i = ZAZ + C^T beta       (= P_i^T A P_i, using W_{i-1} beta = -C),
 *     W_i alpha = m              (eq. (3); P_{i-1}^T r_i = 0).
 *   At k = 0: W = ZAZ, beta = 0.  Cholesky of the lower triangle as in sw().
 *
 * Per element, in this order and rounding (contract off):
 *   t = dinv_i * AZ(i,j)  (t = AZ(i,j) without preconditioner),
 *   u = t - c * z_j(i),   z_{j+1}(i) = g * u (j = 1) or g2 * u - z_{j-1}(i),
 * with g = 1/h and g2 = 2 g.
 */
static void cheb_basis(const orc_op *A, int prec, const double *dinv, const double *r, int s,
                       double c, double g, double g2, double *P) {
  int64_t n = A->n;
  prec_apply(prec, n, dinv, r, P);                       /* z_1 = B^{-1} r */
  for (int j = 1; j <= s; ++j) {
    const double *zj = P + (int64_t)(j - 1) * n;
    double *az = P + (int64_t)(s + j - 1) * n;
    orc_apply(A, zj, az);                                /* AZ(:,j) = A z_j */
    if (j == s) break;
    double *zn = P + (int64_t)j * n;
    const double *zm = j >= 2 ? P + (int64_t)(j - 2) * n : NULL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double t = (prec == ORC_PREC_JACOBI) ? dinv[i] * az[i] : az[i];   /* (K z_j)(i) */
      double cz = c * zj[i];
      double u = t - cz;
      if (j == 1) {
        zn[i] = g * u;
      } else {
        double v = g2 * u;
        zn[i] = v - zm[i];
      }
    }
  }
}

int orc_sstep_cheb(const orc_op *A, int prec, const double *b, double *x, int s, double lo,
                   double hi, double rtol, int maxit, int fixed_outer, orc_result *res,
                   orc_trace *tr) {
  res->status = ORC_EINVAL;
  res->outer = res->cg_equiv = 0;
  res->hist_len = 0;
  res->true_rel = NAN;
  if (tr) tr->len = 0;
  if (!op_check(A) || s < 1 || s > ORC_SMAX || maxit < 0 || (A->n > 0 && s > A->n) ||
      !(hi > lo))
    return ORC_EINVAL;
  int64_t n = A->n;
  double *r = malloc((size_t)n * sizeof(double));
  double *tmp = malloc((size_t)n * sizeof(double));
  double *dinv = malloc((size_t)n * sizeof(double));
  double *P1 = calloc((size_t)n * 2 * s, sizeof(double));
  double *P2 = calloc((size_t)n * 2 * s, sizeof(double));
  if (!r || !tmp || !dinv || !P1 || !P2) {
    free(r); free(tmp); free(dinv); free(P1); free(P2);
    res->status = ORC_ENOMEM;
    return ORC_ENOMEM;
  }
  op_diag(A, dinv);
  for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / dinv[i];
  const double c = 0.5 * (hi + lo), h = 0.5 * (hi - lo);
  const double g = 1.0 / h, g2 = 2.0 * g;

  double bn = nrm2(n, b);
  int status = ORC_NOT_CONVERGED;
  if (bn == 0.0) {
    memset(x, 0, (size_t)n * sizeof(double));
    hist_push(res, 0.0);
    res->status = ORC_OK;
    res->true_rel = 0.0;
    free(r); free(tmp); free(dinv); free(P1); free(P2);
    return ORC_OK;
  }
  residual(A, b, x, r, tmp);                 /* r = b - A x0 */
  double rn = nrm2(n, r);
  hist_push(res, rn / bn);
  int outer_max = fixed_outer > 0 ? fixed_outer : (maxit + s - 1) / s;
  if (fixed_outer <= 0 && rn <= rtol * bn) { status = ORC_OK; outer_max = 0; }

  double m[ORC_SMAX], alpha[ORC_SMAX];
  double ZAZ[ORC_SMAX * ORC_SMAX], ZAP[ORC_SMAX * ORC_SMAX], C[ORC_SMAX * ORC_SMAX];
  double beta[ORC_SMAX * ORC_SMAX], W[ORC_SMAX * ORC_SMAX];
  double L[ORC_SMAX * ORC_SMAX], Lprev[ORC_SMAX * ORC_SMAX];
  double *Pcur = P2, *Pold = P1;             /* k even writes P2, k odd P1 */
  for (int k = 0; k < outer_max; ++k) {
    cheb_basis(A, prec, dinv, r, s, c, g, g2, Pcur);
    /* block Gram: Z^T [AZ | AP_{i-1} | r] */
    for (int a = 0; a < s; ++a) {
      const double *za = Pcur + (int64_t)a * n;
      m[a] = orc_dot(n, za, r);
      for (int q = 0; q < s; ++q) {
        ZAZ[a * s + q] = orc_dot(n, za, Pcur + (int64_t)(s + q) * n);
        ZAP[a * s + q] = k > 0 ? orc_dot(n, za, Pold + (int64_t)(s + q) * n) : 0.0;
      }
    }
    int bad = 0;
    if (k == 0) {
      for (int i = 0; i < s * s; ++i) { W[i] = ZAZ[i]; beta[i] = 0.0; }
    } else {
      /* C(l,j) = AP_{i-1}(:,l)^T z_j;  W_{i-1} beta = -C, column by column */
      for (int l = 0; l < s; ++l)
        for (int j = 0; j < s; ++j) C[l * s + j] = ZAP[j * s + l];
      for (int j = 0; j < s; ++j) {
        double col[ORC_SMAX];
        for (int i = 0; i < s; ++i) col[i] = -C[i * s + j];
        chol_solve(s, Lprev, col);
        for (int i = 0; i < s; ++i) {
          beta[i * s + j] = col[i];
          if (!isfinite(col[i])) bad = 1;
        }
      }
      /* W = ZAZ + C^T beta */
      for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) {
          double acc = 0.0;
          for (int l = 0; l < s; ++l) acc += C[l * s + i] * beta[l * s + j];
          W[i * s + j] = ZAZ[i * s + j] + acc;
        }
    }
    if (!bad) bad = chol(s, W, L);
    if (!bad) {
      for (int i = 0; i < s; ++i) alpha[i] = m[i];   /* W alpha = m */
      chol_solve(s, L, alpha);
      for (int i = 0; i < s; ++i) if (!isfinite(alpha[i])) bad = 1;
    }
    if (bad) { status = ORC_BREAKDOWN; break; }
    block_update(n, s, k, beta, alpha, Pcur, Pold, x, r);
    if (tr && k < tr->cap) {
      /* vm holds m(1..s) followed by the diagonal ZAZ(a,a) */
      for (int a = 0; a < s; ++a) {
        tr->vm[(size_t)k * 2 * s + a] = m[a];
        tr->vm[(size_t)k * 2 * s + s + a] = ZAZ[a * s + a];
      }
      memcpy(tr->alpha + (size_t)k * s, alpha, sizeof(double) * s);
      memcpy(tr->beta + (size_t)k * s * s, beta, sizeof(double) * s * s);
      memcpy(tr->W + (size_t)k * s * s, W, sizeof(double) * s * s);
      if (tr->P) memcpy(tr->P + (size_t)k * 2 * s * n, Pcur, sizeof(double) * 2 * s * n);
      tr->len = k + 1;
    }
    memcpy(Lprev, L, sizeof(L));
    double *t = Pcur; Pcur = Pold; Pold = t;
    res->outer = k + 1;
    rn = nrm2(n, r);
    hist_push(res, rn / bn);
    if (fixed_outer <= 0 && rn <= rtol * bn) { status = ORC_OK; break; }
  }
  if (fixed_outer > 0 && status != ORC_BREAKDOWN)
    status = (rn <= rtol * bn) ? ORC_OK : ORC_NOT_CONVERGED;
  residual(A, b, x, r, tmp);
  res->true_rel = nrm2(n, r) / bn;
  res->cg_equiv = res->outer * s;
  res->status = status;
  free(r); free(tmp); free(dinv); free(P1); free(P2);
  return status;
}

/* The Chebyshev basis of one outer iteration on its own (tests): P is n x 2s
 * column-major, [Z | AZ] for z_1 = B^{-1} r. */
int orc_cheb_basis(const orc_op *A, int prec, const double *r, int s, double lo, double hi,
                   double *P) {
  if (!op_check(A) || s < 1 || s > ORC_SMAX || !(hi > lo)) return ORC_EINVAL;
  double *dinv = malloc((size_t)A->n * sizeof(double));
  if (!dinv) return ORC_ENOMEM;
  op_diag(A, dinv);
  for (int64_t i = 0; i < A->n; ++i) dinv[i] = 1.0 / dinv[i];
  const double c = 0.5 * (hi + lo), h = 0.5 * (hi - lo);
  const double g = 1.0 / h;
  cheb_basis(A, prec, dinv, r, s, c, g, 2.0 * g, P);
  free(dinv);
  return ORC_OK;
}

/* Largest diagonal entry of the operator (exact: a maximum of stored or
 * computed diagonal values).  The default basis interval without a
 * preconditioner is [0, 2 max_i a_ii], which encloses the spectrum of a
 * weakly diagonally dominant SPD matrix (Gershgorin); with the Jacobi
 * preconditioner it is [0, 2]. */
double orc_max_diag(const orc_op *A) {
  double *d = malloc((size_t)A->n * sizeof(double));
  if (!d) return NAN;
  op_diag(A, d);
  double mx = -INFINITY;
  for (int64_t i = 0; i < A->n; ++i) if (d[i] > mx) mx = d[i];
  free(d);
  return mx;
}

/* Dense Cholesky solve of W y = c for a caller's s x s SPD matrix (test use:
 * exposes the same factorisation the solver uses). Returns 0 or 1. */
int orc_spd_solve(int s, const double *W, double *c) {
  double L[ORC_SMAX * ORC_SMAX];
  if (s < 1 || s > ORC_SMAX) return -1;
  if (chol(s, W, L)) return 1;
  chol_solve(s, L, c);
  return 0;
}

/* Alg. 4 followed by Alg. 5 on their own, for tests: P is n x 2s
 * column-major, vm has 2s entries. */
int orc_mpk_cvm(const orc_op *A, int prec, const double *r, int s, double *P, double *vm) {
  if (!op_check(A) || s < 1 || s > ORC_SMAX) return ORC_EINVAL;
  double *dinv = malloc((size_t)A->n * sizeof(double));
  if (!dinv) return ORC_ENOMEM;
  op_diag(A, dinv);
  for (int64_t i = 0; i < A->n; ++i) dinv[i] = 1.0 / dinv[i];
  mpk(A, prec, dinv, r, s, P);
  cvm(A->n, s, P, r, vm);
  free(dinv);
  return ORC_OK;
}

/* Alg. 6 on its own, for tests: factors W_{i-1} and runs sw().  Returns 0
 * or 1 on breakdown. */
int orc_sw(int s, const double *vm, const double *alpha_prev, const double *Wprev,
           double *beta, double *W, double *alpha) {
  double Lp[ORC_SMAX * ORC_SMAX], L[ORC_SMAX * ORC_SMAX];
  if (s < 1 || s > ORC_SMAX) return -1;
  if (chol(s, Wprev, Lp)) return 1;
  return sw(s, vm, alpha_prev, Lp, beta, W, L, alpha);
}

int orc_smax(void) { return ORC_SMAX; }

/* Threads of the oracle's parallel loops from now on (timing runs). */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}
