// Aggregation AMG preconditioner: the one-time hierarchy build on the host
// and the V-cycle application B^-1 y on the GPU.
//
// The paper preconditions its weak-scaling runs with an algebraic multigrid
// whose B^-1 is weighted-Jacobi sweeps on each level of a hierarchy of
// coarser matrices built from A (Sec. III-A, Sec. V-B).  The hierarchy here
// is smoothed aggregation (Vanek, Mandel and Brezina, 1996):
//   strength   j != i strong for i when a_ij^2 >= theta_l^2 |a_ii a_jj|,
//              theta_l = theta 2^-l on level l (coarse couplings are weaker
//              relative to their diagonals; a fixed theta stalls 3D
//              hierarchies after one level);
//   aggregates three passes over the rows in index order: a row whose strong
//              neighbours are all free starts an aggregate with them; a row
//              still free joins the first-pass aggregate of its strongest
//              aggregated strong neighbour (weights within a relative 1e-9
//              are ties, won by the smallest column: rounding in a coarse
//              level's Galerkin sums must not decide); a row still free
//              starts an aggregate with its free strong neighbours;
//   P          (I - omega_p D^-1 A) P_t, P_t(i, agg(i)) = 1, omega_p =
//              4 / (3 rho_G), rho_G = max_i sum_j |a_ij| / |a_ii|;
//   coarse     A_c = P^T A P, R = P^T; stop at max_coarse rows, max_levels
//              levels, or when a level keeps more than 90 % of its rows; the
//              coarsest level is solved with its dense inverse.
// The build runs once per matrix on the host (integer graph work and sparse
// products); every solve-time step is a GPU kernel.  The V-cycle on level l:
//   z = omega D^-1 y, then sweeps-1 more sweeps z += omega D^-1 (y - A z);
//   r = y - A z; y_c = R r; z_c = V-cycle(l+1, y_c); z += P z_c;
//   sweeps post-sweeps z += omega D^-1 (y - A z).
// Same sweeps before and after an exact coarse solve: B^-1 is symmetric.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "engine.hpp"

namespace ssp {

namespace {

// ---- device side ---------------------------------------------------------

// z = omega D^-1 y (the first pre-smoothing sweep, from a zero guess).
__global__ __launch_bounds__(kWG) void k_amg_scale(int64_t n, double w, const double *dinv,
                                                   const double *y, double *z) {
#pragma clang fp contract(off)
  int64_t lo, hi;
  block_chunk(n, logical_block(), gridDim.x, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) {
    const double t = dinv[i] * y[i];
    z[i] = w * t;
  }
}

// z = Ainv y for the coarsest level (dense, row-major, n <= SSP_AMG_DENSE_MAX).
__global__ __launch_bounds__(kWG) void k_amg_dense(int n, const double *Ainv, const double *y,
                                                   double *z) {
#pragma clang fp contract(off)
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
    double acc = 0.0;
    const double *row = Ainv + (int64_t)i * n;
    for (int j = 0; j < n; ++j) {
      const double t = row[j] * y[j];
      acc += t;
    }
    z[i] = acc;
  }
}

// Epilogues of the level operators (no stopping check: a V-cycle always runs
// to the end).
struct EpiAmgSweep {   // zout = z + omega D^-1 (y - A z)
  static constexpr int NP = 0;
  static constexpr bool kCheck = false;
  const double *y, *z, *dinv;
  double w;
  double *zout;
  __device__ __forceinline__ void row(int64_t i, double v, double *) const {
#pragma clang fp contract(off)
    const double d = y[i] - v;
    const double e = dinv[i] * d;
    const double f = w * e;
    zout[i] = z[i] + f;
  }
  __device__ __forceinline__ void finish(DevState *, const double *) const {}
};
struct EpiAmgResid {   // r = y - A z
  static constexpr int NP = 0;
  static constexpr bool kCheck = false;
  const double *y;
  double *r;
  __device__ __forceinline__ void row(int64_t i, double v, double *) const { r[i] = y[i] - v; }
  __device__ __forceinline__ void finish(DevState *, const double *) const {}
};
struct EpiAmgAdd {     // z += P z_c
  static constexpr int NP = 0;
  static constexpr bool kCheck = false;
  double *z;
  __device__ __forceinline__ void row(int64_t i, double v, double *) const { z[i] = z[i] + v; }
  __device__ __forceinline__ void finish(DevState *, const double *) const {}
};

// ---- host side: the hierarchy build ---------------------------------------

struct HostCsr {
  int64_t n = 0, m = 0;   // rows, columns
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
};

HostCsr transpose(const HostCsr &A) {
  HostCsr T;
  T.n = A.m;
  T.m = A.n;
  T.rp.assign(T.n + 1, 0);
  for (int32_t c : A.ci) T.rp[c + 1] += 1;
  for (int64_t i = 0; i < T.n; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(A.ci.size());
  T.v.resize(A.v.size());
  std::vector<int64_t> pos(T.rp.begin(), T.rp.end() - 1);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int64_t q = pos[A.ci[k]]++;
      T.ci[q] = (int32_t)i;
      T.v[q] = A.v[k];
    }
  return T;
}

// C = A B (sparse accumulator per row; columns of each row in first-touch
// order, then sorted).
HostCsr multiply(const HostCsr &A, const HostCsr &B) {
  HostCsr C;
  C.n = A.n;
  C.m = B.m;
  C.rp.assign(C.n + 1, 0);
  std::vector<double> acc(B.m, 0.0);
  std::vector<int64_t> mark(B.m, -1);
  std::vector<int32_t> cols;
  for (int64_t i = 0; i < A.n; ++i) {
    cols.clear();
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int32_t a = A.ci[k];
      const double av = A.v[k];
      for (int64_t q = B.rp[a]; q < B.rp[a + 1]; ++q) {
        const int32_t c = B.ci[q];
        if (mark[c] != i) {
          mark[c] = i;
          acc[c] = 0.0;
          cols.push_back(c);
        }
        acc[c] += av * B.v[q];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t c : cols) {
      C.ci.push_back(c);
      C.v.push_back(acc[c]);
    }
    C.rp[i + 1] = (int64_t)C.ci.size();
  }
  return C;
}

std::vector<double> diagonal(const HostCsr &A) {
  std::vector<double> d(A.n, 0.0);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i) d[i] += A.v[k];
  return d;
}

constexpr double kTie = 1e-9;   // relative width of a tie between neighbour weights

// Aggregate index per row (three passes); returns the aggregate count.
int64_t aggregate(const HostCsr &A, const std::vector<double> &d, double theta,
                  std::vector<int64_t> &agg) {
  const int64_t n = A.n;
  const double t2 = theta * theta;
  auto strong = [&](int64_t i, int64_t k) {
    const int32_t j = A.ci[k];
    if (j == i) return false;
    const double a = A.v[k];
    return a * a >= t2 * std::fabs(d[i] * d[j]);
  };
  agg.assign(n, -1);
  int64_t nc = 0;
  for (int64_t i = 0; i < n; ++i) {   // pass 1
    if (agg[i] >= 0) continue;
    bool free_nb = true;
    for (int64_t k = A.rp[i]; k < A.rp[i + 1] && free_nb; ++k)
      if (strong(i, k) && agg[A.ci[k]] >= 0) free_nb = false;
    if (!free_nb) continue;
    agg[i] = nc;
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (strong(i, k)) agg[A.ci[k]] = nc;
    ++nc;
  }
  const std::vector<int64_t> first = agg;
  for (int64_t i = 0; i < n; ++i) {   // pass 2
    if (agg[i] >= 0) continue;
    int64_t best = -1;
    double bw = -1.0;
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      if (!strong(i, k)) continue;
      const int64_t j = A.ci[k];
      if (first[j] < 0) continue;
      const double w = std::fabs(A.v[k]);
      if (best < 0 || w > bw * (1.0 + kTie) || (w >= bw * (1.0 - kTie) && j < best)) {
        best = j;
        bw = w;
      }
    }
    if (best >= 0) agg[i] = first[best];
  }
  for (int64_t i = 0; i < n; ++i) {   // pass 3
    if (agg[i] >= 0) continue;
    agg[i] = nc;
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (strong(i, k) && agg[A.ci[k]] < 0) agg[A.ci[k]] = nc;
    ++nc;
  }
  return nc;
}

// P = P_t - omega_p D^-1 (A P_t).
HostCsr prolongator(const HostCsr &A, const std::vector<double> &d,
                    const std::vector<int64_t> &agg, int64_t nc) {
  double rho = 0.0;   // Gershgorin bound of rho(D^-1 A)
  for (int64_t i = 0; i < A.n; ++i) {
    double s = 0.0;
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) s += std::fabs(A.v[k]);
    rho = std::max(rho, s / std::fabs(d[i]));
  }
  const double wp = 4.0 / (3.0 * rho);
  HostCsr Pt;
  Pt.n = A.n;
  Pt.m = nc;
  Pt.rp.resize(A.n + 1);
  Pt.ci.resize(A.n);
  Pt.v.assign(A.n, 1.0);
  for (int64_t i = 0; i < A.n; ++i) {
    Pt.rp[i] = i;
    Pt.ci[i] = (int32_t)agg[i];
  }
  Pt.rp[A.n] = A.n;
  HostCsr AP = multiply(A, Pt);
  HostCsr P;
  P.n = A.n;
  P.m = nc;
  P.rp.assign(A.n + 1, 0);
  for (int64_t i = 0; i < A.n; ++i) {
    bool own = false;
    const double di = 1.0 / d[i];
    for (int64_t k = AP.rp[i]; k < AP.rp[i + 1]; ++k) {
      const int32_t c = AP.ci[k];
      const double t = wp * (di * AP.v[k]);
      double v = -t;
      if (c == agg[i]) {
        v = 1.0 - t;
        own = true;
      }
      P.ci.push_back(c);
      P.v.push_back(v);
    }
    if (!own) {   // a row of A P_t without its own aggregate's column
      P.ci.push_back((int32_t)agg[i]);
      P.v.push_back(1.0);
      // keep the row sorted
      const int64_t b0 = P.rp[i];
      std::vector<std::pair<int32_t, double>> row;
      for (int64_t k = b0; k < (int64_t)P.ci.size(); ++k) row.push_back({P.ci[k], P.v[k]});
      std::sort(row.begin(), row.end());
      for (size_t k = 0; k < row.size(); ++k) {
        P.ci[b0 + k] = row[k].first;
        P.v[b0 + k] = row[k].second;
      }
    }
    P.rp[i + 1] = (int64_t)P.ci.size();
  }
  return P;
}

// Inverse of a small SPD matrix (Cholesky, then the columns of L^-T L^-1).
bool dense_inverse(const HostCsr &A, std::vector<double> &inv) {
  const int64_t n = A.n;
  std::vector<double> M(n * n, 0.0), L(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) M[i * n + A.ci[k]] += A.v[k];
  for (int64_t j = 0; j < n; ++j) {
    double s = M[j * n + j];
    for (int64_t q = 0; q < j; ++q) s -= L[j * n + q] * L[j * n + q];
    if (!(s > 0.0) || !std::isfinite(s)) return false;
    L[j * n + j] = std::sqrt(s);
    for (int64_t i = j + 1; i < n; ++i) {
      double t = M[i * n + j];
      for (int64_t q = 0; q < j; ++q) t -= L[i * n + q] * L[j * n + q];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  inv.assign(n * n, 0.0);
  std::vector<double> col(n);
  for (int64_t c = 0; c < n; ++c) {
    for (int64_t i = 0; i < n; ++i) {   // L y = e_c
      double t = (i == c) ? 1.0 : 0.0;
      for (int64_t q = 0; q < i; ++q) t -= L[i * n + q] * col[q];
      col[i] = t / L[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {   // L^T x = y
      double t = col[i];
      for (int64_t q = i + 1; q < n; ++q) t -= L[q * n + i] * col[q];
      col[i] = t / L[i * n + i];
    }
    for (int64_t i = 0; i < n; ++i) inv[i * n + c] = col[i];
  }
  return true;
}

// The levels of the hierarchy from the fine matrix F: As[0] = F, then
// P_l, R_l = P_l^T, A_{l+1} = R_l A_l P_l until a stopping rule holds.
// Returns false (with the reason) for a non-positive diagonal entry.
bool build_levels(const HostCsr &F, double theta, int64_t max_coarse, int max_levels,
                  std::vector<HostCsr> &As, std::vector<HostCsr> &Ps, std::vector<HostCsr> &Rs,
                  std::vector<std::vector<int64_t>> &aggs, std::string &err) {
  As.assign(1, F);
  Ps.clear();
  Rs.clear();
  aggs.clear();
  while (As.back().n > max_coarse && (int)As.size() < max_levels) {
    const HostCsr &Al = As.back();
    const std::vector<double> d = diagonal(Al);
    for (double di : d)
      if (!(di > 0.0)) {
        err = "a diagonal entry is not positive";
        return false;
      }
    std::vector<int64_t> agg;
    const int64_t nc = aggregate(Al, d, std::ldexp(theta, -(int)(As.size() - 1)), agg);
    if (nc == 0 || (double)nc >= 0.9 * (double)Al.n) break;
    HostCsr P = prolongator(Al, d, agg, nc);
    HostCsr R = transpose(P);
    HostCsr Ac = multiply(R, multiply(Al, P));
    Ps.push_back(std::move(P));
    Rs.push_back(std::move(R));
    aggs.push_back(std::move(agg));
    As.push_back(std::move(Ac));
  }
  return true;
}

}  // namespace

// ---- the device hierarchy -------------------------------------------------

struct AmgLevel {
  int64_t n = 0;
  CsrArgs<double> A{}, P{}, R{};   // A unused on level 0 (the matrix itself)
  double *dinv = nullptr;
  double *y = nullptr, *z = nullptr, *z2 = nullptr, *r = nullptr;
  std::vector<void *> owned;
};

struct AmgHier {
  double omega = 2.0 / 3.0;
  int sweeps = 1;
  std::vector<AmgLevel> lv;
  double *coarse_inv = nullptr;
  int64_t coarse_n = 0;
  std::vector<int64_t> rows;
};

namespace {

template <typename T>
int upload(ssp_handle *h, AmgLevel &L, T *&dst, const T *src, size_t count) {
  if (hipMalloc(&dst, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, SSP_ENOMEM, "ssp_set_amg: device allocation failed");
  }
  L.owned.push_back((void *)dst);
  if (count && src)
    HIPCHK(h, hipMemcpy(dst, src, sizeof(T) * count, hipMemcpyHostToDevice));
  return SSP_OK;
}

// Level matrices run in the LDS-staged CSR form: their rows are long (the
// Galerkin operators of a 3D hierarchy hold 30-90 entries per row, the
// restrictions 30-190), which a thread per row would read uncoalesced.
int upload_csr(ssp_handle *h, AmgLevel &L, CsrArgs<double> &dst, const HostCsr &S) {
  std::vector<int32_t> rp32(S.rp.size());
  int64_t maxrow = 0;
  for (size_t i = 0; i < S.rp.size(); ++i) {
    rp32[i] = (int32_t)S.rp[i];
    if (i > 0) maxrow = std::max<int64_t>(maxrow, S.rp[i] - S.rp[i - 1]);
  }
  memset(&dst, 0, sizeof(dst));
  dst.n = S.n;
  dst.variant = CSR_STAGED;
  int64_t R = maxrow > 0 ? kCsrLds / maxrow : kCsrRowsMax;
  R = std::max<int64_t>(1, std::min<int64_t>(R, kCsrRowsMax));
  dst.rows_per_rb = (int)R;
  dst.nrb = (S.n + R - 1) / R;
  int32_t *rp = nullptr, *ci = nullptr;
  double *v = nullptr;
  int rc = upload(h, L, rp, rp32.data(), rp32.size());
  if (!rc) rc = upload(h, L, ci, S.ci.data(), S.ci.size());
  if (!rc) rc = upload(h, L, v, S.v.data(), S.v.size());
  dst.rowptr = rp;
  dst.colind = ci;
  dst.val = v;
  return rc;
}

// The V-cycle's epilogues reduce nothing and check no status, so the
// kernels never touch the control block or the partial sums passed to them.
template <class Epi>
void level_op(ssp_handle *h, const CsrArgs<double> &M, const double *x, const Epi &epi) {
  const int G = (int)std::max<int64_t>(1, std::min<int64_t>(M.nrb, kGridMax));
  k_csr<CSR_STAGED, double, Epi><<<G, kWG, 0, h->stream>>>(M, x, 1.0, epi, h->st,
                                                           h->ws.partials);
}

// z = B^-1 y on level l (z, y device vectors of the level's size).
int vcycle(ssp_handle *h, const ssp_matrix *A, AmgHier &H, size_t l, const double *y,
           double *z) {
  const size_t last = H.lv.size() - 1;
  if (l == last) {
    const int n = (int)H.coarse_n;
    k_amg_dense<<<std::max(1, std::min(64, (n + kWG - 1) / kWG)), kWG, 0, h->stream>>>(
        n, H.coarse_inv, y, z);
    LAUNCHCHK(h);
    return SSP_OK;
  }
  AmgLevel &L = H.lv[l];
  const int64_t n = L.n;
  const double w = H.omega;
  // the level operator (level 0: the matrix in its selected kernel form)
  auto op = [&](const double *x, auto epi) -> int {
    if (l == 0) return launch_op<double>(h, A, x, epi, 3);
    level_op(h, L.A, x, epi);
    LAUNCHCHK(h);
    return SSP_OK;
  };
  // each sweep writes the other of the two buffers z, z2; the cycle makes
  // 2 sweeps - 1 of those swaps, so starting in z2 it ends in z
  double *buf[2] = {z, L.z2};
  int cur = 1;
  k_amg_scale<<<grid_rows(n), kWG, 0, h->stream>>>(n, w, L.dinv, y, buf[cur]);
  LAUNCHCHK(h);
  int rc = SSP_OK;
  for (int q = 1; q < H.sweeps && !rc; ++q, cur ^= 1)
    rc = op(buf[cur], EpiAmgSweep{y, buf[cur], L.dinv, w, buf[cur ^ 1]});
  if (!rc) rc = op(buf[cur], EpiAmgResid{y, L.r});
  if (rc) return rc;
  AmgLevel &C = H.lv[l + 1];
  level_op(h, L.R, L.r, EpiStore<double>{C.y});
  LAUNCHCHK(h);
  rc = vcycle(h, A, H, l + 1, C.y, C.z);
  if (rc) return rc;
  level_op(h, L.P, C.z, EpiAmgAdd{buf[cur]});
  LAUNCHCHK(h);
  for (int q = 0; q < H.sweeps && !rc; ++q, cur ^= 1)
    rc = op(buf[cur], EpiAmgSweep{y, buf[cur], L.dinv, w, buf[cur ^ 1]});
  return rc;
}

}  // namespace

int amg_vcycle(ssp_handle *h, const ssp_matrix *A, const double *y, double *z) {
  if (!A->amg) return fail(h, SSP_EINVAL, "the matrix has no AMG hierarchy");
  return vcycle(h, A, *A->amg, 0, y, z);
}

void amg_free(ssp_matrix *A) {
  if (!A || !A->amg) return;
  for (AmgLevel &L : A->amg->lv)
    for (void *p : L.owned) (void)hipFree(p);
  delete A->amg;
  A->amg = nullptr;
}

}  // namespace ssp

using namespace ssp;

extern "C" {

int ssp_set_amg(ssp_handle *h, ssp_matrix *A, const ssp_amg_opts *opts) {
  if (!h) return SSP_EINVAL;
  if (!A || A->h != h) return fail(h, SSP_EINVAL, "ssp_set_amg: matrix is NULL or belongs to another handle");
  if (A->kind != 0)
    return fail(h, SSP_EUNSUPPORTED, "ssp_set_amg: the AMG hierarchy is built for CSR matrices");
  const double theta = (opts && opts->theta > 0.0) ? opts->theta : 0.08;
  const double omega = (opts && opts->omega > 0.0) ? opts->omega : 2.0 / 3.0;
  const int sweeps = (opts && opts->sweeps > 0) ? opts->sweeps : 1;
  const int64_t max_coarse = (opts && opts->max_coarse > 0) ? opts->max_coarse : 64;
  const int max_levels = (opts && opts->max_levels > 0) ? opts->max_levels : 10;
  if (!(theta < 1.0) || !(omega < 2.0) || sweeps > 16 || max_levels > SSP_AMG_MAX_LEVELS ||
      max_coarse > SSP_AMG_DENSE_MAX)
    return fail(h, SSP_EINVAL, "ssp_set_amg: theta < 1, omega < 2, sweeps <= 16, max_levels <= " +
                                   std::to_string(SSP_AMG_MAX_LEVELS) + ", max_coarse <= " +
                                   std::to_string(SSP_AMG_DENSE_MAX));
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int rc = SSP_OK;
  // the fine matrix on the host
  HostCsr F;
  F.n = F.m = A->n;
  {
    std::vector<int32_t> rp(A->n + 1);
    HIPCHK(h, hipMemcpy(rp.data(), A->csr.rowptr, sizeof(int32_t) * (A->n + 1),
                        hipMemcpyDeviceToHost));
    F.rp.assign(rp.begin(), rp.end());
    const int64_t nnz = rp[A->n];
    F.ci.resize(nnz);
    F.v.resize(nnz);
    HIPCHK(h, hipMemcpy(F.ci.data(), A->csr.colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(F.v.data(), A->csr.val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
  }
  amg_free(A);
  std::vector<HostCsr> As, Ps, Rs;
  std::vector<std::vector<int64_t>> aggs;
  std::string why;
  if (!build_levels(F, theta, max_coarse, max_levels, As, Ps, Rs, aggs, why))
    return fail(h, SSP_EINVAL, "ssp_set_amg: " + why);
  AmgHier *H = new AmgHier;
  H->omega = omega;
  H->sweeps = sweeps;
  if (As.back().n > SSP_AMG_DENSE_MAX) {
    delete H;
    return fail(h, SSP_EUNSUPPORTED, "ssp_set_amg: the coarsest level has " +
                                         std::to_string(As.back().n) + " rows (at most " +
                                         std::to_string(SSP_AMG_DENSE_MAX) + ")");
  }
  std::vector<double> inv;
  if (!dense_inverse(As.back(), inv)) {
    delete H;
    return fail(h, SSP_EINVAL, "ssp_set_amg: the coarsest matrix is not positive definite");
  }
  H->lv.resize(As.size());
  for (size_t l = 0; l < As.size(); ++l) {
    AmgLevel &L = H->lv[l];
    L.n = As[l].n;
    H->rows.push_back(L.n);
    std::vector<double> d = diagonal(As[l]);
    for (double &di : d) di = 1.0 / di;
    rc = upload(h, L, L.dinv, d.data(), d.size());
    if (!rc && l > 0) rc = upload_csr(h, L, L.A, As[l]);
    if (!rc && l + 1 < As.size()) rc = upload_csr(h, L, L.P, Ps[l]);
    if (!rc && l + 1 < As.size()) rc = upload_csr(h, L, L.R, Rs[l]);
    if (!rc) rc = upload(h, L, L.y, (const double *)nullptr, L.n);
    if (!rc) rc = upload(h, L, L.z, (const double *)nullptr, L.n);
    if (!rc) rc = upload(h, L, L.z2, (const double *)nullptr, L.n);
    if (!rc) rc = upload(h, L, L.r, (const double *)nullptr, L.n);
    if (rc) {
      A->amg = H;
      amg_free(A);
      return rc;
    }
  }
  H->coarse_n = As.back().n;
  rc = upload(h, H->lv.back(), H->coarse_inv, inv.data(), inv.size());
  A->amg = H;
  if (rc) {
    amg_free(A);
    return rc;
  }
  A->prec = SSP_PREC_AMG;
  return SSP_OK;
}

int ssp_amg_levels(const ssp_matrix *A, int *levels, int64_t *rows) {
  if (!A || !levels) return SSP_EINVAL;
  if (!A->amg) {
    *levels = 0;
    return SSP_OK;
  }
  *levels = (int)A->amg->rows.size();
  if (rows)
    for (size_t l = 0; l < A->amg->rows.size(); ++l) rows[l] = A->amg->rows[l];
  return SSP_OK;
}

int ssp_amg_apply(ssp_handle *h, const ssp_matrix *A, const double *y, double *z) {
  if (!h) return SSP_EINVAL;
  if (!A || A->h != h) return fail(h, SSP_EINVAL, "ssp_amg_apply: matrix is NULL or belongs to another handle");
  if (!A->amg) return fail(h, SSP_EINVAL, "ssp_amg_apply: the matrix has no AMG hierarchy");
  if (!y || !z || y == z) return fail(h, SSP_EINVAL, "ssp_amg_apply: need distinct vectors");
  HIPCHK(h, hipSetDevice(h->device));
  return amg_vcycle(h, A, y, z);
}

}  // extern "C"
