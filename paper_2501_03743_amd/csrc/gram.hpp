// s-step CG on a Chebyshev basis (the stabilised bases of the related work,
// Sec. IV; Sec. II-A: the monomial basis of Alg. 4 loses linear independence
// as s grows): the basis recurrence as an operator epilogue, the one-pass
// block Gram product on the FP64 matrix cores, and the s x s algebra that
// replaces Alg. 6's moment recurrence.
//
// With K = B^-1 A, an interval [lo, hi] enclosing its spectrum, centre
// c = (hi + lo)/2, half-width h = (hi - lo)/2, g = 1/h:
//   z_1 = B^-1 r,  z_2 = g (K z_1 - c z_1),  z_{j+1} = 2g (K z_j - c z_j) - z_{j-1},
// so z_{j+1} = T_j((K - cI)/h) z_1 and the columns span the same Krylov
// space as Alg. 4's.  AZ(:,j) = A z_j is the operator's output and K z_j =
// B^-1 AZ(:,j) reuses it.  The moments of Alg. 5 describe only a monomial
// basis, so the s x (2s+1) inner products
//   G = Z^T [AZ | AP_{i-1} | r]
// are formed directly, in one pass over the rows, and
//   k = 0:  W = Z^T A Z, beta = 0;
//   k > 0:  W_{i-1} beta = -C with C = P_{i-1}^T A Z (A-conjugacy of P_i and
//           P_{i-1}),  W = Z^T A Z + C^T beta (= P_i^T A P_i),
//   then W = L L^T and W alpha = Z^T r (eq. (3): P_{i-1}^T r_i = 0),
// followed by Alg. 3's block update unchanged.
#pragma once

#include "kernels.hpp"

namespace ssp {

// Basis recurrence, powers j < s: AZ(:,j) = A z_j and
// z_{j+1} = w (B^-1 AZ(:,j) - c z_j) [- z_{j-1}], with w = g for j = 1 and 2g
// after (zm = nullptr for j = 1).  Rounded in this order, without
// contraction.
template <typename T>
struct EpiCheb {
  static constexpr int NP = 0;
  static constexpr bool kCheck = true;
  T *az, *znext;
  const T *zj, *zm;
  Prec<T> pc;
  T c, w;
  __device__ __forceinline__ void row(int64_t i, T v, double *) const {
#pragma clang fp contract(off)
    az[i] = v;
    const T t = pc.apply(i, v);
    const T cz = c * zj[i];
    const T u = t - cz;
    const T wu = w * u;
    znext[i] = zm ? wu - zm[i] : wu;
  }
  __device__ __forceinline__ void finish(DevState *, const double *) const {}
};

// FP64 matrix-core product D(16x16) += A(16x4) B(4x16).  Operand layout
// (gfx950, checked on the device): lane l holds A(l % 16, l / 16) and
// B(l / 16, l % 16); D(4 v + l / 16, l % 16) is element v of lane l's
// accumulator.
typedef double dbl4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ dbl4 mfma_f64(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kGramRows = 64;     // rows per wavefront step
constexpr int kGramGrid = 1024;   // workgroups of the Gram pass (4 per CU)

template <int S>
struct GramShape {
  static constexpr int M = 2 * S + 1;         // columns of [AZ | AP_old | r]
  static constexpr int NT = (M + 15) / 16;    // 16-wide output tiles
  static constexpr int NP = S * M;            // inner products per workgroup
};

// 16 consecutive entries [q, q + 16) of column `col`, as FP64; entries at
// rows >= n read 0 (their addresses are clamped into the column).
template <typename T>
__device__ __forceinline__ void gram_load16(const T *__restrict__ col, int64_t q, int64_t n,
                                            bool full, double (&v)[16]) {
  if (full) {
    if constexpr (sizeof(T) == 8) {
      const double2 *p = reinterpret_cast<const double2 *>(col + q);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double2 t = p[u];
        v[2 * u] = t.x;
        v[2 * u + 1] = t.y;
      }
    } else {
      const float4 *p = reinterpret_cast<const float4 *>(col + q);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 t = p[u];
        v[4 * u] = t.x;
        v[4 * u + 1] = t.y;
        v[4 * u + 2] = t.z;
        v[4 * u + 3] = t.w;
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t row = q + u;
      const T t = col[row < n ? row : n - 1];
      v[u] = row < n ? (double)t : 0.0;
    }
  }
}

// One pass of the block Gram product G = Z^T [AZ | AP_old | r] over all rows:
// each wavefront takes 64-row steps; lane (kq = l / 16, m = l % 16) loads
// rows 16 kq .. 16 kq + 15 of column m of Z (A operand, m < s) and of column
// m of each 16-wide tile of [AZ | AP_old | r] (B operand), and the 16
// matrix-core products t = 0..15 of a step contract rows 16 kq + t over
// kq = 0..3 -- every lane supplies its own loaded values, no transpose.  The
// four wavefronts' tiles are summed in a fixed order and each workgroup
// stores its s (2s+1) sums at partials[c * G + b], c = a (2s+1) + q.
// first = 1 at k = 0 (no AP_old: those columns read as 0).
template <int S, typename T>
__global__ __launch_bounds__(kWG) void k_gram(int64_t n, int64_t ld, const T *__restrict__ Pc,
                                              const T *__restrict__ Po, const T *__restrict__ r,
                                              int first, DevState *st, double *partials) {
  using GS = GramShape<S>;
  if (st->status != ST_RUNNING) return;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int kq = lane / 16, m = lane % 16;
  const int W = kWG / kWave;
  dbl4 acc[GS::NT];
#pragma unroll
  for (int t = 0; t < GS::NT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
  // this lane's columns: A operand z_m (m < s); B operand per tile
  const T *xa = m < S ? Pc + (int64_t)m * ld : nullptr;
  const T *yb[GS::NT];
#pragma unroll
  for (int t = 0; t < GS::NT; ++t) {
    const int q = t * 16 + m;
    yb[t] = q < S ? Pc + (int64_t)(S + q) * ld
            : (q < 2 * S) ? (first ? nullptr : Po + (int64_t)q * ld)
            : (q == 2 * S) ? r : nullptr;
  }
  const int64_t steps = (n + kGramRows - 1) / kGramRows;
  for (int64_t c = (int64_t)blockIdx.x * W + wave; c < steps; c += (int64_t)gridDim.x * W) {
    const int64_t row0 = c * kGramRows;
    const bool full = row0 + kGramRows <= n;
    const int64_t q = row0 + 16 * kq;
    double xv[16];
    if (xa) gram_load16<T>(xa, q, n, full, xv);
    else {
#pragma unroll
      for (int u = 0; u < 16; ++u) xv[u] = 0.0;
    }
#pragma unroll
    for (int t = 0; t < GS::NT; ++t) {
      double yv[16];
      if (yb[t]) gram_load16<T>(yb[t], q, n, full, yv);
      else {
#pragma unroll
        for (int u = 0; u < 16; ++u) yv[u] = 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[t] = mfma_f64(xv[u], yv[u], acc[t]);
    }
  }
  // fixed-order sum of the wavefronts' tiles, then the workgroup's partials
  __shared__ double red[kWG / kWave][GS::NT][4][kWave];
#pragma unroll
  for (int t = 0; t < GS::NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][t][v][lane] = acc[t][v];
  __syncthreads();
  for (int e = threadIdx.x; e < GS::NT * 256; e += kWG) {
    const int t = e / 256, l = (e % 256) / 4, v = e % 4;
    const int i = 4 * v + l / 16, j = t * 16 + l % 16;   // D(i, j) of tile t
    if (i < S && j < GS::M) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < kWG / kWave; ++w) sum += red[w][t][v][l];
      partials[(int64_t)(i * GS::M + j) * gridDim.x + blockIdx.x] = sum;
    }
  }
}

// Sum over G partials per component, 1024 threads: wavefront w reduces the
// components w, w + 16, ...; lane l adds g = l, l + 64, ... in order, then a
// fixed shuffle tree.  Deterministic.
constexpr int kFinWG = 1024;

template <int NP>
__device__ __forceinline__ void reduce_partials_wide(const double *part, int G, double *tot) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  constexpr int NW = kFinWG / kWave;
  constexpr int U = kGramGrid / kWave;
  for (int c = wave; c < NP; c += NW) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int g = lane + u * kWave;
      const double t = part[(int64_t)c * G + (g < G ? g : G - 1)];
      v[u] = g < G ? t : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
    s = wave_sum(s);
    if (lane == 0) tot[c] = s;
  }
}

// ||r||^2 of the previous block update from its G <= kGridMax partials,
// 1024 threads, fixed order; every thread gets the total.
__device__ __forceinline__ double reduce_rr_wide(const double *part, int G) {
  __shared__ double red[kFinWG / kWave];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  constexpr int U = (kGridMax + kFinWG - 1) / kFinWG;
  double v = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int g = threadIdx.x + u * kFinWG;
    const double t = part[g < G ? g : G - 1];
    v += g < G ? t : 0.0;
  }
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kFinWG / kWave; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Finalisation of the Gram pass (one workgroup of kFinWG threads): the
// previous block update's stopping test first (within a polling batch, as
// the monomial path does), then the s x s algebra above.  Breakdown on a
// Cholesky pivot <= s 2^-52 |W_jj| or any non-finite value, as for Alg. 6.
// Writes alpha, beta, W, L, and vm = (Z^T r, diag(Z^T A Z)) for traces.
template <int S>
__global__ __launch_bounds__(kFinWG) void k_gram_finalize(DevState *st, const double *partials,
                                                         int G, const double *rr_part, int rr_G,
                                                         double *hist) {
#pragma clang fp contract(off)
  using GS = GramShape<S>;
  if (st->status != ST_RUNNING) return;
  __shared__ double g[GS::NP];
  __shared__ double Lp[S * S], L[S * S], beta[S * S], W[S * S], C[S * S], alpha[S];
  __shared__ int bad;
  const int tid = threadIdx.x;
  int fail = 0;   // per-thread flag; decisions use __syncthreads_or
  const double eps = 2.220446049250313e-16;  // 2^-52
  if (rr_part) {   // uniform
    const double rr = reduce_rr_wide(rr_part, rr_G);
    if (tid == 0) fin_update(st, rr, hist);
    __syncthreads();
    if (st->status != ST_RUNNING) return;   // the same value for every thread
  }
  const int k = st->k;   // after the previous update's count
  reduce_partials_wide<GS::NP>(partials, G, g);
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int e = tid; e < S * S; e += kFinWG) {
    Lp[e] = st->L[e];
    L[e] = 0.0;
    const int l = e / S, j = e % S;
    C[e] = g[j * GS::M + S + l];          // C(l, j) = AP_old(:,l)^T z_j
  }
  __syncthreads();
  if (k > 0) {
    // W_{i-1} beta = -C, thread j solves column j with the kept factor
    if (tid < S) {
      const int j = tid;
      double col[S];
#pragma unroll
      for (int i = 0; i < S; ++i) col[i] = -C[i * S + j];
#pragma unroll
      for (int i = 0; i < S; ++i) {
        double v = col[i];
#pragma unroll
        for (int q = 0; q < i; ++q) v -= Lp[i * S + q] * col[q];
        col[i] = v / Lp[i * S + i];
      }
#pragma unroll
      for (int i = S - 1; i >= 0; --i) {
        double v = col[i];
#pragma unroll
        for (int q = i + 1; q < S; ++q) v -= Lp[q * S + i] * col[q];
        col[i] = v / Lp[i * S + i];
      }
      bool ok = true;
#pragma unroll
      for (int i = 0; i < S; ++i) {
        beta[i * S + j] = col[i];
        ok = ok && isfinite(col[i]);
      }
      if (!ok) bad = 1;
    }
    __syncthreads();
    // W = Z^T A Z + C^T beta
    for (int e = tid; e < S * S; e += kFinWG) {
      const int i = e / S, j = e % S;
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < S; ++l) acc += C[l * S + i] * beta[l * S + j];
      W[e] = g[i * GS::M + j] + acc;
    }
  } else {
    for (int e = tid; e < S * S; e += kFinWG) {
      const int i = e / S, j = e % S;
      W[e] = g[i * GS::M + j];
      beta[e] = 0.0;
    }
  }
  __syncthreads();
  if (bad) goto breakdown;
  // Cholesky of the lower triangle, one column at a time (the pivot by one
  // thread, the column below it by S - j - 1 threads), then W alpha = Z^T r
  for (int j = 0; j < S; ++j) {
    if (tid == 0) {
      const double wjj = W[j * S + j];
      double d = wjj;
      for (int q = 0; q < j; ++q) d -= L[j * S + q] * L[j * S + q];
      if (!isfinite(d) || d <= (double)S * eps * fabs(wjj)) fail = 1;
      else L[j * S + j] = sqrt(d);
    }
    if (__syncthreads_or(fail)) goto breakdown;
    if (tid > j && tid < S) {
      double v = W[tid * S + j];
      for (int q = 0; q < j; ++q) v -= L[tid * S + q] * L[j * S + q];
      v = v / L[j * S + j];
      L[tid * S + j] = v;
      if (!isfinite(v)) fail = 1;
    }
    if (__syncthreads_or(fail)) goto breakdown;
  }
  if (tid == 0) {
    double a[S];
    for (int i = 0; i < S; ++i) {
      double v = g[i * GS::M + 2 * S];
      for (int q = 0; q < i; ++q) v -= L[i * S + q] * a[q];
      a[i] = v / L[i * S + i];
    }
    for (int i = S - 1; i >= 0; --i) {
      double v = a[i];
      for (int q = i + 1; q < S; ++q) v -= L[q * S + i] * a[q];
      a[i] = v / L[i * S + i];
      if (!isfinite(a[i])) fail = 1;
    }
    for (int i = 0; i < S; ++i) alpha[i] = a[i];
  }
  if (__syncthreads_or(fail)) goto breakdown;
  if (tid < S) {
    st->alpha[tid] = alpha[tid];
    st->vm[tid] = g[tid * GS::M + 2 * S];
    st->vm[S + tid] = g[tid * GS::M + tid];
  }
  for (int e = tid; e < S * S; e += kFinWG) {
    st->beta[e] = beta[e];
    st->W[e] = W[e];
    st->L[e] = L[e];
  }
  return;
breakdown:
  if (tid == 0) st->status = ST_BREAKDOWN;
}

// Totals of the Gram pass's partial sums on their own (the stand-alone basis
// call): out[c] = sum over the G workgroups of component c.
template <int S>
__global__ __launch_bounds__(kFinWG) void k_gram_totals(const double *partials, int G,
                                                       double *out) {
  __shared__ double g[GramShape<S>::NP];
  reduce_partials_wide<GramShape<S>::NP>(partials, G, g);
  __syncthreads();
  for (int c = threadIdx.x; c < GramShape<S>::NP; c += kFinWG) out[c] = g[c];
}

}  // namespace ssp
