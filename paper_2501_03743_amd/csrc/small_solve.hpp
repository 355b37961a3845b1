// The s x s part of one outer iteration, run on the GPU by the last workgroup
// of the matrix-powers kernel as soon as the 2s moments are reduced.
//
//   k = 0 (Alg. 3, start-up):  W(i,j) = vm(i+j), beta = 0.
//   k > 0 (Alg. 6):            moment recurrence for rhs(s..2s-1) with
//                              alpha_{i-1}; b1(i,j) = -rhs(i+j-1) over the full
//                              s x s range; W_{i-1} beta = b1 with the kept
//                              Cholesky factor of W_{i-1}; W = Hankel(vm) - b1 beta.
//   then W = L L^T (unpivoted, lower triangle) and W alpha = vm(1:s) (eq. (3)).
//
// Breakdown (status ST_BREAKDOWN, no update is applied): |alpha_{i-1}(s)| <=
// 1e-300, a Cholesky pivot (before the square root) <= s * 2^-52 * |W_jj|, or
// any non-finite value.
#pragma once

#include "common.hpp"

namespace ssp {

// Called by all kWG threads of one workgroup.  vm holds the 2s moments (the
// same values in every thread).
__device__ void small_solve(DevState *st, int s, const double *vm) {
  __shared__ double s_vm[2 * kSMax];
  __shared__ double s_ap[kSMax];              // alpha_{i-1}
  __shared__ double s_Lp[kSMax * kSMax];      // factor of W_{i-1}
  __shared__ double s_rhs[2 * kSMax];
  __shared__ double s_b1[kSMax * kSMax];
  __shared__ double s_beta[kSMax * kSMax];
  __shared__ double s_W[kSMax * kSMax];
  __shared__ double s_L[kSMax * kSMax];
  __shared__ double s_col[kSMax][kSMax + 1];  // per-column solve scratch
  __shared__ double s_alpha[kSMax];
  int bad = 0;  // per-thread flag; decisions use __syncthreads_or (uniform, race-free)
  const int tid = threadIdx.x;
  const int k = st->k;
  const int ss = s * s;
  const double eps = 2.220446049250313e-16;  // 2^-52

  if (tid < 2 * s) s_vm[tid] = vm[tid];
  if (tid < s) s_ap[tid] = st->alpha[tid];
  for (int i = tid; i < ss; i += kWG) {
    s_Lp[i] = st->L[i];
    s_L[i] = 0.0;
  }
  __syncthreads();

  if (k > 0) {
    if (tid == 0) {
      const double as = s_ap[s - 1];
      if (!(fabs(as) > 1e-300) || !isfinite(as)) bad = 1;
      for (int m = 0; m < 2 * s - 1; ++m) s_rhs[m] = 0.0;
      // rhs(s-1+i) = -(vm(i) + sum_{j<i} rhs(s-1+j) alpha(s-i+j)) / alpha(s)
      for (int i = 1; i <= s && !bad; ++i) {
        double t = s_vm[i - 1];
        for (int j = 1; j <= i - 1; ++j) t += s_rhs[s - 2 + j] * s_ap[s - i + j - 1];
        const double v = -t / as;
        s_rhs[s - 2 + i] = v;
        if (!isfinite(v)) bad = 1;
      }
    }
    if (__syncthreads_or(bad)) goto fail;
    for (int idx = tid; idx < ss; idx += kWG) {
      const int i = idx / s, j = idx % s;
      s_b1[idx] = -s_rhs[i + j];
    }
    __syncthreads();
    // W_{i-1} beta = b1: lane j solves column j
    if (tid < s) {
      const int j = tid;
      for (int i = 0; i < s; ++i) {
        double v = s_b1[i * s + j];
        for (int q = 0; q < i; ++q) v -= s_Lp[i * s + q] * s_col[j][q];
        s_col[j][i] = v / s_Lp[i * s + i];
      }
      for (int i = s - 1; i >= 0; --i) {
        double v = s_col[j][i];
        for (int q = i + 1; q < s; ++q) v -= s_Lp[q * s + i] * s_col[j][q];
        s_col[j][i] = v / s_Lp[i * s + i];
      }
      for (int i = 0; i < s; ++i) s_beta[i * s + j] = s_col[j][i];
    }
    __syncthreads();
    for (int idx = tid; idx < ss; idx += kWG) {
      const int i = idx / s, j = idx % s;
      double acc = 0.0;
      for (int q = 0; q < s; ++q) acc += s_b1[i * s + q] * s_beta[q * s + j];
      s_W[idx] = s_vm[i + j + 1] - acc;
    }
  } else {
    for (int idx = tid; idx < ss; idx += kWG) {
      const int i = idx / s, j = idx % s;
      s_W[idx] = s_vm[i + j + 1];
      s_beta[idx] = 0.0;
    }
  }
  __syncthreads();

  // Cholesky of the lower triangle, one column at a time
  for (int j = 0; j < s; ++j) {
    if (tid == 0) {
      const double wjj = s_W[j * s + j];
      double d = wjj;
      for (int q = 0; q < j; ++q) d -= s_L[j * s + q] * s_L[j * s + q];
      if (!isfinite(d) || d <= (double)s * eps * fabs(wjj)) bad = 1;
      else s_L[j * s + j] = sqrt(d);
    }
    if (__syncthreads_or(bad)) goto fail;
    if (tid > j && tid < s) {
      const int i = tid;
      double v = s_W[i * s + j];
      for (int q = 0; q < j; ++q) v -= s_L[i * s + q] * s_L[j * s + q];
      v = v / s_L[j * s + j];
      s_L[i * s + j] = v;
      if (!isfinite(v)) bad = 1;
    }
    if (__syncthreads_or(bad)) goto fail;
  }
  // W alpha = vm(1:s)
  if (tid == 0) {
    for (int i = 0; i < s; ++i) {
      double v = s_vm[i];
      for (int q = 0; q < i; ++q) v -= s_L[i * s + q] * s_alpha[q];
      s_alpha[i] = v / s_L[i * s + i];
    }
    for (int i = s - 1; i >= 0; --i) {
      double v = s_alpha[i];
      for (int q = i + 1; q < s; ++q) v -= s_L[q * s + i] * s_alpha[q];
      s_alpha[i] = v / s_L[i * s + i];
      if (!isfinite(s_alpha[i])) bad = 1;
    }
  }
  if (__syncthreads_or(bad)) goto fail;
  if (tid < 2 * s) st->vm[tid] = s_vm[tid];
  if (tid < s) st->alpha[tid] = s_alpha[tid];
  for (int i = tid; i < ss; i += kWG) {
    st->beta[i] = s_beta[i];
    st->W[i] = s_W[i];
    st->L[i] = s_L[i];
  }
  return;
fail:
  if (tid == 0) st->status = ST_BREAKDOWN;
}

// The same s x s part for small s, in the registers of ONE thread: the same
// operations in the same order as small_solve, without the workgroup's
// barriers (for s <= 6 the serial arithmetic is a few hundred flops, far
// cheaper than a dozen barriers).  Called by one thread only.
template <int S>
__device__ void small_solve_serial(DevState *st, const double *vm_in) {
#pragma clang fp contract(off)
  const double eps = 2.220446049250313e-16;  // 2^-52
  double vm[2 * S], beta[S][S], W[S][S], L[S][S], alpha[S];
#pragma unroll
  for (int i = 0; i < 2 * S; ++i) vm[i] = vm_in[i];
  const int k = st->k;
  if (k > 0) {
    double ap[S], Lp[S][S], rhs[2 * S];
#pragma unroll
    for (int i = 0; i < S; ++i) ap[i] = st->alpha[i];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) Lp[i][j] = st->L[i * S + j];
    const double as = ap[S - 1];
    if (!(fabs(as) > 1e-300) || !isfinite(as)) goto fail;
#pragma unroll
    for (int m = 0; m < 2 * S; ++m) rhs[m] = 0.0;
    // rhs(s-1+i) = -(vm(i) + sum_{j<i} rhs(s-1+j) alpha(s-i+j)) / alpha(s)
#pragma unroll
    for (int i = 1; i <= S; ++i) {
      double t = vm[i - 1];
#pragma unroll
      for (int j = 1; j <= i - 1; ++j) t += rhs[S - 2 + j] * ap[S - i + j - 1];
      const double v = -t / as;
      rhs[S - 2 + i] = v;
      if (!isfinite(v)) goto fail;
    }
    // W_{i-1} beta = b1, b1(i,j) = -rhs(i+j-1), column by column
#pragma unroll
    for (int j = 0; j < S; ++j) {
      double col[S];
#pragma unroll
      for (int i = 0; i < S; ++i) {
        double v = -rhs[i + j];
#pragma unroll
        for (int q = 0; q < i; ++q) v -= Lp[i][q] * col[q];
        col[i] = v / Lp[i][i];
      }
#pragma unroll
      for (int i = S - 1; i >= 0; --i) {
        double v = col[i];
#pragma unroll
        for (int q = i + 1; q < S; ++q) v -= Lp[q][i] * col[q];
        col[i] = v / Lp[i][i];
      }
#pragma unroll
      for (int i = 0; i < S; ++i) beta[i][j] = col[i];
    }
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < S; ++q) acc += (-rhs[i + q]) * beta[q][j];
        W[i][j] = vm[i + j + 1] - acc;
      }
  } else {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) {
        W[i][j] = vm[i + j + 1];
        beta[i][j] = 0.0;
      }
  }
  // Cholesky of the lower triangle, one column at a time
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int j = 0; j < S; ++j) L[i][j] = 0.0;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const double wjj = W[j][j];
    double d = wjj;
#pragma unroll
    for (int q = 0; q < j; ++q) d -= L[j][q] * L[j][q];
    if (!isfinite(d) || d <= (double)S * eps * fabs(wjj)) goto fail;
    L[j][j] = sqrt(d);
#pragma unroll
    for (int i = j + 1; i < S; ++i) {
      double v = W[i][j];
#pragma unroll
      for (int q = 0; q < j; ++q) v -= L[i][q] * L[j][q];
      v = v / L[j][j];
      L[i][j] = v;
      if (!isfinite(v)) goto fail;
    }
  }
  // W alpha = vm(1:s)
#pragma unroll
  for (int i = 0; i < S; ++i) {
    double v = vm[i];
#pragma unroll
    for (int q = 0; q < i; ++q) v -= L[i][q] * alpha[q];
    alpha[i] = v / L[i][i];
  }
#pragma unroll
  for (int i = S - 1; i >= 0; --i) {
    double v = alpha[i];
#pragma unroll
    for (int q = i + 1; q < S; ++q) v -= L[q][i] * alpha[q];
    alpha[i] = v / L[i][i];
    if (!isfinite(alpha[i])) goto fail;
  }
#pragma unroll
  for (int i = 0; i < 2 * S; ++i) st->vm[i] = vm[i];
#pragma unroll
  for (int i = 0; i < S; ++i) st->alpha[i] = alpha[i];
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int j = 0; j < S; ++j) {
      st->beta[i * S + j] = beta[i][j];
      st->W[i * S + j] = W[i][j];
      st->L[i * S + j] = L[i][j];
    }
  return;
fail:
  st->status = ST_BREAKDOWN;
}

// Dispatch: serial registers for small s, the workgroup version otherwise.
// Called by all threads of the workgroup.
template <int S>
__device__ __forceinline__ void small_solve_t(DevState *st, const double *vm) {
  if constexpr (S <= 6) {
    if (threadIdx.x == 0) small_solve_serial<S>(st, vm);
  } else {
    small_solve(st, S, vm);
  }
}

}  // namespace ssp
