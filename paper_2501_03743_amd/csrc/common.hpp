// Shared device-side definitions of libsstep: launch geometry, the device
// control block of a solve, and block-level reduction helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssp {

constexpr int kSMax = 16;         // largest s (s x s moment matrices)
constexpr int kWG = 256;          // threads per workgroup of every streaming kernel
constexpr int kWave = 64;         // CDNA wavefront
constexpr int kXcd = 8;           // MI355X: 8 accelerator dies, round-robin dispatch
constexpr int64_t kInfinityCache = 256ll << 20;  // memory-side last-level cache (bytes)
constexpr int kGridMax = 2048;    // workgroups of a streaming launch (8 per CU)
constexpr int64_t kColumnStagger = 17 * 256;  // bytes added to block leading dimensions
constexpr int kCsrLds = 4096;     // FP64 products staged in LDS per CSR row block
constexpr int kCsrRowsMax = 1024; // rows per CSR row block
constexpr int kSellPad = 32;      // padding entries (per lane) after the last sliced-ELL slice

// Solve status kept on the device.
enum : int {
  ST_RUNNING = 0,
  ST_CONVERGED = 1,
  ST_MAXIT = 2,
  ST_BREAKDOWN = 3,
  ST_ZERO_RHS = 4,
};

// Device control block of one solve.  Written only by the single-workgroup
// finalisation kernels; read by every kernel to skip work after a stop.
struct DevState {
  int status;
  int k;              // outer iterations completed
  int outer_max;
  int fixed;          // fixed-iteration mode: no stopping test
  int s;
  int hist_cap;
  int ir_refine;      // iterative refinement: index of the current outer step
  int ir_max_refine;
  int ir_hist_cap;
  int ir_inner_total; // batched solves: inner outer iterations over all refinements
  double ir_bb;       // ||b||^2 of the FP64 system
  double ir_rtol;     // outer (FP64) relative tolerance
  double ir_inner_rtol; // inner solves: relative reduction of the inner residual
  double bb;          // ||b||^2
  double rr;          // ||r||^2 after the latest update
  double rtol;
  double rho;         // PCG: u^T r
  double pcg_alpha;
  double pcg_beta;
  double true_rr;     // ||b - A x||^2 at exit
  double vm[2 * kSMax];
  double alpha[kSMax];
  double beta[kSMax * kSMax];   // beta(l, j) at [l * s + j]
  double W[kSMax * kSMax];      // row-major
  double L[kSMax * kSMax];      // lower Cholesky factor of W
};

// Workgroups are dispatched round-robin over the 8 XCDs; this maps the
// hardware index to a logical index so that logically consecutive workgroups
// run on the same XCD and share its L2 (neighbouring grid planes).
__device__ __forceinline__ int logical_block() {
  const int G = gridDim.x, b = blockIdx.x;
  const int q = G / kXcd, rem = G % kXcd;
  const int xcd = b % kXcd, local = b / kXcd;
  return (xcd < rem) ? xcd * (q + 1) + local : rem * (q + 1) + (xcd - rem) * q + local;
}

// Contiguous chunk [lo, hi) of `items` for logical block lb of G.
__device__ __forceinline__ void block_chunk(int64_t items, int lb, int G, int64_t &lo,
                                            int64_t &hi) {
  const int64_t per = (items + G - 1) / G;
  lo = (int64_t)lb * per;
  hi = lo + per;
  if (lo > items) lo = items;
  if (hi > items) hi = items;
}

// XCD-interleaved schedule of `items` for the calling workgroup.  The items
// are split into kXcd contiguous ranges, one per XCD (the hardware deals
// workgroups out round-robin over the XCDs), and each range is dealt out in
// pieces of `piece` items to that XCD's workgroups in turn, so that at any
// time an XCD's workgroups stream one compact region (HBM pages and the XCD's
// L2 shared by neighbours) rather than one distant region each.  The
// workgroup's pieces start at first, first + stride, ... below end.  Grids
// smaller than kXcd take contiguous chunks.  G and b are the grid size and
// the hardware block index (a batch tile passes the grid of the single solve
// it reproduces and its tile index).
struct XcdSched {
  int64_t first, stride, end;
};
__device__ __forceinline__ XcdSched xcd_sched(int64_t items, int64_t piece, int G, int b) {
  XcdSched s;
  int64_t lo, hi;
  if (G < kXcd) {
    block_chunk(items, b, G, lo, hi);
    s.first = lo;
    s.stride = piece;
  } else {
    const int q = G / kXcd, rem = G % kXcd;
    const int xcd = b % kXcd, local = b / kXcd;
    const int qx = xcd < rem ? q + 1 : q;
    block_chunk(items, xcd, kXcd, lo, hi);
    s.first = lo + (int64_t)local * piece;
    s.stride = (int64_t)qx * piece;
  }
  s.end = hi;
  return s;
}

// Loads and stores of data that is not read again soon (the updates'
// stream-once columns and vectors).  The non-temporal hint keeps them from
// displacing what the next kernels read again from the caches: a matrix that
// fits the 256 MB memory-side cache then stays there from one iteration to
// the next (128^3 7-point CSR: the first matrix power after the update
// 50 -> 32 us).  Values are unchanged; only the cache policy differs.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_stream(T *p, T v) {
  __builtin_nontemporal_store(v, p);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sums NP per-thread values over the workgroup and stores them, component-
// major, at out[c * stride]; fixed order, so the result is deterministic.
template <int NP>
__device__ __forceinline__ void block_store_sums(const double (&v)[NP], double *out,
                                                 int64_t stride) {
  __shared__ double red[kWG / kWave][NP > 0 ? NP : 1];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    double t = wave_sum(v[c]);
    if (lane == 0) red[wid][c] = t;
  }
  __syncthreads();
  if (threadIdx.x < NP) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWG / kWave; ++w) t += red[w][threadIdx.x];
    out[threadIdx.x * stride] = t;
  }
}

// In a single-workgroup finalisation kernel: totals[c] = sum over the G
// per-workgroup partials of component c (stored at part[c * G + g]), in a
// fixed order.  All loads of a thread are issued before they are summed.
// Every thread gets the totals.
template <int NP>
__device__ void reduce_partials(const double *part, int G, double (&totals)[NP]) {
  __shared__ double red[kWG / kWave][NP > 0 ? NP : 1];
  constexpr int U = kGridMax / kWG;
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  double v[NP][U];
#pragma unroll
  for (int c = 0; c < NP; ++c)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int g = threadIdx.x + u * kWG;
      const double t = part[(int64_t)c * G + (g < G ? g : G - 1)];  // always a valid address
      v[c][u] = (g < G) ? t : 0.0;
    }
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) t += v[c][u];
    t = wave_sum(t);
    if (lane == 0) red[wid][c] = t;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWG / kWave; ++w) t += red[w][c];
    totals[c] = t;
  }
  __syncthreads();
}

// Fast floor division of non-negative 64-bit values (< 2^52) by a runtime
// divisor, through a double reciprocal and one correction step.
struct FastDiv {
  int64_t d;
  double inv;
};
__device__ __forceinline__ int64_t fdiv(int64_t a, const FastDiv &f, int64_t &rem) {
  int64_t q = (int64_t)((double)a * f.inv);
  int64_t r = a - q * f.d;
  if (r < 0) { q -= 1; r += f.d; }
  else if (r >= f.d) { q += 1; r -= f.d; }
  rem = r;
  return q;
}

}  // namespace ssp
