// Operator application on gfx950: CSR (two kernel forms) and matrix-free
// grid stencils, in FP64 or FP32.  Each visitor walks a range of rows and
// hands (row, (A x)_row) to a functor that runs in the thread owning the row.
//
// Rounding: products are rounded, then summed in the order of the stored
// columns (CSR) or of the stencil definition (matrix-free); FMA contraction
// is off, so the FP64 results are bitwise equal to a plain sequential
// evaluation of the same definition.
#pragma once

#include "common.hpp"

namespace ssp {

enum : int { CSR_STAGED = 0, CSR_ROW = 1, CSR_SELL = 2 };
enum : int { K_2D5 = 1, K_3D7 = 2, K_3D27 = 3, K_VARK = 4 };

template <typename T>
struct CsrArgs {
  int64_t n;
  const int32_t *rowptr;
  const int32_t *colind;
  const T *val;
  int rows_per_rb;   // rows per LDS row block (CSR_STAGED, <= kCsrRowsMax)
  int64_t nrb;       // number of row blocks
  int variant;       // CSR_STAGED, CSR_ROW or CSR_SELL, chosen per matrix by timing
  // sliced ELL copy (CSR_SELL): slice sl holds rows 64 sl .. 64 sl + 63; entry
  // u of its row `lane` is at slice_off[sl] + 64 u + lane, u < slice_w[sl];
  // entries past a row's end have column -1 and value 0
  const int32_t *sell_col;
  const T *sell_val;
  const int64_t *slice_off;
  const int32_t *slice_w;
  int64_t nslices;
  int sell_xcd;      // 1: slices dealt out XCD-interleaved (matrix larger than the
                     // memory-side cache), 0: a contiguous chunk per workgroup
  int sell_wmax;     // widest slice (entries per row)
};

template <typename T>
struct StencilArgs {
  int64_t n;
  int nx, ny, nz;
  FastDiv fx, fy;    // divisions by nx and ny
  T diag, off;
  const T *k;        // cell coefficients (variable-coefficient kind)
};

// Jacobi (or identity) preconditioner: z = dinv .* v.
template <typename T>
struct Prec {
  const T *dinv;     // nullptr: the constant dc
  T dc;
  __device__ __forceinline__ T apply(int64_t i, T v) const {
#pragma clang fp contract(off)
    return (dinv ? dinv[i] : dc) * v;
  }
};

// Rows of one CSR row block (at most kCsrLds stored entries) are staged as
// products val*x in LDS: every thread first issues all its coalesced loads of
// colind and val, then all its gathers of x, so each workgroup keeps up to
// kCsrLds/kWG independent loads in flight.  Each thread then sums its rows in
// column order.  Rows longer than the staging buffer fall back to a direct
// per-thread loop.  Walks row blocks [rb0, rb1); all threads must call it.
template <typename T, class F>
__device__ __forceinline__ void csr_rows_staged(const CsrArgs<T> &A, const T *__restrict__ x,
                                                int64_t rb0, int64_t rb1, F &&f, T xs = T(1)) {
#pragma clang fp contract(off)
  constexpr int kPer = kCsrLds / kWG;
  __shared__ T prod[kCsrLds];
  for (int64_t rb = rb0; rb < rb1; ++rb) {
    const int64_t r0 = rb * A.rows_per_rb;
    const int64_t r1 = (r0 + A.rows_per_rb < A.n) ? r0 + A.rows_per_rb : A.n;
    const int e0 = A.rowptr[r0];
    const int cnt = A.rowptr[r1] - e0;
    if (cnt <= kCsrLds) {
      // entries past the block's end re-read its last entry (cnt >= 1 here
      // unless the block is empty, which stores nothing), so the loads and
      // gathers need no branches and are all in flight together
      int ci[kPer];
      T vv[kPer];
      const int last = cnt > 0 ? cnt - 1 : 0;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + u * kWG;
        const int ec = e < cnt ? e : last;
        ci[u] = A.colind[e0 + ec];
        vv[u] = A.val[e0 + ec];
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) vv[u] = vv[u] * (xs * x[ci[u]]);
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + u * kWG;
        if (e < cnt) prod[e] = vv[u];
      }
      __syncthreads();
      for (int64_t row = r0 + threadIdx.x; row < r1; row += kWG) {
        const int a = A.rowptr[row] - e0, b = A.rowptr[row + 1] - e0;
        T acc = 0;
        for (int e = a; e < b; ++e) acc += prod[e];
        f(row, acc);
      }
      __syncthreads();
    } else {
      for (int64_t row = r0 + threadIdx.x; row < r1; row += kWG) {
        T acc = 0;
        for (int e = A.rowptr[row]; e < A.rowptr[row + 1]; ++e) {
          const T t = A.val[e] * (xs * x[A.colind[e]]);
          acc += t;
        }
        f(row, acc);
      }
    }
  }
}

// Loads, gathers and sums one row in chunks of U stored entries.  Every load
// of a chunk is issued before any product is summed: entries past the row's
// end re-read its last entry (a valid address, so no load needs a branch and
// all of them are in flight together) and are left out of the sum, which
// therefore has the same terms, order and rounding as a sequential product.
template <typename T, int U>
__device__ __forceinline__ T csr_row_sum(const CsrArgs<T> &A, const T *__restrict__ x, int a,
                                         int b, T xs) {
#pragma clang fp contract(off)
  T acc = 0;
  for (int e = a; e < b; e += U) {
    int ci[U];
    T vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int eu = (e + u < b) ? e + u : b - 1;
      ci[u] = A.colind[eu];
      vv[u] = A.val[eu];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) vv[u] = vv[u] * (xs * x[ci[u]]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T t = acc + vv[u];
      acc = (e + u < b) ? t : acc;
    }
  }
  return acc;
}

struct NoPre {};

// One thread per row over rows [r0, r1) (consecutive rows in consecutive
// threads): the epilogue's loads (pre(i)) and the row's first U entries and
// their gathers are all issued before any product is summed.  No LDS, no
// barriers; suits short rows.  Each row's sum has the same order and rounding
// as a sequential product.
template <typename T, class Pre, class F>
__device__ __forceinline__ void csr_rows_direct(const CsrArgs<T> &A, const T *__restrict__ x,
                                                int64_t r0, int64_t r1, Pre &&pre, F &&f,
                                                T xs = T(1)) {
  constexpr int U = 8;
  int64_t row = r0 + threadIdx.x;
  if (row >= r1) return;
  int a = A.rowptr[row], b = A.rowptr[row + 1];
  for (; row < r1; row += kWG) {
    // the next row's pointers are loaded before this row's entries, so the
    // two load chains overlap (the last step re-reads a valid pointer)
    const int64_t nr = (row + kWG < r1) ? row + kWG : row;
    const int na = A.rowptr[nr], nb = A.rowptr[nr + 1];
    const auto p = pre(row);
    f(row, csr_row_sum<T, U>(A, x, a, b, xs), p);
    a = na;
    b = nb;
  }
}

// Same, for a functor f(row, value) without prefetched epilogue data.
template <typename T, class F>
__device__ __forceinline__ void csr_rows_direct(const CsrArgs<T> &A, const T *__restrict__ x,
                                                int64_t r0, int64_t r1, F &&f) {
  csr_rows_direct(
      A, x, r0, r1, [](int64_t) { return NoPre{}; },
      [&](int64_t i, T v, const NoPre &) { f(i, v); });
}

// Sliced ELL form: each wavefront takes whole slices of 64 rows (one row per
// lane); the slice width is uniform across the wavefront, so the loop has no
// divergence, and entry u of the 64 rows is one coalesced load of the
// column indices and one of the values, independent of any row pointer.
// Padded entries (column -1) are masked out of the sum: each row's sum has
// the same terms, order and rounding as the CSR product.

// Address of stored entry u of the slice row `lane`.  Entries past the
// slice width re-read its last entry, and a slice of width 0 reads entry 0 of
// the arrays (which always hold at least one entry, not necessarily
// initialised): every address is valid, so the loads need no branches.
__device__ __forceinline__ int64_t sell_entry(int64_t off, int w, int u, int lane) {
  const int uu = (u < w) ? u : w - 1;
  return (w > 0) ? off + (int64_t)uu * kWave + lane : 0;
}

// Sliced-ELL product: the workgroup takes pieces of 4 consecutive slices,
// one per wavefront: its contiguous chunk in order, or, for a matrix larger
// than the memory-side cache, XCD-interleaved pieces (an XCD's workgroups
// then stream neighbouring slices together, which keeps HBM pages and the
// gathered x shared; measured 8 % faster at 256^3, 2 % slower on a
// cache-resident 128^3 matrix).  The headers (offset, width) of up to 64 of
// a wavefront's slices are read once, one per lane, and broadcast when a
// slice is processed.  The column indices of the next slice's first U
// entries are loaded right after the current slice's gathers and values, so
// they are in flight while the current slice is summed and stored, and the
// next gathers can be issued at once (prefetching the later passes of wide
// slices as well measured no faster on the 27-point matrix).  Only entries
// inside the width with a column >= 0 enter a sum (the others gather the
// row's own x): each row's sum has the same terms, order and rounding as the
// CSR product.
template <bool NT, typename V>
__device__ __forceinline__ V sell_ld(const V *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// Slice widths with a dedicated straight-line kernel (sell_rows_narrow): the
// 2D 5-point, 3D 7-point and 27-point operators.  0 = none (the general loop).
__host__ __device__ constexpr int sell_narrow_width(int wmax) {
  return (wmax == 5 || wmax == 7 || wmax == 27) ? wmax : 0;
}

// Sliced-ELL product for a matrix whose widest slice has exactly UW entries
// per row: each wavefront takes PAIR of its slices per step and issues, with
// no branch in between, their column loads, their value loads, their
// gathers, then the sums and stores; a step leaves no load in flight, so the
// compiler's wait counts stay tight (the general loop, whose column prefetch
// crosses iterations, ends each slice waiting for every load).  One slice per
// step: two ran no faster at 256^3 and fetched 30 % more (the second slice of
// a wavefront is a grid plane away, so its gathers miss the L2).  Entry u of a
// slice is read at the compile-time offset u * 64 from the slice's start:
// for a slice narrower than UW the entries past its width lie in the next
// slice, or in the kSellPad padding entries after the last one -- valid
// addresses whose values are masked out of the sums, which therefore have
// the same terms, order and rounding as the CSR product.  The schedule is the
// general loop's (XCD-interleaved pieces for a matrix larger than the
// memory-side cache).  Measured at 256^3: 7-point 352 -> 333 us per matrix
// power, fetching 0.97x the algorithmic bytes; 27-point 1243 -> 1111 us.
constexpr int kSellPair = 1;
template <bool NT, int PAIR, int UW, typename T, class Pre, class F>
__device__ __forceinline__ void sell_rows_narrow(const CsrArgs<T> &A, const T *__restrict__ x,
                                                 Pre &&pre, F &&f, T xs) {
#pragma clang fp contract(off)
  constexpr int U = UW;
  constexpr int WS = kWG / kWave;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  int64_t first, WSX, s1;
  if (A.sell_xcd) {
    const XcdSched sc = xcd_sched(A.nslices, WS, gridDim.x, blockIdx.x);
    first = sc.first + wave;
    WSX = sc.stride;
    s1 = sc.end;
  } else {
    int64_t s0;
    block_chunk(A.nslices, logical_block(), gridDim.x, s0, s1);
    first = s0 + wave;
    WSX = WS;
  }
  for (int64_t g0 = first; g0 < s1; g0 += WSX * kWave) {
    const int64_t left = (s1 - g0 + WSX - 1) / WSX;
    const int cnt = left < kWave ? (int)left : kWave;
    const int64_t hs = g0 + WSX * (lane < cnt ? lane : cnt - 1);
    const int64_t hoff = A.slice_off[hs];
    const int hw = A.slice_w[hs];
    const int hlo = (int)(uint32_t)hoff, hhi = (int)(hoff >> 32);
    auto header = [&](int t, int64_t &off, int &w) {
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(hlo, t);
      const int64_t hi = __builtin_amdgcn_readlane(hhi, t);
      off = (int64_t)((uint64_t)hi << 32 | lo);
      w = __builtin_amdgcn_readlane(hw, t);
    };
    for (int t = 0; t < cnt; t += PAIR) {
      int64_t off[PAIR], row[PAIR], rowc[PAIR];
      int w[PAIR];
      bool live[PAIR];
      int cc[PAIR][U];
      T vv[PAIR][U], xg[PAIR][U];
      bool ok[PAIR][U];
#pragma unroll
      for (int q = 0; q < PAIR; ++q) {
        const int tq = t + q < cnt ? t + q : t;   // a missing second slice repeats the first
        header(tq, off[q], w[q]);
        row[q] = (g0 + WSX * tq) * kWave + lane;
        live[q] = row[q] < A.n && (q == 0 || t + q < cnt);
        rowc[q] = row[q] < A.n ? row[q] : A.n - 1;
      }
      // U = the widest slice: every entry u < U of a slice of width w < U
      // lies in the next slice (or the padding after the last one), a valid
      // address at a compile-time offset, masked out below
#pragma unroll
      for (int q = 0; q < PAIR; ++q) {
        const int32_t *cp = A.sell_col + off[q] + lane;
#pragma unroll
        for (int u = 0; u < U; ++u) cc[q][u] = sell_ld<NT>(cp + u * kWave);
      }
#pragma unroll
      for (int q = 0; q < PAIR; ++q) {
        const T *vp = A.sell_val + off[q] + lane;
#pragma unroll
        for (int u = 0; u < U; ++u) vv[q][u] = sell_ld<NT>(vp + u * kWave);
      }
#pragma unroll
      for (int q = 0; q < PAIR; ++q)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          ok[q][u] = (u < w[q]) && cc[q][u] >= 0;
          xg[q][u] = x[ok[q][u] ? cc[q][u] : (int)rowc[q]];
        }
#pragma unroll
      for (int q = 0; q < PAIR; ++q) {
        const auto p = pre(rowc[q]);
        T acc = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const T pu = vv[q][u] * (xs * xg[q][u]);
          const T sum = acc + pu;
          acc = ok[q][u] ? sum : acc;
        }
        if (live[q]) f(row[q], acc, p);
      }
    }
  }
}

template <bool NT, typename T, class Pre, class F>
__device__ __forceinline__ void sell_rows(const CsrArgs<T> &A, const T *__restrict__ x, Pre &&pre,
                                          F &&f, T xs) {
#pragma clang fp contract(off)
  constexpr int U = 8;
  constexpr int WS = kWG / kWave;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  // the workgroup's slices: pieces of WS slices (one per wavefront) at
  // first, first + WSX, ... below s1
  int64_t first, WSX, s1;
  if (A.sell_xcd) {
    const XcdSched sc = xcd_sched(A.nslices, WS, gridDim.x, blockIdx.x);
    first = sc.first + wave;
    WSX = sc.stride;
    s1 = sc.end;
  } else {
    int64_t s0;
    block_chunk(A.nslices, logical_block(), gridDim.x, s0, s1);
    first = s0 + wave;
    WSX = WS;
  }
  for (int64_t g0 = first; g0 < s1; g0 += WSX * kWave) {
    // this wavefront's slices g0 + WSX t, t < cnt (cnt >= 1 since g0 < s1)
    const int64_t left = (s1 - g0 + WSX - 1) / WSX;
    const int cnt = left < kWave ? (int)left : kWave;
    const int64_t hs = g0 + WSX * (lane < cnt ? lane : cnt - 1);
    const int64_t hoff = A.slice_off[hs];
    const int hw = A.slice_w[hs];
    const int hlo = (int)(uint32_t)hoff, hhi = (int)(hoff >> 32);
    auto header = [&](int t, int64_t &off, int &w) {
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(hlo, t);
      const int64_t hi = __builtin_amdgcn_readlane(hhi, t);
      off = (int64_t)((uint64_t)hi << 32 | lo);
      w = __builtin_amdgcn_readlane(hw, t);
    };
    int64_t off;
    int w;
    header(0, off, w);
    int cc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cc[u] = sell_ld<NT>(&A.sell_col[sell_entry(off, w, u, lane)]);
    for (int t = 0; t < cnt; ++t) {
      const int64_t row = (g0 + WSX * t) * kWave + lane;
      const bool live = row < A.n;
      const int64_t rowc = live ? row : A.n - 1;
      const auto p = pre(rowc);
      const int64_t so = off;   // this slice's header (off, w move on to the next slice)
      const int sw = w;
      T acc = 0;
      for (int u0 = 0; u0 < (sw > 0 ? sw : 1); u0 += U) {
        if (u0 > 0) {
#pragma unroll
          for (int u = 0; u < U; ++u) cc[u] = sell_ld<NT>(&A.sell_col[sell_entry(so, sw, u0 + u, lane)]);
        }
        T xg[U], vv[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          ok[u] = (u0 + u < sw) && cc[u] >= 0;
          xg[u] = x[ok[u] ? cc[u] : (int)rowc];
          vv[u] = sell_ld<NT>(&A.sell_val[sell_entry(so, sw, u0 + u, lane)]);
        }
        if (u0 + U >= sw) {
          // last pass of this slice: start on the next slice's columns
          header(t + 1 < cnt ? t + 1 : t, off, w);
#pragma unroll
          for (int u = 0; u < U; ++u) cc[u] = sell_ld<NT>(&A.sell_col[sell_entry(off, w, u, lane)]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const T pu = vv[u] * (xs * xg[u]);
          const T sum = acc + pu;
          acc = ok[u] ? sum : acc;
        }
      }
      if (live) f(row, acc, p);
    }
  }
}

// The workgroup's share of a whole-matrix product (contiguous chunk).  The
// kernel form is a template parameter, so the row form carries neither the
// staging buffer nor its registers (occupancy).
template <int VARIANT, typename T, class Pre, class F>
__device__ __forceinline__ void csr_rows(const CsrArgs<T> &A, const T *__restrict__ x, Pre &&pre,
                                         F &&f, T xs) {
  if constexpr (VARIANT == CSR_ROW) {
    int64_t r0, r1;
    block_chunk(A.n, logical_block(), gridDim.x, r0, r1);
    csr_rows_direct(A, x, r0, r1, pre, f, xs);
  } else if constexpr (VARIANT == CSR_SELL) {
    // a matrix larger than the memory-side cache streams its entries with the
    // non-temporal hint (they are not reused before they would be evicted);
    // a cache-resident one keeps them cached across the matrix powers
    const int nw = sell_narrow_width(A.sell_wmax);
    if (nw == 7) {
      if (A.sell_xcd) sell_rows_narrow<true, kSellPair, 7>(A, x, pre, f, xs);
      else sell_rows_narrow<false, kSellPair, 7>(A, x, pre, f, xs);
    } else if (nw == 27) {
      if (A.sell_xcd) sell_rows_narrow<true, kSellPair, 27>(A, x, pre, f, xs);
      else sell_rows_narrow<false, kSellPair, 27>(A, x, pre, f, xs);
    } else if (nw == 5) {
      if (A.sell_xcd) sell_rows_narrow<true, kSellPair, 5>(A, x, pre, f, xs);
      else sell_rows_narrow<false, kSellPair, 5>(A, x, pre, f, xs);
    } else {
      if (A.sell_xcd) sell_rows<true>(A, x, pre, f, xs);
      else sell_rows<false>(A, x, pre, f, xs);
    }
  } else {
    int64_t rb0, rb1;
    block_chunk(A.nrb, logical_block(), gridDim.x, rb0, rb1);
    csr_rows_staged(A, x, rb0, rb1, [&](int64_t i, T v) { f(i, v, pre(i)); }, xs);
  }
}

// Harmonic mean of two cell coefficients: the face weight of the
// variable-coefficient 7-point operator for -div(k grad u).
template <typename T>
__device__ __forceinline__ T face_weight(T kp, T kq) {
#pragma clang fp contract(off)
  const T num = T(2) * kp * kq;
  return num / (kp + kq);
}

// Matrix-free grid operators over points [p0, p1); neighbour order follows
// the definitions (Dirichlet: neighbours outside the grid are absent).
// Every visitor applies the operator to xs * x, forming each xs * x[q] as a
// rounded value first: with xs = 1 that is x itself, and with the constant
// Jacobi scaling c it reproduces the product of the stored vector z = c * x
// bit for bit, so a block column z never has to be written.
template <int KIND, typename T, class F>
__device__ __forceinline__ void stencil_rows(const StencilArgs<T> &S, const T *__restrict__ x,
                                             int64_t p0, int64_t p1, F &&f, T xs = T(1)) {
#pragma clang fp contract(off)
  const int nx = S.nx, ny = S.ny, nz = S.nz;
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += kWG) {
    int64_t rx, ry;
    const int64_t yz = fdiv(p, S.fx, rx);
    const int64_t zq = fdiv(yz, S.fy, ry);
    const int xq = (int)rx, yq = (int)ry, z = (int)zq;
    T acc;
    if constexpr (KIND == K_3D27) {
      // all 26 neighbour loads first (out-of-grid ones re-read x[p]), then
      // the sum over the neighbours inside the grid in definition order
      T v[27];
      bool in[27];
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const bool ok = z + dz >= 0 && z + dz < nz && yq + dy >= 0 && yq + dy < ny &&
                        xq + dx >= 0 && xq + dx < nx && t != 13;
        in[t] = ok;
        v[t] = xs * x[ok ? p + dz * sz + dy * sy + dx : p];
      }
      T nb = 0;
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const T u = nb + v[t];
        nb = in[t] ? u : nb;
      }
      const T d = S.diag * v[13];
      const T o = S.off * nb;
      acc = d + o;
    } else if constexpr (KIND == K_VARK) {
      const T kp = S.k[p];
      const bool in[6] = {z > 0, yq > 0, xq > 0, xq < nx - 1, yq < ny - 1, z < nz - 1};
      const int64_t q[6] = {p - sz, p - sy, p - 1, p + 1, p + sy, p + sz};
      T kq[6], xv[6];
#pragma unroll
      for (int f6 = 0; f6 < 6; ++f6) {
        const int64_t qq = in[f6] ? q[f6] : p;
        kq[f6] = S.k[qq];
        xv[f6] = xs * x[qq];
      }
      const T xp = xs * x[p];
      T dsum = 0, nb = 0;
#pragma unroll
      for (int f6 = 0; f6 < 6; ++f6) {
        const T w = face_weight(kp, kq[f6]);
        const T t = w * xv[f6];
        const T nb1 = nb + t;
        const T ds1 = dsum + (in[f6] ? w : kp);
        nb = in[f6] ? nb1 : nb;
        dsum = ds1;
      }
      const T d = dsum * xp;
      acc = d - nb;
    } else {
      const T xm = xs * x[xq > 0 ? p - 1 : p], xpl = xs * x[xq < nx - 1 ? p + 1 : p];
      const T ym = xs * x[yq > 0 ? p - sy : p], ypl = xs * x[yq < ny - 1 ? p + sy : p];
      T zm = 0, zpl = 0;
      if constexpr (KIND == K_3D7) {
        zm = xs * x[z > 0 ? p - sz : p];
        zpl = xs * x[z < nz - 1 ? p + sz : p];
      }
      const T xc = xs * x[p];
      T nb = 0;
      nb = xq > 0 ? nb + xm : nb;
      nb = xq < nx - 1 ? nb + xpl : nb;
      nb = yq > 0 ? nb + ym : nb;
      nb = yq < ny - 1 ? nb + ypl : nb;
      if constexpr (KIND == K_3D7) {
        nb = z > 0 ? nb + zm : nb;
        nb = z < nz - 1 ? nb + zpl : nb;
      }
      const T d = S.diag * xc;
      const T o = S.off * nb;
      acc = d + o;
    }
    f(p, acc);
  }
}

// Tiling of the LDS-staged 3D stencil kernels: a workgroup owns a kTX x kTY
// block of a grid plane (one point per thread) and marches through zchunk
// planes, keeping planes z-1, z, z+1 (with a one-cell halo) in LDS, so every
// x value is read from memory about 1.5x instead of once per neighbour.
constexpr int kTX = 64, kTY = kWG / kTX;
struct Tiling3 {
  int ntx, nty, ntz, zchunk;
};

// False when the kind is not tiled or a plane has more tiles than a launch
// may hold.  Only the 27-point operator is tiled: its 26 neighbour gathers
// made the cache-served kernel L2-bound (256^3: 1.75x faster tiled), while
// the 7-point kernel runs faster cache-served (128^3: 11.3 vs 14.7 us per
// product) and 2D and variable-coefficient operators are not tiled.
inline bool stencil_tiling(int kind, int nx, int ny, int nz, Tiling3 &t) {
  if (kind != K_3D27) return false;
  t.ntx = (nx + kTX - 1) / kTX;
  t.nty = (ny + kTY - 1) / kTY;
  const int64_t plane = (int64_t)t.ntx * t.nty;
  if (plane > kGridMax) return false;
  int64_t ntz = kGridMax / plane;          // fill the launch ...
  const int64_t by_depth = nz / 8;         // ... but march at least 8 planes
  if (ntz > by_depth) ntz = by_depth;
  if (ntz < 1) ntz = 1;
  t.zchunk = (int)((nz + ntz - 1) / ntz);
  t.ntz = (nz + t.zchunk - 1) / t.zchunk;
  return true;
}

}  // namespace ssp
