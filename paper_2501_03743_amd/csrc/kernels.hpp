// Streaming kernels of libsstep (gfx950): operator application with fused
// epilogues (matrix powers, moments, residuals), the fused block update, and
// the standard-CG kernels.
//
// Every operator kernel visits each row once and hands (row, (A x)_row) to an
// epilogue functor that writes the outputs of that row and accumulates the
// per-thread partial sums of the inner products the step needs.  Each
// workgroup stores its sums; a single-workgroup finalisation kernel launched
// next on the same stream reduces them in a fixed order (deterministic
// results) and finishes the step on the GPU (moments -> s x s solve, residual
// norm -> stopping test), so no host round trip is needed inside an
// iteration.  The kernel boundary orders the two: no device-scope fences or
// atomics in the streaming kernels.
#pragma once

#include "common.hpp"
#include "small_solve.hpp"

namespace ssp {

// --------------------------------------------------------------------------
// Operators
// --------------------------------------------------------------------------

struct CsrArgs {
  int64_t n;
  const int32_t *rowptr;
  const int32_t *colind;
  const double *val;
  int rows_per_rb;   // rows per LDS row block (<= kCsrRowsMax)
  int64_t nrb;       // number of row blocks
  int variant;       // CSR_STAGED or CSR_ROW (chosen per matrix by timing)
};

enum : int { CSR_STAGED = 0, CSR_ROW = 1 };

struct StencilArgs {
  int64_t n;
  int nx, ny, nz;
  FastDiv fx, fy;    // divisions by nx and ny
  double diag, off;
  const double *k;   // variable coefficient (VARK)
};

enum : int { K_2D5 = 1, K_3D7 = 2, K_3D27 = 3, K_VARK = 4 };

// Rows of one CSR row block (at most kCsrLds stored entries) are staged as
// products val*x in LDS: every thread first issues all its coalesced loads of
// colind and val, then all its gathers of x, so each workgroup keeps up to
// kCsrLds/kWG independent loads in flight.  Each thread then sums its rows in
// column order (products rounded, then added: bitwise equal to a sequential
// row-order CSR product without FMA contraction).  Rows longer than the
// staging buffer fall back to a direct per-thread loop.
template <class F>
__device__ __forceinline__ void csr_rows_staged(const CsrArgs &A, const double *__restrict__ x, F &&f) {
#pragma clang fp contract(off)
  constexpr int kPer = kCsrLds / kWG;
  __shared__ double prod[kCsrLds];
  int64_t rb0, rb1;
  block_chunk(A.nrb, logical_block(), gridDim.x, rb0, rb1);
  for (int64_t rb = rb0; rb < rb1; ++rb) {
    const int64_t r0 = rb * A.rows_per_rb;
    const int64_t r1 = (r0 + A.rows_per_rb < A.n) ? r0 + A.rows_per_rb : A.n;
    const int e0 = A.rowptr[r0];
    const int cnt = A.rowptr[r1] - e0;
    if (cnt <= kCsrLds) {
      int ci[kPer];
      double vv[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + u * kWG;
        if (e < cnt) {
          ci[u] = A.colind[e0 + e];
          vv[u] = A.val[e0 + e];
        }
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + u * kWG;
        if (e < cnt) vv[u] = vv[u] * x[ci[u]];
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + u * kWG;
        if (e < cnt) prod[e] = vv[u];
      }
      __syncthreads();
      for (int64_t row = r0 + threadIdx.x; row < r1; row += kWG) {
        const int a = A.rowptr[row] - e0, b = A.rowptr[row + 1] - e0;
        double acc = 0.0;
        for (int e = a; e < b; ++e) acc += prod[e];
        f(row, acc);
      }
      __syncthreads();
    } else {
      for (int64_t row = r0 + threadIdx.x; row < r1; row += kWG) {
        double acc = 0.0;
        for (int e = A.rowptr[row]; e < A.rowptr[row + 1]; ++e) {
          const double t = A.val[e] * x[A.colind[e]];
          acc += t;
        }
        f(row, acc);
      }
    }
  }
}

// One thread per row, rows of a workgroup contiguous: each thread issues the
// loads of up to 8 stored entries of its row at once, then their gathers,
// then sums in column order (same rounding as the staged form).  No LDS and
// no barriers; suits short rows.
template <class F>
__device__ __forceinline__ void csr_rows_direct(const CsrArgs &A, const double *__restrict__ x,
                                                F &&f) {
#pragma clang fp contract(off)
  constexpr int U = 8;
  int64_t r0, r1;
  block_chunk(A.n, logical_block(), gridDim.x, r0, r1);
  for (int64_t row = r0 + threadIdx.x; row < r1; row += kWG) {
    const int a = A.rowptr[row], b = A.rowptr[row + 1];
    double acc = 0.0;
    for (int e = a; e < b; e += U) {
      int ci[U];
      double vv[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e + u < b) {
          ci[u] = A.colind[e + u];
          vv[u] = A.val[e + u];
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e + u < b) vv[u] = vv[u] * x[ci[u]];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e + u < b) acc += vv[u];
    }
    f(row, acc);
  }
}

template <class F>
__device__ __forceinline__ void csr_rows(const CsrArgs &A, const double *__restrict__ x, F &&f) {
  if (A.variant == CSR_ROW) csr_rows_direct(A, x, f);
  else csr_rows_staged(A, x, f);
}

// Matrix-free grid operators; neighbour order and rounding follow the
// definitions (Dirichlet: neighbours outside the grid are absent).
template <int KIND, class F>
__device__ __forceinline__ void stencil_rows(const StencilArgs &S, const double *__restrict__ x,
                                             F &&f) {
#pragma clang fp contract(off)
  int64_t p0, p1;
  block_chunk(S.n, logical_block(), gridDim.x, p0, p1);
  const int nx = S.nx, ny = S.ny, nz = S.nz;
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += kWG) {
    int64_t rx, ry;
    const int64_t yz = fdiv(p, S.fx, rx);
    const int64_t zq = fdiv(yz, S.fy, ry);
    const int xq = (int)rx, yq = (int)ry, z = (int)zq;
    double acc;
    if constexpr (KIND == K_3D27) {
      double nb = 0.0;
      for (int dz = -1; dz <= 1; ++dz) {
        const int qz = z + dz;
        if (qz < 0 || qz >= nz) continue;
        for (int dy = -1; dy <= 1; ++dy) {
          const int qy = yq + dy;
          if (qy < 0 || qy >= ny) continue;
          const double *row = x + (int64_t)qz * sz + (int64_t)qy * sy;
          for (int dx = -1; dx <= 1; ++dx) {
            const int qx = xq + dx;
            if (qx < 0 || qx >= nx) continue;
            if (dx == 0 && dy == 0 && dz == 0) continue;
            nb += row[qx];
          }
        }
      }
      const double d = S.diag * x[p];
      const double o = S.off * nb;
      acc = d + o;
    } else if constexpr (KIND == K_VARK) {
      const double kp = S.k[p];
      const bool in[6] = {z > 0, yq > 0, xq > 0, xq < nx - 1, yq < ny - 1, z < nz - 1};
      const int64_t q[6] = {p - sz, p - sy, p - 1, p + 1, p + sy, p + sz};
      double dsum = 0.0, nb = 0.0;
#pragma unroll
      for (int f6 = 0; f6 < 6; ++f6) {
        if (in[f6]) {
          const double kq = S.k[q[f6]];
          const double num = 2.0 * kp * kq;
          const double w = num / (kp + kq);
          dsum += w;
          const double t = w * x[q[f6]];
          nb += t;
        } else {
          dsum += kp;
        }
      }
      const double d = dsum * x[p];
      acc = d - nb;
    } else {
      double nb = 0.0;
      if (xq > 0) nb += x[p - 1];
      if (xq < nx - 1) nb += x[p + 1];
      if (yq > 0) nb += x[p - sy];
      if (yq < ny - 1) nb += x[p + sy];
      if constexpr (KIND == K_3D7) {
        if (z > 0) nb += x[p - sz];
        if (z < nz - 1) nb += x[p + sz];
      }
      const double d = S.diag * x[p];
      const double o = S.off * nb;
      acc = d + o;
    }
    f(p, acc);
  }
}

// --------------------------------------------------------------------------
// Epilogues
// --------------------------------------------------------------------------

// Jacobi (or identity) preconditioner: z = dinv .* v.
struct Prec {
  const double *dinv;  // nullptr: constant dc
  double dc;
  __device__ __forceinline__ double apply(int64_t i, double v) const {
#pragma clang fp contract(off)
    return (dinv ? dinv[i] : dc) * v;
  }
};

struct EpiStore {
  static constexpr int NP = 0;
  static constexpr bool kCheck = false;
  double *y;
  __device__ __forceinline__ void row(int64_t i, double v, double *) const { y[i] = v; }
  __device__ __forceinline__ void finish(DevState *, const double *) const {}
};

// Matrix powers, power j < s: AZ(:,j) = A Z(:,j), Z(:,j+1) = B^-1 AZ(:,j).
struct EpiMpk {
  static constexpr int NP = 0;
  static constexpr bool kCheck = true;
  double *az, *znext;
  Prec pc;
  __device__ __forceinline__ void row(int64_t i, double v, double *) const {
    az[i] = v;
    znext[i] = pc.apply(i, v);
  }
  __device__ __forceinline__ void finish(DevState *, const double *) const {}
};

// Last power j = s, fused with Alg. 5: AZ(:,s) = A Z(:,s) and the partial
// sums of vm(a) = Z(:,a)^T r and vm(s+a) = Z(:,a)^T AZ(:,s), a = 1..s.  The
// last workgroup reduces them and runs the s x s solve.
template <int S>
struct EpiMpkLast {
  static constexpr int NP = 2 * S;
  static constexpr bool kCheck = true;
  double *az;
  const double *Z;  // column a at Z + a*ld
  int64_t ld;
  const double *r;
  int solve;        // 0: only store vm (the stand-alone Alg. 4 + Alg. 5 call)
  __device__ __forceinline__ void row(int64_t i, double v, double *part) const {
    az[i] = v;
    const double ri = r[i];
#pragma unroll
    for (int a = 0; a < S; ++a) {
      const double za = Z[(int64_t)a * ld + i];
      part[a] += za * ri;
      part[S + a] += za * v;
    }
  }
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (solve) {
      small_solve(st, S, tot);
    } else if (threadIdx.x < NP) {
      st->vm[threadIdx.x] = tot[threadIdx.x];
    }
  }
};

// r = b - A x, z1 = B^-1 r, with ||b||^2 and ||r||^2; initialises the solve.
struct EpiInit {
  static constexpr int NP = 2;
  static constexpr bool kCheck = false;
  const double *b;
  double *r, *z1;
  Prec pc;
  double *hist;
  __device__ __forceinline__ void row(int64_t i, double v, double *part) const {
#pragma clang fp contract(off)
    const double bi = b[i];
    const double ri = bi - v;
    r[i] = ri;
    z1[i] = pc.apply(i, ri);
    part[0] += bi * bi;
    part[1] += ri * ri;
  }
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (threadIdx.x == 0) {
      const double bb = tot[0], rr = tot[1];
      st->bb = bb;
      st->rr = rr;
      st->k = 0;
      const double bn = sqrt(bb), rn = sqrt(rr);
      if (st->hist_cap > 0) hist[0] = bb > 0.0 ? rn / bn : 0.0;
      int status = ST_RUNNING;
      if (bb == 0.0) status = ST_ZERO_RHS;
      else if (!st->fixed && rn <= st->rtol * bn) status = ST_CONVERGED;
      else if (st->outer_max <= 0) status = ST_MAXIT;
      st->status = status;
    }
  }
};

// PCG start (Alg. 1): r = b - A x, p = u = B^-1 r, rho = u^T r.
struct EpiPcgInit {
  static constexpr int NP = 3;
  static constexpr bool kCheck = false;
  const double *b;
  double *r, *p;
  Prec pc;
  double *hist;
  __device__ __forceinline__ void row(int64_t i, double v, double *part) const {
#pragma clang fp contract(off)
    const double bi = b[i];
    const double ri = bi - v;
    const double ui = pc.apply(i, ri);
    r[i] = ri;
    p[i] = ui;
    part[0] += bi * bi;
    part[1] += ri * ri;
    part[2] += ui * ri;
  }
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (threadIdx.x == 0) {
      const double bb = tot[0], rr = tot[1];
      st->bb = bb;
      st->rr = rr;
      st->rho = tot[2];
      st->k = 0;
      const double bn = sqrt(bb), rn = sqrt(rr);
      if (st->hist_cap > 0) hist[0] = bb > 0.0 ? rn / bn : 0.0;
      int status = ST_RUNNING;
      if (bb == 0.0) status = ST_ZERO_RHS;
      else if (!st->fixed && rn <= st->rtol * bn) status = ST_CONVERGED;
      else if (st->outer_max <= 0) status = ST_MAXIT;
      st->status = status;
    }
  }
};

// PCG: s = A p with p^T s; alpha = rho / p^T s.
struct EpiPcgSpmv {
  static constexpr int NP = 1;
  static constexpr bool kCheck = true;
  const double *p;
  double *sv;
  __device__ __forceinline__ void row(int64_t i, double v, double *part) const {
    sv[i] = v;
    part[0] += p[i] * v;
  }
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (threadIdx.x == 0) {
      const double ps = tot[0];
      const double a = st->rho / ps;
      if (!(ps > 0.0) || !isfinite(a)) st->status = ST_BREAKDOWN;
      else st->pcg_alpha = a;
    }
  }
};

// ||b - A x||^2 of the final iterate (runs whatever the status).
struct EpiTrueRes {
  static constexpr int NP = 1;
  static constexpr bool kCheck = false;
  const double *b;
  __device__ __forceinline__ void row(int64_t i, double v, double *part) const {
#pragma clang fp contract(off)
    const double t = b[i] - v;
    part[0] += t * t;
  }
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (threadIdx.x == 0) st->true_rr = tot[0];
  }
};

// --------------------------------------------------------------------------
// Kernels
// --------------------------------------------------------------------------

template <class Epi>
__device__ __forceinline__ void epi_tail(const double (&part)[Epi::NP > 0 ? Epi::NP : 1],
                                         double *partials) {
  if constexpr (Epi::NP > 0) {
    double v[Epi::NP];
#pragma unroll
    for (int c = 0; c < Epi::NP; ++c) v[c] = part[c];
    block_store_sums<Epi::NP>(v, partials + blockIdx.x, gridDim.x);
  }
}

// Finalisation of a reducing step: one workgroup reduces the G partials and
// applies the step's finish() (s x s solve, stopping test, ...).
template <class Fin>
__global__ __launch_bounds__(kWG) void k_finalize(Fin fin, DevState *st, const double *partials,
                                                  int G) {
  if (Fin::kCheck && st->status != ST_RUNNING) return;
  double tot[Fin::NP];
  reduce_partials<Fin::NP>(partials, G, tot);
  fin.finish(st, tot);
}

template <class Epi>
__global__ __launch_bounds__(kWG) void k_csr(CsrArgs A, const double *__restrict__ x, Epi epi,
                                             DevState *st, double *partials) {
  if (Epi::kCheck && st->status != ST_RUNNING) return;
  double part[Epi::NP > 0 ? Epi::NP : 1];
#pragma unroll
  for (int c = 0; c < (Epi::NP > 0 ? Epi::NP : 1); ++c) part[c] = 0.0;
  csr_rows(A, x, [&](int64_t i, double v) { epi.row(i, v, part); });
  epi_tail<Epi>(part, partials);
}

template <int KIND, class Epi>
__global__ __launch_bounds__(kWG) void k_stencil(StencilArgs S, const double *__restrict__ x,
                                                 Epi epi, DevState *st, double *partials) {
  if (Epi::kCheck && st->status != ST_RUNNING) return;
  double part[Epi::NP > 0 ? Epi::NP : 1];
#pragma unroll
  for (int c = 0; c < (Epi::NP > 0 ? Epi::NP : 1); ++c) part[c] = 0.0;
  stencil_rows<KIND>(S, x, [&](int64_t i, double v) { epi.row(i, v, part); });
  epi_tail<Epi>(part, partials);
}

// Fused block update (Alg. 3, in the order of its four update lines), one
// thread per row computing all s outputs:
//   P  = Z  + P_old  beta          (skipped at k = 0: P_old = 0)
//   x  = x  + P alpha
//   AP = AZ + AP_old beta
//   r  = r  - AP alpha
// then z1 = B^-1 r for the next matrix powers (column 1 of the other block,
// whose row was just read by the same thread) and the partial sums of
// ||r||^2 (finished by FinUpdate).
template <int S>
__global__ __launch_bounds__(kWG) void k_update(int64_t n, int64_t ld, double *__restrict__ Pc,
                                                double *__restrict__ Po, double *__restrict__ x,
                                                double *__restrict__ r, Prec pc, DevState *st,
                                                double *partials) {
#pragma clang fp contract(off)
  if (st->status != ST_RUNNING) return;
  const int k = st->k;
  double alpha[S], beta[S][S];
#pragma unroll
  for (int j = 0; j < S; ++j) alpha[j] = st->alpha[j];
  if (k > 0) {
#pragma unroll
    for (int l = 0; l < S; ++l)
#pragma unroll
      for (int j = 0; j < S; ++j) beta[l][j] = st->beta[l * S + j];
  }
  double part[1] = {0.0};
  int64_t lo, hi;
  block_chunk(n, logical_block(), gridDim.x, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) {
    double p[S], ap[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
      p[j] = Pc[(int64_t)j * ld + i];
      ap[j] = Pc[(int64_t)(S + j) * ld + i];
    }
    if (k > 0) {
      double po[S], apo[S];
#pragma unroll
      for (int l = 0; l < S; ++l) {
        po[l] = Po[(int64_t)l * ld + i];
        apo[l] = Po[(int64_t)(S + l) * ld + i];
      }
#pragma unroll
      for (int j = 0; j < S; ++j) {
        double a = p[j], b = ap[j];
#pragma unroll
        for (int l = 0; l < S; ++l) {
          const double t = po[l] * beta[l][j];
          a += t;
          const double u = apo[l] * beta[l][j];
          b += u;
        }
        p[j] = a;
        ap[j] = b;
      }
#pragma unroll
      for (int j = 0; j < S; ++j) {
        Pc[(int64_t)j * ld + i] = p[j];
        Pc[(int64_t)(S + j) * ld + i] = ap[j];
      }
    }
    double dx = 0.0, dr = 0.0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const double t = p[j] * alpha[j];
      dx += t;
      const double u = ap[j] * alpha[j];
      dr += u;
    }
    const double xi = x[i] + dx;
    const double ri = r[i] - dr;
    x[i] = xi;
    r[i] = ri;
    Po[i] = pc.apply(i, ri);
    part[0] += ri * ri;
  }
  double v[1] = {part[0]};
  block_store_sums<1>(v, partials + blockIdx.x, gridDim.x);
}

// After the block update: ||r||^2, history entry, stopping test, k += 1.
struct FinUpdate {
  static constexpr int NP = 1;
  static constexpr bool kCheck = true;
  double *hist;
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (threadIdx.x == 0) {
      const double rr = tot[0];
      const int kk = st->k + 1;
      st->rr = rr;
      st->k = kk;
      const double rn = sqrt(rr), bn = sqrt(st->bb);
      if (kk < st->hist_cap) hist[kk] = rn / bn;
      const bool conv = rn <= st->rtol * bn;
      if (!st->fixed && conv) st->status = ST_CONVERGED;
      else if (kk >= st->outer_max) st->status = (st->fixed && conv) ? ST_CONVERGED : ST_MAXIT;
    }
  }
};

// PCG (Alg. 1) update: x += alpha p, r -= alpha s, u = B^-1 r; partial sums
// of u^T r and ||r||^2 (finished by FinPcgUpdate).
__global__ __launch_bounds__(kWG) void k_pcg_update(int64_t n, double *__restrict__ x,
                                                    double *__restrict__ r,
                                                    const double *__restrict__ p,
                                                    const double *__restrict__ sv, Prec pc,
                                                    DevState *st, double *partials) {
#pragma clang fp contract(off)
  if (st->status != ST_RUNNING) return;
  const double a = st->pcg_alpha;
  double ur = 0.0, rr = 0.0;
  int64_t lo, hi;
  block_chunk(n, logical_block(), gridDim.x, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) {
    const double ap = a * p[i];
    const double xi = x[i] + ap;
    const double as = a * sv[i];
    const double ri = r[i] - as;
    x[i] = xi;
    r[i] = ri;
    const double ui = pc.apply(i, ri);
    ur += ui * ri;
    rr += ri * ri;
  }
  double v[2] = {ur, rr};
  block_store_sums<2>(v, partials + blockIdx.x, gridDim.x);
}

// After the PCG update: beta = u_{k+1}^T r_{k+1} / u_k^T r_k, history entry,
// stopping test, k += 1.
struct FinPcgUpdate {
  static constexpr int NP = 2;
  static constexpr bool kCheck = true;
  double *hist;
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (threadIdx.x == 0) {
      const double urn = tot[0], rrn = tot[1];
      st->pcg_beta = urn / st->rho;
      st->rho = urn;
      st->rr = rrn;
      const int kk = st->k + 1;
      st->k = kk;
      const double rn = sqrt(rrn), bn = sqrt(st->bb);
      if (kk < st->hist_cap) hist[kk] = rn / bn;
      const bool conv = rn <= st->rtol * bn;
      if (!st->fixed && conv) st->status = ST_CONVERGED;
      else if (kk >= st->outer_max) st->status = (st->fixed && conv) ? ST_CONVERGED : ST_MAXIT;
    }
  }
};

// PCG direction: p = u + beta p with u = B^-1 r recomputed from r.
__global__ __launch_bounds__(kWG) void k_pcg_direction(int64_t n, const double *__restrict__ r,
                                                       double *__restrict__ p, Prec pc,
                                                       const DevState *st) {
#pragma clang fp contract(off)
  // the new direction only matters while the iteration continues
  if (st->status != ST_RUNNING) return;
  const double b = st->pcg_beta;
  int64_t lo, hi;
  block_chunk(n, logical_block(), gridDim.x, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) {
    const double ui = pc.apply(i, r[i]);
    const double t = b * p[i];
    p[i] = ui + t;
  }
}

// z = B^-1 v on its own (first column of the stand-alone matrix powers).
__global__ __launch_bounds__(kWG) void k_prec(int64_t n, const double *__restrict__ v,
                                              double *__restrict__ z, Prec pc) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) z[i] = pc.apply(i, v[i]);
}

// Jacobi: dinv_i = 1 / a_ii from a CSR matrix (sum of diagonal entries; a
// missing or non-positive diagonal gives a non-finite or negative value,
// which the solve reports as a breakdown).
__global__ __launch_bounds__(kWG) void k_csr_dinv(int64_t n, const int32_t *rowptr,
                                                  const int32_t *colind, const double *val,
                                                  double *dinv) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e)
    if (colind[e] == i) d += val[e];
  dinv[i] = 1.0 / d;
}

// Jacobi for the variable-coefficient stencil: the diagonal is the sum of the
// six face weights.
__global__ __launch_bounds__(kWG) void k_vark_dinv(StencilArgs S, double *dinv) {
#pragma clang fp contract(off)
  const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (p >= S.n) return;
  int64_t rx, ry;
  const int64_t yz = fdiv(p, S.fx, rx);
  const int64_t zq = fdiv(yz, S.fy, ry);
  const int xq = (int)rx, yq = (int)ry, z = (int)zq;
  const int nx = S.nx, ny = S.ny, nz = S.nz;
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  const double kp = S.k[p];
  const bool in[6] = {z > 0, yq > 0, xq > 0, xq < nx - 1, yq < ny - 1, z < nz - 1};
  const int64_t q[6] = {p - sz, p - sy, p - 1, p + 1, p + sy, p + sz};
  double dsum = 0.0;
  for (int f = 0; f < 6; ++f) {
    if (in[f]) {
      const double kq = S.k[q[f]];
      const double num = 2.0 * kp * kq;
      dsum += num / (kp + kq);
    } else {
      dsum += kp;
    }
  }
  dinv[p] = 1.0 / dsum;
}

// Row lengths of a stencil operator in CSR form (rowptr is their prefix sum).
template <int KIND>
__global__ __launch_bounds__(kWG) void k_stencil_rowlen(StencilArgs S, int32_t *len) {
  const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (p >= S.n) return;
  int64_t rx, ry;
  const int64_t yz = fdiv(p, S.fx, rx);
  const int64_t zq = fdiv(yz, S.fy, ry);
  const int xq = (int)rx, yq = (int)ry, z = (int)zq;
  const int cx = 1 + (xq > 0) + (xq < S.nx - 1);
  const int cy = 1 + (yq > 0) + (yq < S.ny - 1);
  const int cz = (KIND == K_2D5) ? 1 : 1 + (z > 0) + (z < S.nz - 1);
  int c;
  if (KIND == K_3D27) c = cx * cy * cz;
  else c = 1 + (cx - 1) + (cy - 1) + (cz - 1);
  len[p] = c;
}

// Fills colind/val of a stencil operator in CSR form, columns ascending.
template <int KIND>
__global__ __launch_bounds__(kWG) void k_stencil_fill(StencilArgs S, const int32_t *rowptr,
                                                      int32_t *colind, double *val) {
#pragma clang fp contract(off)
  const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (p >= S.n) return;
  int64_t rx, ry;
  const int64_t yz = fdiv(p, S.fx, rx);
  const int64_t zq = fdiv(yz, S.fy, ry);
  const int xq = (int)rx, yq = (int)ry, z = (int)zq;
  const int nx = S.nx, ny = S.ny, nz = S.nz;
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  int e = rowptr[p];
  if constexpr (KIND == K_3D27) {
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int qx = xq + dx, qy = yq + dy, qz = z + dz;
          if (qx < 0 || qx >= nx || qy < 0 || qy >= ny || qz < 0 || qz >= nz) continue;
          colind[e] = (int32_t)(qx + sy * qy + sz * qz);
          val[e] = (dx == 0 && dy == 0 && dz == 0) ? S.diag : S.off;
          ++e;
        }
  } else {
    const bool in[6] = {KIND != K_2D5 && z > 0, yq > 0, xq > 0, xq < nx - 1, yq < ny - 1,
                        KIND != K_2D5 && z < nz - 1};
    const int64_t q[6] = {p - sz, p - sy, p - 1, p + 1, p + sy, p + sz};
    double w[6];
    double dsum = 0.0;
    if constexpr (KIND == K_VARK) {
      const double kp = S.k[p];
      for (int f = 0; f < 6; ++f) {
        if (in[f]) {
          const double kq = S.k[q[f]];
          const double num = 2.0 * kp * kq;
          w[f] = num / (kp + kq);
        } else {
          w[f] = kp;
        }
        dsum += w[f];
      }
    }
    for (int f = 0; f < 3; ++f)
      if (in[f]) {
        colind[e] = (int32_t)q[f];
        val[e] = (KIND == K_VARK) ? -w[f] : S.off;
        ++e;
      }
    colind[e] = (int32_t)p;
    val[e] = (KIND == K_VARK) ? dsum : S.diag;
    ++e;
    for (int f = 3; f < 6; ++f)
      if (in[f]) {
        colind[e] = (int32_t)q[f];
        val[e] = (KIND == K_VARK) ? -w[f] : S.off;
        ++e;
      }
  }
}

// Longest row of a CSR matrix (one atomicMax per workgroup).
__global__ __launch_bounds__(kWG) void k_csr_maxrow(int64_t n, const int32_t *rowptr,
                                                    int *out) {
  __shared__ int m[kWG];
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  m[threadIdx.x] = (i < n) ? rowptr[i + 1] - rowptr[i] : 0;
  __syncthreads();
  for (int o = kWG / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) m[threadIdx.x] = max(m[threadIdx.x], m[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, m[0]);
}

// CSR validation: rowptr[0] = 0, monotone, columns in range and strictly
// ascending per row, a positive diagonal entry.  Sets *bad on a violation.
__global__ __launch_bounds__(kWG) void k_csr_validate(int64_t n, int64_t nnz,
                                                      const int32_t *rowptr,
                                                      const int32_t *colind, const double *val,
                                                      int *bad) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  const int a = rowptr[i], b = rowptr[i + 1];
  int ok = (a >= 0) && (b >= a) && (b <= nnz) && (i > 0 || a == 0) && (i < n - 1 || b == nnz);
  double d = 0.0;
  if (ok) {
    int prev = -1;
    for (int e = a; e < b; ++e) {
      const int c = colind[e];
      if (c < 0 || c >= n || c <= prev) { ok = 0; break; }
      prev = c;
      if (c == i) d += val[e];
    }
  }
  if (!(d > 0.0)) ok = 0;
  if (!ok) atomicOr(bad, 1);
}

}  // namespace ssp
