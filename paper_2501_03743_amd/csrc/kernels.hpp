// Streaming kernels of libsstep (gfx950): operator application with fused
// epilogues (matrix powers, moments, residuals), the fused block update, the
// standard-CG kernels and the iterative-refinement glue.
//
// Every operator kernel visits each row once and hands (row, (A x)_row) to an
// epilogue functor that writes the outputs of that row and accumulates the
// per-thread partial sums of the inner products the step needs.  Each
// workgroup stores its sums; a single-workgroup finalisation kernel launched
// next on the same stream reduces them in a fixed order (deterministic
// results) and finishes the step on the GPU (moments -> s x s solve, residual
// norm -> stopping test), so no host round trip is needed inside an
// iteration.  The kernel boundary orders the two: there are no device-scope
// fences or atomics in the streaming kernels.
//
// T is the precision of the matrix and of the vectors (double, or float for
// the inner solves of mixed-precision refinement); inner products, moments
// and the s x s algebra are always FP64.
#pragma once

#include "common.hpp"
#include "operators.hpp"
#include "small_solve.hpp"

namespace ssp {

// --------------------------------------------------------------------------
// Epilogues (row functors) and their finalisations
// --------------------------------------------------------------------------

template <typename T>
struct EpiStore {
  static constexpr int NP = 0;
  static constexpr bool kCheck = false;
  T *y;
  __device__ __forceinline__ void row(int64_t i, T v, double *) const { y[i] = v; }
  __device__ __forceinline__ void finish(DevState *, const double *) const {}
};

// Matrix powers, power j < s (Alg. 4): AZ(:,j) = A Z(:,j), Z(:,j+1) = B^-1 AZ(:,j).
// With a constant Jacobi scaling c, Z(:,j+1) = c AZ(:,j) is not stored
// (znext = nullptr): its readers form c * AZ(i,j) themselves, the same
// rounded value.
template <typename T>
struct EpiMpk {
  static constexpr int NP = 0;
  static constexpr bool kCheck = true;
  T *az, *znext;
  Prec<T> pc;
  __device__ __forceinline__ void row(int64_t i, T v, double *) const {
    az[i] = v;
    if (znext) znext[i] = pc.apply(i, v);
  }
  __device__ __forceinline__ void finish(DevState *, const double *) const {}
};

// Last power j = s, fused with Alg. 5: AZ(:,s) = A Z(:,s) and the partial
// sums of vm(a) = Z(:,a)^T r and vm(s+a) = Z(:,a)^T AZ(:,s), a = 1..s, in
// FP64 (FP32 products are exact in FP64).  Finalised by the s x s solve.
// After a block update: ||r||^2 = rr, history entry, stopping test, k += 1
// (thread 0).
__device__ __forceinline__ void fin_update(DevState *st, double rr, double *hist) {
  const int kk = st->k + 1;
  st->rr = rr;
  st->k = kk;
  const double rn = sqrt(rr), bn = sqrt(st->bb);
  if (kk < st->hist_cap) hist[kk] = rn / bn;
  const bool conv = rn <= st->rtol * bn;
  if (!st->fixed && conv) st->status = ST_CONVERGED;
  else if (kk >= st->outer_max) st->status = (st->fixed && conv) ? ST_CONVERGED : ST_MAXIT;
}

template <int S, typename T>
struct EpiMpkLast {
  static constexpr int NP = 2 * S;
  static constexpr bool kCheck = true;
  T *az;
  const T *Z;       // the block: Z(:,a) at column a-1, AZ(:,a) at column S+a-1
  int64_t ld;
  const T *r;
  int solve;        // 0: only store vm (the stand-alone Alg. 4 + Alg. 5 call)
  T zc;             // 0: Z stored; else the constant Jacobi scaling c, with
                    // Z(:,1) = c r and Z(:,a) = c AZ(:,a-1) formed here
  // the previous block update's ||r||^2 partials, finished here first (its
  // stopping test) instead of by a launch of their own; nullptr: none
  const double *rr_part;
  int rr_G;
  double *hist;
  __device__ __forceinline__ void row(int64_t i, T v, double *part) const {
#pragma clang fp contract(off)
    az[i] = v;
    const T rt = r[i];
    const double ri = (double)rt;
    const double vi = (double)v;
#pragma unroll
    for (int a = 0; a < S; ++a) {
      const double za = (zc == T(0)) ? (double)Z[(int64_t)a * ld + i]
                        : (a == 0) ? (double)(zc * rt)
                                   : (double)(zc * Z[(int64_t)(S + a - 1) * ld + i]);
      part[a] += za * ri;
      part[S + a] += za * vi;
    }
  }
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (rr_part) {   // uniform
      double rr[1];
      reduce_partials<1>(rr_part, rr_G, rr);
      if (threadIdx.x == 0) fin_update(st, rr[0], hist);
      __syncthreads();
      if (st->status != ST_RUNNING) return;   // the same value for every thread
    }
    if (solve) {
      small_solve_t<S>(st, tot);
    } else if (threadIdx.x < NP) {
      st->vm[threadIdx.x] = tot[threadIdx.x];
    }
  }
};

// Epilogue data that can be loaded before the row's product is formed.  By
// default there is none; the last matrix power prefetches Z(i,1..s) and r(i).
template <class Epi>
__device__ __forceinline__ NoPre epi_pre(const Epi &, int64_t) {
  return NoPre{};
}
template <class Epi, typename T>
__device__ __forceinline__ void epi_row(const Epi &e, int64_t i, T v, const NoPre &, double *part) {
  e.row(i, v, part);
}
template <int S>
struct LastPre {
  double z[S];
  double r;
};
template <int S, typename T>
__device__ __forceinline__ LastPre<S> epi_pre(const EpiMpkLast<S, T> &e, int64_t i) {
#pragma clang fp contract(off)
  LastPre<S> p;
  const T ri = e.r[i];
  if (e.zc == T(0)) {
#pragma unroll
    for (int a = 0; a < S; ++a) p.z[a] = (double)e.Z[(int64_t)a * e.ld + i];
  } else {
    p.z[0] = (double)(e.zc * ri);
#pragma unroll
    for (int a = 1; a < S; ++a) p.z[a] = (double)(e.zc * e.Z[(int64_t)(S + a - 1) * e.ld + i]);
  }
  p.r = (double)ri;
  return p;
}
template <int S, typename T>
__device__ __forceinline__ void epi_row(const EpiMpkLast<S, T> &e, int64_t i, T v,
                                        const LastPre<S> &p, double *part) {
#pragma clang fp contract(off)
  e.az[i] = v;
  const double vi = (double)v;
#pragma unroll
  for (int a = 0; a < S; ++a) {
    part[a] += p.z[a] * p.r;
    part[S + a] += p.z[a] * vi;
  }
}

// Sets the status after the residual norms of a starting iterate are known.
__device__ __forceinline__ void start_status(DevState *st, double bb, double rr, double *hist) {
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

// r = b - A x, z1 = B^-1 r, with ||b||^2 and ||r||^2 (FP64 solve start).
struct EpiInit {
  static constexpr int NP = 2;
  static constexpr bool kCheck = false;
  const double *b;
  double *r, *z1;
  Prec<double> pc;
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
    if (threadIdx.x == 0) start_status(st, tot[0], tot[1], hist);
  }
};

// PCG start (Alg. 1): r = b - A x, p = u = B^-1 r, rho = u^T r.
struct EpiPcgInit {
  static constexpr int NP = 3;
  static constexpr bool kCheck = false;
  const double *b;
  double *r, *p;
  Prec<double> pc;
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
      st->rho = tot[2];
      start_status(st, tot[0], tot[1], hist);
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
#pragma clang fp contract(off)
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

// PFCG start (Alg. 2): r = b - A x0 (and u = B^-1 r when the Jacobi scaling
// is a stored vector), ||b||^2 and ||r||^2.  rho_{-1} = 1: with p and s
// zero, the general step then gives exactly the paper's first step
// (gamma = 0, p_0 = u_0, s_0 = w_0, rho_0 = beta_0).
struct EpiPfcgInit {
  static constexpr int NP = 2;
  static constexpr bool kCheck = false;
  const double *b;
  double *r, *u;     // u: nullptr for a constant scaling (never stored)
  Prec<double> pc;
  double *hist;
  __device__ __forceinline__ void row(int64_t i, double v, double *part) const {
#pragma clang fp contract(off)
    const double bi = b[i];
    const double ri = bi - v;
    r[i] = ri;
    if (u) u[i] = pc.apply(i, ri);
    part[0] += bi * bi;
    part[1] += ri * ri;
  }
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (threadIdx.x == 0) {
      st->rho = 1.0;
      start_status(st, tot[0], tot[1], hist);
    }
  }
};

// PFCG step, first half (Alg. 2): w = A u with u = B^-1 r, and the three
// coupled dot products alpha = u^T r, beta = u^T w, gamma = u^T s_{k-1} in
// the same pass (one reduction).  For a constant scaling c the operator is
// applied to c r (the visitor's scale) and u_i = c r_i is formed here with
// the same rounding.  The finalisation forms rho_k = beta - gamma^2/rho_{k-1}
// and the two coefficients of the update.
struct EpiPfcgSpmv {
  static constexpr int NP = 3;
  static constexpr bool kCheck = true;
  const double *r, *u, *sv;   // u: stored B^-1 r, or nullptr (constant c)
  double *w;
  double c;
  // the previous update's ||r||^2 partials, finished here first (its
  // stopping test) instead of by a launch of their own; nullptr: none
  const double *rr_part;
  int rr_G;
  double *hist;
  __device__ __forceinline__ void row(int64_t i, double v, double *part) const {
#pragma clang fp contract(off)
    w[i] = v;
    const double ri = r[i];
    const double ui = u ? u[i] : c * ri;
    part[0] += ui * ri;
    part[1] += ui * v;
    part[2] += ui * sv[i];
  }
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
#pragma clang fp contract(off)
    if (rr_part) {   // uniform
      double rr[1];
      reduce_partials<1>(rr_part, rr_G, rr);
      if (threadIdx.x == 0) fin_update(st, rr[0], hist);
      __syncthreads();
      if (st->status != ST_RUNNING) return;   // the same value for every thread
    }
    if (threadIdx.x == 0) {
      const double alpha = tot[0], beta = tot[1], gamma = tot[2];
      const double rho_prev = st->rho;
      const double rho = beta - gamma * gamma / rho_prev;
      const double g = gamma / rho_prev;       // gamma_k / rho_{k-1}
      const double step = alpha / rho;         // alpha_k / rho_k
      if (!(rho > 0.0) || !isfinite(step) || !isfinite(g)) {
        st->status = ST_BREAKDOWN;
      } else {
        st->rho = rho;
        st->pcg_alpha = step;
        st->pcg_beta = g;
      }
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

// Judge of a warm start x0: ||b||^2 and ||b - A x0||^2 (runs whatever the
// status; the host compares them before the solve starts).
struct EpiWarmCheck {
  static constexpr int NP = 2;
  static constexpr bool kCheck = false;
  const double *b;
  __device__ __forceinline__ void row(int64_t i, double v, double *part) const {
#pragma clang fp contract(off)
    const double bi = b[i];
    const double t = bi - v;
    part[0] += bi * bi;
    part[1] += t * t;
  }
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (threadIdx.x == 0) {
      st->bb = tot[0];
      st->true_rr = tot[1];
    }
  }
};

// One damped Jacobi sweep xout = xin + omega B^-1 (b - A xin) (smooths a
// predicted initial guess before it is judged).
struct EpiJacobiSweep {
  static constexpr int NP = 0;
  static constexpr bool kCheck = false;
  const double *b, *xin;
  double *xout;
  Prec<double> pc;
  double omega;
  __device__ __forceinline__ void row(int64_t i, double v, double *) const {
#pragma clang fp contract(off)
    const double t = pc.apply(i, b[i] - v);
    const double u = omega * t;
    xout[i] = xin[i] + u;
  }
  __device__ __forceinline__ void finish(DevState *, const double *) const {}
};

// Iterative refinement, outer step: the FP64 residual r = b - A x of the
// current FP64 iterate, rounded to FP32 as the right-hand side of the next
// inner solve; the inner iterate d starts at 0, so the inner residual is that
// right-hand side and z1 = B^-1 r in FP32.  Partial sums: ||b||^2, ||r||^2 in
// FP64, and ||r32||^2.  The finalisation applies the outer stopping test and
// prepares the inner solve (its stopping test is relative to ||r32||).
struct EpiIrResidual {
  static constexpr int NP = 3;
  static constexpr bool kCheck = false;
  const double *b;
  float *r32, *z1, *d32;
  Prec<float> pc;
  double *hist;     // one entry per refinement step
  __device__ __forceinline__ void row(int64_t i, double v, double *part) const {
#pragma clang fp contract(off)
    const double bi = b[i];
    const double ri = bi - v;
    const float rf = (float)ri;
    r32[i] = rf;
    z1[i] = pc.apply(i, rf);
    d32[i] = 0.0f;
    part[0] += bi * bi;
    part[1] += ri * ri;
    part[2] += (double)rf * (double)rf;
  }
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (threadIdx.x != 0) return;
    const double bb = tot[0], rr = tot[1], rr32 = tot[2];
    const int j = st->ir_refine;
    if (j == 0) st->ir_bb = bb;
    const double bn = sqrt(st->ir_bb), rn = sqrt(rr);
    if (j < st->ir_hist_cap) hist[j] = bb > 0.0 ? rn / bn : 0.0;
    st->true_rr = rr;
    st->bb = rr32;
    st->rr = rr32;
    st->k = 0;
    // the inner solve reduces its residual by ir_inner_rtol, but not below
    // half of what the outer test still needs (no over-solving at the end)
    const double need = 0.5 * st->ir_rtol * bn / sqrt(rr32);
    st->rtol = need > st->ir_inner_rtol ? need : st->ir_inner_rtol;
    if (bb == 0.0) st->status = ST_ZERO_RHS;
    else if (rn <= st->ir_rtol * bn) st->status = ST_CONVERGED;
    else if (j >= st->ir_max_refine) st->status = ST_MAXIT;
    else if (!(rr32 > 0.0) || !isfinite(rr)) st->status = ST_BREAKDOWN;
    else st->status = ST_RUNNING;   // run the inner solve
  }
};

// --------------------------------------------------------------------------
// Kernels
// --------------------------------------------------------------------------

// Partial sums are stored at the workgroup's logical index, i.e. in the
// order of the row chunks, so any launch that splits rows into the same
// chunks (the batched solver included) reduces them in the same order.
template <class Epi>
__device__ __forceinline__ void epi_tail(const double (&part)[Epi::NP > 0 ? Epi::NP : 1],
                                         double *partials) {
  if constexpr (Epi::NP > 0) {
    double v[Epi::NP];
#pragma unroll
    for (int c = 0; c < Epi::NP; ++c) v[c] = part[c];
    block_store_sums<Epi::NP>(v, partials + logical_block(), gridDim.x);
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

template <int VARIANT, typename T, class Epi>
__global__ __launch_bounds__(kWG) void k_csr(CsrArgs<T> A, const T *__restrict__ x, T xs, Epi epi,
                                             DevState *st, double *partials) {
  if (Epi::kCheck && st->status != ST_RUNNING) return;
  double part[Epi::NP > 0 ? Epi::NP : 1];
#pragma unroll
  for (int c = 0; c < (Epi::NP > 0 ? Epi::NP : 1); ++c) part[c] = 0.0;
  csr_rows<VARIANT>(
      A, x, [&](int64_t i) { return epi_pre(epi, i); },
      [&](int64_t i, T v, const auto &p) { epi_row(epi, i, v, p, part); }, xs);
  epi_tail<Epi>(part, partials);
}

template <int KIND, typename T, class Epi>
__global__ __launch_bounds__(kWG) void k_stencil(StencilArgs<T> S, const T *__restrict__ x, T xs,
                                                 Epi epi, DevState *st, double *partials) {
  if (Epi::kCheck && st->status != ST_RUNNING) return;
  double part[Epi::NP > 0 ? Epi::NP : 1];
#pragma unroll
  for (int c = 0; c < (Epi::NP > 0 ? Epi::NP : 1); ++c) part[c] = 0.0;
  int64_t p0, p1;
  block_chunk(S.n, logical_block(), gridDim.x, p0, p1);
  stencil_rows<KIND>(S, x, p0, p1, [&](int64_t i, T v) { epi.row(i, v, part); }, xs);
  epi_tail<Epi>(part, partials);
}

// LDS-staged 3D stencils (7- and 27-point, constant coefficients): the same
// operator and epilogues as k_stencil, the same terms in the same order per
// point (neighbours outside the grid masked out), but each x value is
// brought into LDS once per plane tile instead of being gathered through the
// caches by every neighbour.
template <int KIND, typename T, class Epi>
__global__ __launch_bounds__(kWG) void k_stencil_tiled(StencilArgs<T> S, const T *__restrict__ x,
                                                       T xs, Epi epi, DevState *st,
                                                       double *partials, Tiling3 tl) {
#pragma clang fp contract(off)
  if (Epi::kCheck && st->status != ST_RUNNING) return;
  constexpr int HX = kTX + 2, HY = kTY + 2;
  __shared__ T pl[3][HY][HX];
  double part[Epi::NP > 0 ? Epi::NP : 1];
#pragma unroll
  for (int c = 0; c < (Epi::NP > 0 ? Epi::NP : 1); ++c) part[c] = 0.0;
  const int nx = S.nx, ny = S.ny, nz = S.nz;
  const int b = logical_block();
  const int tx = b % tl.ntx, ty = (b / tl.ntx) % tl.nty, tz = b / (tl.ntx * tl.nty);
  const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * tl.zchunk;
  const int z1 = (z0 + tl.zchunk < nz) ? z0 + tl.zchunk : nz;
  const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool mine = gx < nx && gy < ny;
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  // plane z (z >= -1) into slot (z + 3) % 3; cells outside the grid hold 0
  // and are never summed
  auto load = [&](int z) {
    T(*dst)[HX] = pl[(z + 3) % 3];
    for (int e = threadIdx.x; e < HX * HY; e += kWG) {
      const int hy = e / HX, hx = e - hy * HX;
      const int qx = x0 + hx - 1, qy = y0 + hy - 1;
      const bool ok = z >= 0 && z < nz && qx >= 0 && qx < nx && qy >= 0 && qy < ny;
      const int64_t q = ok ? (int64_t)z * sz + (int64_t)qy * sy + qx : 0;
      const T v = xs * x[q];
      dst[hy][hx] = ok ? v : T(0);
    }
  };
  if (z0 < z1) {
    load(z0 - 1);
    load(z0);
  }
  for (int z = z0; z < z1; ++z) {
    load(z + 1);
    __syncthreads();
    if (mine) {
      const int sm = (z + 2) % 3, sc = z % 3, sp = (z + 1) % 3;
      T acc;
      if constexpr (KIND == K_3D27) {
        T nb = 0;
#pragma unroll
        for (int t = 0; t < 27; ++t) {
          const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
          const bool ok = t != 13 && z + dz >= 0 && z + dz < nz && gy + dy >= 0 &&
                          gy + dy < ny && gx + dx >= 0 && gx + dx < nx;
          const int sl = dz < 0 ? sm : (dz == 0 ? sc : sp);
          const T u = nb + pl[sl][ly + 1 + dy][lx + 1 + dx];
          nb = ok ? u : nb;
        }
        const T d = S.diag * pl[sc][ly + 1][lx + 1];
        const T o = S.off * nb;
        acc = d + o;
      } else {
        T nb = 0;
        nb = gx > 0 ? nb + pl[sc][ly + 1][lx] : nb;
        nb = gx < nx - 1 ? nb + pl[sc][ly + 1][lx + 2] : nb;
        nb = gy > 0 ? nb + pl[sc][ly][lx + 1] : nb;
        nb = gy < ny - 1 ? nb + pl[sc][ly + 2][lx + 1] : nb;
        nb = z > 0 ? nb + pl[sm][ly + 1][lx + 1] : nb;
        nb = z < nz - 1 ? nb + pl[sp][ly + 1][lx + 1] : nb;
        const T d = S.diag * pl[sc][ly + 1][lx + 1];
        const T o = S.off * nb;
        acc = d + o;
      }
      epi.row((int64_t)z * sz + (int64_t)gy * sy + gx, acc, part);
    }
    __syncthreads();
  }
  epi_tail<Epi>(part, partials);
}

// Fused block update (Alg. 3, in the order of its four update lines), one
// thread per row computing all s outputs, arithmetic in FP64:
//   P  = Z  + P_old  beta          (skipped at k = 0: P_old = 0)
//   x  = x  + P alpha
//   AP = AZ + AP_old beta
//   r  = r  - AP alpha
// then z1 = B^-1 r for the next matrix powers (column 1 of the other block,
// whose row was just read by the same thread) and the partial sums of
// ||r||^2 (finished by FinUpdate).  With T = float the new P and AP are
// rounded to FP32 before they update x and r, as stored.
template <int S, typename T>
struct UpdateCoef {
  int k;
  double alpha[S], beta[S][S];
  __device__ __forceinline__ void load(const DevState *st) {
    k = st->k;
#pragma unroll
    for (int j = 0; j < S; ++j) alpha[j] = st->alpha[j];
    if (k > 0) {
#pragma unroll
      for (int l = 0; l < S; ++l)
#pragma unroll
        for (int j = 0; j < S; ++j) beta[l][j] = st->beta[l * S + j];
    }
  }
};

// The rows [lo, hi) of the block update; returns this thread's partial ||r||^2.
// zc = 0: Z is stored in the block and z1 = B^-1 r_new is written for the
// next matrix powers; zc = c (constant Jacobi scaling): Z(:,1) = c r and
// Z(:,j) = c AZ(:,j-1) are formed from values the update reads anyway, and
// no z1 is written.
template <int S, typename T>
__device__ __forceinline__ double update_rows(const UpdateCoef<S, T> &c, int64_t lo, int64_t hi,
                                              int64_t ld, T *__restrict__ Pc,
                                              T *__restrict__ Po, T *__restrict__ x,
                                              T *__restrict__ r, const Prec<T> &pc, T zc) {
#pragma clang fp contract(off)
  double part = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) {
    double p[S], ap[S];
    const T r0 = r[i];
    T azs[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
      azs[j] = ld_stream(&Pc[(int64_t)(S + j) * ld + i]);
      ap[j] = (double)azs[j];
    }
    if (zc == T(0)) {
#pragma unroll
      for (int j = 0; j < S; ++j) p[j] = (double)ld_stream(&Pc[(int64_t)j * ld + i]);
    } else {
      p[0] = (double)(zc * r0);
#pragma unroll
      for (int j = 1; j < S; ++j) p[j] = (double)(zc * azs[j - 1]);
    }
    if (c.k > 0) {
      double po[S], apo[S];
#pragma unroll
      for (int l = 0; l < S; ++l) {
        po[l] = (double)ld_stream(&Po[(int64_t)l * ld + i]);
        apo[l] = (double)ld_stream(&Po[(int64_t)(S + l) * ld + i]);
      }
#pragma unroll
      for (int j = 0; j < S; ++j) {
        double a = p[j], b = ap[j];
#pragma unroll
        for (int l = 0; l < S; ++l) {
          const double t = po[l] * c.beta[l][j];
          a += t;
          const double u = apo[l] * c.beta[l][j];
          b += u;
        }
        const T as = (T)a, bs = (T)b;
        st_stream(&Pc[(int64_t)j * ld + i], as);
        st_stream(&Pc[(int64_t)(S + j) * ld + i], bs);
        p[j] = (double)as;
        ap[j] = (double)bs;
      }
    } else if (zc != T(0)) {
      // k = 0: P = Z must be stored for the next iteration's P_old beta
#pragma unroll
      for (int j = 0; j < S; ++j) st_stream(&Pc[(int64_t)j * ld + i], (T)p[j]);
    }
    double dx = 0.0, dr = 0.0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const double t = p[j] * c.alpha[j];
      dx += t;
      const double u = ap[j] * c.alpha[j];
      dr += u;
    }
    const T xi = (T)((double)ld_stream(&x[i]) + dx);
    const T ri = (T)((double)r0 - dr);
    st_stream(&x[i], xi);
    r[i] = ri;
    if (zc == T(0)) Po[i] = pc.apply(i, ri);
    part += (double)ri * (double)ri;
  }
  return part;
}

// The rows are dealt out in XCD-interleaved pieces of kWG (one row per
// thread per piece); the partial is stored at the hardware block index.
template <int S, typename T>
__global__ __launch_bounds__(kWG) void k_update(int64_t n, int64_t ld, T *__restrict__ Pc,
                                                T *__restrict__ Po, T *__restrict__ x,
                                                T *__restrict__ r, Prec<T> pc, T zc, DevState *st,
                                                double *partials) {
  if (st->status != ST_RUNNING) return;
  UpdateCoef<S, T> c;
  c.load(st);
  const XcdSched sc = xcd_sched(n, kWG, gridDim.x, blockIdx.x);
  double acc = 0.0;
  for (int64_t b0 = sc.first; b0 < sc.end; b0 += sc.stride) {
    const int64_t b1 = b0 + kWG < sc.end ? b0 + kWG : sc.end;
    acc += update_rows<S, T>(c, b0, b1, ld, Pc, Po, x, r, pc, zc);
  }
  double v[1] = {acc};
  block_store_sums<1>(v, partials + blockIdx.x, gridDim.x);
}

// After the block update: ||r||^2, history entry, stopping test, k += 1.
struct FinUpdate {
  static constexpr int NP = 1;
  static constexpr bool kCheck = true;
  double *hist;
  __device__ __forceinline__ void finish(DevState *st, const double *tot) const {
    if (threadIdx.x == 0) fin_update(st, tot[0], hist);
  }
};

// PCG (Alg. 1) update: x += alpha p, r -= alpha s, u = B^-1 r; partial sums
// of u^T r and ||r||^2 (finished by FinPcgUpdate).
static __global__ __attribute__((unused)) __launch_bounds__(kWG) void k_pcg_update(int64_t n, double *__restrict__ x,
                                                    double *__restrict__ r,
                                                    const double *__restrict__ p,
                                                    const double *__restrict__ sv,
                                                    Prec<double> pc, DevState *st,
                                                    double *partials) {
#pragma clang fp contract(off)
  if (st->status != ST_RUNNING) return;
  const double a = st->pcg_alpha;
  double ur = 0.0, rr = 0.0;
  int64_t lo, hi;
  block_chunk(n, logical_block(), gridDim.x, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) {
    // x and s = A p are not read again soon (non-temporal); p and r are
    // read by the next kernels
    const double ap = a * p[i];
    const double xi = ld_stream(&x[i]) + ap;
    const double as = a * ld_stream(&sv[i]);
    const double ri = r[i] - as;
    st_stream(&x[i], xi);
    r[i] = ri;
    const double ui = pc.apply(i, ri);
    ur += ui * ri;
    rr += ri * ri;
  }
  double v[2] = {ur, rr};
  block_store_sums<2>(v, partials + logical_block(), gridDim.x);
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

// PFCG step, second half (Alg. 2): p = u - g p, x += a p, s = w - g s,
// r -= a s (u = B^-1 r of the old r; stored u is refreshed from the new r),
// with ||r||^2 partials finished by FinUpdate.  Rows in XCD-interleaved
// pieces; the partial is stored at the hardware block index.
static __global__ __attribute__((unused)) __launch_bounds__(kWG) void k_pfcg_update(
    int64_t n, double *__restrict__ x, double *__restrict__ r, double *__restrict__ p,
    double *__restrict__ sv, const double *__restrict__ w, double *__restrict__ u,
    Prec<double> pc, DevState *st, double *partials) {
#pragma clang fp contract(off)
  if (st->status != ST_RUNNING) return;
  const double a = st->pcg_alpha, g = st->pcg_beta;
  const XcdSched sc = xcd_sched(n, kWG, gridDim.x, blockIdx.x);
  double rr = 0.0;
  for (int64_t b0 = sc.first; b0 < sc.end; b0 += sc.stride) {
    const int64_t b1 = b0 + kWG < sc.end ? b0 + kWG : sc.end;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kWG) {
      // plain loads and stores: PFCG's five vectors (84 MB at 128^3) fit the
      // memory-side cache, and non-temporal hints here measured slower
      const double ri = r[i];
      const double ui = u ? u[i] : pc.dc * ri;
      const double gp = g * p[i];
      const double pn = ui - gp;
      const double ap = a * pn;
      const double xn = x[i] + ap;
      const double gs = g * sv[i];
      const double sn = w[i] - gs;
      const double as = a * sn;
      const double rn = ri - as;
      p[i] = pn;
      x[i] = xn;
      sv[i] = sn;
      r[i] = rn;
      if (u) u[i] = pc.apply(i, rn);
      rr += rn * rn;
    }
  }
  double v[1] = {rr};
  block_store_sums<1>(v, partials + blockIdx.x, gridDim.x);
}

// PCG direction: p = u + beta p with u = B^-1 r recomputed from r.
static __global__ __attribute__((unused)) __launch_bounds__(kWG) void k_pcg_direction(int64_t n, const double *__restrict__ r,
                                                       double *__restrict__ p, Prec<double> pc,
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

// Iterative refinement: x += d (FP32 correction added in FP64).
static __global__ __attribute__((unused)) __launch_bounds__(kWG) void k_ir_add(int64_t n, double *__restrict__ x,
                                                const float *__restrict__ d) {
  int64_t lo, hi;
  block_chunk(n, logical_block(), gridDim.x, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) x[i] = x[i] + (double)d[i];
}

// z = B^-1 v on its own (first column of the stand-alone matrix powers).
// The row grid is capped, so each workgroup covers a chunk of rows.
template <typename T>
__global__ __launch_bounds__(kWG) void k_prec(int64_t n, const T *__restrict__ v,
                                              T *__restrict__ z, Prec<T> pc) {
  int64_t lo, hi;
  block_chunk(n, logical_block(), gridDim.x, lo, hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) z[i] = pc.apply(i, v[i]);
}

}  // namespace ssp
