// Host-side engine of libsstep: handle and matrix objects, workspaces, the
// device control block, profiling, and the launch sequences of one outer
// iteration.  Shared by the C-ABI translation unit and the per-precision
// instantiation units (inst_f64.hip, inst_f32.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "gram.hpp"
#include "kernels.hpp"
#include "temporal.hpp"
#include "sstep.h"

namespace ssp {

// Workspace of the solves of one handle (grown on demand, reused).
struct Workspace {
  int64_t n = 0, ld = 0;
  int s = 0;
  double *P1 = nullptr, *P2 = nullptr;     // n x 2s FP64 blocks, column-major, leading dim ld
  double *r = nullptr;
  double *pcg_p = nullptr, *pcg_s = nullptr;
  int64_t n32 = 0, ld32 = 0;
  int s32 = 0;
  float *Q1 = nullptr, *Q2 = nullptr;       // FP32 blocks of the inner solves
  float *r32 = nullptr, *d32 = nullptr;
  double *partials = nullptr;              // kGridMax x 2*kSMax
  double *partials_rr = nullptr;           // kGridMax: the block update's ||r||^2
  double *partials_gram = nullptr;         // kGramGrid x s(2s+1): the block Gram pass
  double *hist = nullptr;
  int hist_cap = 0;
};

}  // namespace ssp

struct ssp_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  ssp::Workspace ws;
  ssp::DevState *st = nullptr;     // device control block
  ssp::DevState *h_init = nullptr; // pinned staging for the control block
  ssp::DevState *h_read = nullptr; // pinned readback
  // results of the last solve
  int last_outer = 0, last_s = 1;
  double last_true_rel = NAN;
  std::vector<double> last_hist;
  int last_restarts = 0;           // residual-replacement restarts of the last solve
  int last_warm_kept = -1;         // warm-start judge: 1 kept, 0 fell back, -1 none
  double last_warm_rel0 = NAN;
  // profiling (HIP events around launches)
  bool prof_on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_cls;
  std::vector<int> ev_iter;        // outer iteration of the launch (-1: outside the loop)
  int prof_iter = -1;
  size_t ev_used = 0;
  int prof_launch[SSP_PROFILE_CLASSES] = {};
  double prof_ms[SSP_PROFILE_CLASSES] = {};
  // batched solves: one device buffer for every per-system array
  void *batch_mem = nullptr;
  size_t batch_bytes = 0;
};

namespace ssp {
struct AmgHier;
}

struct ssp_matrix {
  ssp_handle *h = nullptr;
  int kind = 0;                    // 0 = CSR, else SSP_STENCIL_*
  int64_t n = 0, nnz = 0;
  ssp::CsrArgs<double> csr{};
  ssp::CsrArgs<float> csr32{};     // FP32 values (built on first mixed-precision use)
  int32_t *own_rowptr = nullptr, *own_colind = nullptr;
  double *own_val = nullptr;
  float *val32 = nullptr;
  int32_t *sell_col = nullptr;     // sliced ELL copy (library-owned)
  double *sell_val = nullptr;
  float *sell_val32 = nullptr;
  int64_t *slice_off = nullptr;
  int32_t *slice_w = nullptr;
  int64_t sell_entries = 0;
  ssp::StencilArgs<double> sten{};
  ssp::StencilArgs<float> sten32{};
  float *k32 = nullptr;
  double *dinv = nullptr;          // Jacobi vector (CSR, variable coefficient)
  float *dinv32 = nullptr;
  double dconst = 1.0;             // Jacobi constant (constant-diagonal stencils)
  bool has32 = false;
  int prec = SSP_PREC_JACOBI;
  ssp::AmgHier *amg = nullptr;     // AMG hierarchy (ssp_set_amg)
  int tb = 1;                      // temporally blocked powers: 0 never, 1 where they
                                   // fill the GPU, 2 wherever they apply
};

namespace ssp {

inline int fail(ssp_handle *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  return code;
}

#define HIPCHK(h, call)                                                               \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ssp::fail((h), SSP_EHIP, std::string("HIP error ") + hipGetErrorString(e_) + \
                                          " (line " + std::to_string(__LINE__) + ")"); \
  } while (0)

#define LAUNCHCHK(h) HIPCHK(h, hipGetLastError())

template <typename T> struct Prec;

// z = B^-1 y by one AMG V-cycle (amg.hip); and the hierarchy's release.
int amg_vcycle(ssp_handle *h, const ssp_matrix *A, const double *y, double *z);
void amg_free(ssp_matrix *A);

// The pointwise preconditioner of the fused epilogues.  With the AMG
// preconditioner they apply the identity and a V-cycle runs after them.
inline Prec<double> prec_of(const ssp_matrix *A, double *) {
  if (A->prec == SSP_PREC_NONE || A->prec == SSP_PREC_AMG) return Prec<double>{nullptr, 1.0};
  if (A->dinv) return Prec<double>{A->dinv, 0.0};
  return Prec<double>{nullptr, A->dconst};
}
inline Prec<float> prec_of(const ssp_matrix *A, float *) {
  if (A->prec == SSP_PREC_NONE || A->prec == SSP_PREC_AMG) return Prec<float>{nullptr, 1.0f};
  if (A->dinv32) return Prec<float>{A->dinv32, 0.0f};
  return Prec<float>{nullptr, (float)A->dconst};
}

inline const CsrArgs<double> &csr_of(const ssp_matrix *A, double *) { return A->csr; }
inline const CsrArgs<float> &csr_of(const ssp_matrix *A, float *) { return A->csr32; }
inline const StencilArgs<double> &sten_of(const ssp_matrix *A, double *) { return A->sten; }
inline const StencilArgs<float> &sten_of(const ssp_matrix *A, float *) { return A->sten32; }

inline int grid_rows(int64_t n) {
  int64_t g = (n + kWG - 1) / kWG;
  if (g > kGridMax) g = kGridMax;
  if (g < 1) g = 1;
  return (int)g;
}

inline bool tiled_of(const ssp_matrix *A, Tiling3 &t) {
  return A->kind != 0 && stencil_tiling(A->kind == SSP_STENCIL_3D7 ? K_3D7
                                        : A->kind == SSP_STENCIL_3D27 ? K_3D27 : 0,
                                        A->sten.nx, A->sten.ny, A->sten.nz, t);
}

inline int grid_of(const ssp_matrix *A) {
  Tiling3 t;
  if (tiled_of(A, t)) return t.ntx * t.nty * t.ntz;
  if (A->kind == 0 && A->csr.variant == CSR_SELL) {
    int64_t g = (A->csr.nslices + kWG / kWave - 1) / (kWG / kWave);
    if (g > kGridMax) g = kGridMax;
    return (int)std::max<int64_t>(g, 1);
  }
  if (A->kind == 0 && A->csr.variant == CSR_STAGED) {
    int64_t g = A->csr.nrb;
    if (g > kGridMax) g = kGridMax;
    return (int)std::max<int64_t>(g, 1);
  }
  return grid_rows(A->n);
}

// Profiling classes: 0 matrix powers j < s and plain SpMV, 1 last power with
// moments and s x s solve, 2 vector/block updates, 3 other, 4 the block Gram
// pass of the Chebyshev basis.
inline void prof_begin(ssp_handle *h, int cls) {
  if (!h->prof_on) return;
  if (h->ev_used + 2 > h->ev.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      h->ev.push_back(e);
    }
    h->ev_cls.resize(h->ev.size() / 2 + 64);
    h->ev_iter.resize(h->ev.size() / 2 + 64);
  }
  h->ev_cls[h->ev_used / 2] = cls;
  h->ev_iter[h->ev_used / 2] = h->prof_iter;
  (void)hipEventRecord(h->ev[h->ev_used], h->stream);
}

inline void prof_end(ssp_handle *h) {
  if (!h->prof_on || h->ev_used + 2 > h->ev.size()) return;
  (void)hipEventRecord(h->ev[h->ev_used + 1], h->stream);
  h->ev_used += 2;
}

// Launches of iterations enqueued after the stop (no-op kernels) are skipped:
// the averages describe launches that did the work.
inline void prof_collect(ssp_handle *h, int iters_done) {
  if (!h->prof_on) return;
  for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
    if (h->ev_iter[i / 2] >= iters_done) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) == hipSuccess) {
      const int c = h->ev_cls[i / 2];
      h->prof_launch[c] += 1;
      h->prof_ms[c] += ms;
    }
  }
  h->ev_used = 0;
}

// Operator launch (CSR or stencil kind) with epilogue Epi, followed by the
// finalisation kernel when Epi reduces.  The control block and the partial
// sums are the handle's unless `ctl` names others (the allocation-free
// entry point passes its static scratch).
struct Ctl {
  DevState *st;
  double *partials;
};
template <typename T, class Epi>
int launch_op(ssp_handle *h, const ssp_matrix *A, const T *x, const Epi &epi, int cls,
              T xs = T(1), const Ctl *ctl = nullptr) {
  const int G = grid_of(A);
  T *tag = nullptr;
  DevState *const st = ctl ? ctl->st : h->st;
  double *const partials = ctl ? ctl->partials : h->ws.partials;
  prof_begin(h, cls);
  switch (A->kind) {
    case 0:
      if (A->csr.variant == CSR_ROW)
        k_csr<CSR_ROW, T, Epi><<<G, kWG, 0, h->stream>>>(csr_of(A, tag), x, xs, epi, st,
                                                          partials);
      else if (A->csr.variant == CSR_SELL)
        k_csr<CSR_SELL, T, Epi><<<G, kWG, 0, h->stream>>>(csr_of(A, tag), x, xs, epi, st,
                                                           partials);
      else
        k_csr<CSR_STAGED, T, Epi><<<G, kWG, 0, h->stream>>>(csr_of(A, tag), x, xs, epi, st,
                                                             partials);
      break;
    case SSP_STENCIL_2D5:
      k_stencil<K_2D5, T, Epi><<<G, kWG, 0, h->stream>>>(sten_of(A, tag), x, xs, epi, st,
                                                          partials);
      break;
    case SSP_STENCIL_3D7:
    case SSP_STENCIL_3D27: {
      Tiling3 tl;
      const bool tiled = tiled_of(A, tl);
      if (A->kind == SSP_STENCIL_3D7) {
        if (tiled)
          k_stencil_tiled<K_3D7, T, Epi><<<G, kWG, 0, h->stream>>>(sten_of(A, tag), x, xs, epi,
                                                                    st, partials, tl);
        else
          k_stencil<K_3D7, T, Epi><<<G, kWG, 0, h->stream>>>(sten_of(A, tag), x, xs, epi, st,
                                                              partials);
      } else {
        if (tiled)
          k_stencil_tiled<K_3D27, T, Epi><<<G, kWG, 0, h->stream>>>(sten_of(A, tag), x, xs, epi,
                                                                     st, partials, tl);
        else
          k_stencil<K_3D27, T, Epi><<<G, kWG, 0, h->stream>>>(sten_of(A, tag), x, xs, epi,
                                                               st, partials);
      }
      break;
    }
    case SSP_STENCIL_3D7_VARK:
      k_stencil<K_VARK, T, Epi><<<G, kWG, 0, h->stream>>>(sten_of(A, tag), x, xs, epi, st,
                                                           partials);
      break;
    default:
      return fail(h, SSP_EINVAL, "unknown operator kind " + std::to_string(A->kind));
  }
  if constexpr (Epi::NP > 0) {
    k_finalize<Epi><<<1, kWG, 0, h->stream>>>(epi, st, partials, G);
  }
  prof_end(h);
  LAUNCHCHK(h);
  return SSP_OK;
}

// Blocks and vectors of one outer iteration in precision T.
template <typename T>
struct IterBufs {
  T *P1, *P2;       // ping-pong n x 2s blocks
  int64_t ld;
  T *x, *r;
  double cheb_c = 0.0, cheb_g = 0.0;   // Chebyshev basis: centre, 1 / half-width
};

// The temporally blocked powers apply to the 3D 7-point constant-coefficient
// grid (whose Jacobi factor is a constant) for s >= 2, when a plane of
// 32 x 32 tiles fits one launch.  By default they are taken only where their
// launches keep at least three quarters of the compute units busy (on
// smaller grids one launch per power is faster: 64^3 s = 4 2.8 vs 4.9 ms);
// tb = 2 takes them wherever they apply, tb = 0 never.
inline bool tb_usable(const ssp_matrix *A, int s) {
  if (A->kind != SSP_STENCIL_3D7 || s < 2 || A->tb == 0) return false;
  const StencilArgs<double> &S = A->sten;
  const int64_t plane = (int64_t)((S.nx + kTbT - 1) / kTbT) * ((S.ny + kTbT - 1) / kTbT);
  if (plane > kGridMax) return false;
  if (A->tb == 2) return true;
  const int L = s < kTbMaxL ? s : kTbMaxL;
  return tb_grid(tb_tiling(S.nx, S.ny, S.nz, L, 1)) * 4 >= 3 * kCUs;
}

// Workgroups of a blocked-powers kernel resident per compute unit (its
// registers and LDS decide), asked of the runtime once.
template <int L, int SM, typename T>
int tb_per_cu() {
  static int n = -1;
  if (n < 0) {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_mpk_tb7<L, SM, T>, kTbWG, 0) !=
        hipSuccess)
      v = 1;
    n = std::max(v, 1);
  }
  return n;
}

// Launch PASS of the temporally blocked powers of an S-power block and the
// launches after it; G is set to the grid of the last (the one leaving the
// moment partials).
template <int S, int PASS, typename T>
void tb_pass(ssp_handle *h, const ssp_matrix *A, const T *in, const T *r, T c, int j0, T *P,
             int64_t ld, bool store_z, DevState *st, double *partials, int &G) {
  constexpr int L = tb_levels(S, PASS);
  constexpr bool last = PASS == tb_passes(S) - 1;
  T *tag = nullptr;
  const StencilArgs<T> &sa = sten_of(A, tag);
  const TbTiling tl = tb_tiling(sa.nx, sa.ny, sa.nz, L, tb_per_cu<L, last ? S : 0, T>());
  G = tl.ntx * tl.nty * tl.ntz;
  k_mpk_tb7<L, last ? S : 0, T><<<G, kTbWG, 0, h->stream>>>(
      sa, in, c, j0, S, P, ld, store_z ? 1 : 0, r, st, partials, tl);
  if constexpr (!last)
    tb_pass<S, PASS + 1, T>(h, A, P + (int64_t)(S + j0 + L - 1) * ld, r, c, j0 + L, P, ld,
                            store_z, st, partials, G);
}

// AZ(:,1..S) of the block P (and Z(:,2..S) when store_z) from r, with the
// moment partials of Alg. 5 in `partials` (G workgroups).
template <int S, typename T>
int tb_powers(ssp_handle *h, const ssp_matrix *A, const T *r, T c, T *P, int64_t ld,
              bool store_z, DevState *st, double *partials, int &G) {
  tb_pass<S, 0, T>(h, A, r, r, c, 0, P, ld, store_z, st, partials, G);
  LAUNCHCHK(h);
  return SSP_OK;
}

// One outer iteration of the s-step method (Alg. 3): s matrix-power
// launches (Alg. 4; the last fused with Alg. 5 and followed by the s x s
// solve of Alg. 6 on the GPU) and the fused block update.  Within a batch of
// iterations enqueued between two host polls, the stopping test of an
// update runs in the next iteration's last-power finalisation (before its
// s x s solve, which it skips once the test holds); only the batch's last
// update gets a finalisation launch of its own, so the polled status is
// always current.  The powers enqueued after a converging update run
// without effect on x and r, as the kernels after the stop always did.
template <int S, typename T>
int sstep_iteration(ssp_handle *h, const ssp_matrix *A, const IterBufs<T> &B, int k,
                    bool first_in_batch, bool last_in_batch) {
  T *Pc = (k % 2 == 0) ? B.P2 : B.P1;   // Alg. 3: even k fills P2, odd k fills P1
  T *Po = (k % 2 == 0) ? B.P1 : B.P2;
  T *tag = nullptr;
  const Prec<T> pc = prec_of(A, tag);
  // constant Jacobi scaling c (or none, c = 1): the Z columns are never
  // stored; each reader forms c * r or c * AZ(:,j-1), the same rounded values
  // with AMG the block Z is stored and each Z(:,j+1) = B^-1 AZ(:,j) is a
  // V-cycle after the power that produced AZ(:,j)
  constexpr bool kF64 = std::is_same<T, double>::value;
  const bool amg = kF64 && A->prec == SSP_PREC_AMG;
  const T zc = (pc.dinv || amg) ? T(0) : pc.dc;
  bool powers_done = false;
  if constexpr (S >= 2) {
    if (zc != T(0) && tb_usable(A, S)) {
      // the s powers in ceil(s / 4) temporally blocked launches, then the
      // moments' reduction and the s x s solve
      int G = 0;
      prof_begin(h, 0);
      int rc = tb_powers<S, T>(h, A, B.r, zc, Pc, B.ld, false, h->st, h->ws.partials, G);
      prof_end(h);
      if (rc) return rc;
      prof_begin(h, 1);
      k_finalize<EpiMpkLast<S, T>><<<1, kWG, 0, h->stream>>>(
          EpiMpkLast<S, T>{Pc + (int64_t)(2 * S - 1) * B.ld, Pc, B.ld, B.r, 1, zc,
                           first_in_batch ? nullptr : h->ws.partials_rr, grid_rows(A->n),
                           h->ws.hist},
          h->st, h->ws.partials, G);
      prof_end(h);
      LAUNCHCHK(h);
      powers_done = true;
    }
  }
  for (int j = 1; j <= S && !powers_done; ++j) {
    const T *zin;
    T xs = T(1);
    if (zc == T(0)) {
      zin = Pc + (int64_t)(j - 1) * B.ld;
    } else {
      zin = (j == 1) ? B.r : Pc + (int64_t)(S + j - 2) * B.ld;
      xs = zc;
    }
    T *az = Pc + (int64_t)(S + j - 1) * B.ld;
    int rc;
    if (j < S) {
      rc = launch_op<T>(
          h, A, zin, EpiMpk<T>{az, (zc == T(0) && !amg) ? Pc + (int64_t)j * B.ld : nullptr, pc},
          0, xs);
      if constexpr (kF64)
        if (!rc && amg) rc = amg_vcycle(h, A, az, Pc + (int64_t)j * B.ld);
    } else
      rc = launch_op<T>(h, A, zin,
                        EpiMpkLast<S, T>{az, Pc, B.ld, B.r, 1, zc,
                                         first_in_batch ? nullptr : h->ws.partials_rr,
                                         grid_rows(A->n), h->ws.hist},
                        1, xs);
    if (rc) return rc;
  }
  const int G = grid_rows(A->n);
  prof_begin(h, 2);
  k_update<S, T><<<G, kWG, 0, h->stream>>>(A->n, B.ld, Pc, Po, B.x, B.r, pc, zc, h->st,
                                            h->ws.partials_rr);
  if constexpr (kF64)
    if (amg) {   // z_1 = B^-1 r of the next iteration, where the update left r
      LAUNCHCHK(h);
      const int rc = amg_vcycle(h, A, B.r, Po);
      if (rc) return rc;
    }
  if (last_in_batch)
    k_finalize<FinUpdate><<<1, kWG, 0, h->stream>>>(FinUpdate{h->ws.hist}, h->st,
                                                    h->ws.partials_rr, G);
  prof_end(h);
  LAUNCHCHK(h);
  return SSP_OK;
}

// One outer iteration on the Chebyshev basis: s operator launches (the basis
// recurrence in their epilogues; the last stores AZ(:,s) only), the block
// Gram pass on the matrix cores, its finalisation (the previous update's
// stopping test within a polling batch, then the s x s algebra) and Alg. 3's
// block update with the Z columns stored.
inline int gram_grid(int64_t n) {
  const int64_t steps = (n + kGramRows - 1) / kGramRows;
  int64_t g = (steps + kWG / kWave - 1) / (kWG / kWave);
  if (g > kGramGrid) g = kGramGrid;
  return (int)std::max<int64_t>(g, 1);
}

template <int S, typename T>
int sstep_cheb_iteration(ssp_handle *h, const ssp_matrix *A, const IterBufs<T> &B, int k,
                         bool first_in_batch, bool last_in_batch) {
  T *Pc = (k % 2 == 0) ? B.P2 : B.P1;
  T *Po = (k % 2 == 0) ? B.P1 : B.P2;
  T *tag = nullptr;
  const Prec<T> pc = prec_of(A, tag);
  const T c = (T)B.cheb_c, g = (T)B.cheb_g, g2 = (T)(2.0 * B.cheb_g);
  for (int j = 1; j <= S; ++j) {
    T *zj = Pc + (int64_t)(j - 1) * B.ld;
    T *az = Pc + (int64_t)(S + j - 1) * B.ld;
    int rc;
    if (j < S)
      rc = launch_op<T>(h, A, zj,
                        EpiCheb<T>{az, Pc + (int64_t)j * B.ld, zj,
                                   j >= 2 ? Pc + (int64_t)(j - 2) * B.ld : nullptr, pc, c,
                                   j == 1 ? g : g2},
                        0);
    else
      rc = launch_op<T>(h, A, zj, EpiMpk<T>{az, nullptr, pc}, 1);
    if (rc) return rc;
  }
  const int Gg = gram_grid(A->n);
  const int G = grid_rows(A->n);
  prof_begin(h, 4);
  k_gram<S, T><<<Gg, kWG, 0, h->stream>>>(A->n, B.ld, Pc, Po, B.r, k == 0 ? 1 : 0, h->st,
                                           h->ws.partials_gram);
  prof_end(h);
  prof_begin(h, 1);
  k_gram_finalize<S><<<1, kFinWG, 0, h->stream>>>(
      h->st, h->ws.partials_gram, Gg, first_in_batch ? nullptr : h->ws.partials_rr, G,
      h->ws.hist);
  prof_end(h);
  prof_begin(h, 2);
  k_update<S, T><<<G, kWG, 0, h->stream>>>(A->n, B.ld, Pc, Po, B.x, B.r, pc, T(0), h->st,
                                            h->ws.partials_rr);
  if (last_in_batch)
    k_finalize<FinUpdate><<<1, kWG, 0, h->stream>>>(FinUpdate{h->ws.hist}, h->st,
                                                    h->ws.partials_rr, G);
  prof_end(h);
  LAUNCHCHK(h);
  return SSP_OK;
}

// Alg. 4 + Alg. 5 on their own (no solve): the block P and vm in the state.
template <int S>
int mpk_only(ssp_handle *h, const ssp_matrix *A, const double *r, double *P, int64_t ld,
             const Ctl *ctl) {
  double *tag = nullptr;
  const Prec<double> pc = prec_of(A, tag);
  const int G = grid_rows(A->n);
  const bool amg = A->prec == SSP_PREC_AMG;
  if (amg) {
    if (ctl) return fail(h, SSP_EUNSUPPORTED, "the AMG preconditioner allocates no scratch here");
    int rc = amg_vcycle(h, A, r, P);
    if (rc) return rc;
  } else {
    k_prec<double><<<G, kWG, 0, h->stream>>>(A->n, r, P, pc);
  }
  LAUNCHCHK(h);
  if constexpr (S >= 2) {
    if (!ctl && !amg && !pc.dinv && tb_usable(A, S)) {
      int Gt = 0;
      int rc = tb_powers<S, double>(h, A, r, pc.dc, P, ld, true, h->st, h->ws.partials, Gt);
      if (rc) return rc;
      k_finalize<EpiMpkLast<S, double>><<<1, kWG, 0, h->stream>>>(
          EpiMpkLast<S, double>{P + (int64_t)(2 * S - 1) * ld, P, ld, r, 0}, h->st,
          h->ws.partials, Gt);
      LAUNCHCHK(h);
      return SSP_OK;
    }
  }
  for (int j = 1; j <= S; ++j) {
    const double *zin = P + (int64_t)(j - 1) * ld;
    double *az = P + (int64_t)(S + j - 1) * ld;
    int rc;
    if (j < S) {
      rc = launch_op<double>(h, A, zin, EpiMpk<double>{az, amg ? nullptr : P + (int64_t)j * ld, pc},
                             0, 1.0, ctl);
      if (!rc && amg) rc = amg_vcycle(h, A, az, P + (int64_t)j * ld);
    } else
      rc = launch_op<double>(h, A, zin, EpiMpkLast<S, double>{az, P, ld, r, 0}, 1, 1.0, ctl);
    if (rc) return rc;
  }
  return SSP_OK;
}

// The Chebyshev basis of one outer iteration on its own: P = [Z | AZ] for
// z_1 = B^-1 r (columns at P + j ld), and the Gram sums Z^T [AZ | 0 | r]
// reduced into `out` (s (2s+1) doubles, device; the AP_{i-1} part is 0).
template <int S>
int cheb_basis_only(ssp_handle *h, const ssp_matrix *A, const double *r, double *P, int64_t ld,
                    double c, double g, double *out) {
  double *tag = nullptr;
  const Prec<double> pc = prec_of(A, tag);
  k_prec<double><<<grid_rows(A->n), kWG, 0, h->stream>>>(A->n, r, P, pc);
  LAUNCHCHK(h);
  for (int j = 1; j <= S; ++j) {
    double *zj = P + (int64_t)(j - 1) * ld;
    double *az = P + (int64_t)(S + j - 1) * ld;
    int rc;
    if (j < S)
      rc = launch_op<double>(h, A, zj,
                             EpiCheb<double>{az, P + (int64_t)j * ld, zj,
                                             j >= 2 ? P + (int64_t)(j - 2) * ld : nullptr, pc,
                                             c, j == 1 ? g : 2.0 * g},
                             0);
    else
      rc = launch_op<double>(h, A, zj, EpiMpk<double>{az, nullptr, pc}, 1);
    if (rc) return rc;
  }
  const int Gg = gram_grid(A->n);
  k_gram<S, double><<<Gg, kWG, 0, h->stream>>>(A->n, ld, P, nullptr, r, 1, h->st,
                                                h->ws.partials_gram);
  k_gram_totals<S><<<1, kFinWG, 0, h->stream>>>(h->ws.partials_gram, Gg, out);
  LAUNCHCHK(h);
  return SSP_OK;
}

template <typename T>
using iter_fn = int (*)(ssp_handle *, const ssp_matrix *, const IterBufs<T> &, int, bool, bool);
using cheb_basis_fn = int (*)(ssp_handle *, const ssp_matrix *, const double *, double *, int64_t,
                              double, double, double *);
using mpk_fn = int (*)(ssp_handle *, const ssp_matrix *, const double *, double *, int64_t,
                       const Ctl *);

// Defined in inst_f64.hip (s = 1..16) and inst_f32.hip (s = 1..8);
// nullptr for an s out of range.  cheb_*: the Chebyshev-basis iteration.
iter_fn<double> iteration_f64(int s);
iter_fn<float> iteration_f32(int s);
iter_fn<double> cheb_iteration_f64(int s);
cheb_basis_fn cheb_basis_f64(int s);
iter_fn<float> cheb_iteration_f32(int s);
mpk_fn mpk_f64(int s);

constexpr int kSMaxF32 = 8;

// Shared helpers defined in capi.hip.
int ensure_fp32(ssp_handle *h, ssp_matrix *A);
int status_code(int device_status);

}  // namespace ssp
