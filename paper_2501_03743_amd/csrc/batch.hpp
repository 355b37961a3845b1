// Batched persistent solve: many independent systems of uneven size in ONE
// launch.  Each system runs the mixed-precision s-step solve (FP64 outer
// residual and refinement, FP32 matrix powers and block updates, FP64
// moments and s x s algebra) as a state machine of phases:
//
//   RESID  (tiles) r = b - A x in FP64 -> FP32 rhs, z1, d = 0    -> outer test
//   POWER j (tiles, j = 1..s) matrix powers; j = s adds the moments -> s x s solve
//   UPDATE (tiles) fused block update                            -> inner test
//   IRADD  (tiles) x += d                                        -> RESID
//   DONE
//
// A phase is split into tiles of rows.  Persistent workgroups claim runs of
// up to `run` consecutive tiles from any system with unclaimed work (a 64-bit
// word per system packs the phase sequence number and the next tile, so a
// claim can never be applied to the wrong phase), process them, and count
// them done.  The workgroup that
// completes a phase's last tile reduces the phase's partial sums, runs the
// finishing step (stopping tests, the s x s solve) and publishes the next
// phase.  No workgroup ever waits for another: an idle workgroup polls the
// systems, so the schedule cannot deadlock, and every poll loop carries a
// stall guard so the grid always drains.
//
// Memory ordering: tile outputs are released (agent-scope release fence in
// every wave, then the done counter increment); the finishing workgroup and
// the claimers of the next phase acquire (agent-scope acquire fence after the
// atomic) before reading them.  On gfx950 these fences write back and
// invalidate the XCD's L2, so they are taken once per run of tiles.
#pragma once

#include "kernels.hpp"
#include "sstep.h"

namespace ssp {

enum : int { PH_RESID = 0, PH_POWER = 1, PH_UPDATE = 2, PH_IRADD = 3, PH_DONE = 4 };

// Per-system description (read-only in the kernel).
struct BatchSys {
  int kind;                 // 0 = CSR (row form), else SSP_STENCIL_*
  CsrArgs<double> c64;
  CsrArgs<float> c32;
  StencilArgs<double> s64;
  StencilArgs<float> s32;
  Prec<double> pc64;
  Prec<float> pc32;
  const double *b;
  double *x;
  float *Q1, *Q2, *r32, *d32;
  int64_t ld;
  double *partials;         // component-major, stride ntiles
  double *hist;             // FP64 residual per refinement step
  DevState *st;
  int64_t n;
  int64_t tile_rows;
  int ntiles;
  int single;               // 1: the partition of a single solve (tile t = its block t)
};

// Per-system scheduling words (device atomics).
struct BatchSched {
  unsigned long long claim; // (sequence << 32) | next tile
  unsigned done;            // tiles finished in the current phase
  int phase;
  int j;                    // matrix power index
  int pad;
};

struct BatchGlobal {
  unsigned ndone;           // systems in PH_DONE
  unsigned progress;        // tiles finished (stall guard)
  int error;                // 1: a workgroup saw no progress for too long
  int pad;
};

__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// Applies the operator of system y (in precision T) to rows [lo, hi).
template <typename T, class F>
__device__ __forceinline__ void batch_rows(const BatchSys &y, const T *x, int64_t lo, int64_t hi,
                                           F &&f) {
  if constexpr (sizeof(T) == 8) {
    switch (y.kind) {
      case 0: csr_rows_direct(y.c64, x, lo, hi, f); break;
      case SSP_STENCIL_2D5: stencil_rows<K_2D5>(y.s64, x, lo, hi, f); break;
      case SSP_STENCIL_3D7: stencil_rows<K_3D7>(y.s64, x, lo, hi, f); break;
      case SSP_STENCIL_3D27: stencil_rows<K_3D27>(y.s64, x, lo, hi, f); break;
      default: stencil_rows<K_VARK>(y.s64, x, lo, hi, f); break;
    }
  } else {
    switch (y.kind) {
      case 0: csr_rows_direct(y.c32, x, lo, hi, f); break;
      case SSP_STENCIL_2D5: stencil_rows<K_2D5>(y.s32, x, lo, hi, f); break;
      case SSP_STENCIL_3D7: stencil_rows<K_3D7>(y.s32, x, lo, hi, f); break;
      case SSP_STENCIL_3D27: stencil_rows<K_3D27>(y.s32, x, lo, hi, f); break;
      default: stencil_rows<K_VARK>(y.s32, x, lo, hi, f); break;
    }
  }
}

// Processes tile t of the current phase of system y; stores its partial sums.
template <int S>
__device__ void batch_tile(const BatchSys &y, const BatchSched &sc, int t) {
  const int64_t lo0 = (int64_t)t * y.tile_rows;
  const int64_t lo = lo0 < y.n ? lo0 : y.n;
  const int64_t hi = (lo + y.tile_rows < y.n) ? lo + y.tile_rows : y.n;
  const int k = y.st->k;
  float *Pc = (k % 2 == 0) ? y.Q2 : y.Q1;
  float *Po = (k % 2 == 0) ? y.Q1 : y.Q2;
  if (sc.phase == PH_RESID) {
    EpiIrResidual epi{y.b, y.r32, y.Q2, y.d32, y.pc32, y.hist};
    double part[3] = {0.0, 0.0, 0.0};
    batch_rows<double>(y, y.x, lo, hi, [&](int64_t i, double v) { epi.row(i, v, part); });
    block_store_sums<3>(part, y.partials + t, y.ntiles);
  } else if (sc.phase == PH_POWER) {
    const int j = sc.j;
    const float *zin = Pc + (int64_t)(j - 1) * y.ld;
    float *az = Pc + (int64_t)(S + j - 1) * y.ld;
    if (j < S) {
      EpiMpk<float> epi{az, Pc + (int64_t)j * y.ld, y.pc32};
      batch_rows<float>(y, zin, lo, hi, [&](int64_t i, float v) { epi.row(i, v, nullptr); });
    } else {
      EpiMpkLast<S, float> epi{az, Pc, y.ld, y.r32, 1};
      double part[2 * S];
#pragma unroll
      for (int c = 0; c < 2 * S; ++c) part[c] = 0.0;
      batch_rows<float>(y, zin, lo, hi, [&](int64_t i, float v) { epi.row(i, v, part); });
      block_store_sums<2 * S>(part, y.partials + t, y.ntiles);
    }
  } else if (sc.phase == PH_UPDATE) {
    UpdateCoef<S, float> c;
    c.load(y.st);
    double v[1] = {0.0};
    if (y.single) {
      // the rows block t of the single solve's update kernel takes
      const XcdSched xs = xcd_sched(y.n, kWG, y.ntiles, t);
      for (int64_t b0 = xs.first; b0 < xs.end; b0 += xs.stride) {
        const int64_t b1 = b0 + kWG < xs.end ? b0 + kWG : xs.end;
        v[0] += update_rows<S, float>(c, b0, b1, y.ld, Pc, Po, y.d32, y.r32, y.pc32, 0.0f);
      }
    } else {
      v[0] = update_rows<S, float>(c, lo, hi, y.ld, Pc, Po, y.d32, y.r32, y.pc32, 0.0f);
    }
    block_store_sums<1>(v, y.partials + t, y.ntiles);
  } else if (sc.phase == PH_IRADD) {
    for (int64_t i = lo + threadIdx.x; i < hi; i += kWG) y.x[i] = y.x[i] + (double)y.d32[i];
  }
}

// Run by the whole workgroup that finished the last tile of a phase: finish
// the phase and return the next one (j in *jn).
template <int S>
__device__ int batch_transition(const BatchSys &y, const BatchSched &sc, int *jn) {
  DevState *st = y.st;
  __shared__ int next_s, j_s;
  if (sc.phase == PH_RESID) {
    double tot[3];
    reduce_partials<3>(y.partials, y.ntiles, tot);
    EpiIrResidual{y.b, y.r32, y.Q2, y.d32, y.pc32, y.hist}.finish(st, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
      next_s = (st->status == ST_RUNNING) ? PH_POWER : PH_DONE;
      j_s = 1;
    }
  } else if (sc.phase == PH_POWER) {
    if (sc.j < S) {
      if (threadIdx.x == 0) {
        next_s = PH_POWER;
        j_s = sc.j + 1;
      }
    } else {
      double tot[2 * S];
      reduce_partials<2 * S>(y.partials, y.ntiles, tot);
      small_solve_t<S>(st, tot);
      __syncthreads();
      if (threadIdx.x == 0) {
        j_s = 1;
        if (st->status == ST_RUNNING) next_s = PH_UPDATE;
        else next_s = (st->k > 0) ? PH_IRADD : PH_DONE;   // inner breakdown
      }
    }
  } else if (sc.phase == PH_UPDATE) {
    double tot[1];
    reduce_partials<1>(y.partials, y.ntiles, tot);
    FinUpdate{nullptr}.finish(st, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
      st->ir_inner_total += 1;
      next_s = (st->status == ST_RUNNING) ? PH_POWER : PH_IRADD;
      j_s = 1;
    }
  } else {  // PH_IRADD
    if (threadIdx.x == 0) {
      st->ir_refine += 1;
      next_s = PH_RESID;
      j_s = 1;
    }
  }
  __syncthreads();
  *jn = j_s;
  return next_s;
}

// The persistent kernel.  order: 0 = scan systems from the largest, 1 =
// round-robin start per workgroup.  spin_limit bounds the consecutive empty
// polls without any global progress before a workgroup gives up (error).
template <int S>
__global__ __launch_bounds__(kWG) void k_batch(const BatchSys *__restrict__ sys,
                                               BatchSched *sched, BatchGlobal *glob, int nsys,
                                               const int *__restrict__ scan_order, int order,
                                               unsigned spin_limit, int run) {
  __shared__ int s_sys, s_tile, s_cnt, s_exit;
  unsigned idle = 0, last_progress = 0;
  const int start = (order == 1) ? (int)(blockIdx.x % (unsigned)nsys) : 0;
  for (;;) {
    if (threadIdx.x == 0) {
      s_sys = -1;
      s_exit = 0;
      const unsigned nd = __hip_atomic_load(&glob->ndone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int err = __hip_atomic_load(&glob->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (nd >= (unsigned)nsys || err) {
        s_exit = 1;
      } else {
        for (int q = 0; q < nsys && s_sys < 0; ++q) {
          const int i = scan_order[(start + q) % nsys];
          BatchSched *sc = &sched[i];
          const unsigned long long c =
              __hip_atomic_load(&sc->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if ((unsigned)(c & 0xffffffffull) >= (unsigned)sys[i].ntiles) continue;
          const unsigned long long c2 = __hip_atomic_fetch_add(
              &sc->claim, (unsigned long long)run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const unsigned t = (unsigned)(c2 & 0xffffffffull);
          if (t < (unsigned)sys[i].ntiles) {
            s_sys = i;
            s_tile = (int)t;
            s_cnt = (int)min((unsigned)run, (unsigned)sys[i].ntiles - t);
          }
        }
        if (s_sys < 0) {
          const unsigned pr =
              __hip_atomic_load(&glob->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (pr != last_progress) {
            last_progress = pr;
            idle = 0;
          } else if (++idle > spin_limit) {
            __hip_atomic_store(&glob->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_exit = 1;
          }
        }
      }
    }
    __syncthreads();
    if (s_exit) break;
    const int i = s_sys;
    if (i < 0) {
      __builtin_amdgcn_s_sleep(8);
      continue;
    }
    fence_acquire();
    const BatchSys y = sys[i];
    BatchSched sc;
    sc.phase = __hip_atomic_load(&sched[i].phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sc.j = __hip_atomic_load(&sched[i].j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int cnt = s_cnt;
    for (int k = 0; k < cnt; ++k) batch_tile<S>(y, sc, s_tile + k);
    fence_release();
    __syncthreads();
    __shared__ int s_last;
    if (threadIdx.x == 0) {
      const unsigned d = __hip_atomic_fetch_add(&sched[i].done, (unsigned)cnt, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&glob->progress, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_last = (d + (unsigned)cnt == (unsigned)y.ntiles);
    }
    __syncthreads();
    if (!s_last) continue;
    // this workgroup finished the phase: finish it and publish the next one
    fence_acquire();
    int jn = 1;
    const int next = batch_transition<S>(y, sc, &jn);
    fence_release();
    __syncthreads();
    if (threadIdx.x == 0) {
      __hip_atomic_store(&sched[i].done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&sched[i].phase, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&sched[i].j, jn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // this workgroup is the only writer of the sequence bits
      const unsigned long long cur =
          __hip_atomic_load(&sched[i].claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long seq = ((cur >> 32) + 1ull) << 32;
      if (next == PH_DONE) {
        __hip_atomic_store(&sched[i].claim, seq | (unsigned long long)y.ntiles,
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&glob->ndone, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_store(&sched[i].claim, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
  }
}

// Stepped schedule: the same per-system phases, one launch pair per step.
// k_batch_tiles runs every tile of every unfinished system's current phase
// (work item g is tile tile_idx[g] of system tile_sys[g]); k_batch_step then
// finishes each system's phase (one workgroup per system).  Kernel
// boundaries order the phases, so no fences or claims are needed, and a
// tile's arithmetic is the persistent kernel's exactly.
template <int S>
__global__ __launch_bounds__(kWG) void k_batch_tiles(const BatchSys *__restrict__ sys,
                                                     const BatchSched *__restrict__ sched,
                                                     const int *__restrict__ tile_sys,
                                                     const int *__restrict__ tile_idx) {
  const int i = tile_sys[blockIdx.x];
  BatchSched sc;
  sc.phase = sched[i].phase;
  sc.j = sched[i].j;
  if (sc.phase == PH_DONE) return;
  batch_tile<S>(sys[i], sc, tile_idx[blockIdx.x]);
}

template <int S>
__global__ __launch_bounds__(kWG) void k_batch_step(const BatchSys *__restrict__ sys,
                                                    BatchSched *sched, BatchGlobal *glob) {
  const int i = blockIdx.x;
  BatchSched sc;
  sc.phase = sched[i].phase;
  sc.j = sched[i].j;
  if (sc.phase == PH_DONE) return;
  int jn = 1;
  const int next = batch_transition<S>(sys[i], sc, &jn);
  if (threadIdx.x == 0) {
    sched[i].phase = next;
    sched[i].j = jn;
    if (next == PH_DONE) atomicAdd(&glob->ndone, 1u);
  }
}

}  // namespace ssp
