// Temporally blocked matrix powers of the 3D 7-point constant-coefficient
// operator: the communication-avoiding form of Alg. 4 (Sec. IV) on one GPU.
//
// One launch computes L consecutive powers.  A workgroup owns a 32 x 32
// column of the grid and a chunk of z planes and marches through the planes;
// at march step t it loads plane t of the input and computes plane t - l of
// power l, l = 1..L (each power one plane behind the one it reads).  Every
// level keeps its last planes in an LDS ring, over the tile widened by L - l
// cells on each side, which is exactly what the next level reads, so a
// level's input never leaves the compute unit.  Only the tile's own points
// (and only planes of its chunk) are stored; the widened borders are
// recomputed by the neighbouring workgroups.  Per point the arithmetic is the
// matrix-free kernel's (neighbours scaled by c and rounded first, summed in
// the order x-, x+, y-, y+, z-, z+, only those inside the grid; diag * centre
// + off * sum), so every power is bitwise equal to the one-launch-per-power
// path's.  The launch that computes the last power also forms Alg. 5's
// moments z_a^T r and z_a^T AZ(:,s) per point (the same products as the
// fused last power) and leaves per-workgroup partial sums; only their
// reduction order differs.
//
// Nothing a launch stores is read back by it (the moments take z_a from the
// rings, deep enough to still hold the plane they need, or from columns of
// earlier launches), so the barriers between levels order LDS only and never
// wait for global stores in flight; the next input plane is loaded into
// registers one step ahead.
#pragma once

#include "kernels.hpp"

namespace ssp {

constexpr int kTbT = 32;     // tile edge (x and y) of the stored points
constexpr int kTbWG = 1024;  // threads per workgroup
constexpr int kCUs = 256;     // MI355X compute units
constexpr int kTbMaxL = 4;   // powers per launch (FP64 rings of 4 levels: 144 KB of LDS)

// LDS rings of a launch of L levels: level l < L (level 0 is the input) keeps
// its last D_l planes over the (kTbT + 2 (L - l))^2 region: three for the
// next level's stencil, more where the moments still need plane t - L
// (D_l = L - l + 1 for l >= 1).
__host__ __device__ constexpr int tb_edge(int L, int l) { return kTbT + 2 * (L - l); }
__host__ __device__ constexpr int tb_depth(int L, int l) {
  return (l >= 1 && L - l + 1 > 3) ? L - l + 1 : 3;
}
__host__ __device__ constexpr int tb_lds_off(int L, int l) {
  int s = 0;
  for (int m = 0; m < l; ++m) s += tb_depth(L, m) * tb_edge(L, m) * tb_edge(L, m);
  return s;
}
__host__ __device__ constexpr int tb_lds_elems(int L) { return tb_lds_off(L, L); }

// Launches of an s-power block: ceil(s / 4) launches of nearly equal level
// counts, the longer ones first (s = 5: 3 + 2; s = 8: 4 + 4).
__host__ __device__ constexpr int tb_passes(int s) { return (s + kTbMaxL - 1) / kTbMaxL; }
__host__ __device__ constexpr int tb_levels(int s, int pass) {
  return s / tb_passes(s) + (pass < s % tb_passes(s) ? 1 : 0);
}

struct TbTiling {
  int ntx, nty, ntz, zchunk;
};

// Ring slot of plane p (p >= -kTbMaxL - 1) in a ring of D planes.
__device__ __forceinline__ int tb_slot(int p, int D) { return (p + 2 * D * kTbMaxL) % D; }

// Workgroup barrier that orders LDS accesses only: outstanding global loads
// and stores stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroup sums of NP values, stored component-major at out[c * stride]
// (the kTbWG-thread form of block_store_sums).
template <int NP>
__device__ __forceinline__ void tb_store_sums(const double (&v)[NP], double *out, int64_t stride) {
  __shared__ double red[kTbWG / kWave][NP];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    const double t = wave_sum(v[c]);
    if (lane == 0) red[wid][c] = t;
  }
  __syncthreads();
  if (threadIdx.x < NP) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kTbWG / kWave; ++w) t += red[w][threadIdx.x];
    out[threadIdx.x * stride] = t;
  }
}

// Powers j0 + 1 .. j0 + L of the block P (AZ(:,j) at column S + j - 1, Z(:,j)
// at column j - 1, leading dimension ld) from the input column `in`
// (r for j0 = 0, else AZ(:,j0)), each level's input scaled by c (the
// constant Jacobi factor, or 1): AZ(:,j) = A (c AZ(:,j-1)).  store_z: also
// store Z(:,j+1) = c AZ(:,j) for j < S (the explicit block of the stand-alone
// Alg. 4 + 5 call).  SM = S when this launch computes the last power: then
// the moments vm(a) = z_a^T r, vm(S+a) = z_a^T AZ(:,S), a < S, with z_0 = c r
// and z_a = c AZ(:,a), go to partials[c * G + g]; SM = 0 otherwise.
template <int L, int SM, typename T>
__global__ __launch_bounds__(kTbWG) void k_mpk_tb7(StencilArgs<T> A, const T *__restrict__ in,
                                                   T c, int j0, int S, T *P, int64_t ld,
                                                   int store_z, const T *__restrict__ r,
                                                   DevState *st, double *partials, TbTiling tl) {
#pragma clang fp contract(off)
  if (st->status != ST_RUNNING) return;
  __shared__ T lds[tb_lds_elems(L)];
  constexpr int NP = SM > 0 ? 2 * SM : 1;
  constexpr int E0 = tb_edge(L, 0);
  constexpr int NPF = (E0 * E0 + kTbWG - 1) / kTbWG;   // input values per thread and plane
  double part[NP];
#pragma unroll
  for (int a = 0; a < NP; ++a) part[a] = 0.0;
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  const int b = logical_block();   // x-y neighbours run on the same XCD
  const int tx = b % tl.ntx, ty = (b / tl.ntx) % tl.nty, tz = b / (tl.ntx * tl.nty);
  const int x0 = tx * kTbT, y0 = ty * kTbT, z0 = tz * tl.zchunk;
  const int z1 = (z0 + tl.zchunk < nz) ? z0 + tl.zchunk : nz;
  const int t0 = z0 - L, t1 = z1 - 1 + L;   // input planes of the chunk
  // the input plane of the next step, held in registers while a step runs
  T pf[NPF];
  auto fetch = [&](int pz) {
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int e = threadIdx.x + k * kTbWG;
      const int hy = e / E0, hx = e - hy * E0;
      const int gx = x0 - L + hx, gy = y0 - L + hy;
      if (pz >= 0 && pz < nz && e < E0 * E0 && gx >= 0 && gx < nx && gy >= 0 && gy < ny)
        pf[k] = in[(int64_t)pz * sz + (int64_t)gy * sy + gx];
    }
  };
  auto put = [&](int pz) {
    T *R = lds + tb_slot(pz, 3) * E0 * E0;
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int e = threadIdx.x + k * kTbWG;
      const int hy = e / E0, hx = e - hy * E0;
      const int gx = x0 - L + hx, gy = y0 - L + hy;
      if (pz >= 0 && pz < nz && e < E0 * E0 && gx >= 0 && gx < nx && gy >= 0 && gy < ny)
        R[e] = c * pf[k];
    }
  };
  // the moment inputs of the next step's level-L point (one point per
  // thread: kTbT^2 == kTbWG): r and, beyond the first launch, the columns
  // AZ(:,a), a <= j0, of earlier launches
  static_assert(kTbT * kTbT == kTbWG, "level L: one point per thread");
  T mr = T(0);
  T mz[SM > 0 ? SM : 1];
#pragma unroll
  for (int a = 0; a < (SM > 0 ? SM : 1); ++a) mz[a] = T(0);
  auto mfetch = [&](int pz) {
    if constexpr (SM > 0) {
      const int gx = x0 + (int)threadIdx.x % kTbT, gy = y0 + (int)threadIdx.x / kTbT;
      if (pz >= z0 && pz < z1 && gx < nx && gy < ny) {
        const int64_t q = (int64_t)pz * sz + (int64_t)gy * sy + gx;
        mr = r[q];
#pragma unroll
        for (int a = 1; a < SM; ++a)
          if (a <= j0) mz[a] = P[(int64_t)(SM + a - 1) * ld + q];
      }
    }
  };
  if (z0 < z1) {
    fetch(t0);
    mfetch(t0 - L);
  }
  for (int t = t0; z0 < z1 && t <= t1; ++t) {
    // level 0: plane t of the input (its ring slot held plane t - 3, last
    // read by level 1 in the previous step)
    put(t);
    if (t < t1) fetch(t + 1);
    lds_barrier();
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      const int p = t - l;
      const int h = L - l;
      const int lo = (z0 - h > 0) ? z0 - h : 0;
      const int hi = (z1 + h - 1 < nz - 1) ? z1 + h - 1 : nz - 1;
      if (p >= lo && p <= hi) {
        const int E = tb_edge(L, l), Ep = E + 2;
        const int Dp = tb_depth(L, l - 1);
        const T *Rp = lds + tb_lds_off(L, l - 1);
        const T *Rm = Rp + tb_slot(p - 1, Dp) * Ep * Ep;
        const T *Rc = Rp + tb_slot(p, Dp) * Ep * Ep;
        const T *Rn = Rp + tb_slot(p + 1, Dp) * Ep * Ep;
        T *Rw = lds + tb_lds_off(L, l < L ? l : 0) + tb_slot(p, tb_depth(L, l < L ? l : 0)) * E * E;
        const int jj = j0 + l;
        T *az = P + (int64_t)(S + jj - 1) * ld;
        for (int e = threadIdx.x; e < E * E; e += kTbWG) {
          const int hy = e / E, hx = e - hy * E;
          const int gx = x0 - h + hx, gy = y0 - h + hy;
          if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
          const int ce = (hy + 1) * Ep + hx + 1;
          const T xc = Rc[ce];
          const T xm = Rc[ce - 1], xpl = Rc[ce + 1];
          const T ym = Rc[ce - Ep], ypl = Rc[ce + Ep];
          const T zm = Rm[ce], zpl = Rn[ce];
          T nb = 0;
          nb = gx > 0 ? nb + xm : nb;
          nb = gx < nx - 1 ? nb + xpl : nb;
          nb = gy > 0 ? nb + ym : nb;
          nb = gy < ny - 1 ? nb + ypl : nb;
          nb = p > 0 ? nb + zm : nb;
          nb = p < nz - 1 ? nb + zpl : nb;
          const T d = A.diag * xc;
          const T o = A.off * nb;
          const T v = d + o;
          if (l < L) Rw[e] = c * v;
          const bool own = hx >= h && hx < h + kTbT && hy >= h && hy < h + kTbT && p >= z0 &&
                           p < z1;
          if (!own) continue;
          const int64_t q = (int64_t)p * sz + (int64_t)gy * sy + gx;
          az[q] = v;
          if (store_z && jj < S) P[(int64_t)jj * ld + q] = c * v;
          if constexpr (SM > 0) {
            if (l == L) {
              // z_a at this point: c r and the input column from memory
              // (read-only here), the levels of this launch from their rings
              const T rt = mr;
              const double ri = (double)rt, vi = (double)v;
#pragma unroll
              for (int a = 0; a < SM; ++a) {
                const int la = a - j0;
                double za;
                if (a == 0) {
                  za = (double)(c * rt);
                } else if (la <= 0) {
                  za = (double)(c * mz[a]);
                } else {
                  za = 0.0;
#pragma unroll
                  for (int m = 1; m < L; ++m) {
                    if (la == m) {
                      const int Em = tb_edge(L, m), off = L - m;
                      za = (double)lds[tb_lds_off(L, m) + tb_slot(p, tb_depth(L, m)) * Em * Em +
                                       (hy + off) * Em + hx + off];
                    }
                  }
                }
                const double t1v = za * ri;
                part[a] += t1v;
                const double t2v = za * vi;
                part[SM + a] += t2v;
              }
            }
          }
        }
      }
      if (l == L) mfetch(t + 1 - L);
      lds_barrier();
    }
  }
  if constexpr (SM > 0) tb_store_sums<NP>(part, partials + b, gridDim.x);
}

// Tiling of the temporally blocked launch: 32 x 32 columns, and as many z
// chunks as fill the GPU in one round of workgroups (per_cu resident per
// compute unit; a second, partial round would double the time), each chunk
// at least 2L planes deep.
inline TbTiling tb_tiling(int nx, int ny, int nz, int L, int per_cu) {
  TbTiling t;
  t.ntx = (nx + kTbT - 1) / kTbT;
  t.nty = (ny + kTbT - 1) / kTbT;
  const int64_t plane = (int64_t)t.ntx * t.nty;
  int64_t ntz = std::max<int64_t>(1, (int64_t)kCUs * std::max(per_cu, 1) / plane);
  const int64_t deep = std::max<int64_t>(1, nz / (2 * L));
  if (ntz > deep) ntz = deep;
  if (ntz * plane > kGridMax) ntz = std::max<int64_t>(1, kGridMax / plane);
  t.zchunk = (int)((nz + ntz - 1) / ntz);
  t.ntz = (nz + t.zchunk - 1) / t.zchunk;
  return t;
}

// Workgroups of the tiling (the grid of the launch).
inline int64_t tb_grid(const TbTiling &t) { return (int64_t)t.ntx * t.nty * t.ntz; }

}  // namespace ssp
