// Matrix set-up kernels of libsstep: Jacobi vectors, CSR validation and
// statistics, stencil-to-CSR materialisation, FP64 -> FP32 copies.
#pragma once

#include "common.hpp"
#include "operators.hpp"

namespace ssp {

// FP32 copy of an FP64 array (matrix values, Jacobi vector, coefficients).
__global__ __launch_bounds__(kWG) void k_to_float(int64_t n, const double *__restrict__ a,
                                                  float *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
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
__global__ __launch_bounds__(kWG) void k_vark_dinv(StencilArgs<double> S, double *dinv) {
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
  for (int f = 0; f < 6; ++f) dsum += in[f] ? face_weight(kp, S.k[q[f]]) : kp;
  dinv[p] = 1.0 / dsum;
}

// Fills colind/val of a stencil operator in CSR form, columns ascending.
template <int KIND>
__global__ __launch_bounds__(kWG) void k_stencil_fill(StencilArgs<double> S, const int32_t *rowptr,
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
        w[f] = in[f] ? face_weight(kp, S.k[q[f]]) : kp;
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

// Sets *differs if some dinv[i] is not bitwise equal to dinv[0].
__global__ __launch_bounds__(kWG) void k_all_equal(int64_t n, const double *__restrict__ v,
                                                   int *differs) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  if (__double_as_longlong(v[i]) != __double_as_longlong(v[0])) atomicOr(differs, 1);
}

// Largest 1 / dinv_i (the largest diagonal entry) over the finite positive
// values, as the bit pattern of a non-negative double (which orders like the
// integer): one atomicMax per workgroup on *out (zeroed by the caller).
__global__ __launch_bounds__(kWG) void k_max_recip(int64_t n, const double *__restrict__ dinv,
                                                   unsigned long long *out) {
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
    const double d = 1.0 / dinv[i];
    if (isfinite(d) && d > m) m = d;
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const double o = __shfl_xor(m, off, kWave);
    m = o > m ? o : m;
  }
  __shared__ double red[kWG / kWave];
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int w = 1; w < kWG / kWave; ++w) b = red[w] > b ? red[w] : b;
    unsigned long long bits;
    memcpy(&bits, &b, sizeof(bits));
    atomicMax(out, bits);
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
      if (c < 0 || c >= n || c <= prev) {
        ok = 0;
        break;
      }
      prev = c;
      if (c == i) d += val[e];
    }
  }
  if (!(d > 0.0)) ok = 0;
  if (!ok) atomicOr(bad, 1);
}

// Sliced ELL set-up: the width of slice sl is its longest row.
__global__ __launch_bounds__(kWG) void k_sell_width(int64_t n, int64_t nslices,
                                                    const int32_t *__restrict__ rowptr,
                                                    int32_t *__restrict__ width) {
  const int64_t sl = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (sl >= nslices) return;
  int w = 0;
  for (int l = 0; l < kWave; ++l) {
    const int64_t r = sl * kWave + l;
    if (r < n) w = max(w, rowptr[r + 1] - rowptr[r]);
  }
  width[sl] = w;
}

// One thread per (padded) row: its entries in slice order, then padding
// (column -1, value 0) up to the slice width.
__global__ __launch_bounds__(kWG) void k_sell_fill(int64_t n, int64_t nslices,
                                                   const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ colind,
                                                   const double *__restrict__ val,
                                                   const int64_t *__restrict__ slice_off,
                                                   const int32_t *__restrict__ width,
                                                   int32_t *__restrict__ scol,
                                                   double *__restrict__ sval) {
  const int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (r >= nslices * kWave) return;
  const int64_t sl = r / kWave;
  const int lane = (int)(r - sl * kWave);
  const int w = width[sl];
  const int a = r < n ? rowptr[r] : 0;
  const int len = r < n ? rowptr[r + 1] - a : 0;
  for (int u = 0; u < w; ++u) {
    const int64_t e = slice_off[sl] + (int64_t)u * kWave + lane;
    if (u < len) {
      scol[e] = colind[a + u];
      sval[e] = val[a + u];
    } else {
      scol[e] = -1;
      sval[e] = 0.0;
    }
  }
}

}  // namespace ssp
