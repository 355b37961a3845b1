// Streaming reference kernels for the roofline figures: the bandwidth a plain
// read (and a plain copy) of a large array reaches on this device, measured
// with the library's own launch geometry.
#pragma once

#include "common.hpp"

namespace ssp {

// Reads n doubles (16-byte loads, grid-strided) and stores one sum per
// workgroup (so the loads cannot be removed).
__global__ __launch_bounds__(kWG) void k_stream_read(int64_t n, const double *__restrict__ src,
                                                     double *__restrict__ part) {
  const double2 *s2 = reinterpret_cast<const double2 *>(src);
  const int64_t n2 = n / 2;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n2; i += (int64_t)gridDim.x * kWG) {
    const double2 v = s2[i];
    acc += v.x + v.y;
  }
  double t[1] = {acc};
  block_store_sums<1>(t, part + blockIdx.x, gridDim.x);
}

// dst = src, 16-byte loads and stores, grid-strided.
__global__ __launch_bounds__(kWG) void k_stream_copy(int64_t n, const double *__restrict__ src,
                                                     double *__restrict__ dst) {
  const double2 *s2 = reinterpret_cast<const double2 *>(src);
  double2 *d2 = reinterpret_cast<double2 *>(dst);
  const int64_t n2 = n / 2;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n2; i += (int64_t)gridDim.x * kWG)
    d2[i] = s2[i];
}

}  // namespace ssp
