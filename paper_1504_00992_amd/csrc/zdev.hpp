// Device-side complex helpers and wavefront / workgroup reductions (CDNA4,
// 64-lane wavefronts).
#pragma once

#include "internal.hpp"

namespace tebd {

__device__ __forceinline__ zt zmake(double re, double im) { return make_double2(re, im); }
__device__ __forceinline__ zt zconj(zt a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ zt zadd(zt a, zt b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ zt zsub(zt a, zt b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ zt zscale(zt a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ zt zmul(zt a, zt b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ zt zcmul(zt a, zt b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double zabs2(zt a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum over the workgroup; every thread receives the result.  `red` must hold
// one double per wavefront; the call contains two barriers.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) t += red[i];
  __syncthreads();
  return t;
}

}  // namespace tebd
