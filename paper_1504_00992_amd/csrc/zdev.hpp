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
// re + i im += conj(u) y, as four fused multiply-adds
__device__ __forceinline__ void zdot_acc(zt u, zt y, double& re, double& im) {
  re = fma(u.x, y.x, fma(u.y, y.y, re));
  im = fma(u.x, y.y, fma(-u.y, y.x, im));
}
// The two outputs of a real plane rotation of complex x, y:
// cs x - sn y and sn x + cs y, with fused multiply-adds.
__device__ __forceinline__ zt zrot_lo(zt x, zt y, double cs, double sn) {
  return make_double2(fma(cs, x.x, -sn * y.x), fma(cs, x.y, -sn * y.y));
}
__device__ __forceinline__ zt zrot_hi(zt x, zt y, double cs, double sn) {
  return make_double2(fma(sn, x.x, cs * y.x), fma(sn, x.y, cs * y.y));
}
// y - u d, as four fused multiply-adds
__device__ __forceinline__ zt zsub_mul(zt y, zt u, zt d) {
  return make_double2(fma(-u.x, d.x, fma(u.y, d.y, y.x)), fma(-u.x, d.y, fma(-u.y, d.x, y.y)));
}
// *p when c holds, else 0, without selecting between addresses (a select of
// an LDS or global address with a local's address would put the local in
// scratch memory).
__device__ __forceinline__ zt zload_if(bool c, const zt* p) {
  zt v = make_double2(0.0, 0.0);
  if (c) v = *p;
  return v;
}

// Wavefront sum of a double, result in every lane.  DPP moves on the two
// 32-bit halves: quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror and
// row_mirror give every lane its 16-lane row sum; row_bcast15 into rows 1, 3
// and row_bcast31 into rows 2, 3 leave the total in lane 63, which is read
// back as a uniform value.  (GFX9 DPP controls; no LDS traffic.)
// With every row enabled each lane receives a valid source lane for the
// row-local patterns used here, so the destination's old value is never kept
// and needs no initialisation; masked rows (the row broadcasts) keep 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double v) {
  if constexpr (ROW_MASK == 0xf) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
  } else {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xb1>(v);
  v += dpp_move<0x4e>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  v += dpp_move<0x142, 0xa>(v);
  v += dpp_move<0x143, 0xc>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
// Sum over aligned groups of g lanes (g a power of two), result in every
// lane of the group: DPP quad_perm [1,0,3,2] and [2,3,0,1], then
// row_half_mirror and row_mirror pair the halves of 8- and 16-lane groups;
// wider groups cross rows with shuffles.
__device__ __forceinline__ double group_sum(double v, int g) {
  if (g >= 2) v += dpp_move<0xb1>(v);
  if (g >= 4) v += dpp_move<0x4e>(v);
  if (g >= 8) v += dpp_move<0x141>(v);
  if (g >= 16) v += dpp_move<0x140>(v);
  for (int off = 16; off < g; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Wavefront maximum of non-negative values (uniform result): the row_bcast
// steps of wave_sum with max in place of +; masked-off rows see 0, which
// cannot exceed a non-negative maximum.
__device__ __forceinline__ double wave_max_nonneg(double v) {
  v = fmax(v, dpp_move<0xb1>(v));
  v = fmax(v, dpp_move<0x4e>(v));
  v = fmax(v, dpp_move<0x141>(v));
  v = fmax(v, dpp_move<0x140>(v));
  v = fmax(v, dpp_move<0x142, 0xa>(v));
  v = fmax(v, dpp_move<0x143, 0xc>(v));
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Inclusive scan of int32 values over the wavefront with an associative op
// and its identity: DPP row_shr 1, 2, 4, 8 within each 16-lane row (a lane
// whose source lies before its row's start reads the identity), then
// row_bcast15 into rows 1 and 3 and row_bcast31 into rows 2 and 3 (the other
// rows read the identity).  Lane 63 ends with the reduction of all 64.
template <class Op>
__device__ __forceinline__ int32_t wave_scan_i32(int32_t v, int32_t identity, Op op) {
  v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x111, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x112, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x114, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x118, 0xf, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x142, 0xa, 0xf, false));
  v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x143, 0xc, 0xf, false));
  return v;
}

// Uniform read of lane `src` (src uniform across the wavefront).
__device__ __forceinline__ double read_lane(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
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
