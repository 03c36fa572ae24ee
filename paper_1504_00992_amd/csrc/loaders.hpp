// Operand loaders and result stores shared by the contraction kernels.
//
// A loader maps a logical operand element to memory: A loaders take (r, k),
// B loaders (k, c), and say which index is contiguous so that the
// global->LDS copy of the tile engine is coalesced.  Stores receive (r, c)
// of the result tile, only in range.  Diagonal lambda scalings, conjugation
// and the index permutations of the bond update live here.
#pragma once

#include "zgemm.hpp"

namespace tebd {

__device__ __forceinline__ double inv_floor(const double* lam, int idx, double floor_) {
  if (lam == nullptr) return 1.0;
  const double v = lam[idx];
  return v > floor_ ? 1.0 / v : 0.0;
}

struct LdThetaA {  // (r = i*chi_l + a, k = g)
  const zt* gk;
  const double* lam_l;
  const double* lam_m;
  int chi_l, cap;
  static constexpr bool contig_k = true;
  __device__ zt operator()(int r, int k) const {
    const int i = r / chi_l, a = r - i * chi_l;
    double s = lam_m[k];
    if (lam_l) s *= lam_l[a];
    return zscale(gk[(size_t(i) * cap + a) * cap + k], s);
  }
};

struct LdThetaB {  // (k = g, c = j*chi_r + b)
  const zt* gk1;
  const double* lam_r;
  int chi_r, cap;
  static constexpr bool contig_n = true;
  __device__ zt operator()(int k, int c) const {
    const int j = c / chi_r, b = c - j * chi_r;
    const zt v = gk1[(size_t(j) * cap + k) * cap + b];
    return lam_r ? zscale(v, lam_r[b]) : v;
  }
};

struct StTheta {
  zt* T;
  int chi_l, chi_r, dr;
  __device__ void operator()(int r, int c, zt v) {
    const int i = r / chi_l, a = r - i * chi_l;
    const int j = c / chi_r, b = c - j * chi_r;
    T[(size_t(i) * dr + j) * (size_t(chi_l) * chi_r) + size_t(a) * chi_r + b] = v;
  }
};

// Theta of one member into its gate group's block: row (i j), column
// col0 + (a chi_r + b), leading dimension ld (the group's columns).
struct StThetaGroup {
  zt* T;
  int64_t ld;
  int col0, chi_l, chi_r, dr;
  __device__ void operator()(int r, int c, zt v) {
    const int i = r / chi_l, a = r - i * chi_l;
    const int j = c / chi_r, b = c - j * chi_r;
    T[(size_t(i) * dr + j) * ld + col0 + size_t(a) * chi_r + b] = v;
  }
};

struct LdRowB {  // B[k][c] = p[k*ld + c]
  const zt* p;
  int64_t ld;
  static constexpr bool contig_n = true;
  __device__ zt operator()(int k, int c) const { return p[size_t(k) * ld + c]; }
};

struct LdRowA {  // A[r][k] = p[r*ld + k]
  const zt* p;
  int64_t ld;
  static constexpr bool contig_k = true;
  __device__ zt operator()(int r, int k) const { return p[size_t(r) * ld + k]; }
};

struct LdAdjA {  // (r, k) -> conj(p[k*ld + r]): the adjoint of a row-major matrix
  const zt* p;
  int64_t ld;
  static constexpr bool contig_k = false;
  __device__ zt operator()(int r, int k) const { return zconj(p[size_t(k) * ld + r]); }
};

struct LdColB {  // B[k][c] = p[c*ld + k] (column-major)
  const zt* p;
  int64_t ld;
  static constexpr bool contig_n = false;
  __device__ zt operator()(int k, int c) const { return p[size_t(c) * ld + k]; }
};

struct LdColA {  // A[r][k] = p[k*ld + r] (column-major)
  const zt* p;
  int64_t ld;
  static constexpr bool contig_k = false;
  __device__ zt operator()(int r, int k) const { return p[size_t(k) * ld + r]; }
};

struct LdAdjColA {  // (r, k) -> conj(p[r*ld + k]): the adjoint of a column-major matrix
  const zt* p;
  int64_t ld;
  static constexpr bool contig_k = true;
  __device__ zt operator()(int r, int k) const { return zconj(p[size_t(r) * ld + k]); }
};

// complex64 copies of A for the FP32 products
struct LdRowAf {  // A[r][k] = p[r*ld + k]
  const float2* p;
  int64_t ld;
  static constexpr bool contig_k = true;
  __device__ float2 operator()(int r, int k) const { return p[size_t(r) * ld + k]; }
};

struct LdAdjAf {  // (r, k) -> conj(p[k*ld + r])
  const float2* p;
  int64_t ld;
  static constexpr bool contig_k = false;
  __device__ float2 operator()(int r, int k) const {
    const float2 v = p[size_t(k) * ld + r];
    return make_float2(v.x, -v.y);
  }
};

struct StCol {  // C[r][c] -> p[c*ld + r]
  zt* p;
  int64_t ld;
  __device__ void operator()(int r, int c, zt v) { p[size_t(c) * ld + r] = v; }
};

struct StRow {  // C[r][c] -> p[r*ld + c]
  zt* p;
  int64_t ld;
  __device__ void operator()(int r, int c, zt v) { p[size_t(r) * ld + c] = v; }
};

}  // namespace tebd
