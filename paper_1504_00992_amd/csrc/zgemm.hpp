// Complex FP64 tile engine on CDNA4 matrix cores.
//
// One workgroup computes a BM x BN tile of C = op(A) op(B) (complex128) with
// v_mfma_f64_16x16x4_f64.  A complex product is four real products:
//   Re C += Re A Re B - Im A Im B,   Im C += Re A Im B + Im A Re B,
// so each 16x16x4 complex step issues four MFMAs into two accumulators.
// Operand access goes through small loader functors, so the same engine
// serves every contraction of the bond update (Theta build, gate, sketch,
// power iteration, projection, singular-vector formation); the loaders
// encode layouts, conjugation and diagonal scalings, and say which index is
// contiguous in memory so the global->LDS copy is coalesced.
//
// MFMA operand layout (16x16x4 f64, 64 lanes): lane t supplies A[t%16][t/16]
// and B[t/16][t%16]; accumulator element r of lane t is C[t/16 + 4r][t%16].
#pragma once

#include "zdev.hpp"

namespace tebd {

typedef double v4d __attribute__((ext_vector_type(4)));

template <int BM_, int BN_, int BK_, int WGM_, int WGN_>
struct ZCfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WGM = WGM_, WGN = WGN_;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int FM = WM / 16, FN = WN / 16;
  static constexpr int LDA = BM + 1, LDB = BN + 1;  // +1 element breaks LDS bank aliasing
  static constexpr int NA = BM * BK / NT, NB = BK * BN / NT;
  static constexpr size_t lds_elems = size_t(BK) * LDA + size_t(BK) * LDB;
  static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert((BM * BK) % NT == 0 && (BK * BN) % NT == 0, "tile must split evenly");
  static_assert(BK % 4 == 0, "K step is a multiple of the MFMA depth");
};

// Loader contract:
//   A loader: zt operator()(int r, int k) const;  static constexpr bool contig_k
//   B loader: zt operator()(int k, int c) const;  static constexpr bool contig_n
//   Store:    void operator()(int r, int c, zt v);  (only called in range)
template <class Cfg, class LA, class LB>
__device__ __forceinline__ void zgemm_load(int M, int N, int K, int m0, int n0, int k0,
                                           const LA& la, const LB& lb, zt (&ra)[Cfg::NA],
                                           zt (&rb)[Cfg::NB]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < Cfg::NA; ++s) {
    const int e = tid + s * Cfg::NT;
    int r, k;
    if (LA::contig_k) {
      k = e % Cfg::BK;
      r = e / Cfg::BK;
    } else {
      r = e % Cfg::BM;
      k = e / Cfg::BM;
    }
    const int gr = m0 + r, gk = k0 + k;
    ra[s] = (gr < M && gk < K) ? la(gr, gk) : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int s = 0; s < Cfg::NB; ++s) {
    const int e = tid + s * Cfg::NT;
    int k, c;
    if (LB::contig_n) {
      c = e % Cfg::BN;
      k = e / Cfg::BN;
    } else {
      k = e % Cfg::BK;
      c = e / Cfg::BK;
    }
    const int gk = k0 + k, gc = n0 + c;
    rb[s] = (gk < K && gc < N) ? lb(gk, gc) : make_double2(0.0, 0.0);
  }
}

template <class Cfg, class LA, class LB>
__device__ __forceinline__ void zgemm_stage(zt* As, zt* Bs, const zt (&ra)[Cfg::NA],
                                            const zt (&rb)[Cfg::NB]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < Cfg::NA; ++s) {
    const int e = tid + s * Cfg::NT;
    int r, k;
    if (LA::contig_k) {
      k = e % Cfg::BK;
      r = e / Cfg::BK;
    } else {
      r = e % Cfg::BM;
      k = e / Cfg::BM;
    }
    As[k * Cfg::LDA + r] = ra[s];
  }
#pragma unroll
  for (int s = 0; s < Cfg::NB; ++s) {
    const int e = tid + s * Cfg::NT;
    int k, c;
    if (LB::contig_n) {
      c = e % Cfg::BN;
      k = e / Cfg::BN;
    } else {
      k = e % Cfg::BK;
      c = e / Cfg::BK;
    }
    Bs[k * Cfg::LDB + c] = rb[s];
  }
}

// C tile at (m0, n0) of size up to BM x BN; K loop over the whole depth.
template <class Cfg, class LA, class LB, class ST>
__device__ void zgemm_tile(int M, int N, int K, int m0, int n0, const LA& la, const LB& lb,
                           ST& st, zt* smem) {
  zt* As = smem;
  zt* Bs = smem + Cfg::BK * Cfg::LDA;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave / Cfg::WGN, wc = wave % Cfg::WGN;
  v4d accr[Cfg::FM][Cfg::FN], acci[Cfg::FM][Cfg::FN];
#pragma unroll
  for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::FN; ++j) {
      accr[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      acci[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  zt ra[Cfg::NA], rb[Cfg::NB];
  if (K > 0) zgemm_load<Cfg>(M, N, K, m0, n0, 0, la, lb, ra, rb);
  for (int k0 = 0; k0 < K; k0 += Cfg::BK) {
    zgemm_stage<Cfg, LA, LB>(As, Bs, ra, rb);
    __syncthreads();
    if (k0 + Cfg::BK < K) zgemm_load<Cfg>(M, N, K, m0, n0, k0 + Cfg::BK, la, lb, ra, rb);
#pragma unroll
    for (int kk = 0; kk < Cfg::BK; kk += 4) {
      const int ka = kk + (lane >> 4);
      double ar[Cfg::FM], ai[Cfg::FM], nai[Cfg::FM], br[Cfg::FN], bi[Cfg::FN];
#pragma unroll
      for (int i = 0; i < Cfg::FM; ++i) {
        const zt a = As[ka * Cfg::LDA + wr * Cfg::WM + i * 16 + (lane & 15)];
        ar[i] = a.x;
        ai[i] = a.y;
        nai[i] = -a.y;
      }
#pragma unroll
      for (int j = 0; j < Cfg::FN; ++j) {
        const zt b = Bs[ka * Cfg::LDB + wc * Cfg::WN + j * 16 + (lane & 15)];
        br[j] = b.x;
        bi[j] = b.y;
      }
#pragma unroll
      for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::FN; ++j) {
          accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], accr[i][j], 0, 0, 0);
          acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], acci[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::FN; ++j) {
          accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[i], bi[j], accr[i][j], 0, 0, 0);
          acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], acci[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * Cfg::WM + i * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wc * Cfg::WN + j * 16 + (lane & 15);
        if (row < M && col < N) st(row, col, make_double2(accr[i][j][r], acci[i][j][r]));
      }
}

// 16 x 16 tile of C = op(A) op(B) by the four wavefronts of a 256-thread
// workgroup, each over every fourth k-step of 4 (wavefront w: k in
// [4w, 4w + 4), [4w + 16, 4w + 20), ...), with the operands read by each
// lane straight into its matrix-core registers (lane t: A[t % 16][k + t / 16]
// and B[k + t / 16][t % 16]), four k-steps in flight.  No LDS staging and no
// barrier in the loop; the four partial tiles meet in LDS (red: 2048
// doubles) and are added in wavefront order.  The chain of dependent matrix-
// core steps is a quarter of a single wavefront's over the full depth.
template <class LA, class LB, class ST>
__device__ void zgemm_tile_split16(int M, int N, int K, int m0, int n0, const LA& la,
                                   const LB& lb, ST& st, double* red) {
  constexpr int U = 4;  // k-steps loaded ahead
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = m0 + (lane & 15), c = n0 + (lane & 15), kl = lane >> 4;
  const bool rin = r < M, cin = c < N;
  const zt zero = make_double2(0.0, 0.0);
  v4d accr = {0.0, 0.0, 0.0, 0.0}, acci = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 4 * wave; k0 < K; k0 += 16 * U) {
    zt a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + 16 * u + kl;
      a[u] = (rin && k < K) ? la(r, k) : zero;
      b[u] = (cin && k < K) ? lb(k, c) : zero;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[u].x, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[u].y, acci, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[u].y, b[u].y, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, b[u].x, acci, 0, 0, 0);
    }
  }
  // red[((w * 4 + i) * 2 + part) * 64 + lane]: element i of lane's
  // accumulators, C[lane / 16 + 4 i][lane % 16]
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    red[((wave * 4 + i) * 2 + 0) * 64 + lane] = accr[i];
    red[((wave * 4 + i) * 2 + 1) * 64 + lane] = acci[i];
  }
  __syncthreads();
  {
    const int e = threadIdx.x, row = e >> 4, col = e & 15;
    const int t = (row & 3) * 16 + col, i = row >> 2;
    double vr = 0.0, vi = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      vr += red[((w * 4 + i) * 2 + 0) * 64 + t];
      vi += red[((w * 4 + i) * 2 + 1) * 64 + t];
    }
    if (m0 + row < M && n0 + col < N) st(m0 + row, n0 + col, make_double2(vr, vi));
  }
  __syncthreads();  // red is read before the next tile writes it
}

// Complex FP32 variant for the mixed-precision sketch and power-iteration
// products: the same tiles and loaders (FP64 operands are rounded to FP32
// when staged into LDS), v_mfma_f32_16x16x4_f32 with FP32 accumulation.
// This instruction's 16 x 16 result keeps lane t's four rows contiguous:
// element r of lane t is C[4 (t/16) + r][t % 16].  Results are widened to
// FP64 when stored.
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 to_f32(zt v) { return make_float2(float(v.x), float(v.y)); }
__device__ __forceinline__ float2 to_f32(float2 v) { return v; }

template <class T>
__device__ __forceinline__ T zero_of() {
  T z;
  z.x = 0;
  z.y = 0;
  return z;
}

// Operand registers of the FP32 engine: the loader's element type (complex128
// operands are rounded when staged, complex64 ones pass through).
template <class Cfg, class LA, class LB, class TA, class TB>
__device__ __forceinline__ void cgemm_load(int M, int N, int K, int m0, int n0, int k0,
                                           const LA& la, const LB& lb, TA (&ra)[Cfg::NA],
                                           TB (&rb)[Cfg::NB]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < Cfg::NA; ++s) {
    const int e = tid + s * Cfg::NT;
    int r, k;
    if (LA::contig_k) {
      k = e % Cfg::BK;
      r = e / Cfg::BK;
    } else {
      r = e % Cfg::BM;
      k = e / Cfg::BM;
    }
    const int gr = m0 + r, gk = k0 + k;
    ra[s] = (gr < M && gk < K) ? la(gr, gk) : zero_of<TA>();
  }
#pragma unroll
  for (int s = 0; s < Cfg::NB; ++s) {
    const int e = tid + s * Cfg::NT;
    int k, c;
    if (LB::contig_n) {
      c = e % Cfg::BN;
      k = e / Cfg::BN;
    } else {
      k = e % Cfg::BK;
      c = e / Cfg::BK;
    }
    const int gk = k0 + k, gc = n0 + c;
    rb[s] = (gk < K && gc < N) ? lb(gk, gc) : zero_of<TB>();
  }
}

template <class Cfg, class LA, class LB, class TA, class TB>
__device__ __forceinline__ void cgemm_stage(float2* As, float2* Bs, const TA (&ra)[Cfg::NA],
                                            const TB (&rb)[Cfg::NB]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < Cfg::NA; ++s) {
    const int e = tid + s * Cfg::NT;
    int r, k;
    if (LA::contig_k) {
      k = e % Cfg::BK;
      r = e / Cfg::BK;
    } else {
      r = e % Cfg::BM;
      k = e / Cfg::BM;
    }
    As[k * Cfg::LDA + r] = to_f32(ra[s]);
  }
#pragma unroll
  for (int s = 0; s < Cfg::NB; ++s) {
    const int e = tid + s * Cfg::NT;
    int k, c;
    if (LB::contig_n) {
      c = e % Cfg::BN;
      k = e / Cfg::BN;
    } else {
      k = e % Cfg::BK;
      c = e / Cfg::BK;
    }
    Bs[k * Cfg::LDB + c] = to_f32(rb[s]);
  }
}

template <class Cfg, class LA, class LB, class ST>
__device__ void cgemm_tile(int M, int N, int K, int m0, int n0, const LA& la, const LB& lb,
                           ST& st, float2* smem) {
  float2* As = smem;
  float2* Bs = smem + Cfg::BK * Cfg::LDA;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave / Cfg::WGN, wc = wave % Cfg::WGN;
  v4f accr[Cfg::FM][Cfg::FN], acci[Cfg::FM][Cfg::FN];
#pragma unroll
  for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::FN; ++j) {
      accr[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
      acci[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  using TA = decltype(la(0, 0));
  using TB = decltype(lb(0, 0));
  TA ra[Cfg::NA];
  TB rb[Cfg::NB];
  if (K > 0) cgemm_load<Cfg>(M, N, K, m0, n0, 0, la, lb, ra, rb);
  for (int k0 = 0; k0 < K; k0 += Cfg::BK) {
    cgemm_stage<Cfg, LA, LB>(As, Bs, ra, rb);
    __syncthreads();
    if (k0 + Cfg::BK < K) cgemm_load<Cfg>(M, N, K, m0, n0, k0 + Cfg::BK, la, lb, ra, rb);
#pragma unroll
    for (int kk = 0; kk < Cfg::BK; kk += 4) {
      const int ka = kk + (lane >> 4);
      float ar[Cfg::FM], ai[Cfg::FM], nai[Cfg::FM], br[Cfg::FN], bi[Cfg::FN];
#pragma unroll
      for (int i = 0; i < Cfg::FM; ++i) {
        const float2 a = As[ka * Cfg::LDA + wr * Cfg::WM + i * 16 + (lane & 15)];
        ar[i] = a.x;
        ai[i] = a.y;
        nai[i] = -a.y;
      }
#pragma unroll
      for (int j = 0; j < Cfg::FN; ++j) {
        const float2 b = Bs[ka * Cfg::LDB + wc * Cfg::WN + j * 16 + (lane & 15)];
        br[j] = b.x;
        bi[j] = b.y;
      }
#pragma unroll
      for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::FN; ++j) {
          accr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], br[j], accr[i][j], 0, 0, 0);
          acci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bi[j], acci[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::FN; ++j) {
          accr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai[i], bi[j], accr[i][j], 0, 0, 0);
          acci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], br[j], acci[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < Cfg::FM; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * Cfg::WM + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wc * Cfg::WN + j * 16 + (lane & 15);
        if (row < M && col < N)
          st(row, col, make_double2(double(accr[i][j][r]), double(acci[i][j][r])));
      }
}

}  // namespace tebd
