// Dense complex contractions of the bond update on FP64 matrix cores.
//
// * Theta build, Eq. (deftheta): one GEMM per bond,
//     Theta[(i,a),(j,c)] = sum_g (lam_l[a] G_k[i][a][g] lam_m[g]) (G_k+1[j][g][c] lam_r[c]),
//   with the diagonal lambdas folded into the operand loads, written in the
//   layout T[(i j)][(a c)] that the gate product reads.
// * Gate update, Eq. (defupdatetheta): A = G T as (dl dr) x (dl dr) times
//   (dl dr) x (chi_l chi_r), scattered into the blocked matrix of Sec. II.B,
//   A[(i,a),(j,c)], with partial sums of |A|^2 for ||A||_F^2.  The chains
//   that share a bond's gate run as one product over all their columns
//   (their T side by side), so each output tile reads its gate rows once
//   for many chains.
// * Sketch and power iteration, Alg. 1: Y = A Omega, Yt = A^H Q, Y = A Q~.
// * Singular vectors, Sec. IV steps i-iii: U = Q X and V^H = (Q_B W)^H for the
//   kept chi' columns, with the lambda^-1 reabsorption of the TEBD update
//   folded into the store.
//
// Scheduling: problem sizes live on the device, so every contraction kind
// runs as one persistent launch over a global queue of output tiles (32 x 32
// for Theta, the sketches and U, V^H; 64 x 16 or 64 x 64 for the gate
// groups; 64 x 64 for the others; prefix sums over problems
// built by k_schedule).  Workgroup i takes the
// virtual index (i mod 8) * G/8 + i / 8, so the consecutive tiles of one
// problem, which share operand rows, land on the same XCD and its L2.
#include "kinds.hpp"
#include "loaders.hpp"

namespace tebd {

using Cfg64 = ZCfg<64, 64, 16, 2, 2>;
// Sketch and power-iteration products: 32 x 32 tiles (kSketchTileM/N).
using CfgSk = ZCfg<kSketchTileM, kSketchTileN, 16, 2, 2>;
// Theta's contraction depth is the old bond dimension chi_m, often 1 to a
// few dozen: K slabs of 8 instead of 16 (the least that 32 x 32 tiles of
// 256 threads stage evenly), and 32 x 32 tiles like the sketches.
using CfgTheta = ZCfg<32, 32, 8, 2, 2>;

hipError_t launch_schedule(Prob* probs, const Common& c, hipStream_t s) {
  if (c.bounds_dev)
    TEBD_LAUNCH("k_schedule<tebd::Prob, true>", (k_schedule<Prob, true>), dim3(1), dim3(kScheduleThreads), 0, s, probs,
                       c.nprob, c.tebd, c.offs, c.bounds_dev);
  else
    TEBD_LAUNCH("k_schedule<tebd::Prob, false>", (k_schedule<Prob, false>), dim3(1), dim3(kScheduleThreads), 0, s, probs,
                       c.nprob, c.tebd, c.offs, static_cast<int32_t*>(nullptr));
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Gaussian test matrix Omega (Alg. 1, first step), generated tile by tile
// over the n x l tile queue.  Philox4x32-10 (Salmon et al., SC'11): ten
// rounds on the counter (r, c, problem id, stream id) with key
// (seed low, seed high), the key advanced by the Weyl constants before every
// round but the first; the first two output words give u = (x + 1/2) 2^-32
// and z = sqrt(-2 ln u1) exp(2 pi i u2) / sqrt(2).
__device__ __forceinline__ void philox10(uint32_t x[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t hi0 = __umulhi(M0, x[0]), lo0 = M0 * x[0];
    const uint32_t hi1 = __umulhi(M1, x[2]), lo1 = M1 * x[2];
    const uint32_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
  }
}

// Entry (r, c) of problem pid's Gaussian stream.
__device__ __forceinline__ zt gauss_entry(int r, int c, int pid, uint32_t sid, uint64_t seed) {
  uint32_t x[4] = {uint32_t(r), uint32_t(c), uint32_t(pid), sid};
  philox10(x, uint32_t(seed & 0xffffffffu), uint32_t(seed >> 32));
  const double u1 = (double(x[0]) + 0.5) * 0x1p-32;
  const double u2 = (double(x[1]) + 0.5) * 0x1p-32;
  const double rad = sqrt(-2.0 * log(u1)) * 0.70710678118654752440;
  double sn, cs;
  sincos(2.0 * M_PI * u2, &sn, &cs);
  return make_double2(rad * cs, rad * sn);
}

__device__ __forceinline__ void omega_tile(Prob& P, int M, int N, int m0, int n0, uint64_t seed,
                                           uint32_t sid) {
  if (P.om_ext) return;
  zt* om = const_cast<zt*>(P.om);
  constexpr int TM = kSketchTileM, TN = kSketchTileN;  // the n x l queue's tiles
  for (int e = threadIdx.x; e < TM * TN; e += 256) {
    const int r = m0 + e / TN, c = n0 + e % TN;
    if (r >= M || c >= N) continue;
    om[size_t(r) * P.ldom + c] = gauss_entry(r, c, P.pid, sid, seed);
  }
}

__global__ __launch_bounds__(256) void k_omega(Prob* probs, const int32_t* offs, int nprob,
                                               int tebd, uint64_t seed, uint32_t sid) {
  for_each_tile<TK_SKN>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
    omega_tile(P, M, N, m0, n0, seed, sid);
  });
}

// --------------------------------------------------------------------------
// Accuracy Check probes (Sec. IV, Alg. 2): B = A Omega_r with Omega_r the
// next r columns (from ac_col) of the problem's Gaussian stream, generated
// while the operand tile is staged; B lands in the columns of Y after the
// current basis (Y has room for r more).
struct LdProbeB {  // (k, c) -> Gaussian entry (k, col0 + c)
  int col0, pid;
  uint32_t sid;
  uint64_t seed;
  static constexpr bool contig_n = true;
  __device__ zt operator()(int k, int c) const { return gauss_entry(k, col0 + c, pid, sid, seed); }
};

__global__ __launch_bounds__(256) void k_acc_probe(Prob* probs, const int32_t* offs, int nprob,
                                                   int tebd, uint64_t seed, uint32_t sid) {
  __shared__ zt smem[CfgSk::lds_elems];
  for_each_tile<TK_ACB>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
    LdRowA la{P.A, P.lda};
    LdProbeB lb{P.ac_col, P.pid, sid, seed};
    StCol st{P.Y + size_t(P.l) * P.m, P.m};
    zgemm_tile<CfgSk>(M, N, P.n, m0, n0, la, lb, st, smem);
  });
}

hipError_t launch_acc_probe(Prob* probs, const Common& c, hipStream_t s) {
  TEBD_LAUNCH("k_acc_probe", k_acc_probe, dim3(grid_for(c, TK_ACB)), dim3(256), 0, s, probs,
              c.offs, c.nprob, c.tebd, c.seed, c.stream_id);
  return hipGetLastError();
}

hipError_t launch_omega(Prob* probs, const Common& c, hipStream_t s) {
  TEBD_LAUNCH("k_omega", k_omega, dim3(grid_for(c, TK_SKN)), dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd,
                     c.seed, c.stream_id);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Theta build

__global__ __launch_bounds__(256) void k_theta(Prob* probs, const int32_t* offs, int nprob) {
  __shared__ zt smem[CfgTheta::lds_elems];
  for_each_tile<TK_THETA>(probs, offs, nprob, 1, [&](Prob& P, int M, int N, int m0, int n0, int) {
    LdThetaA la{P.gk, P.lam_l, P.lam_mid, P.chi_l, P.chi_cap};
    LdThetaB lb{P.gk1, P.lam_r, P.chi_r, P.chi_cap};
    StThetaGroup st{P.T, P.gtot, P.gcol0, P.chi_l, P.chi_r, P.dr};
    zgemm_tile<CfgTheta>(M, N, P.chi_m, m0, n0, la, lb, st, smem);
  });
}

// --------------------------------------------------------------------------
// Gate update
struct LdGate {
  const zt* g;
  int ld;
  static constexpr bool contig_k = true;
  __device__ zt operator()(int r, int k) const { return g[size_t(r) * ld + k]; }
};

// Where the gate product's column c of a group lands: the member that owns
// it and the address of its entry (i, j) = (0, 0) in the member's A, with
// the strides of i and j (rows (i j) of the product go to A[(i, a)][(j, b)]).
struct GateCol {
  zt* base;
  float2* basef;  // the same entry of the member's complex64 copy of A (FP32 products), or null
  int32_t si, sj;
};

template <int BN>
struct StGateGroup {
  const GateCol* col;  // the tile's BN columns
  double* f2;          // |A|^2 of the tile's entries, BM x BN row-major
  int m0, n0, dr;
  __device__ void operator()(int r, int c, zt v) {
    const GateCol& g = col[c - n0];
    const int i = r / dr, j = r - i * dr;
    const size_t o = size_t(i) * g.si + size_t(j) * g.sj;
    g.base[o] = v;
    if (g.basef) g.basef[o] = make_float2(float(v.x), float(v.y));
    f2[(r - m0) * BN + (c - n0)] = zabs2(v);
  }
};

// One 16 x 16 tile of the group product, its depth d_l d_r split
// between the workgroup's four wavefronts (zgemm_tile_split16).
__device__ __forceinline__ void gate_group_tile(Prob* probs, int lead, int M, int N, int m0,
                                                      int n0, double* f2, double* red,
                                                      GateCol* cols, double* csum) {
  constexpr int BM = kGateTileM, BN = kGateTileN;
  const Prob& L = probs[lead];
  const int tid = threadIdx.x, gn = L.gn, gs = L.gstride;
  if (tid < BN) {
    const int c = n0 + tid;
    GateCol g{nullptr, nullptr, 0, 0};
    if (c < N) {
      int q = 0;
      for (int k = 1; k < gn; ++k)
        if (probs[lead + k * gs].gcol0 <= c) q = k;
      const Prob& Q = probs[lead + q * gs];
      const int lc = c - Q.gcol0, a = lc / Q.chi_r, b = lc - a * Q.chi_r;
      g.base = Q.A + size_t(a) * Q.n + b;
      g.basef = Q.Af ? Q.Af + size_t(a) * Q.n + b : nullptr;
      g.si = Q.chi_l * Q.n;
      g.sj = Q.chi_r;
    }
    cols[tid] = g;
  }
  __syncthreads();
  LdGate la{L.gate, L.gate_ld};
  LdRowB lb{L.T, L.gtot};
  StGateGroup<BN> st{cols, f2, m0, n0, L.dr};
  const int K = L.dl * L.dr;
  const int ncol = N - n0 < BN ? N - n0 : BN;
  zgemm_tile_split16(M, N, K, m0, n0, la, lb, st, red);  // ends with a barrier: f2 is written
  const int rows = M - m0 < BM ? M - m0 : BM;
  if (tid < ncol) {
    double sum = 0.0;
    for (int r = 0; r < rows; ++r) sum += f2[r * BN + tid];
    csum[tid] = sum;
  }
  __syncthreads();
  if (tid < gn) {
    Prob& Q = probs[lead + tid * gs];
    const int q0 = Q.gcol0, q1 = tid + 1 < gn ? probs[lead + (tid + 1) * gs].gcol0 : L.gtot;
    const int lo = q0 > n0 ? q0 : n0, hi = q1 < n0 + ncol ? q1 : n0 + ncol;
    if (lo < hi) {
      double sum = 0.0;
      for (int c = lo; c < hi; ++c) sum += csum[c - n0];
      const int first = q0 / BN, ntouch = (q1 - 1) / BN - first + 1;
      Q.part[(m0 / BM) * ntouch + (n0 / BN - first)] = sum;
    }
  }
  __syncthreads();  // the column table and the LDS are free for the next tile
}

__global__ __launch_bounds__(256) void k_gate(Prob* probs, const int32_t* offs, int nprob) {
  __shared__ double f2[kGateTileM * kGateTileN];
  __shared__ double red[2048];
  __shared__ GateCol cols[kGateTileN];
  __shared__ double csum[kGateTileN];
  for_each_tile<TK_GATE>(probs, offs, nprob, 1, [&](Prob& P, int M, int N, int m0, int n0, int) {
    gate_group_tile(probs, int(&P - probs), M, N, m0, n0, f2, red, cols, csum);
  });
}

hipError_t launch_theta_gate(Prob* probs, const Common& c, hipStream_t s) {
  TEBD_LAUNCH("k_theta", k_theta, dim3(grid_for(c, TK_THETA)), dim3(256), 0, s, probs, c.offs, c.nprob);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  TEBD_LAUNCH("k_gate", k_gate, dim3(grid_for(c, TK_GATE)), dim3(256), 0, s, probs,
              c.offs, c.nprob);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Sketch / power iteration / projection products

template <int WHICH>
__global__ __launch_bounds__(256) void k_sketch(Prob* probs, const int32_t* offs, int nprob,
                                                int tebd) {
  __shared__ zt smem[CfgSk::lds_elems];
  if (WHICH == SK_Y_FROM_OMEGA) {
    for_each_tile<TK_SKM>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdRowA la{P.A, P.lda};
      LdRowB lb{P.om, P.ldom};
      StCol st{P.Y, P.m};
      zgemm_tile<CfgSk>(M, N, P.n, m0, n0, la, lb, st, smem);
    });
  } else if (WHICH == SK_YT_FROM_Y) {
    for_each_tile<TK_SKN>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdAdjA la{P.A, P.lda};
      LdColB lb{P.Y, P.m};
      StCol st{P.Yt, P.n};
      zgemm_tile<CfgSk>(M, N, P.m, m0, n0, la, lb, st, smem);
    });
  } else {
    for_each_tile<TK_SKM>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdRowA la{P.A, P.lda};
      LdColB lb{P.Yt, P.n};
      StCol st{P.Y, P.m};
      zgemm_tile<CfgSk>(M, N, P.n, m0, n0, la, lb, st, smem);
    });
  }
}

// Mixed precision (sketch and power-iteration products only): complex FP32
// MFMA with FP32 accumulation; Y and Yt stay FP64 for the QR that follows.
template <int WHICH>
__global__ __launch_bounds__(256) void k_sketch_f32(Prob* probs, const int32_t* offs, int nprob,
                                                    int tebd) {
  __shared__ float2 smem[CfgSk::lds_elems];
  // A from its complex64 copy when there is one (half the bytes), else
  // rounded from complex128 when staged
  if (WHICH == SK_Y_FROM_OMEGA) {
    for_each_tile<TK_SKM>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdRowB lb{P.om, P.ldom};
      StCol st{P.Y, P.m};
      if (P.Af)
        cgemm_tile<CfgSk>(M, N, P.n, m0, n0, LdRowAf{P.Af, P.n}, lb, st, smem);
      else
        cgemm_tile<CfgSk>(M, N, P.n, m0, n0, LdRowA{P.A, P.lda}, lb, st, smem);
    });
  } else if (WHICH == SK_YT_FROM_Y) {
    for_each_tile<TK_SKN>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdColB lb{P.Y, P.m};
      StCol st{P.Yt, P.n};
      if (P.Af)
        cgemm_tile<CfgSk>(M, N, P.m, m0, n0, LdAdjAf{P.Af, P.n}, lb, st, smem);
      else
        cgemm_tile<CfgSk>(M, N, P.m, m0, n0, LdAdjA{P.A, P.lda}, lb, st, smem);
    });
  } else {
    for_each_tile<TK_SKM>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdColB lb{P.Yt, P.n};
      StCol st{P.Y, P.m};
      if (P.Af)
        cgemm_tile<CfgSk>(M, N, P.n, m0, n0, LdRowAf{P.Af, P.n}, lb, st, smem);
      else
        cgemm_tile<CfgSk>(M, N, P.n, m0, n0, LdRowA{P.A, P.lda}, lb, st, smem);
    });
  }
}

hipError_t launch_sketch_f32(Prob* probs, const Common& c, int which, hipStream_t s) {
  const dim3 g(grid_for(c, which == SK_YT_FROM_Y ? TK_SKN : TK_SKM));
  if (which == SK_Y_FROM_OMEGA)
    TEBD_LAUNCH("k_sketch_f32<0>", k_sketch_f32<SK_Y_FROM_OMEGA>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
  else if (which == SK_YT_FROM_Y)
    TEBD_LAUNCH("k_sketch_f32<1>", k_sketch_f32<SK_YT_FROM_Y>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
  else
    TEBD_LAUNCH("k_sketch_f32<2>", k_sketch_f32<SK_Y_FROM_YT>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Gram-based QR (CholeskyQR2) of the large problems, the tile-queue parts:
// G = Y^H Y into C (l x l), and Q = Y R^-1 into Qc with R^-1 (upper
// triangular, from k_chol) in J.  WHICH selects the m x l sketch Y (bit 1 of
// P.chol) or the n x l sketch Yt (bit 2); in the second pass only the
// problems whose first pass succeeded take part.
template <int WHICH>
__global__ __launch_bounds__(256) void k_gram(Prob* probs, const int32_t* offs, int nprob, int tebd,
                                              int pass) {
  __shared__ zt smem[CfgSk::lds_elems];
  for_each_tile<TK_GRAM>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
    if (!(P.chol & (WHICH ? 2 : 1)) || (pass && !P.chol_ok)) return;
    const int rows = WHICH ? P.n : P.m;
    const zt* Yc = WHICH ? P.Yt : P.Y;
    LdAdjColA la{Yc, rows};
    LdColB lb{Yc, rows};
    StCol st{P.C, P.l};
    zgemm_tile<CfgSk>(M, N, rows, m0, n0, la, lb, st, smem);
  });
}

template <int WHICH>
__global__ __launch_bounds__(256) void k_qapply(Prob* probs, const int32_t* offs, int nprob,
                                                int tebd) {
  __shared__ zt smem[CfgSk::lds_elems];
  for_each_tile<WHICH ? TK_QAPN : TK_QAPM>(probs, offs, nprob, tebd,
                                           [&](Prob& P, int M, int N, int m0, int n0, int) {
    if (!P.chol_ok) return;
    const int rows = WHICH ? P.n : P.m;
    LdColA la{WHICH ? P.Yt : P.Y, rows};
    LdColB lb{P.J, P.l};
    StCol st{P.Qc, rows};
    zgemm_tile<CfgSk>(M, N, P.l, m0, n0, la, lb, st, smem);
  });
}

hipError_t launch_gram(Prob* probs, const Common& c, int which, int pass, hipStream_t s) {
  const dim3 g(grid_for(c, TK_GRAM));
  if (which)
    TEBD_LAUNCH("k_gram<1>", k_gram<1>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd, pass);
  else
    TEBD_LAUNCH("k_gram<0>", k_gram<0>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd, pass);
  return hipGetLastError();
}

hipError_t launch_qapply(Prob* probs, const Common& c, int which, hipStream_t s) {
  if (which)
    TEBD_LAUNCH("k_qapply<1>", k_qapply<1>, dim3(grid_for(c, TK_QAPN)), dim3(256), 0, s, probs,
                c.offs, c.nprob, c.tebd);
  else
    TEBD_LAUNCH("k_qapply<0>", k_qapply<0>, dim3(grid_for(c, TK_QAPM)), dim3(256), 0, s, probs,
                c.offs, c.nprob, c.tebd);
  return hipGetLastError();
}

// The FP64 sketch products on 64 x 64 output tiles (fewer operand reloads
// for large problems; chosen per launch by the autotune cache).
template <int WHICH, class Cfg, int KM, int KN>
__device__ __forceinline__ void sketch_tiles(Prob* probs, const int32_t* offs, int nprob, int tebd,
                                             zt* smem) {
  if (WHICH == SK_Y_FROM_OMEGA) {
    for_each_tile<KM>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdRowA la{P.A, P.lda};
      LdRowB lb{P.om, P.ldom};
      StCol st{P.Y, P.m};
      zgemm_tile<Cfg>(M, N, P.n, m0, n0, la, lb, st, smem);
    });
  } else if (WHICH == SK_YT_FROM_Y) {
    for_each_tile<KN>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdAdjA la{P.A, P.lda};
      LdColB lb{P.Y, P.m};
      StCol st{P.Yt, P.n};
      zgemm_tile<Cfg>(M, N, P.m, m0, n0, la, lb, st, smem);
    });
  } else {
    for_each_tile<KM>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdRowA la{P.A, P.lda};
      LdColB lb{P.Yt, P.n};
      StCol st{P.Y, P.m};
      zgemm_tile<Cfg>(M, N, P.n, m0, n0, la, lb, st, smem);
    });
  }
}

template <int WHICH>
__global__ __launch_bounds__(256) void k_sketch_wide(Prob* probs, const int32_t* offs, int nprob,
                                                     int tebd) {
  __shared__ zt smem[Cfg64::lds_elems];
  sketch_tiles<WHICH, Cfg64, TK_SKM_W, TK_SKN_W>(probs, offs, nprob, tebd, smem);
}

// The FP64 sketch products on 16 x 16 tiles, each split over the depth
// between the four wavefronts (zgemm_tile_split16; chosen per launch by the
// autotune cache).
template <int WHICH>
__global__ __launch_bounds__(256) void k_sketch_split(Prob* probs, const int32_t* offs, int nprob,
                                                      int tebd) {
  __shared__ double red[2048];
  if (WHICH == SK_Y_FROM_OMEGA) {
    for_each_tile<TK_SKM_S>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdRowA la{P.A, P.lda};
      LdRowB lb{P.om, P.ldom};
      StCol st{P.Y, P.m};
      zgemm_tile_split16(M, N, P.n, m0, n0, la, lb, st, red);
    });
  } else if (WHICH == SK_YT_FROM_Y) {
    for_each_tile<TK_SKN_S>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdAdjA la{P.A, P.lda};
      LdColB lb{P.Y, P.m};
      StCol st{P.Yt, P.n};
      zgemm_tile_split16(M, N, P.m, m0, n0, la, lb, st, red);
    });
  } else {
    for_each_tile<TK_SKM_S>(probs, offs, nprob, tebd, [&](Prob& P, int M, int N, int m0, int n0, int) {
      LdRowA la{P.A, P.lda};
      LdColB lb{P.Yt, P.n};
      StCol st{P.Y, P.m};
      zgemm_tile_split16(M, N, P.n, m0, n0, la, lb, st, red);
    });
  }
}

// Autotune cache: variant per (precision, rows bucket, width bucket): 0 the
// 32 x 32 tiles, 1 the 64 x 64 tiles, 2 the split-depth 16 x 16 tiles; -1
// (unset) means the 32 x 32 tiles.  Written by tebd_tune_set between calls.
namespace {
constexpr int kTuneRows[6] = {128, 256, 512, 1024, 2048, 8192};
constexpr int kTuneWidth[5] = {32, 64, 80, 128, 256};
int8_t g_tune[3][6][5] = {};
bool g_tune_init = false;

int tune_bucket(const int* bounds, int nb, int v) {
  for (int i = 0; i < nb; ++i)
    if (v <= bounds[i]) return i;
  return -1;
}
}  // namespace

int sketch_variant(int table, int max_rows, int width) {
  if (table == 1 || !g_tune_init) return 0;
  const int br = tune_bucket(kTuneRows, 6, max_rows), bw = tune_bucket(kTuneWidth, 5, width);
  if (br < 0 || bw < 0) return 0;
  const int v = g_tune[table][br][bw];
  return v < 0 ? 0 : v;
}

hipError_t launch_sketch(Prob* probs, const Common& c, int which, hipStream_t s) {
  // a TEBD sweep reads its own table under the MPS capacities, so that every
  // rank mode (host bounds or none, graph capture) takes the same variant
  const bool sweep = c.tune_rows > 0;
  const int rows = sweep ? c.tune_rows : (c.mmax > c.nmax ? c.mmax : c.nmax);
  const int variant = sketch_variant(sweep ? 2 : 0, rows, sweep ? c.tune_width : c.lmax);
  if (variant == 1) {
    const dim3 g(grid_for(c, which == SK_YT_FROM_Y ? TK_SKN_W : TK_SKM_W));
    if (which == SK_Y_FROM_OMEGA)
      TEBD_LAUNCH("k_sketch_wide<0>", k_sketch_wide<SK_Y_FROM_OMEGA>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
    else if (which == SK_YT_FROM_Y)
      TEBD_LAUNCH("k_sketch_wide<1>", k_sketch_wide<SK_YT_FROM_Y>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
    else
      TEBD_LAUNCH("k_sketch_wide<2>", k_sketch_wide<SK_Y_FROM_YT>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
    return hipGetLastError();
  }
  if (variant == 2) {
    const dim3 g(grid_for(c, which == SK_YT_FROM_Y ? TK_SKN_S : TK_SKM_S));
    if (which == SK_Y_FROM_OMEGA)
      TEBD_LAUNCH("k_sketch_split<0>", k_sketch_split<SK_Y_FROM_OMEGA>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
    else if (which == SK_YT_FROM_Y)
      TEBD_LAUNCH("k_sketch_split<1>", k_sketch_split<SK_YT_FROM_Y>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
    else
      TEBD_LAUNCH("k_sketch_split<2>", k_sketch_split<SK_Y_FROM_YT>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
    return hipGetLastError();
  }
  const dim3 g(grid_for(c, which == SK_YT_FROM_Y ? TK_SKN : TK_SKM));
  if (which == SK_Y_FROM_OMEGA)
    TEBD_LAUNCH("k_sketch<0>", k_sketch<SK_Y_FROM_OMEGA>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
  else if (which == SK_YT_FROM_Y)
    TEBD_LAUNCH("k_sketch<1>", k_sketch<SK_YT_FROM_Y>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
  else
    TEBD_LAUNCH("k_sketch<2>", k_sketch<SK_Y_FROM_YT>, g, dim3(256), 0, s, probs, c.offs, c.nprob, c.tebd);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Kept singular vectors and lambda^-1 reabsorption
// (r, k) -> Q[k*ld + r]: the range finder's Q, whose columns pair with those
// of B^H = A^H Q; the QR of B^H keeps column order (its recorded permutation
// is the identity), so no permutation is applied here.
struct LdQP {
  const zt* p;
  int64_t ld;
  static constexpr bool contig_k = false;
  __device__ zt operator()(int r, int k) const { return p[size_t(k) * ld + r]; }
};
struct LdSmallColB {  // B[k][c] = X[c*l + k], zero for c >= l
  const zt* p;
  int l;
  static constexpr bool contig_n = false;
  __device__ zt operator()(int k, int c) const {
    return c < l ? p[size_t(c) * l + k] : make_double2(0.0, 0.0);
  }
};
struct LdSmallAdjA {  // A[g][k] = conj(W[g*l + k]), zero for g >= l
  const zt* p;
  int l;
  static constexpr bool contig_k = true;
  __device__ zt operator()(int g, int k) const {
    return g < l ? zconj(p[size_t(g) * l + k]) : make_double2(0.0, 0.0);
  }
};
struct LdQbAdjB {  // B[k][c] = conj(Q_B[c][k]) = conj(p[k*ld + c])
  const zt* p;
  int64_t ld;
  static constexpr bool contig_n = true;
  __device__ zt operator()(int k, int c) const { return zconj(p[size_t(k) * ld + c]); }
};

struct StU {  // standalone: U[r][g], zero beyond chi'
  zt* U;
  int64_t ldu;
  int chi;
  __device__ void operator()(int r, int g, zt v) {
    U[size_t(r) * ldu + g] = g < chi ? v : make_double2(0.0, 0.0);
  }
};
struct StVH {
  zt* VH;
  int64_t ldvh;
  int chi;
  __device__ void operator()(int g, int c, zt v) {
    VH[size_t(g) * ldvh + c] = g < chi ? v : make_double2(0.0, 0.0);
  }
};
struct StGammaL {  // Gamma'_k[i][a][g] = U[(i,a), g] / lam_l[a]
  zt* gk;
  const double* lam_l;
  double floor_;
  int chi_l, cap, chi;
  __device__ void operator()(int r, int g, zt v) {
    const int i = r / chi_l, a = r - i * chi_l;
    gk[(size_t(i) * cap + a) * cap + g] =
        g < chi ? zscale(v, inv_floor(lam_l, a, floor_)) : make_double2(0.0, 0.0);
  }
};
struct StGammaR {  // Gamma'_k+1[j][g][b] = V^H[g, (j,b)] / lam_r[b]
  zt* gk1;
  const double* lam_r;
  double floor_;
  int chi_r, cap, chi;
  __device__ void operator()(int g, int c, zt v) {
    const int j = c / chi_r, b = c - j * chi_r;
    gk1[(size_t(j) * cap + g) * cap + b] =
        g < chi ? zscale(v, inv_floor(lam_r, b, floor_)) : make_double2(0.0, 0.0);
  }
};

// Tiles entirely beyond chi' only write zeros (no contraction).  In TEBD the
// column range is the padded MPS capacity, so stale entries are cleared.
// U and V^H are independent: one launch walks the tiles of both.
template <int TEBD_>
__device__ __forceinline__ void form_u_tile(Prob& P, int M, int N, int m0, int n0, zt* smem) {
  if (P.retry) return;  // adaptive rank: stage 2 will write this problem
  const int chi = P.chi_new;
  const int Keff = (n0 >= chi) ? 0 : P.l;
  LdQP la{P.Y, P.m};
  LdSmallColB lb{P.X, P.l};
  if (TEBD_) {
    StGammaL st{P.gk, P.lam_l, P.lambda_floor, P.chi_l, P.chi_cap, chi};
    zgemm_tile<CfgSk>(M, N, Keff, m0, n0, la, lb, st, smem);
  } else {
    StU st{P.U, P.ldu, chi};
    zgemm_tile<CfgSk>(M, N, Keff, m0, n0, la, lb, st, smem);
  }
}

template <int TEBD_>
__device__ __forceinline__ void form_vh_tile(Prob& P, int M, int N, int m0, int n0, zt* smem) {
  if (P.retry) return;
  const int chi = P.chi_new;
  const int Keff = (m0 >= chi) ? 0 : P.l;
  LdSmallAdjA la{P.W, P.l};
  LdQbAdjB lb{P.Yt, P.n};
  if (TEBD_) {
    StGammaR st{P.gk1, P.lam_r, P.lambda_floor, P.chi_r, P.chi_cap, chi};
    zgemm_tile<CfgSk>(M, N, Keff, m0, n0, la, lb, st, smem);
  } else {
    StVH st{P.VH, P.ldvh, chi};
    zgemm_tile<CfgSk>(M, N, Keff, m0, n0, la, lb, st, smem);
  }
}

template <int TEBD_>
__global__ __launch_bounds__(256) void k_form_uv(Prob* probs, const int32_t* offs, int nprob) {
  __shared__ zt smem[CfgSk::lds_elems];
  for_each_tile2<TK_FORMU, TK_FORMV>(
      probs, offs, nprob, TEBD_,
      [&](Prob& P, int M, int N, int m0, int n0, int) { form_u_tile<TEBD_>(P, M, N, m0, n0, smem); },
      [&](Prob& P, int M, int N, int m0, int n0, int) { form_vh_tile<TEBD_>(P, M, N, m0, n0, smem); });
}

hipError_t launch_form_uv(Prob* probs, const Common& c, hipStream_t s) {
  const dim3 g(grid_for(c, TK_FORMU, TK_FORMV));
  if (c.tebd)
    TEBD_LAUNCH("k_form_uv<1>", k_form_uv<1>, g, dim3(256), 0, s, probs, c.offs, c.nprob);
  else
    TEBD_LAUNCH("k_form_uv<0>", k_form_uv<0>, g, dim3(256), 0, s, probs, c.offs, c.nprob);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Recording for the adjoint: every triplet the RRSVD computed (not only the
// kept ones) with plain U and V^H (no reabsorption), the singular values and
// the geometry, written once per bond in the pass that finishes it.
__global__ __launch_bounds__(256) void k_tape_uv(Prob* probs, const int32_t* offs, int nprob) {
  __shared__ zt smem[Cfg64::lds_elems];
  auto tape_u = [&](Prob& P, int M, int N, int m0, int n0, int) {
    if (P.retry) return;
    LdQP la{P.Y, P.m};
    LdSmallColB lb{P.X, P.l};
    StRow st{P.tape_u, P.tape_ldu};
    zgemm_tile<Cfg64>(M, N, P.l, m0, n0, la, lb, st, smem);
  };
  auto tape_vh = [&](Prob& P, int M, int N, int m0, int n0, int) {
    if (P.retry) return;
    LdSmallAdjA la{P.W, P.l};
    LdQbAdjB lb{P.Yt, P.n};
    StRow st{P.tape_vh, P.tape_ldvh};
    zgemm_tile<Cfg64>(M, N, P.l, m0, n0, la, lb, st, smem);
  };
  for_each_tile2<TK_TAPEU, TK_TAPEV>(probs, offs, nprob, 1, tape_u, tape_vh);
}

// One wavefront per problem: header and singular values.  A problem the
// planner rejected (l = 0 in the first pass) gets an invalid header; in the
// second pass of the adaptive scheme only re-run problems write.
__global__ __launch_bounds__(64) void k_tape_meta(Prob* probs, int pass2, int n_sites) {
  Prob& P = probs[blockIdx.x];
  if (!P.tape_hdr) return;
  const int lane = threadIdx.x;
  const bool done = P.l > 0 && !P.retry;
  const bool bad = !pass2 && P.l == 0;
  if (!done && !bad) return;
  for (int j = lane; j < P.l; j += 64) P.tape_sig[j] = P.sig[j];
  if (lane == 0) {
    int32_t* h = P.tape_hdr;
    h[TH_VALID] = done ? 1 : 0;
    h[TH_L] = P.l;
    h[TH_K] = done ? P.chi_new : 0;
    h[TH_M] = P.m;
    h[TH_N] = P.n;
    h[TH_CHI_L] = P.chi_l;
    h[TH_CHI_M] = P.chi_m;
    h[TH_CHI_R] = P.chi_r;
    h[TH_DL] = P.dl;
    h[TH_DR] = P.dr;
    h[TH_CHAIN] = P.pid / (n_sites - 1);
    h[TH_BOND] = P.pid % (n_sites - 1);
    h[TH_LCAP] = P.tape_ldu;
  }
}

hipError_t launch_tape(Prob* probs, const Common& c, hipStream_t s) {
  TEBD_LAUNCH("k_tape_uv", k_tape_uv, dim3(grid_for(c, TK_TAPEU, TK_TAPEV)), dim3(256), 0, s, probs,
                     c.offs, c.nprob);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  TEBD_LAUNCH("k_tape_meta", k_tape_meta, dim3(c.nprob), dim3(64), 0, s, probs, c.pass2, c.nsites);
  return hipGetLastError();
}

}  // namespace tebd

extern "C" tebd_status tebd_tune_set(int32_t precision, int32_t max_rows, int32_t width,
                                     int32_t variant) {
  using namespace tebd;
  if (precision < 0 || precision > 2 || variant < -1 || variant > 2 ||
      (precision == 1 && variant > 0))
    return TEBD_ERR_ARG;
  const int br = tune_bucket(kTuneRows, 6, max_rows), bw = tune_bucket(kTuneWidth, 5, width);
  if (max_rows < 1 || width < 1 || br < 0 || bw < 0) return TEBD_ERR_SHAPE;
  if (!g_tune_init) {
    for (auto& a : g_tune)
      for (auto& b : a)
        for (auto& v : b) v = -1;
    g_tune_init = true;
  }
  g_tune[precision][br][bw] = int8_t(variant);
  return TEBD_OK;
}

extern "C" int32_t tebd_tune_get(int32_t precision, int32_t max_rows, int32_t width) {
  using namespace tebd;
  if (precision < 0 || precision > 2 || max_rows < 1 || width < 1) return -1;
  const int br = tune_bucket(kTuneRows, 6, max_rows), bw = tune_bucket(kTuneWidth, 5, width);
  if (br < 0 || bw < 0 || !g_tune_init) return -1;
  return g_tune[precision][br][bw];
}
