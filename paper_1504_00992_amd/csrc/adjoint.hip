// Reverse mode of one TEBD sweep: every bond update of the sweep undone at
// once, batched over bonds and chains like the forward.
//
// The paper does not differentiate its method; this is the derivative of
// the bond update it defines (Sec. II.B: Theta of Eq. deftheta, the gate of
// Eq. defupdatetheta, the truncated SVD of the blocked matrix, the
// renormalised lambda' and the lambda^-1 reabsorption), given the tape the
// recorded forward wrote: the l triplets (U, s, V^H) its RRSVD computed, of
// which the first k were kept.
//
// Cotangents follow zbar = dL/dRe z + i dL/dIm z.  Per bond, with Ubar and
// Vbar^H the reabsorbed cotangents of Gamma'_k and Gamma'_k+1 (zero beyond
// column / row k) and sbar that of the kept s through lambda' = s/||s||:
//   M1 = U^H Ubar, M2 = V^H Vbar                                 (l x k)
//   D  = (J + J^H) S + S (K + K^H) + 1/2 S^-1 (L^H - L) + diag(sbar)
//        - M1 S^-1 - S^-1 M2^H,  J = F o M1, K = F o M2, L = I o M2  (l x l)
//   Abar = (U D + Ubar S^-1) V^H + U (S^-1 Vbar^H)    (one GEMM over 2 l)
// with F_ij = (s_j^2 - s_i^2) / ((s_j^2 - s_i^2)^2 + eta^2), eta = 1e-12 s_1^2.
// Triplets computed but not kept enter with zero cotangent, so the kept
// ones stay coupled to the part of the discarded spectrum the sketch saw;
// the rest enters through the projector terms folded into D.  Then
//   Theta-bar = G^H Abar,  Gbar += Abar Theta^H       (gate, Eq. defupdatetheta)
//   R1 = Theta-bar (Gamma_k+1 lambda_r)^H,  R2 = (lambda_l Gamma_k lambda_m)^H Theta-bar
// give the cotangents of Gamma_k, Gamma_k+1, lambda_m and contributions to
// those of lambda_l and lambda_r (Eq. deftheta).
//
// All GEMM-shaped steps are 64 x 64 tiles on FP64 MFMA over persistent tile
// queues; the elementwise and reduction steps run one workgroup per bond.
// Every sum has a fixed order, so results do not depend on scheduling.
#include "loaders.hpp"
#include "tilequeue.hpp"

namespace tebd {

using CfgA = ZCfg<64, 64, 16, 2, 2>;

__device__ __forceinline__ double lam_or_one(const double* lam, int i) {
  return lam ? lam[i] : 1.0;
}

template <>
struct TileKinds<AdjProb> {
  static constexpr int count = TA_COUNT;
  static constexpr int tile_m(int) { return 64; }
  static constexpr int tile_n(int) { return 64; }
  static constexpr bool col_major(int) { return false; }
  __device__ static __forceinline__ void shape(int kind, const AdjProb& P, int, int& M, int& N) {
    M = N = 0;
    if (P.L == 0) return;
    switch (kind) {
      case TA_M1:
      case TA_M2:
        M = P.L;
        N = P.k;
        break;
      case TA_THETA:
      case TA_ABAR:
        M = P.m;
        N = P.n;
        break;
      case TA_X:
        M = P.m;
        N = P.L;
        break;
      case TA_GADJ:
        M = P.dl * P.dr;
        N = P.chi_l * P.chi_r;
        break;
      case TA_GBAR: {
        const int d2 = P.dl * P.dr;
        M = 64 * ((d2 + 63) / 64) * P.nchunk;
        N = d2;
        break;
      }
      case TA_R1:
        M = P.m;
        N = P.chi_m;
        break;
      case TA_R2:
        M = P.chi_m;
        N = P.n;
        break;
      default:
        break;
    }
  }
};

// --------------------------------------------------------------------------
// Planning: one thread per bond of the sweep.  The tape slot must describe
// the same bond of the same state, else the bond is skipped and flagged.
__global__ void k_adj_plan(AdjProb* probs, int nprob, int nb, int parity, tebd_mps mps,
                           const zt* gates, int64_t gstride, const char* tape, size_t slot_bytes,
                           int64_t mcap, int64_t lcap, zt* gamma_bar, double* lambda_bar,
                           zt* gate_bar, int32_t* status, double lambda_floor, char* slab_base,
                           size_t slab_sz, int64_t nchunk_cap) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  const int N = mps.n_sites, cap = mps.chi_max, dmax = mps.d_max;
  const int chain = p / nb, bond = parity + 2 * (p - chain * nb);
  const int32_t* chi = mps.chi + size_t(chain) * (N + 1);
  AdjProb P;
  P.chain = chain;
  P.bond = bond;
  P.chi_l = chi[bond];
  P.chi_m = chi[bond + 1];
  P.chi_r = chi[bond + 2];
  P.dl = mps.d[bond];
  P.dr = mps.d[bond + 1];
  P.m = P.dl * P.chi_l;
  P.n = P.dr * P.chi_r;
  int32_t* hdr;
  double* sig;
  zt* U;
  zt* VH;
  tape_slot(const_cast<char*>(tape) + size_t(p) * slot_bytes, mcap, lcap, hdr, sig, U, VH);
  const int L = hdr[TH_L], k = hdr[TH_K];
  const bool ok = hdr[TH_VALID] == 1 && hdr[TH_CHAIN] == chain && hdr[TH_BOND] == bond &&
                  hdr[TH_CHI_L] == P.chi_l && hdr[TH_CHI_M] == P.chi_m &&
                  hdr[TH_CHI_R] == P.chi_r && hdr[TH_DL] == P.dl && hdr[TH_DR] == P.dr &&
                  hdr[TH_LCAP] == lcap && L >= 1 && L <= lcap && k >= 1 && k <= L && k <= cap &&
                  P.chi_l >= 1 && P.chi_l <= cap && P.chi_m >= 1 && P.chi_m <= cap &&
                  P.chi_r >= 1 && P.chi_r <= cap && P.dl >= 1 && P.dl <= dmax && P.dr >= 1 &&
                  P.dr <= dmax;
  P.L = ok ? L : 0;
  P.k = ok ? k : 0;
  P.nchunk = (P.chi_l * P.chi_r + kGateChunk - 1) / kGateChunk;
  if (P.nchunk > nchunk_cap) P.nchunk = int32_t(nchunk_cap);
  P.ldu = int32_t(lcap);
  P.ldvh = int32_t(mcap);
  P.ldl = int32_t(lcap);
  P.chi_cap = cap;
  P.gate_ld = dmax * dmax;
  P.dmax = dmax;
  P.lambda_floor = lambda_floor;
  P.eta = ok ? 1e-12 * sig[0] * sig[0] : 0.0;
  P.U = U;
  P.VH = VH;
  P.sig = sig;
  const size_t site_stride = size_t(dmax) * cap * cap;
  const size_t gsz = size_t(dmax) * dmax * dmax * dmax;
  P.gk = reinterpret_cast<const zt*>(mps.gamma) + (size_t(chain) * N + bond) * site_stride;
  P.gk1 = P.gk + site_stride;
  const double* lam_chain = mps.lambda + size_t(chain) * (N - 1) * cap;
  P.lam_l = bond >= 1 ? lam_chain + size_t(bond - 1) * cap : nullptr;
  P.lam_m = lam_chain + size_t(bond) * cap;
  P.lam_r = bond + 1 <= N - 2 ? lam_chain + size_t(bond + 1) * cap : nullptr;
  P.gate = gates + size_t(chain) * gstride + size_t(bond) * gsz;
  P.gbk = gamma_bar + (size_t(chain) * N + bond) * site_stride;
  P.gbk1 = P.gbk + site_stride;
  P.lbar_m = lambda_bar + size_t(chain) * (N - 1) * cap + size_t(bond) * cap;
  P.gate_bar = gate_bar + size_t(chain) * gstride + size_t(bond) * gsz;
  P.status = status + size_t(chain) * (N - 1) + bond;
  // scratch slab
  const size_t z = sizeof(zt), d = sizeof(double);
  const int64_t d2 = int64_t(dmax) * dmax;
  char* c = slab_base + size_t(p) * slab_sz;
  P.sbar = reinterpret_cast<double*>(c);
  c += align256(lcap * d);
  P.sinv = reinterpret_cast<double*>(c);
  c += align256(lcap * d);
  P.lamL = reinterpret_cast<double*>(c);
  c += align256(cap * d);
  P.lamR = reinterpret_cast<double*>(c);
  c += align256(cap * d);
  P.M1 = reinterpret_cast<zt*>(c);
  c += align256(lcap * lcap * z);
  P.M2 = reinterpret_cast<zt*>(c);
  c += align256(lcap * lcap * z);
  P.D = reinterpret_cast<zt*>(c);
  c += align256(lcap * lcap * z);
  P.X = reinterpret_cast<zt*>(c);
  c += align256(mcap * lcap * z);
  P.AbT = reinterpret_cast<zt*>(c);
  c += align256(mcap * mcap * z);
  P.T = reinterpret_cast<zt*>(c);
  c += align256(mcap * mcap * z);
  P.Thb = reinterpret_cast<zt*>(c);
  c += align256(mcap * mcap * z);
  P.R1 = reinterpret_cast<zt*>(c);
  c += align256(mcap * cap * z);
  P.R2 = reinterpret_cast<zt*>(c);
  c += align256(int64_t(cap) * mcap * z);
  P.gpart = reinterpret_cast<zt*>(c);
  probs[p] = P;
  *P.status = ok ? 0 : TEBD_DEV_BAD_STATE;
}

// --------------------------------------------------------------------------
// Per bond: sbar through the renormalisation, 1/s, and the reabsorption's
// contributions to the cotangents of lambda_l and lambda_r:
//   d/dlambda_l[a] of U[(i,a), c] / lambda_l[a] = -Gamma'/lambda_l.
__global__ __launch_bounds__(256) void k_adj_prep(AdjProb* probs) {
  __shared__ double red[4];
  AdjProb& P = probs[blockIdx.x];
  if (P.L == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int L = P.L, k = P.k, cap = P.chi_cap;
  double nk = 0.0, dot = 0.0;
  for (int c = tid; c < k; c += 256) nk += P.sig[c] * P.sig[c];
  nk = block_sum<256>(nk, red);
  const double nrm = sqrt(nk);
  const double inv_n = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int c = tid; c < k; c += 256) dot += P.sig[c] * inv_n * P.lbar_m[c];
  dot = block_sum<256>(dot, red);
  for (int j = tid; j < L; j += 256) {
    const double s = P.sig[j];
    P.sinv[j] = s > 0.0 ? 1.0 / s : 0.0;
    P.sbar[j] = j < k ? (P.lbar_m[j] - s * inv_n * dot) * inv_n : 0.0;
  }
  for (int a = wave; a < P.chi_l; a += 4) {
    double acc = 0.0;
    for (int e = lane; e < P.dl * k; e += 64) {
      const int i = e / k, c = e - i * k;
      const zt g = P.gbk[(size_t(i) * cap + a) * cap + c];
      const zt u = P.U[size_t(i * P.chi_l + a) * P.ldu + c];
      acc += g.x * u.x + g.y * u.y;
    }
    acc = wave_sum(acc);
    const double il = inv_floor(P.lam_l, a, P.lambda_floor);
    if (lane == 0) P.lamL[a] = P.lam_l ? -il * il * acc : 0.0;
  }
  for (int b = wave; b < P.chi_r; b += 4) {
    double acc = 0.0;
    for (int e = lane; e < P.dr * k; e += 64) {
      const int j = e / k, c = e - j * k;
      const zt g = P.gbk1[(size_t(j) * cap + c) * cap + b];
      const zt v = P.VH[size_t(c) * P.ldvh + j * P.chi_r + b];
      acc += g.x * v.x + g.y * v.y;
    }
    acc = wave_sum(acc);
    const double ir = inv_floor(P.lam_r, b, P.lambda_floor);
    if (lane == 0) P.lamR[b] = P.lam_r ? -ir * ir * acc : 0.0;
  }
}

// --------------------------------------------------------------------------
// M1 = U^H Ubar, M2 = V^H Vbar, and Theta rebuilt from the state.
struct LdUbar {  // (r = i*chi_l + a, j) -> Gamma'-bar_k[i][a][j] / lambda_l[a]
  const zt* gb;
  const double* lam_l;
  double floor_;
  int chi_l, cap;
  static constexpr bool contig_n = true;
  __device__ zt operator()(int r, int j) const {
    const int i = r / chi_l, a = r - i * chi_l;
    return zscale(gb[(size_t(i) * cap + a) * cap + j], inv_floor(lam_l, a, floor_));
  }
};
struct LdVbar {  // (c = jj*chi_r + b, j) -> conj(Gamma'-bar_k+1[jj][j][b] / lambda_r[b])
  const zt* gb1;
  const double* lam_r;
  double floor_;
  int chi_r, cap;
  static constexpr bool contig_n = false;
  __device__ zt operator()(int c, int j) const {
    const int jj = c / chi_r, b = c - jj * chi_r;
    return zconj(zscale(gb1[(size_t(jj) * cap + j) * cap + b], inv_floor(lam_r, b, floor_)));
  }
};

__global__ __launch_bounds__(256) void k_adj_m12_theta(AdjProb* probs, const int32_t* offs,
                                                       int nprob) {
  __shared__ zt smem[CfgA::lds_elems];
  for_each_tile<TA_M1>(probs, offs, nprob, 0, [&](AdjProb& P, int M, int N, int m0, int n0, int) {
    LdAdjA la{P.U, P.ldu};
    LdUbar lb{P.gbk, P.lam_l, P.lambda_floor, P.chi_l, P.chi_cap};
    StRow st{P.M1, P.ldl};
    zgemm_tile<CfgA>(M, N, P.m, m0, n0, la, lb, st, smem);
  });
  for_each_tile<TA_M2>(probs, offs, nprob, 0, [&](AdjProb& P, int M, int N, int m0, int n0, int) {
    LdRowA la{P.VH, P.ldvh};
    LdVbar lb{P.gbk1, P.lam_r, P.lambda_floor, P.chi_r, P.chi_cap};
    StRow st{P.M2, P.ldl};
    zgemm_tile<CfgA>(M, N, P.n, m0, n0, la, lb, st, smem);
  });
  for_each_tile<TA_THETA>(probs, offs, nprob, 0, [&](AdjProb& P, int M, int N, int m0, int n0, int) {
    LdThetaA la{P.gk, P.lam_l, P.lam_m, P.chi_l, P.chi_cap};
    LdThetaB lb{P.gk1, P.lam_r, P.chi_r, P.chi_cap};
    StTheta st{P.T, P.chi_l, P.chi_r, P.dr};
    zgemm_tile<CfgA>(M, N, P.chi_m, m0, n0, la, lb, st, smem);
  });
}

// --------------------------------------------------------------------------
// D (l x l), one workgroup per bond.
__global__ __launch_bounds__(256) void k_adj_core(AdjProb* probs) {
  AdjProb& P = probs[blockIdx.x];
  if (P.L == 0) return;
  const int L = P.L, k = P.k, ld = P.ldl;
  const double eta2 = P.eta * P.eta;
  for (int e = threadIdx.x; e < L * L; e += 256) {
    const int i = e / L, j = e - i * L;
    const double si = P.sig[i], sj = P.sig[j];
    const double dd = sj * sj - si * si;
    const double f = i == j ? 0.0 : dd / (dd * dd + eta2);  // F_ij; F_ji = -F_ij
    const zt m1ij = zload_if(j < k, P.M1 + size_t(i) * ld + j);
    const zt m1ji = zload_if(i < k, P.M1 + size_t(j) * ld + i);
    const zt m2ij = zload_if(j < k, P.M2 + size_t(i) * ld + j);
    const zt m2ji = zload_if(i < k, P.M2 + size_t(j) * ld + i);
    // (J_ij + conj(J_ji)) s_j + s_i (K_ij + conj(K_ji)), J = F o M1, K = F o M2
    const zt jj = zsub(zscale(m1ij, f), zscale(zconj(m1ji), f));
    const zt kk = zsub(zscale(m2ij, f), zscale(zconj(m2ji), f));
    zt v = zadd(zscale(jj, sj), zscale(kk, si));
    const double ii = P.sinv[i], ij = P.sinv[j];
    if (i == j) {
      v.x += P.sbar[i];
      if (i < k) v.y -= ii * m2ij.y;  // 1/2 S^-1 (L^H - L)
    }
    v = zsub(v, zscale(m1ij, ij));        // - M1 S^-1
    v = zsub(v, zscale(zconj(m2ji), ii));  // - S^-1 M2^H
    P.D[size_t(i) * ld + j] = v;
  }
}

// --------------------------------------------------------------------------
// X = U D + Ubar S^-1  (m x l)
struct StXadd {
  zt* X;
  int64_t ld;
  const zt* gb;
  const double* lam_l;
  const double* sinv;
  double floor_;
  int chi_l, cap, k;
  __device__ void operator()(int r, int j, zt v) {
    if (j < k) {
      const int i = r / chi_l, a = r - i * chi_l;
      const zt ub = zscale(gb[(size_t(i) * cap + a) * cap + j], inv_floor(lam_l, a, floor_));
      v = zadd(v, zscale(ub, sinv[j]));
    }
    X[size_t(r) * ld + j] = v;
  }
};

__global__ __launch_bounds__(256) void k_adj_x(AdjProb* probs, const int32_t* offs, int nprob) {
  __shared__ zt smem[CfgA::lds_elems];
  for_each_tile<TA_X>(probs, offs, nprob, 0, [&](AdjProb& P, int M, int N, int m0, int n0, int) {
    LdRowA la{P.U, P.ldu};
    LdRowB lb{P.D, P.ldl};
    StXadd st{P.X, P.ldl, P.gbk, P.lam_l, P.sinv, P.lambda_floor, P.chi_l, P.chi_cap, P.k};
    zgemm_tile<CfgA>(M, N, P.L, m0, n0, la, lb, st, smem);
  });
}

// --------------------------------------------------------------------------
// Abar = [X | U] [V^H ; S^-1 Vbar^H], stored as [(i j)][(a c)] for the gate.
struct LdXU {  // (r, kk): kk < l -> X[r][kk], else U[r][kk - l]
  const zt* X;
  int64_t ldx;
  const zt* U;
  int64_t ldu;
  int L;
  static constexpr bool contig_k = true;
  __device__ zt operator()(int r, int kk) const {
    return kk < L ? X[size_t(r) * ldx + kk] : U[size_t(r) * ldu + (kk - L)];
  }
};
struct LdVhY {  // (kk, c): kk < l -> V^H[kk][c], else S^-1 Vbar^H (rows < k)
  const zt* VH;
  int64_t ldvh;
  const zt* gb1;
  const double* lam_r;
  const double* sinv;
  double floor_;
  int chi_r, cap, L, k;
  static constexpr bool contig_n = true;
  __device__ zt operator()(int kk, int c) const {
    if (kk < L) return VH[size_t(kk) * ldvh + c];
    const int j = kk - L;
    if (j >= k) return make_double2(0.0, 0.0);
    const int jj = c / chi_r, b = c - jj * chi_r;
    return zscale(gb1[(size_t(jj) * cap + j) * cap + b], inv_floor(lam_r, b, floor_) * sinv[j]);
  }
};

__global__ __launch_bounds__(256) void k_adj_abar(AdjProb* probs, const int32_t* offs, int nprob) {
  __shared__ zt smem[CfgA::lds_elems];
  for_each_tile<TA_ABAR>(probs, offs, nprob, 0, [&](AdjProb& P, int M, int N, int m0, int n0, int) {
    LdXU la{P.X, P.ldl, P.U, P.ldu, P.L};
    LdVhY lb{P.VH, P.ldvh, P.gbk1, P.lam_r, P.sinv, P.lambda_floor, P.chi_r, P.chi_cap, P.L, P.k};
    StTheta st{P.AbT, P.chi_l, P.chi_r, P.dr};
    zgemm_tile<CfgA>(M, N, 2 * P.L, m0, n0, la, lb, st, smem);
  });
}

// --------------------------------------------------------------------------
// Gate: Theta-bar = G^H Abar (blocked layout) and the per-chunk partial sums
// of Gbar = Abar Theta^H over K-chunks of the (alpha beta) index.
struct StBlocked {  // (r = i*dr + j, c = a*chi_r + b) -> p[(i*chi_l + a)*n + j*chi_r + b]
  zt* p;
  int chi_l, chi_r, dr, n;
  __device__ void operator()(int r, int c, zt v) {
    const int i = r / dr, j = r - i * dr;
    const int a = c / chi_r, b = c - a * chi_r;
    p[(size_t(i) * chi_l + a) * n + size_t(j) * chi_r + b] = v;
  }
};
struct LdAdjB {  // B[k][c] = conj(p[c*ld + k])
  const zt* p;
  int64_t ld;
  static constexpr bool contig_n = false;
  __device__ zt operator()(int k, int c) const { return zconj(p[size_t(c) * ld + k]); }
};

__global__ __launch_bounds__(256) void k_adj_gate(AdjProb* probs, const int32_t* offs, int nprob) {
  __shared__ zt smem[CfgA::lds_elems];
  for_each_tile<TA_GADJ>(probs, offs, nprob, 0, [&](AdjProb& P, int M, int N, int m0, int n0, int) {
    LdAdjA la{P.gate, P.gate_ld};
    LdRowB lb{P.AbT, N};
    StBlocked st{P.Thb, P.chi_l, P.chi_r, P.dr, P.n};
    zgemm_tile<CfgA>(M, N, M, m0, n0, la, lb, st, smem);
  });
  for_each_tile<TA_GBAR>(probs, offs, nprob, 0, [&](AdjProb& P, int, int N, int m0, int n0, int) {
    const int d2 = P.dl * P.dr;
    const int rows = 64 * ((d2 + 63) / 64);
    const int chunk = m0 / rows;
    const int kc0 = chunk * kGateChunk;
    const int ab = P.chi_l * P.chi_r;
    const int len = min(kGateChunk, ab - kc0);
    LdRowA la{P.AbT + kc0, ab};
    LdAdjB lb{P.T + kc0, ab};
    StRow st{P.gpart + size_t(chunk) * d2 * d2, d2};
    zgemm_tile<CfgA>(d2, N, len, m0 - chunk * rows, n0, la, lb, st, smem);
  });
}

// --------------------------------------------------------------------------
// R1 = Theta-bar (Gamma_k+1 lambda_r)^H, R2 = (lambda_l Gamma_k lambda_m)^H Theta-bar
struct LdGtAdj {  // (kk = j*chi_r + b, g) -> conj(Gamma_k+1[j][g][b]) lambda_r[b]
  const zt* gk1;
  const double* lam_r;
  int chi_r, cap;
  static constexpr bool contig_n = false;
  __device__ zt operator()(int kk, int g) const {
    const int j = kk / chi_r, b = kk - j * chi_r;
    return zscale(zconj(gk1[(size_t(j) * cap + g) * cap + b]), lam_or_one(lam_r, b));
  }
};
struct LdGsAdj {  // (g, kk = i*chi_l + a) -> conj(lambda_l[a] Gamma_k[i][a][g] lambda_m[g])
  const zt* gk;
  const double* lam_l;
  const double* lam_m;
  int chi_l, cap;
  static constexpr bool contig_k = false;
  __device__ zt operator()(int g, int kk) const {
    const int i = kk / chi_l, a = kk - i * chi_l;
    return zscale(zconj(gk[(size_t(i) * cap + a) * cap + g]), lam_or_one(lam_l, a) * lam_m[g]);
  }
};

__global__ __launch_bounds__(256) void k_adj_r(AdjProb* probs, const int32_t* offs, int nprob) {
  __shared__ zt smem[CfgA::lds_elems];
  for_each_tile<TA_R1>(probs, offs, nprob, 0, [&](AdjProb& P, int M, int N, int m0, int n0, int) {
    LdRowA la{P.Thb, P.n};
    LdGtAdj lb{P.gk1, P.lam_r, P.chi_r, P.chi_cap};
    StRow st{P.R1, P.chi_cap};
    zgemm_tile<CfgA>(M, N, P.n, m0, n0, la, lb, st, smem);
  });
  for_each_tile<TA_R2>(probs, offs, nprob, 0, [&](AdjProb& P, int M, int N, int m0, int n0, int) {
    LdGsAdj la{P.gk, P.lam_l, P.lam_m, P.chi_l, P.chi_cap};
    LdRowB lb{P.Thb, P.n};
    StRow st{P.R2, P.ldvh};
    zgemm_tile<CfgA>(M, N, P.m, m0, n0, la, lb, st, smem);
  });
}

// --------------------------------------------------------------------------
// Per bond: the cotangents of Gamma_k, Gamma_k+1 (whole padded blocks) and
// lambda_m, and the Theta parts of the lambda_l / lambda_r contributions.
__global__ __launch_bounds__(256) void k_adj_finish(AdjProb* probs) {
  AdjProb& P = probs[blockIdx.x];
  if (P.L == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cap = P.chi_cap, cl = P.chi_l, cm = P.chi_m, cr = P.chi_r;
  if (P.lam_l) {
    for (int a = wave; a < cl; a += 4) {
      double acc = 0.0;
      for (int e = lane; e < P.dl * cm; e += 64) {
        const int i = e / cm, g = e - i * cm;
        const zt r = P.R1[size_t(i * cl + a) * cap + g];
        const zt x = P.gk[(size_t(i) * cap + a) * cap + g];
        acc += (r.x * x.x + r.y * x.y) * P.lam_m[g];
      }
      acc = wave_sum(acc);
      if (lane == 0) P.lamL[a] += acc;
    }
  }
  for (int g = wave; g < cm; g += 4) {
    double acc = 0.0;
    for (int e = lane; e < P.dl * cl; e += 64) {
      const int i = e / cl, a = e - i * cl;
      const zt r = P.R1[size_t(i * cl + a) * cap + g];
      const zt x = P.gk[(size_t(i) * cap + a) * cap + g];
      acc += (r.x * x.x + r.y * x.y) * lam_or_one(P.lam_l, a);
    }
    acc = wave_sum(acc);
    if (lane == 0) P.lbar_m[g] = acc;
  }
  if (P.lam_r) {
    for (int b = wave; b < cr; b += 4) {
      double acc = 0.0;
      for (int e = lane; e < P.dr * cm; e += 64) {
        const int j = e / cm, g = e - j * cm;
        const zt r = P.R2[size_t(g) * P.ldvh + j * cr + b];
        const zt x = P.gk1[(size_t(j) * cap + g) * cap + b];
        acc += r.x * x.x + r.y * x.y;
      }
      acc = wave_sum(acc);
      if (lane == 0) P.lamR[b] += acc;
    }
  }
  for (int g = cm + tid; g < cap; g += 256) P.lbar_m[g] = 0.0;
  const int blk = P.dmax * cap * cap;
  for (int e = tid; e < blk; e += 256) {
    const int i = e / (cap * cap), rem = e - i * cap * cap, a = rem / cap, g = rem - a * cap;
    zt v = make_double2(0.0, 0.0);
    if (i < P.dl && a < cl && g < cm)
      v = zscale(P.R1[size_t(i * cl + a) * cap + g], lam_or_one(P.lam_l, a) * P.lam_m[g]);
    P.gbk[e] = v;
  }
  for (int e = tid; e < blk; e += 256) {
    const int j = e / (cap * cap), rem = e - j * cap * cap, g = rem / cap, b = rem - g * cap;
    zt v = make_double2(0.0, 0.0);
    if (j < P.dr && g < cm && b < cr)
      v = zscale(P.R2[size_t(g) * P.ldvh + j * cr + b], lam_or_one(P.lam_r, b));
    P.gbk1[e] = v;
  }
}

// --------------------------------------------------------------------------
// Gate cotangents: one workgroup per bond of the parity; chains in order.
// With a zero chain stride every chain shares one gate and one sum.
__global__ __launch_bounds__(256) void k_adj_gsum(const AdjProb* probs, int n_chains, int nb,
                                                  int64_t gstride) {
  const int bi = blockIdx.x;
  const AdjProb& P0 = probs[bi];
  if (P0.dl < 1 || P0.dl > P0.dmax || P0.dr < 1 || P0.dr > P0.dmax) return;
  const int d2 = P0.dl * P0.dr, ld = P0.gate_ld;
  for (int e = threadIdx.x; e < d2 * d2; e += 256) {
    const int r = e / d2, c = e - r * d2;
    if (gstride == 0) {
      zt acc = P0.gate_bar[size_t(r) * ld + c];
      for (int ch = 0; ch < n_chains; ++ch) {
        const AdjProb& P = probs[size_t(ch) * nb + bi];
        if (P.L == 0) continue;
        for (int q = 0; q < P.nchunk; ++q) acc = zadd(acc, P.gpart[size_t(q) * d2 * d2 + e]);
      }
      P0.gate_bar[size_t(r) * ld + c] = acc;
    } else {
      for (int ch = 0; ch < n_chains; ++ch) {
        const AdjProb& P = probs[size_t(ch) * nb + bi];
        if (P.L == 0) continue;
        zt acc = P.gate_bar[size_t(r) * ld + c];
        for (int q = 0; q < P.nchunk; ++q) acc = zadd(acc, P.gpart[size_t(q) * d2 * d2 + e]);
        P.gate_bar[size_t(r) * ld + c] = acc;
      }
    }
  }
}

// Cotangents of the lambdas the sweep only read (bonds of the other
// parity): add the contributions of the update on the right (its lambda_l)
// and on the left (its lambda_r), in that order.
__global__ __launch_bounds__(64) void k_adj_lambda(const AdjProb* probs, tebd_mps mps, int parity,
                                                   int nb, double* lambda_bar) {
  const int N = mps.n_sites, cap = mps.chi_max;
  const int chain = blockIdx.x / (N - 1), t = blockIdx.x - chain * (N - 1);
  if ((t & 1) == parity) return;
  const int chi_t = mps.chi[size_t(chain) * (N + 1) + t + 1];
  const AdjProb* right = t + 1 <= N - 2 ? probs + size_t(chain) * nb + (t + 1 - parity) / 2 : nullptr;
  const AdjProb* left = t - 1 >= 0 ? probs + size_t(chain) * nb + (t - 1 - parity) / 2 : nullptr;
  if (right && right->L == 0) right = nullptr;
  if (left && left->L == 0) left = nullptr;
  double* lb = lambda_bar + size_t(chain) * (N - 1) * cap + size_t(t) * cap;
  for (int e = threadIdx.x; e < chi_t && e < cap; e += 64) {
    double v = lb[e];
    if (right) v += right->lamL[e];
    if (left) v += left->lamR[e];
    lb[e] = v;
  }
}

hipError_t launch_adjoint(AdjProb* probs, const AdjCommon& c, const tebd_mps& mps_in,
                          const zt* gates, const char* tape, size_t slot_bytes, int64_t mcap,
                          int64_t lcap, zt* gamma_bar, double* lambda_bar, zt* gate_bar,
                          int32_t* status, double lambda_floor, char* slab_base, size_t slab_sz,
                          int64_t nchunk_cap, hipStream_t s) {
  hipError_t e;
#define TRY(name, ...)               \
  do {                               \
    TEBD_LAUNCH(name, __VA_ARGS__);  \
    e = hipGetLastError();           \
    if (e != hipSuccess) return e;   \
  } while (0)
  const dim3 g(c.grid), pb(c.nprob);
  TRY("k_adj_plan", k_adj_plan, dim3((c.nprob + 63) / 64), dim3(64), 0, s, probs, c.nprob, c.nb, c.parity,
      mps_in, gates, c.gate_chain_stride, tape, slot_bytes, mcap, lcap, gamma_bar, lambda_bar,
      gate_bar, status, lambda_floor, slab_base, slab_sz, nchunk_cap);
  TRY("k_schedule<tebd::AdjProb, false>", k_schedule<AdjProb>, dim3(1), dim3(kScheduleThreads), 0, s, probs, c.nprob, 0, c.offs,
      static_cast<int32_t*>(nullptr));
  TRY("k_adj_prep", k_adj_prep, pb, dim3(256), 0, s, probs);
  TRY("k_adj_m12_theta", k_adj_m12_theta, g, dim3(256), 0, s, probs, c.offs, c.nprob);
  TRY("k_adj_core", k_adj_core, pb, dim3(256), 0, s, probs);
  TRY("k_adj_x", k_adj_x, g, dim3(256), 0, s, probs, c.offs, c.nprob);
  TRY("k_adj_abar", k_adj_abar, g, dim3(256), 0, s, probs, c.offs, c.nprob);
  TRY("k_adj_gate", k_adj_gate, g, dim3(256), 0, s, probs, c.offs, c.nprob);
  TRY("k_adj_r", k_adj_r, g, dim3(256), 0, s, probs, c.offs, c.nprob);
  TRY("k_adj_finish", k_adj_finish, pb, dim3(256), 0, s, probs);
  TRY("k_adj_gsum", k_adj_gsum, dim3(c.nb), dim3(256), 0, s, probs, c.n_chains, c.nb, c.gate_chain_stride);
  TRY("k_adj_lambda", k_adj_lambda, dim3(c.n_chains * (c.n_sites - 1)), dim3(64), 0, s, probs, mps_in,
      c.parity, c.nb, lambda_bar);
#undef TRY
  return hipSuccess;
}

}  // namespace tebd
