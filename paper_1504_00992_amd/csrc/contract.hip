// Dense complex contractions of the bond update on FP64 matrix cores.
//
// * Theta build, Eq. (deftheta): one GEMM per bond,
//     Theta[(i,a),(j,c)] = sum_g (lam_l[a] G_k[i][a][g] lam_m[g]) (G_k+1[j][g][c] lam_r[c]),
//   with the diagonal lambdas folded into the operand loads, written in the
//   layout T[(i j)][(a c)] that the gate product reads.
// * Gate update, Eq. (defupdatetheta): A = G T as (dl dr) x (dl dr) times
//   (dl dr) x (chi_l chi_r), scattered into the blocked matrix of Sec. II.B,
//   A[(i,a),(j,c)], with per-tile partial sums of |A|^2 for ||A||_F^2.
// * Sketch and power iteration, Alg. 1: Y = A Omega, Yt = A^H Q, Y = A Q~.
// * Singular vectors, Sec. IV steps i-iii: U = Q X and V^H = (Q_B W)^H for the
//   kept chi' columns, with the lambda^-1 reabsorption of the TEBD update
//   folded into the store.
#include "zgemm.hpp"

namespace tebd {

using Cfg64 = ZCfg<64, 64, 16, 2, 2>;

__device__ __forceinline__ double inv_floor(const double* lam, int idx, double floor_) {
  if (lam == nullptr) return 1.0;
  const double v = lam[idx];
  return v > floor_ ? 1.0 / v : 0.0;
}

// --------------------------------------------------------------------------
// Theta build
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

__global__ __launch_bounds__(256) void k_theta(Prob* probs) {
  __shared__ zt smem[Cfg64::lds_elems];
  const Prob& P = probs[blockIdx.z];
  if (P.l == 0) return;
  const int M = P.dl * P.chi_l, N = P.dr * P.chi_r, K = P.chi_m;
  const int m0 = blockIdx.y * Cfg64::BM, n0 = blockIdx.x * Cfg64::BN;
  if (m0 >= M || n0 >= N) return;
  LdThetaA la{P.gk, P.lam_l, P.lam_mid, P.chi_l, P.chi_cap};
  LdThetaB lb{P.gk1, P.lam_r, P.chi_r, P.chi_cap};
  StTheta st{P.T, P.chi_l, P.chi_r, P.dr};
  zgemm_tile<Cfg64>(M, N, K, m0, n0, la, lb, st, smem);
}

// --------------------------------------------------------------------------
// Gate update
struct LdGate {
  const zt* g;
  int ld;
  static constexpr bool contig_k = true;
  __device__ zt operator()(int r, int k) const { return g[size_t(r) * ld + k]; }
};
struct LdRowB {  // B[k][c] = p[k*ld + c]
  const zt* p;
  int64_t ld;
  static constexpr bool contig_n = true;
  __device__ zt operator()(int k, int c) const { return p[size_t(k) * ld + c]; }
};
struct StGate {
  zt* A;
  int chi_l, chi_r, dr, n;
  double acc;
  __device__ void operator()(int r, int c, zt v) {
    const int i = r / dr, j = r - i * dr;
    const int a = c / chi_r, b = c - a * chi_r;
    A[(size_t(i) * chi_l + a) * n + size_t(j) * chi_r + b] = v;
    acc += zabs2(v);
  }
};

__global__ __launch_bounds__(256) void k_gate(Prob* probs) {
  __shared__ zt smem[Cfg64::lds_elems];
  __shared__ double red[4];
  const Prob& P = probs[blockIdx.z];
  if (P.l == 0) return;
  const int M = P.dl * P.dr, N = P.chi_l * P.chi_r, K = P.dl * P.dr;
  const int m0 = blockIdx.y * Cfg64::BM, n0 = blockIdx.x * Cfg64::BN;
  if (m0 >= M || n0 >= N) return;
  LdGate la{P.gate, P.gate_ld};
  LdRowB lb{P.T, N};
  StGate st{P.A, P.chi_l, P.chi_r, P.dr, P.n, 0.0};
  zgemm_tile<Cfg64>(M, N, K, m0, n0, la, lb, st, smem);
  const double s = block_sum<256>(st.acc, red);
  if (threadIdx.x == 0) {
    const int tiles_n = (N + Cfg64::BN - 1) / Cfg64::BN;
    P.part[blockIdx.y * tiles_n + blockIdx.x] = s;
  }
}

hipError_t launch_theta_gate(Prob* probs, const Common& c, hipStream_t s) {
  const int cap = c.dmax * c.chimax;
  dim3 g1((cap + 63) / 64, (cap + 63) / 64, c.nprob);
  hipLaunchKernelGGL(k_theta, g1, dim3(256), 0, s, probs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int d2 = c.dmax * c.dmax, x2 = c.chimax * c.chimax;
  dim3 g2((x2 + 63) / 64, (d2 + 63) / 64, c.nprob);
  hipLaunchKernelGGL(k_gate, g2, dim3(256), 0, s, probs);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Sketch / power iteration / projection products
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
struct StCol {  // C[r][c] -> p[c*ld + r]
  zt* p;
  int64_t ld;
  __device__ void operator()(int r, int c, zt v) { p[size_t(c) * ld + r] = v; }
};

template <int WHICH>
__global__ __launch_bounds__(256) void k_sketch(Prob* probs) {
  __shared__ zt smem[Cfg64::lds_elems];
  const Prob& P = probs[blockIdx.z];
  if (P.l == 0) return;
  const int m0 = blockIdx.y * Cfg64::BM, n0 = blockIdx.x * Cfg64::BN;
  if (WHICH == SK_Y_FROM_OMEGA) {
    const int M = P.m, N = P.l, K = P.n;
    if (m0 >= M || n0 >= N) return;
    LdRowA la{P.A, P.lda};
    LdRowB lb{P.om, P.ldom};
    StCol st{P.Y, P.m};
    zgemm_tile<Cfg64>(M, N, K, m0, n0, la, lb, st, smem);
  } else if (WHICH == SK_YT_FROM_Y) {
    const int M = P.n, N = P.l, K = P.m;
    if (m0 >= M || n0 >= N) return;
    LdAdjA la{P.A, P.lda};
    LdColB lb{P.Y, P.m};
    StCol st{P.Yt, P.n};
    zgemm_tile<Cfg64>(M, N, K, m0, n0, la, lb, st, smem);
  } else {
    const int M = P.m, N = P.l, K = P.n;
    if (m0 >= M || n0 >= N) return;
    LdRowA la{P.A, P.lda};
    LdColB lb{P.Yt, P.n};
    StCol st{P.Y, P.m};
    zgemm_tile<Cfg64>(M, N, K, m0, n0, la, lb, st, smem);
  }
}

hipError_t launch_sketch(Prob* probs, const Common& c, int which, hipStream_t s) {
  const int rows = (which == SK_YT_FROM_Y) ? c.nmax : c.mmax;
  dim3 g((c.lmax + 63) / 64, (rows + 63) / 64, c.nprob);
  if (which == SK_Y_FROM_OMEGA)
    hipLaunchKernelGGL(k_sketch<SK_Y_FROM_OMEGA>, g, dim3(256), 0, s, probs);
  else if (which == SK_YT_FROM_Y)
    hipLaunchKernelGGL(k_sketch<SK_YT_FROM_Y>, g, dim3(256), 0, s, probs);
  else
    hipLaunchKernelGGL(k_sketch<SK_Y_FROM_YT>, g, dim3(256), 0, s, probs);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Kept singular vectors and lambda^-1 reabsorption
struct LdQ {  // (r, k) -> Q[k*ld + r] (column-major Q, rows r)
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

// Tiles entirely beyond chi' only write zeros (no contraction).
template <int TEBD_>
__global__ __launch_bounds__(256) void k_form_u(Prob* probs) {
  __shared__ zt smem[Cfg64::lds_elems];
  const Prob& P = probs[blockIdx.z];
  if (P.l == 0) return;
  // TEBD: clear every padded column of Gamma'_k beyond chi'
  const int M = P.m, N = TEBD_ ? P.chi_cap : P.kcap, K = P.l;
  const int m0 = blockIdx.y * Cfg64::BM, n0 = blockIdx.x * Cfg64::BN;
  if (m0 >= M || n0 >= N) return;
  const int chi = P.chi_new;
  const int Keff = (n0 >= chi) ? 0 : K;
  LdQ la{P.Y, P.m};
  LdSmallColB lb{P.X, P.l};
  if (TEBD_) {
    StGammaL st{P.gk, P.lam_l, P.lambda_floor, P.chi_l, P.chi_cap, chi};
    zgemm_tile<Cfg64>(M, N, Keff, m0, n0, la, lb, st, smem);
  } else {
    StU st{P.U, P.ldu, chi};
    zgemm_tile<Cfg64>(M, N, Keff, m0, n0, la, lb, st, smem);
  }
}

template <int TEBD_>
__global__ __launch_bounds__(256) void k_form_vh(Prob* probs) {
  __shared__ zt smem[Cfg64::lds_elems];
  const Prob& P = probs[blockIdx.z];
  if (P.l == 0) return;
  const int M = TEBD_ ? P.chi_cap : P.kcap, N = P.n, K = P.l;
  const int m0 = blockIdx.y * Cfg64::BM, n0 = blockIdx.x * Cfg64::BN;
  if (m0 >= M || n0 >= N) return;
  const int chi = P.chi_new;
  const int Keff = (m0 >= chi) ? 0 : K;
  LdSmallAdjA la{P.W, P.l};
  LdQbAdjB lb{P.Yt, P.n};
  if (TEBD_) {
    StGammaR st{P.gk1, P.lam_r, P.lambda_floor, P.chi_r, P.chi_cap, chi};
    zgemm_tile<Cfg64>(M, N, Keff, m0, n0, la, lb, st, smem);
  } else {
    StVH st{P.VH, P.ldvh, chi};
    zgemm_tile<Cfg64>(M, N, Keff, m0, n0, la, lb, st, smem);
  }
}

hipError_t launch_form_uv(Prob* probs, const Common& c, hipStream_t s) {
  const int kc = c.tebd ? c.chimax : c.kcap;
  dim3 gu((kc + 63) / 64, (c.mmax + 63) / 64, c.nprob);
  dim3 gv((c.nmax + 63) / 64, (kc + 63) / 64, c.nprob);
  if (c.tebd) {
    hipLaunchKernelGGL(k_form_u<1>, gu, dim3(256), 0, s, probs);
    hipLaunchKernelGGL(k_form_vh<1>, gv, dim3(256), 0, s, probs);
  } else {
    hipLaunchKernelGGL(k_form_u<0>, gu, dim3(256), 0, s, probs);
    hipLaunchKernelGGL(k_form_vh<0>, gv, dim3(256), 0, s, probs);
  }
  return hipGetLastError();
}

}  // namespace tebd
