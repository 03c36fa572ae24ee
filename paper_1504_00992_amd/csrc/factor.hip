// Wavefront-level kernels of the RRSVD pipeline (one workgroup per problem):
// planning of a TEBD sweep, ||A||_F^2, Householder QR with explicit Q, the small SVD by one-sided Jacobi, and the truncation
// rule with lambda renormalisation.
//
// Paper: Tamascelli, Rosenbach, Plenio, arXiv:1504.00992.  QR steps of Alg. 1
// (the paper leaves the QR method open; Householder reflections are used
// because the sketch of a TEBD Theta is often rank deficient), the SVD of
// B = Q^H A of Sec. IV step ii (computed as B^H = Q_B R_B, then a one-sided
// Jacobi SVD of R_B^H, which keeps small singular values to high relative
// accuracy), and the discarded weight of Sec. II.C, Eq. (defdiscweigt),
// evaluated with the Frobenius identity of Sec. IV.
#include <cfloat>
#include <type_traits>

#include "kinds.hpp"

namespace tebd {

// --------------------------------------------------------------------------
// TEBD sweep planning: one thread per (chain, bond of the parity), problems
// numbered chain-major.  Chains that share a bond's gate form gate groups
// (up to kGateGroup consecutive chains; their problems nb apart): the
// group's Theta matrices sit side by side in one row-major block, and one
// gate product covers all their columns, reading the gate once per output
// tile instead of once per chain.  The Theta blocks are laid out bond-major.
//
// Columns chi_l chi_r of chain ch in its gate group (0 when its bond or
// local dimensions are out of range: such a problem is skipped, and has no
// columns in the group).
__device__ __forceinline__ int group_cols(const tebd_mps& mps, int ch, int bond) {
  const int32_t* chi = mps.chi + size_t(ch) * (mps.n_sites + 1);
  const int cl = chi[bond], cm = chi[bond + 1], cr = chi[bond + 2], cap = mps.chi_max;
  const int dl = mps.d[bond], dr = mps.d[bond + 1];
  const bool ok = cl >= 1 && cl <= cap && cm >= 1 && cm <= cap && cr >= 1 && cr <= cap &&
                  dl >= 1 && dl <= mps.d_max && dr >= 1 && dr <= mps.d_max;
  return ok ? cl * cr : 0;
}

__host__ __device__ __forceinline__ int qr_class(int rows, int l);

// Plan item t (the thread layout below) of a sweep: writes one descriptor.
// Called by whole wavefronts (the group sums are lane shuffles).
__device__ __forceinline__ void plan_item(int t, Prob* probs, int nprob, const tebd_mps& mps,
                                          const zt* gates, int64_t gate_chain_stride, int parity,
                                          int single_chain, int single_bond, int kcap, int p_over,
                                          char* slab_base, size_t slab_sz, int64_t mcap,
                                          int64_t ncap, int64_t lcap, int64_t lslab,
                                          int64_t npart_cap, double* disc, int32_t* status,
                                          double lambda_floor, int mixed, int adaptive, char* tape,
                                          size_t tape_stride, char* theta_base,
                                          size_t theta_stride, int chol) {
  // Items run group by group: a group's chains are the lanes of one aligned
  // kGateGroup-lane segment of a wavefront, so its column offsets are a
  // segmented prefix sum over the lanes.
  const int N = mps.n_sites, cap = mps.chi_max, dmax = mps.d_max;
  const int nb = (N - 1 - parity + 1) / 2;
  int chain, bond, bi = 0, p = 0;
  bool live;
  if (single_chain >= 0) {
    chain = single_chain;
    bond = single_bond;
    live = t == 0;
  } else {
    const int ncb = (mps.n_chains + kGateGroup - 1) / kGateGroup;
    const int g = t / kGateGroup;
    bi = g / ncb;
    chain = (g - bi * ncb) * kGateGroup + (t - g * kGateGroup);
    bond = parity + 2 * bi;
    live = bi < nb && chain < mps.n_chains;
    p = chain * nb + bi;
  }
  const int w = live ? group_cols(mps, chain, bond) : 0;
  int incl = w;
#pragma unroll
  for (int off = 1; off < kGateGroup; off <<= 1) {
    const int v = __shfl_up(incl, off, kGateGroup);
    if ((threadIdx.x & (kGateGroup - 1)) >= off) incl += v;
  }
  int gtot = __shfl(incl, kGateGroup - 1, kGateGroup), gcol0 = incl - w;
  // gate group: chains c0 .. c0 + gsz - 1 of this bond when they share the
  // gate, else this problem alone
  int c0 = chain, gsz = 1;
  if (single_chain < 0 && gate_chain_stride == 0) {
    c0 = chain / kGateGroup * kGateGroup;
    gsz = mps.n_chains - c0 < kGateGroup ? mps.n_chains - c0 : kGateGroup;
  } else {
    gcol0 = 0;
    gtot = w;
  }
  if (!live || p >= nprob) return;
  Prob P;
  const int32_t* chi = mps.chi + size_t(chain) * (N + 1);
  const int cl = chi[bond], cm = chi[bond + 1], cr = chi[bond + 2];
  const int dl = mps.d[bond], dr = mps.d[bond + 1];
  const bool bad = cl < 1 || cl > cap || cm < 1 || cm > cap || cr < 1 || cr > cap || dl < 1 ||
                   dl > dmax || dr < 1 || dr > dmax;
  P.chi_l = cl;
  P.chi_m = cm;
  P.chi_r = cr;
  P.dl = dl;
  P.dr = dr;
  P.m = dl * cl;
  P.n = dr * cr;
  int l2 = kcap + p_over;
  if (l2 > P.m) l2 = P.m;
  if (l2 > P.n) l2 = P.n;
  int k1 = kcap, l = l2;
  if (adaptive == 1 || adaptive == 2) {  // first stage: the current bond dimension plus a margin
    const int margin = (cm + 3) / 4 > 4 ? (cm + 3) / 4 : 4;
    k1 = cm + margin < kcap ? cm + margin : kcap;
    l = k1 + p_over;
    if (l > P.m) l = P.m;
    if (l > P.n) l = P.n;
  }
  P.ac_r = 0;
  P.ac_col = 0;
  P.ac_cap = l2;
  P.ac_grow = 0;
  P.chol_ok = 0;
  if (adaptive == 3) {  // Accuracy Check: from the current bond dimension, probes of p columns
    l = cm + p_over;
    if (l > P.m) l = P.m;
    if (l > P.n) l = P.n;
    P.ac_r = p_over < 1 ? 1 : (p_over > kAccMaxR ? kAccMaxR : p_over);
    P.ac_col = l;
    l2 = l;  // no second stage
  }
  P.l = bad ? 0 : l;
  P.k1 = k1;
  P.l1 = l;
  // the Gram-based QR (where the pipeline has it) for the large sketches
  P.chol = chol && !bad ? (qr_class(P.m, l) >= 2 ? 1 : 0) | (qr_class(P.n, l) >= 2 ? 2 : 0) : 0;
  P.l2 = l2;
  P.retry = 0;
  P.kcap = kcap;
  P.pid = chain * (N - 1) + bond;
  P.chi_new = 0;
  P.flags = bad ? TEBD_DEV_BAD_STATE : 0;
  P.npart = 0;
  P.mixed = mixed;
  P.om_ext = 0;
  P.frob2 = 0.0;
  carve_slab(P, slab_base + size_t(p) * slab_sz, mcap, ncap, lslab, 1, mixed, npart_cap);
  P.gcol0 = gcol0;
  P.gtot = gtot;
  P.gn = chain == c0 ? gsz : 0;
  P.gstride = nb;
  P.T = reinterpret_cast<zt*>(theta_base + (size_t(bi) * mps.n_chains + c0) * theta_stride);
  P.lda = P.n;
  P.ldom = P.l;
  P.U = nullptr;
  P.ldu = 0;
  P.S = nullptr;
  P.VH = nullptr;
  P.ldvh = 0;
  P.chi_out = nullptr;
  const size_t site_stride = size_t(dmax) * cap * cap;
  P.gk = mps.gamma ? reinterpret_cast<zt*>(mps.gamma) + (size_t(chain) * N + bond) * site_stride
                   : nullptr;
  P.gk1 = P.gk + site_stride;
  double* lam_chain = mps.lambda + size_t(chain) * (N - 1) * cap;
  P.lam_l = bond >= 1 ? lam_chain + size_t(bond - 1) * cap : nullptr;
  P.lam_mid = lam_chain + size_t(bond) * cap;
  P.lam_r = bond + 1 <= N - 2 ? lam_chain + size_t(bond + 1) * cap : nullptr;
  P.chi_slot = mps.chi + size_t(chain) * (N + 1) + bond + 1;
  // single-bond mode: `gates` is that bond's gate
  P.gate = single_chain >= 0 ? gates
                             : gates + size_t(chain) * gate_chain_stride +
                                   size_t(bond) * dmax * dmax * dmax * dmax;
  P.gate_ld = dmax * dmax;
  P.chi_cap = cap;
  P.lambda_floor = lambda_floor;
  if (tape) {
    tape_slot(tape + size_t(p) * tape_stride, mcap, lcap, P.tape_hdr, P.tape_sig, P.tape_u,
              P.tape_vh);
    P.tape_ldu = int32_t(lcap);
    P.tape_ldvh = int32_t(ncap);
  } else {
    P.tape_u = P.tape_vh = nullptr;
    P.tape_sig = nullptr;
    P.tape_hdr = nullptr;
    P.tape_ldu = P.tape_ldvh = 0;
  }
  if (single_chain >= 0) {
    P.disc = disc;
    P.status = status;
  } else {
    P.disc = disc + size_t(chain) * (N - 1) + bond;
    P.status = status + size_t(chain) * (N - 1) + bond;
  }
  probs[p] = P;
  if (bad) {
    *P.status = TEBD_DEV_BAD_STATE;
    *P.disc = 0.0;
  }
}

__global__ __launch_bounds__(64) void k_plan_sweep(
    Prob* probs, int nprob, tebd_mps mps, const zt* gates, int64_t gate_chain_stride, int parity,
    int single_chain, int single_bond, int kcap, int p_over, char* slab_base, size_t slab_sz,
    int64_t mcap, int64_t ncap, int64_t lcap, int64_t lslab, int64_t npart_cap, double* disc,
    int32_t* status, double lambda_floor, int mixed, int adaptive, char* tape, size_t tape_stride,
    int32_t* retry_count, char* theta_base, size_t theta_stride, int chol) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0 && retry_count) {
    *retry_count = 0;
    retry_count[kAccCountSlot] = 0;  // the Accuracy Check's two round counters
    retry_count[kAccCountSlot + 1] = 0;
    retry_count[kAccCountSlot + 2] = 0;  // and its widest pass
  }
  plan_item(t, probs, nprob, mps, gates, gate_chain_stride, parity, single_chain, single_bond,
            kcap, p_over, slab_base, slab_sz, mcap, ncap, lcap, lslab, npart_cap, disc, status,
            lambda_floor, mixed, adaptive, tape, tape_stride, theta_base, theta_stride, chol);
}

hipError_t launch_plan_sweep(Prob* probs, const Common& c, const tebd_mps& mps, const zt* gates,
                             int64_t gate_chain_stride, int32_t parity, int32_t single_chain,
                             int32_t single_bond, int32_t p_over, char* slab_base,
                             size_t slab_sz, double* disc, int32_t* status, double lambda_floor,
                             int32_t mixed, int32_t adaptive, char* tape, size_t tape_stride,
                             int32_t* retry_count, int64_t lslab, char* theta_base,
                             size_t theta_stride, hipStream_t s) {
  const int64_t mcap = int64_t(c.dmax) * c.chimax;
  const int64_t lcap = c.lmax;
  const int64_t npart_cap = gate_partials_cap(c.dmax * c.dmax, c.chimax * c.chimax);
  // one kGateGroup-lane segment per (bond, block of kGateGroup chains)
  int64_t items = 1;
  if (single_chain < 0) {
    const int64_t nb = c.nprob / mps.n_chains, ncb = (mps.n_chains + kGateGroup - 1) / kGateGroup;
    items = nb * ncb * kGateGroup;
  }
  static_assert(64 % kGateGroup == 0, "segments do not straddle wavefronts");
  TEBD_LAUNCH("k_plan_sweep", k_plan_sweep, dim3((items + 63) / 64), dim3(64), 0, s, probs,
              c.nprob, mps, gates, gate_chain_stride, parity, single_chain, single_bond, c.kcap,
              p_over, slab_base, slab_sz, mcap, mcap, lcap, lslab, npart_cap, disc, status,
              lambda_floor, mixed, adaptive, tape, tape_stride, retry_count, theta_base,
              theta_stride, c.chol);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// ||A||_F^2 for caller-supplied matrices (fixed summation order): workgroup
// (problem, slice) sums |A|^2 over its slice of rows (threads along the
// columns) into part[slice].  With the FP32 products it also writes the
// complex64 copy of A they read.
__global__ __launch_bounds__(256) void k_frob(Prob* probs) {
  __shared__ double red[4];
  const int pi = blockIdx.x / kFrobSlices, sl = blockIdx.x - pi * kFrobSlices;
  Prob& P = probs[pi];
  if (P.l == 0) return;
  const int rs = (P.m + kFrobSlices - 1) / kFrobSlices;
  const int r0 = sl * rs, r1 = r0 + rs < P.m ? r0 + rs : P.m;
  double s = 0.0;
  for (int r = r0; r < r1; ++r) {
    const zt* row = P.A + size_t(r) * P.lda;
    float2* rowf = P.Af ? P.Af + size_t(r) * P.n : nullptr;
    for (int c = threadIdx.x; c < P.n; c += 256) {
      const zt v = row[c];
      s += zabs2(v);
      if (rowf) rowf[c] = make_float2(float(v.x), float(v.y));
    }
  }
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) P.part[sl] = s;
}

hipError_t launch_frob(Prob* probs, const Common& c, hipStream_t s) {
  TEBD_LAUNCH("k_frob", k_frob, dim3(c.nprob * kFrobSlices), dim3(256), 0, s, probs);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Householder QR of a rows x l column-major matrix (ld = rows), in place,
// followed by the explicit thin Q (backward accumulation).  Reflector j is
// H_j = I - 2 u u^H with ||u|| = 1, u supported on rows >= j, chosen so that
// H_j x = beta e_j with beta = -phase(x_j) ||x||; a zero column gives H_j = I.
// With want_r the l x l upper factor (column-major) is written to P.Rb first.
//
// qr_core serves the two larger size classes: problems with
// (l + 2) rows <= kLdsElems keep the whole matrix in LDS; larger ones work
// on the matrix in global memory (L2-resident) with one wavefront per
// trailing column, the column held in registers between its dot product and
// its update when it has at most 64 * kRegRows rows left.  The small
// problems that dominate a TEBD sweep run register-resident (k_qr_reg).
constexpr int kLdsElems = 9600;  // complex elements of LDS a workgroup may claim (150 KiB)
constexpr int kRegRows = 16;

// y_c[j0..rows) -= 2 u (u^H y_c) for one column, by one wavefront.  Rows
// below `skip` are treated as zero on input (they held R entries).
template <int REG>
__device__ __forceinline__ void reflect_column(const zt* __restrict__ u, zt* yc, int j0, int skip,
                                               int rows, int lane, double* nrm_out = nullptr) {
  double nn = 0.0;  // sum |y_c[r]|^2 over r > j0 after the update
  const int nr = rows - j0;
  double dr = 0.0, di = 0.0;
  if (REG > 0 && nr <= 64 * REG) {
    zt cache[REG > 0 ? REG : 1];
#pragma unroll
    for (int i = 0; i < REG; ++i) {
      const int r = j0 + lane + 64 * i;
      cache[i] = (r < rows && r >= skip) ? yc[r] : make_double2(0.0, 0.0);
      if (r < rows) {
        const zt t = zcmul(u[r], cache[i]);
        dr += t.x;
        di += t.y;
      }
    }
    dr = wave_sum(dr);
    di = wave_sum(di);
    const zt d2 = make_double2(2.0 * dr, 2.0 * di);
#pragma unroll
    for (int i = 0; i < REG; ++i) {
      const int r = j0 + lane + 64 * i;
      if (r < rows) {
        const zt v = zsub(cache[i], zmul(u[r], d2));
        yc[r] = v;
        if (r > j0) nn += zabs2(v);
      }
    }
  } else {
    for (int r = j0 + lane; r < rows; r += 64) {
      if (r < skip) continue;
      const zt t = zcmul(u[r], yc[r]);
      dr += t.x;
      di += t.y;
    }
    dr = wave_sum(dr);
    di = wave_sum(di);
    const zt d2 = make_double2(2.0 * dr, 2.0 * di);
    for (int r = j0 + lane; r < rows; r += 64) {
      const zt old = r < skip ? make_double2(0.0, 0.0) : yc[r];
      const zt v = zsub(old, zmul(u[r], d2));
      yc[r] = v;
      if (r > j0) nn += zabs2(v);
    }
  }
  if (nrm_out) {
    nn = wave_sum(nn);
    if (lane == 0) *nrm_out = nn;
  }
}

// Pivot order key of a remaining column: larger for a larger trailing norm
// v; norms that agree to 2^-36 relative count as equal, and then the lower
// position wins.  0 (no candidate) for a NaN norm.  The low byte carries a
// payload (the group of the register QR).  One 64-bit maximum picks the
// pivot, and the norm it returns is v to 2^-36 relative.
__device__ __forceinline__ unsigned long long pivot_key(double v, int pos, int payload) {
  if (!(v >= 0.0)) return 0ull;
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  return (1ull << 63) | (b & 0x7FFFFFFFFFFF0000ull) |
         (static_cast<unsigned long long>(255 - pos) << 8) | static_cast<unsigned>(payload);
}
__device__ __forceinline__ double pivot_key_norm(unsigned long long k) {
  return __longlong_as_double(static_cast<long long>(k & 0x7FFFFFFFFFFF0000ull));
}
__device__ __forceinline__ int pivot_key_pos(unsigned long long k) {
  return 255 - static_cast<int>((k >> 8) & 0xff);
}
__device__ __forceinline__ unsigned long long key_max(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ unsigned long long key_dpp(unsigned long long k) {
  return static_cast<unsigned long long>(
      __double_as_longlong(dpp_move<CTRL, ROW_MASK>(__longlong_as_double(static_cast<long long>(k)))));
}
// Wavefront maximum of keys (uniform result): the row steps of
// wave_max_nonneg, masked-off rows reading 0 (no candidate).
__device__ __forceinline__ unsigned long long key_wave_max(unsigned long long k) {
  k = key_max(k, key_dpp<0xb1>(k));
  k = key_max(k, key_dpp<0x4e>(k));
  k = key_max(k, key_dpp<0x141>(k));
  k = key_max(k, key_dpp<0x140>(k));
  k = key_max(k, key_dpp<0x142, 0xa>(k));
  k = key_max(k, key_dpp<0x143, 0xc>(k));
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(k & 0xffffffffu), 63));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(k >> 32), 63));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}
__device__ __forceinline__ unsigned long long key_max_xor(unsigned long long k, int off) {
  const double o = __shfl_xor(__longlong_as_double(static_cast<long long>(k)), off, 64);
  const unsigned long long ok = static_cast<unsigned long long>(__double_as_longlong(o));
  return ok > k ? ok : k;
}

// Column pivoting for the range-finder QRs of Alg. 1: before step j the
// remaining column with the largest trailing norm (pivot_key order) is
// swapped into place, and the factorisation stops at the first j >= 1 whose
// pivot norm |R_jj| is <= kRankTol |R_00|.  The kept rank r replaces the
// sketch width l of the problem, so later products and the small SVD work on
// the numerical range only.
//
// Work split: column c belongs to wavefront c mod NW.  Step j is prepared by
// the owner of column j alone (pivot search, swap, reflector), published in
// a double-buffered LDS vector, and applied by every wavefront to its own
// trailing columns, which also yields their new trailing norms (double-
// buffered, so the next pivot search reads a stable copy).  One barrier per
// step, two with pivoting; the thin Q is accumulated the same way backwards.
constexpr double kRankTol = 1e-13;

template <int NT, int REG>
__device__ __forceinline__ int qr_core(zt* Y, int rows, int l, zt* u_s /* 2 * rows */,
                                       zt* rdiag, zt* Rb, bool piv, bool allow_stop,
                                       int32_t* perm /* l, or nullptr */,
                                       double* nrm /* 2 * kMaxL */, int* sh_i) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = NT / 64;
  int rank = l;
  double best00 = 0.0;  // squared pivot norm of step 0
  if (piv) {
    for (int c = wave; c < l; c += NW) {
      double s = 0.0;
      for (int r = lane; r < rows; r += 64) s += zabs2(Y[size_t(c) * rows + r]);
      s = wave_sum(s);
      if (lane == 0) nrm[c] = s;
    }
  }
  for (int j = 0; j < l; ++j) {
    double* ncur = nrm + (j & 1) * kMaxL;
    double* nnext = nrm + ((j + 1) & 1) * kMaxL;
    zt* u = u_s + (j & 1) * rows;
    if (piv) __syncthreads();  // trailing norms of step j-1 are complete
    if (wave == (j % NW)) {
      int stop = 0;
      if (piv) {
        unsigned long long bk = 0ull;
        for (int c = j + lane; c < l; c += 64) {
          const unsigned long long k = pivot_key(ncur[c], c, 0);
          bk = k > bk ? k : bk;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) bk = key_max_xor(bk, off);
        const int bi = bk ? pivot_key_pos(bk) : j;
        const double best = pivot_key_norm(bk);  // |R_jj|^2 to 2^-36
        if (j == 0) best00 = best;
        if (allow_stop && j > 0 && !(best > kRankTol * kRankTol * best00)) stop = 1;
        if (!stop && bi != j) {
          zt* ya = Y + size_t(j) * rows;
          zt* yb = Y + size_t(bi) * rows;
          for (int r = lane; r < rows; r += 64) {
            const zt t = ya[r];
            ya[r] = yb[r];
            yb[r] = t;
          }
          if (perm && lane == 0) {
            const int32_t t = perm[j];
            perm[j] = perm[bi];
            perm[bi] = t;
          }
        }
      }
      if (!stop) {
        zt* yj = Y + size_t(j) * rows;
        double s = 0.0;
        for (int r = j + 1 + lane; r < rows; r += 64) s += zabs2(yj[r]);
        s = wave_sum(s);
        const zt alpha = yj[j];
        const double aa = sqrt(zabs2(alpha));
        const double xnorm = sqrt(aa * aa + s);
        zt beta = make_double2(0.0, 0.0), v0 = make_double2(0.0, 0.0);
        double vinv = 0.0;  // 1 / ||x - beta e_j||
        if (xnorm > 0.0) {
          const zt ph = aa > 0.0 ? zscale(alpha, 1.0 / aa) : make_double2(1.0, 0.0);
          beta = zscale(ph, -xnorm);
          v0 = zsub(alpha, beta);
          vinv = 1.0 / sqrt(2.0 * xnorm * (xnorm + aa));
        }
        for (int r = j + lane; r < rows; r += 64) {
          const zt uu = zscale(r == j ? v0 : yj[r], vinv);
          u[r] = uu;
          yj[r] = uu;
        }
        if (lane == 0) rdiag[j] = beta;
      }
      if (lane == 0) sh_i[j & 1] = stop;
    }
    __syncthreads();  // reflector j (or the stop decision) is published
    if (sh_i[j & 1]) {
      rank = j;
      break;
    }
    for (int c = j + 1 + ((wave - (j + 1) % NW + NW) % NW); c < l; c += NW)
      reflect_column<REG>(u, Y + size_t(c) * rows, j, j, rows, lane, piv ? nnext + c : nullptr);
  }
  __syncthreads();
  if (Rb) {
    for (int e = tid; e < rank * rank; e += NT) {
      const int c = e / rank, i = e - c * rank;
      zt v;
      if (i < c)
        v = Y[size_t(c) * rows + i];
      else if (i == c)
        v = rdiag[c];
      else
        v = make_double2(0.0, 0.0);
      Rb[e] = v;
    }
    __syncthreads();
  }
  // Q = H_0 H_1 ... H_{r-1} [I; 0], accumulated from the last reflector: the
  // owner of column j publishes u_j and turns its column into H_j e_j, then
  // every wavefront applies H_j to its columns c > j (row j treated as 0).
  for (int j = rank - 1; j >= 0; --j) {
    zt* u = u_s + (j & 1) * rows;
    if (wave == (j % NW)) {
      zt* yj = Y + size_t(j) * rows;
      for (int r = j + lane; r < rows; r += 64) u[r] = yj[r];
      const zt uj = yj[j];
      for (int r = lane; r < rows; r += 64) {
        zt v = make_double2(0.0, 0.0);
        if (r >= j) {
          v = zscale(zmul(r == j ? uj : yj[r], zconj(uj)), -2.0);
          if (r == j) v.x += 1.0;
        }
        yj[r] = v;
      }
    }
    __syncthreads();
    for (int c = j + 1 + ((wave - (j + 1) % NW + NW) % NW); c < rank; c += NW)
      reflect_column<REG>(u, Y + size_t(c) * rows, j, j + 1, rows, lane);
  }
  __syncthreads();
  return rank;
}

// Column kernels over the strided rows r0, r0 + G, ... < rows, four rows per
// iteration with independent partial sums, so that the LDS loads of four
// rows are in flight together instead of one load latency per row.
__device__ __forceinline__ zt col_dot(const zt* u, const zt* y, int r0, int rows, int G) {
  double a0 = 0.0, b0 = 0.0, a1 = 0.0, b1 = 0.0, a2 = 0.0, b2 = 0.0, a3 = 0.0, b3 = 0.0;
  int r = r0;
  for (; r + 3 * G < rows; r += 4 * G) {
    const zt u0 = u[r], u1 = u[r + G], u2 = u[r + 2 * G], u3 = u[r + 3 * G];
    const zt y0 = y[r], y1 = y[r + G], y2 = y[r + 2 * G], y3 = y[r + 3 * G];
    zdot_acc(u0, y0, a0, b0);
    zdot_acc(u1, y1, a1, b1);
    zdot_acc(u2, y2, a2, b2);
    zdot_acc(u3, y3, a3, b3);
  }
  for (; r < rows; r += G) zdot_acc(u[r], y[r], a0, b0);
  return make_double2((a0 + a1) + (a2 + a3), (b0 + b1) + (b2 + b3));
}

__device__ __forceinline__ double col_norm2(const zt* y, int r0, int rows, int G) {
  double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0;
  int r = r0;
  for (; r + 3 * G < rows; r += 4 * G) {
    n0 += zabs2(y[r]);
    n1 += zabs2(y[r + G]);
    n2 += zabs2(y[r + 2 * G]);
    n3 += zabs2(y[r + 3 * G]);
  }
  for (; r < rows; r += G) n0 += zabs2(y[r]);
  return (n0 + n1) + (n2 + n3);
}

// A problem a gated QR launch leaves alone: gate 1 runs only the bases the
// Accuracy Check grew; gate 2 only what the Gram-based QR did not finish.
__device__ __forceinline__ bool qr_gated(const Prob& P, int gate) {
  return (gate == 1 && !P.ac_grow) || (gate == 2 && P.chol_ok);
}

// Size classes of the batched QR, by (rows, l): 0 and 1 are register-
// resident (512 threads with 8 rows per lane, 1024 threads with 12), 2 keeps
// the matrix in LDS (1024 threads), 3 works on global memory.  The class
// index never decreases when rows or l grow, so a box of sizes
// [rmin, rmax] x [lmin, lmax] reaches exactly the classes between
// qr_class(rmin, lmin) and qr_class(rmax, lmax).
constexpr int kRegGroupMax = 32;  // lanes per column of the register classes

__host__ __device__ __forceinline__ int reg_group(int nt, int l) {
  int lp2 = 1;
  while (lp2 < l) lp2 <<= 1;
  const int g = nt / lp2;
  return g > kRegGroupMax ? kRegGroupMax : g;
}

__host__ __device__ __forceinline__ bool qr_reg_fits(int nt, int rpl, int rows, int l) {
  if (l < 1 || l > kMaxL) return false;
  const int g = reg_group(nt, l);
  return g >= 1 && rows <= g * rpl;
}

__host__ __device__ __forceinline__ int qr_class(int rows, int l) {
  if (qr_reg_fits(512, 8, rows, l)) return 0;
  if (qr_reg_fits(1024, 12, rows, l)) return 1;
  if (int64_t(l + 2) * rows <= kLdsElems) return 2;
  return 3;
}

// Register-resident QR.  Column c of the rows x l matrix belongs to a group
// of G lanes (G = NT / l rounded up to a power of two, at most 32, so a
// group never straddles wavefronts); lane h of the group keeps rows h,
// h + G, ... of the column in registers.  Dot products, updates and
// trailing norms of a column are register arithmetic plus a DPP sum over
// the group; only the reflector is broadcast through LDS, where all groups
// read the same G addresses at a time.  The reflector buffer holds zeros
// outside the reflector's rows, so the row loops run without branches (their
// LDS loads overlap) and rows outside [j, rows) are left exactly unchanged.
//
// Columns never move.  Pivoting picks the unfactored group first in
// pivot_key order, over the positions the swaps of qr_core would have
// produced (each group tracks its own): every trailing group posts its key
// in LDS, and after the barrier each wavefront takes their maximum.  The
// pivot group is recorded as logical column j; R, the pivot order and the
// thin Q are written out in logical order.  Same reflectors (stored
// unnormalised), pivoting rule and rank tolerance as qr_core.
// With pivoting, two barriers per factorisation step (trailing norms,
// reflector); without, one.  Every reflector keeps an LDS slot of its own
// when they all fit (always for 512 threads x 8 rows), and then each group
// accumulates its column of Q with no barrier at all; otherwise two
// alternating buffers serve, and the backward accumulation takes one
// barrier per step.
template <int RPL>
struct RegQrShared {
  // rows x l elements always fit for 512 x 8; 144 KiB for 1024 x 12
  static constexpr int kBuf = RPL <= 8 ? 4096 : 9216;
  zt buf[kBuf];  // reflector slots (zero outside the reflector's rows)
  zt rdiag[kMaxL];
  double tau_s[kMaxL];              // tau of each reflector (H = I - tau v v^H)
  unsigned long long key_s[kMaxL];  // pivot key of each group; 0 once pivoted
  int32_t piv_grp[kMaxL];
};

// The body for one group width G and RPL rows per lane (compile-time
// constants, so the row offsets of the register loops are immediates; RPL
// may be below the class's RS when the rows fit, which shortens every
// register loop); SLOTS: every reflector keeps its own slot
// (G * RPL * l <= RegQrShared<RS>::kBuf); PIV: column pivoting.
template <int NT, int RPL, int G, bool SLOTS, bool PIV, int RS>
__device__ __forceinline__ void qr_reg_body(Prob& P, int rows, int l, zt* Yg, int want_r,
                                            RegQrShared<RS>& sh) {
  constexpr bool piv = PIV;
  constexpr int UST = G * RPL;               // rows a group can hold
  constexpr int KEEP = RPL <= 8 ? RPL : 1;  // reflector rows kept in registers
  auto& rdiag = sh.rdiag;
  auto& key_s = sh.key_s;
  auto& piv_grp = sh.piv_grp;
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = tid / G, h = tid - g * G;
  const bool have = g < l;
  // the QR of B^H keeps every column; without pivoting no rank is revealed
  const bool allow_stop = piv && !want_r;
  const zt zero = make_double2(0.0, 0.0);
  // reflector j: slot j, or the alternating buffers
  constexpr bool slots = SLOTS;
  auto slot = [&](int j) { return sh.buf + (slots ? j : (j & 1)) * UST; };
  zt y[RPL];
  double nn = 0.0;
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = h + G * i;
    y[i] = zload_if(have && r < rows, Yg + size_t(g) * rows + r);
    nn += zabs2(y[i]);
  }
  nn = group_sum(nn, G);
  for (int c = tid; c < l; c += NT) piv_grp[c] = c;
  if (piv && have && h == 0) key_s[g] = pivot_key(nn, g, g);
  __syncthreads();
  // trailing norm (rows >= the next step) and position of this group
  double my_tn = nn;
  int my_pos = g;
  int mine = kMaxL;  // logical column of this group once it has been the pivot
  // Reflectors are kept unnormalised, H_j = I - tau_j v v^H with
  // v = x - beta e_j (x: the column at step j, zero above row j) and
  // tau_j = 2 / ||v||^2 = 1 / (||x|| (||x|| + |x_j|)): rows > j of v are the
  // column itself, so they are written before beta and tau are known.  The
  // group of logical column j keeps x unscaled in its registers and v_j, tau_j
  // in my_v0, my_tau.
  double my_tau = 0.0;
  zt my_v0 = zero;
  // rows > j of v into buffer ub, zeros elsewhere in the group's range (so no
  // earlier reflector survives in the buffer)
  auto write_v = [&](zt* ub, int j) {
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const bool on = h + G * i > j && h + G * i < rows;
      zt w;
      w.x = on ? y[i].x : 0.0;
      w.y = on ? y[i].y : 0.0;
      ub[h + G * i] = w;
    }
  };
  // The rest of reflector j from the column of group p (pn = ||column p,
  // rows >= j||), called by the whole group p after write_v: row j of v,
  // tau_j and R_jj = beta.
  auto finish_reflector = [&](int j, int p, double pn, zt* ub) {
    // row j sits in register j / G of the group's lane j % G (uniform)
    const int i0 = j / G, hj = j - i0 * G, lj = (p * G + hj) & 63;
    double ax = 0.0, ay = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i)
      if (i == i0) {
        ax = read_lane(y[i].x, lj);
        ay = read_lane(y[i].y, lj);
      }
    const zt alpha = make_double2(ax, ay);
    const double a2 = zabs2(alpha);
    const double ia = a2 > 0.0 ? rsqrt(a2) : 0.0;  // 1 / |alpha|
    const double aa = a2 * ia;
    const double xnorm = pn;
    zt beta = zero, v0 = zero;
    double tau = 0.0;
    if (xnorm > 0.0) {
      const zt ph = aa > 0.0 ? zscale(alpha, ia) : make_double2(1.0, 0.0);
      beta = zscale(ph, -xnorm);
      v0 = zsub(alpha, beta);
      tau = 1.0 / (xnorm * (xnorm + aa));
    }
    if (h == hj) ub[j] = v0;
    if (h == 0) {
      rdiag[j] = beta;
      sh.tau_s[j] = tau;
    }
    my_tau = tau;
    my_v0 = v0;
    mine = j;
  };
  auto reflector = [&](int j, int p, double pn, zt* ub) {
    write_v(ub, j);
    finish_reflector(j, p, pn, ub);
  };
  // trailing column: y -= tau_j v (v^H y) with v in ub, zero outside its
  // rows; with want_norm (uniform over the wavefront) the norm of rows > j is
  // returned (else 0); with vout (the next reflector's group) rows > j + 1 of
  // the updated column are written there as the next v, before the norm is
  // reduced
  auto apply = [&](const zt* ub, int j, bool want_norm, zt* vout) {
    const double tau = sh.tau_s[j];
    zt uu[KEEP];  // v kept in registers between the two loops when they fit
    double dr0 = 0.0, di0 = 0.0, dr1 = 0.0, di1 = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const zt u = ub[h + G * i];
      if (i < KEEP) uu[i < KEEP ? i : 0] = u;
      if (i & 1)
        zdot_acc(u, y[i], dr1, di1);
      else
        zdot_acc(u, y[i], dr0, di0);
    }
    const double dr = group_sum(dr0 + dr1, G), di = group_sum(di0 + di1, G);
    const zt d2 = make_double2(tau * dr, tau * di);
    // without the kept copy, the second read of u must not be hoisted
    // above this point (it would hold every row twice in registers)
    if (KEEP < RPL) __builtin_amdgcn_sched_barrier(0);
    double tn = 0.0;
    if (want_norm) {
      double tn0 = 0.0, tn1 = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = h + G * i;
        const zt u = i < KEEP ? uu[i < KEEP ? i : 0] : ub[r];
        y[i] = zsub_mul(y[i], u, d2);
        const double yx = r > j ? y[i].x : 0.0, yy = r > j ? y[i].y : 0.0;
        if (i & 1)
          tn1 = fma(yx, yx, fma(yy, yy, tn1));
        else
          tn0 = fma(yx, yx, fma(yy, yy, tn0));
      }
      if (vout) write_v(vout, j + 1);
      tn = group_sum(tn0 + tn1, G);
    } else {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const zt u = i < KEEP ? uu[i < KEEP ? i : 0] : ub[h + G * i];
        y[i] = zsub_mul(y[i], u, d2);
      }
    }
    return tn;
  };
  int rank = l;
  if constexpr (!piv) {
    // Logical column j is group j, which builds reflector j as soon as its
    // own update by reflector j - 1 is done (with its trailing norm summed
    // in the same pass), while the other groups are still applying j - 1;
    // reflector j + 1 goes to another slot or buffer than reflector j, so
    // one barrier per step suffices.
    if (g == 0) reflector(0, 0, sqrt(nn), slot(0));
    __syncthreads();
    for (int j = 0; j + 1 < l; ++j) {
      if (have && g > j) {
        // the wavefront that holds group j + 1 sums trailing norms
        const bool lead = (tid >> 6) == (((j + 1) * G) >> 6);
        const double tn = apply(slot(j), j, lead, g == j + 1 ? slot(j + 1) : nullptr);
        if (g == j + 1) finish_reflector(j + 1, g, sqrt(tn), slot(j + 1));
      }
      __syncthreads();  // reflector j + 1 is published; reflector j is read
    }
  }
  double best00 = 0.0;  // squared pivot norm of step 0
  for (int j = 0; piv && j < l; ++j) {
    unsigned long long key = 0ull;
    for (int c = lane; c < l; c += 64) key = key_max(key, key_s[c]);
    key = key_wave_max(key);
    if (key == 0ull) {  // only NaN norms left: stop here
      rank = j;
      break;
    }
    const int p = static_cast<int>(key & 0xff), pp = pivot_key_pos(key);
    const double best = pivot_key_norm(key);  // |R_jj|^2 to 2^-36
    if (j == 0) best00 = best;
    if (allow_stop && j > 0 && !(best > kRankTol * kRankTol * best00)) {
      rank = j;
      break;
    }
    if (g == p) reflector(j, p, sqrt(my_tn), slot(j));
    __syncthreads();  // reflector j is published; every key read is done
    if (tid == 0) piv_grp[j] = p;
    if (have && mine == kMaxL) {
      if (my_pos == j) my_pos = pp;  // the swap of qr_core moves it to the pivot's place
      my_tn = apply(slot(j), j, true, nullptr);
      if (h == 0) key_s[g] = pivot_key(my_tn, my_pos, g);
    }
    if (g == p && h == 0) key_s[g] = 0ull;
    __syncthreads();  // the keys of step j + 1 are in
  }
  if (want_r) {
    if (have && mine < rank) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = h + G * i;
        if (r < rank) {  // value selects only (no select between addresses)
          const zt d = rdiag[r];
          const bool up = r < mine, dg = r == mine;
          zt v;
          v.x = up ? y[i].x : (dg ? d.x : 0.0);
          v.y = up ? y[i].y : (dg ? d.y : 0.0);
          P.Rb[size_t(mine) * rank + r] = v;
        }
      }
    }
    for (int c = tid; c < rank; c += NT) P.piv[c] = piv_grp[c];
  }
  // Q = H_0 ... H_{r-1} [I; 0]: the group of logical column c < rank starts
  // from H_c e_c = e_c - tau_c v_c conj(v_c[c]) and applies H_{c-1}, ..., H_0.
  // With a slot per reflector the groups need no barrier.  With the
  // alternating buffers, the group of column j publishes v_j one step
  // ahead, while H_{j+1} is being applied (column j is not touched by H_j or
  // later reflectors): one barrier per step.
  auto start_q = [&](zt* ub) {  // by the group with mine < rank; ub: publish v_c there
    const int c = mine, i0 = c / G, hc = c - i0 * G;
    // -tau_c conj(v_c[c])
    const zt m = make_double2(-my_tau * my_v0.x, my_tau * my_v0.y);
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const bool on = h + G * i > c && h + G * i < rows;
      zt w;
      w.x = on ? y[i].x : 0.0;
      w.y = on ? y[i].y : 0.0;
      if (ub) ub[h + G * i] = w;  // zeros outside [c, rows)
      y[i] = zmul(w, m);
    }
    if (ub && h == hc) ub[c] = my_v0;
#pragma unroll
    for (int i = 0; i < RPL; ++i)
      if (i == i0 && h == hc) {
        y[i] = zmul(my_v0, m);
        y[i].x += 1.0;
      }
  };
  if constexpr (slots) {
    // Every reflector keeps its slot, so any group can accumulate any column,
    // and column c costs c applications.  The columns go out in blocks of the
    // 64 / G groups of a wavefront, costliest block first, dealt to the four
    // SIMDs back and forth (SIMD 0 1 2 3 3 2 1 0 0 1 ..., wavefront w on SIMD
    // w mod 4, the k-th block of a SIMD to its k-th wavefront), so that the
    // SIMDs carry similar sums.  The start H_c e_c comes from slot c: its
    // rows > c are the column as it was when reflector c was built, row c
    // holds v_c[c].  The same operations, in the same order, as when the
    // group of column c accumulates it.
    constexpr int GPW = 64 / G;
    const int nblk = (rank + GPW - 1) / GPW;
    const int wv = tid >> 6, kq = wv >> 2, sq = wv & 3;
    const int dq = 4 * kq + ((kq & 1) ? 3 - sq : sq);  // deal position of this wavefront
    const int qc = dq < nblk ? (nblk - 1 - dq) * GPW + g % GPW : rank;
    if (qc < rank) {
      const zt* vs = slot(qc);
      const zt v0 = vs[qc];
      const double tau = sh.tau_s[qc];
      const zt m = make_double2(-tau * v0.x, tau * v0.y);  // -tau_c conj(v_c[c])
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = h + G * i;
        y[i] = zmul(zload_if(r > qc && r < rows, vs + r), m);
        if (r == qc) {
          y[i] = zmul(v0, m);
          y[i].x += 1.0;
        }
      }
      for (int j = qc - 1; j >= 0; --j) apply(slot(j), j, false, nullptr);
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = h + G * i;
        if (r < rows) Yg[size_t(qc) * rows + r] = y[i];
      }
    }
  } else {
    if (rank > 0 && mine == rank - 1) start_q(slot(rank - 1));
    for (int j = rank - 1; j >= 0; --j) {
      __syncthreads();  // v_j is published; the reads of the other buffer are done
      if (j > 0 && mine == j - 1) start_q(slot(j - 1));
      if (have && mine > j && mine < rank) apply(slot(j), j, false, nullptr);
    }
    if (have && mine < rank) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = h + G * i;
        if (r < rows) Yg[size_t(mine) * rows + r] = y[i];
      }
    }
  }
  if (tid == 0) P.l = rank;
}

template <int NT, int RPL, bool PIV>
__global__ __launch_bounds__(NT) void k_qr_reg(Prob* probs, int which, int want_r, int cls,
                                                 int gate) {
  __shared__ RegQrShared<RPL> sh;
  Prob& P = probs[blockIdx.x];
  const int l = P.l;
  const int rows = which ? P.n : P.m;
  // class from the width the pass started with: P.l shrinks as QRs run
  if (l == 0 || qr_class(rows, P.l1) != cls || qr_gated(P, gate)) return;
  zt* Yg = which ? P.Yt : P.Y;
  // l <= kMaxL, so G >= NT / kMaxL
  static_assert(NT / kMaxL >= 2, "group widths below 2 are not instantiated");
  const int G = reg_group(NT, l);
  auto run = [&](auto gc) {
    constexpr int GC = decltype(gc)::value, HALF = RPL / 2;
    // the revealed rank of the later QRs of a pass is often below the width
    // that set the class: G doubles, and half the rows per lane may do
    if (rows <= GC * HALF) {
      // G * HALF * l <= NT * HALF <= kBuf: every reflector has its slot
      static_assert(NT * HALF <= RegQrShared<RPL>::kBuf, "slots for the half-height body");
      qr_reg_body<NT, HALF, GC, true, PIV>(P, rows, l, Yg, want_r, sh);
    } else if (RPL <= 8 || GC * RPL * l <= RegQrShared<RPL>::kBuf) {
      // 512 x 8: G * 8 * l <= 4096 for every l (G * l <= 512, or G = 32 and l <= 16)
      qr_reg_body<NT, RPL, GC, true, PIV>(P, rows, l, Yg, want_r, sh);
    } else {
      qr_reg_body<NT, RPL, GC, (RPL <= 8), PIV>(P, rows, l, Yg, want_r, sh);
    }
  };
  if (G == 32)
    run(std::integral_constant<int, 32>());
  else if (G == 16)
    run(std::integral_constant<int, 16>());
  else if (G == 8)
    run(std::integral_constant<int, 8>());
  else if (NT / kMaxL <= 4 && G == 4)
    run(std::integral_constant<int, (NT / kMaxL <= 4 ? 4 : 8)>());
  else if (NT / kMaxL <= 2)
    run(std::integral_constant<int, (NT / kMaxL <= 2 ? 2 : 8)>());
}

// Class 2, (l + 2) * rows <= kLdsElems beyond the register classes:
// qr_core's column ownership with 1024 threads (one wavefront per column at
// a time), the matrix in up to 150 KiB of LDS.
template <int NT>
__global__ __launch_bounds__(NT) void k_qr_lds(Prob* probs, int which, int want_r, int pivot,
                                                 int gate) {
  extern __shared__ zt lds[];  // rows * l matrix, then 2 * rows for u
  __shared__ zt rdiag[kMaxL];
  Prob& P = probs[blockIdx.x];
  const int l = P.l;
  const int rows = which ? P.n : P.m;
  if (l == 0 || qr_class(rows, P.l1) != 2 || qr_gated(P, gate)) return;
  __shared__ double nrm[2 * kMaxL];
  __shared__ int sh_i[2];
  zt* Yg = which ? P.Yt : P.Y;
  const int tot = rows * l;
  for (int e = threadIdx.x; e < tot; e += NT) lds[e] = Yg[e];
  __syncthreads();
  __shared__ int32_t perm_s[kMaxL];
  for (int c = threadIdx.x; c < l; c += NT) perm_s[c] = c;
  __syncthreads();
  const int rank = qr_core<NT, 0>(lds, rows, l, lds + tot, rdiag, want_r ? P.Rb : nullptr,
                                  pivot != 0, pivot != 0 && !want_r, want_r ? perm_s : nullptr, nrm,
                                  sh_i);
  if (want_r)
    for (int c = threadIdx.x; c < l; c += NT) P.piv[c] = perm_s[c];
  const int keep = rows * rank;
  for (int e = threadIdx.x; e < keep; e += NT) Yg[e] = lds[e];
  if (threadIdx.x == 0) P.l = rank;
}

// Class 3, everything larger, runs on global memory (L2-resident) with
// 1024 threads, qr_core's column ownership, and each column held in
// registers between its dot product and its update.
// The two reflector buffers live in LDS up to kGlbLdsRows rows (147 KiB)
// and in the problem's slab beyond.
constexpr int kGlbLdsRows = 4608;

template <int NT>
__global__ __launch_bounds__(NT) void k_qr_glb(Prob* probs, int which, int want_r, int pivot,
                                                 int gate) {
  extern __shared__ zt u_lds[];  // 2 * min(rows, kGlbLdsRows)
  __shared__ zt rdiag[kMaxL];
  Prob& P = probs[blockIdx.x];
  const int l = P.l;
  const int rows = which ? P.n : P.m;
  if (l == 0 || qr_class(rows, P.l1) != 3 || qr_gated(P, gate)) return;
  zt* u_s = rows <= kGlbLdsRows ? u_lds : P.qru;
  __shared__ double nrm[2 * kMaxL];
  __shared__ int sh_i[2];
  __shared__ int32_t perm_s[kMaxL];
  for (int c = threadIdx.x; c < l; c += NT) perm_s[c] = c;
  __syncthreads();
  const int rank = qr_core<NT, kRegRows>(which ? P.Yt : P.Y, rows, l, u_s, rdiag,
                                         want_r ? P.Rb : nullptr, pivot != 0,
                                         pivot != 0 && !want_r, want_r ? perm_s : nullptr, nrm,
                                         sh_i);
  if (want_r)
    for (int c = threadIdx.x; c < l; c += NT) P.piv[c] = perm_s[c];
  if (threadIdx.x == 0) P.l = rank;
}

// --------------------------------------------------------------------------
// The size classes of one batched factorisation touch disjoint problems and
// each fills only a few waves per CU, so they run side by side: the first
// class on the caller's stream, the others on side streams (default
// priority) forked from it and joined back with events.  Side streams and
// events are per host thread and device, created on first use.
namespace {
constexpr int kSide = 3;
struct SideStreams {
  bool ready = false;
  hipStream_t st[kSide];
  hipEvent_t fork, join[kSide];
};

hipError_t side_streams(SideStreams*& out) {
  static thread_local SideStreams tab[16];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 16) {
    out = nullptr;
    return hipSuccess;
  }
  SideStreams& ss = tab[dev];
  if (!ss.ready) {
    e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming);
    for (int i = 0; i < kSide && e == hipSuccess; ++i) {
      e = hipStreamCreateWithFlags(&ss.st[i], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ss.join[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) return e;
    ss.ready = true;
  }
  out = &ss;
  return hipSuccess;
}

// Run launches[0..n) (each a callable taking a stream) concurrently after
// everything already enqueued on s; s continues after all of them.  Small
// batches, and the second pass of the adaptive rank (which re-runs only the
// few rejected problems), run them in order on s: there the fork and join
// cost more than the overlap gains.
constexpr int kForkMinProblems = 64;

template <class L>
hipError_t fork_join(hipStream_t s, L* launches, int n, const Common& c) {
  if (n == 0) return hipSuccess;
  SideStreams* ss = nullptr;
  const bool fork = n > 1 && c.nprob >= kForkMinProblems && !c.pass2 && !c.serial;
  hipError_t e = fork ? side_streams(ss) : hipSuccess;
  if (e != hipSuccess) return e;
  if (n == 1 || !ss) {
    for (int i = 0; i < n; ++i) {
      launches[i](s);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  e = hipEventRecord(ss->fork, s);
  if (e != hipSuccess) return e;
  const int side = n - 1 < kSide ? n - 1 : kSide;
  for (int i = 0; i < side; ++i) {
    e = hipStreamWaitEvent(ss->st[i], ss->fork, 0);
    if (e != hipSuccess) return e;
  }
  for (int i = 0; i < n; ++i) {
    hipStream_t t = i == 0 ? s : ss->st[(i - 1) % side];
    launches[i](t);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (int i = 0; i < side; ++i) {
    e = hipEventRecord(ss->join[i], ss->st[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ss->join[i], 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace

hipError_t launch_qr(Prob* probs, const Common& c, int which, int want_r, int pivot,
                     hipStream_t s, int gate) {
  const int rows_max = which ? c.nmax : c.mmax;
  const int rows_min = which ? c.nmin : c.mmin;
  static const hipError_t attr = []() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_qr_glb<1024>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(2 * size_t(kGlbLdsRows) * sizeof(zt)));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_qr_lds<1024>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(size_t(kLdsElems) * sizeof(zt)));
  }();
  if (attr != hipSuccess) return attr;
  typedef void (*Launch)(hipStream_t, Prob*, int, int, int, int, int, int);
  struct Item {
    Launch fn;
    Prob* probs;
    int which, want_r, pivot, nprob, rows, grow;
    void operator()(hipStream_t t) const { fn(t, probs, which, want_r, pivot, nprob, rows, grow); }
  };
  const Launch fns[4] = {
      [](hipStream_t t, Prob* p, int w, int r, int v, int np, int, int g) {
        if (v)
          TEBD_LAUNCH("k_qr_reg<512, 8, true>", (k_qr_reg<512, 8, true>), dim3(np), dim3(512), 0, t, p, w, r, 0, g);
        else
          TEBD_LAUNCH("k_qr_reg<512, 8, false>", (k_qr_reg<512, 8, false>), dim3(np), dim3(512), 0, t, p, w, r, 0, g);
      },
      [](hipStream_t t, Prob* p, int w, int r, int v, int np, int, int g) {
        if (v)
          TEBD_LAUNCH("k_qr_reg<1024, 12, true>", (k_qr_reg<1024, 12, true>), dim3(np), dim3(1024), 0, t, p, w, r, 1, g);
        else
          TEBD_LAUNCH("k_qr_reg<1024, 12, false>", (k_qr_reg<1024, 12, false>), dim3(np), dim3(1024), 0, t, p, w, r, 1, g);
      },
      [](hipStream_t t, Prob* p, int w, int r, int v, int np, int, int g) {
        TEBD_LAUNCH("k_qr_lds<1024>", k_qr_lds<1024>, dim3(np), dim3(1024), size_t(kLdsElems) * sizeof(zt),
                           t, p, w, r, v, g);
      },
      [](hipStream_t t, Prob* p, int w, int r, int v, int np, int rw, int g) {
        TEBD_LAUNCH("k_qr_glb<1024>", k_qr_glb<1024>, dim3(np), dim3(1024),
                    2 * size_t(rw < kGlbLdsRows ? rw : kGlbLdsRows) * sizeof(zt), t,
                           p, w, r, v, g);
      }};
  // the classes between those of the smallest and the largest possible size
  const int lo = qr_class(rows_min, c.lmin), hi = qr_class(rows_max, c.lmax);
  Item items[4];
  int n = 0;
  for (int k = lo; k <= hi; ++k)
    items[n++] = {fns[k], probs, which, want_r, pivot, c.nprob, rows_max, gate};
  return fork_join(s, items, n, c);
}

// --------------------------------------------------------------------------
// Gram-based QR (CholeskyQR2) of the large problems (QR classes 2 and 3):
// two passes of G = Y^H Y (k_gram), G = R^H R by Cholesky, Y <- Y R^-1
// (k_qapply into Qc, then Qc and Y trade places).  The passes are wide
// tile-queue products instead of a workgroup's reflector chain, which is
// what the large problems need.  A Cholesky pivot at or below kCholTol times
// the Gram's largest diagonal (kappa(Y) beyond about 1e7, where CholeskyQR2
// loses orthogonality) refuses the problem: TEBD_DEV_QR_FALLBACK, and the
// Householder kernels (gate 2) take it over from what the passes left in Y,
// which spans the same space.  Bit 1 of P.chol: the m x l sketch is
// eligible, bit 2: the n x l sketch.
constexpr double kCholTol = 1e-14;
constexpr int kCholLdsL = 96;  // Gram in LDS up to this width (147 KiB), else in global memory

__global__ void k_chol_mark(Prob* probs, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  Prob& P = probs[p];
  int f = 0;
  if (P.l > 0) {
    if (qr_class(P.m, P.l1) >= 2) f |= 1;
    if (qr_class(P.n, P.l1) >= 2) f |= 2;
  }
  P.chol = f;
  P.chol_ok = 0;
}

hipError_t launch_chol_mark(Prob* probs, const Common& c, hipStream_t s) {
  TEBD_LAUNCH("k_chol_mark", k_chol_mark, dim3((c.nprob + 63) / 64), dim3(64), 0, s, probs,
              c.nprob);
  return hipGetLastError();
}

// Cholesky G = L L^H of the Gram in C (column-major l x l, lower triangle
// used), then X = R^-1 = (L^-1)^H, upper triangular, into J: column c of
// L^-1 by forward substitution, one wavefront per column, the column held
// across the lanes (lane t keeps rows t, t + 64, ...).
// With want_r (the QR of B^H, whose R_B the small SVD takes): pass 0 writes
// R_1 = L_1^H into Rb, pass 1 replaces it by R_2 R_1 = L_2^H R_1 (so that
// B^H = Q_2 R_2 R_1) and the identity column order into piv.  A pass-1
// refusal puts B^H back into Yt (pass 0 left it in Qc), so that the
// Householder fallback factors B^H itself.
template <int WHICH>
__global__ __launch_bounds__(1024) void k_chol(Prob* probs, int pass, int want_r) {
  Prob& P = probs[blockIdx.x];
  const int l = P.l, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool elig = l > 0 && (P.chol & (WHICH ? 2 : 1)) && (pass == 0 || P.chol_ok);
  if (!elig) {
    if (tid == 0 && pass == 0) P.chol_ok = 0;
    return;
  }
  __shared__ zt g_lds[kCholLdsL * kCholLdsL];
  __shared__ double dmax_s;
  __shared__ int fail_s;
  const bool in_lds = l <= kCholLdsL;
  zt* G = in_lds ? g_lds : P.C;
  if (in_lds)
    for (int e = tid; e < l * l; e += 1024) g_lds[e] = P.C[e];
  __syncthreads();
  if (tid == 0) {
    double dm = 0.0;
    for (int j = 0; j < l; ++j) dm = fmax(dm, G[j + size_t(j) * l].x);
    dmax_s = dm;
    fail_s = !(dm > 0.0) || !isfinite(dm);
  }
  __syncthreads();
  for (int j = 0; j < l && !fail_s; ++j) {
    if (tid == 0) {
      const double d = G[j + size_t(j) * l].x;
      if (!(d > kCholTol * dmax_s) || !isfinite(d))
        fail_s = 1;
      else
        G[j + size_t(j) * l] = make_double2(sqrt(d), 0.0);
    }
    __syncthreads();
    if (fail_s) break;
    const double inv = 1.0 / G[j + size_t(j) * l].x;
    for (int i = j + 1 + tid; i < l; i += 1024) G[i + size_t(j) * l] = zscale(G[i + size_t(j) * l], inv);
    __syncthreads();
    const int nt = l - j - 1;
    for (int e = tid; e < nt * nt; e += 1024) {
      const int kk = e / nt, ii = e - kk * nt;
      if (ii < kk) continue;
      const int k = j + 1 + kk, i = j + 1 + ii;
      const zt lij = G[i + size_t(j) * l], lkj = G[k + size_t(j) * l];
      G[i + size_t(k) * l] = zsub(G[i + size_t(k) * l], zmul(lij, zconj(lkj)));
    }
    __syncthreads();
  }
  if (fail_s) {
    if (tid == 0) {
      P.chol_ok = 0;
      P.flags |= TEBD_DEV_QR_FALLBACK;
      if (want_r && pass == 1) {  // back to B^H (the first pass swapped it into Qc)
        zt* t = WHICH ? P.Yt : P.Y;
        if (WHICH)
          P.Yt = P.Qc;
        else
          P.Y = P.Qc;
        P.Qc = t;
      }
    }
    return;
  }
  if (want_r) {
    // R_B (column-major, upper): pass 0 R_1 = L^H; pass 1 L^H R_1, through X
    zt* Rb = P.Rb;
    if (pass == 0) {
      for (int e = tid; e < l * l; e += 1024) {
        const int c = e / l, r = e - c * l;
        Rb[e] = r <= c ? zconj(G[c + size_t(r) * l]) : make_double2(0.0, 0.0);
      }
    } else {
      zt* T = P.X;
      for (int e = tid; e < l * l; e += 1024) {
        const int c = e / l, r = e - c * l;
        double sr = 0.0, si = 0.0;
        for (int k = r; k <= c; ++k) {  // (L^H)[r][k] = conj(L[k][r])
          const zt a = G[k + size_t(r) * l], b = Rb[k + size_t(c) * l];
          sr += a.x * b.x + a.y * b.y;
          si += a.x * b.y - a.y * b.x;
        }
        T[e] = make_double2(sr, si);
      }
      __syncthreads();
      for (int e = tid; e < l * l; e += 1024) Rb[e] = T[e];
      for (int c = tid; c < l; c += 1024) P.piv[c] = c;
    }
  }
  // X = (L^-1)^H: row c of X holds conj of column c of L^-1
  zt* X = P.J;
  for (int c = wave; c < l; c += 16) {
    zt xr[kMaxL / 64];  // rows lane, lane + 64, ... of column c of L^-1
#pragma unroll
    for (int q = 0; q < kMaxL / 64; ++q) xr[q] = make_double2(0.0, 0.0);
    for (int i = c; i < l; ++i) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < kMaxL / 64; ++q) {
        const int k = lane + 64 * q;
        if (k >= c && k < i) {
          const zt lik = G[i + size_t(k) * l];
          sr += lik.x * xr[q].x - lik.y * xr[q].y;
          si += lik.x * xr[q].y + lik.y * xr[q].x;
        }
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      const double lii = G[i + size_t(i) * l].x;
      const zt x = i == c ? make_double2(1.0 / lii, 0.0) : make_double2(-sr / lii, -si / lii);
#pragma unroll
      for (int q = 0; q < kMaxL / 64; ++q)
        if (lane + 64 * q == i) xr[q] = x;
    }
#pragma unroll
    for (int q = 0; q < kMaxL / 64; ++q) {
      const int i = lane + 64 * q;
      if (i < l) X[c + size_t(i) * l] = i >= c ? zconj(xr[q]) : make_double2(0.0, 0.0);
    }
  }
  if (tid == 0) P.chol_ok = 1;
}

template <int WHICH>
__global__ void k_qswap(Prob* probs, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  Prob& P = probs[p];
  if (!P.chol_ok) return;
  zt* t = WHICH ? P.Yt : P.Y;
  if (WHICH)
    P.Yt = P.Qc;
  else
    P.Y = P.Qc;
  P.Qc = t;
}

hipError_t launch_chol_qr(Prob* probs, const Common& c, int which, hipStream_t s, int want_r) {
  hipError_t e = hipSuccess;
  for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
    e = launch_gram(probs, c, which, pass, s);
    if (e != hipSuccess) break;
    if (which)
      TEBD_LAUNCH("k_chol<1>", k_chol<1>, dim3(c.nprob), dim3(1024), 0, s, probs, pass, want_r);
    else
      TEBD_LAUNCH("k_chol<0>", k_chol<0>, dim3(c.nprob), dim3(1024), 0, s, probs, pass, want_r);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_qapply(probs, c, which, s);
    if (e != hipSuccess) break;
    if (which)
      TEBD_LAUNCH("k_qswap<1>", k_qswap<1>, dim3((c.nprob + 63) / 64), dim3(64), 0, s, probs, c.nprob);
    else
      TEBD_LAUNCH("k_qswap<0>", k_qswap<0>, dim3((c.nprob + 63) / 64), dim3(64), 0, s, probs, c.nprob);
    e = hipGetLastError();
  }
  return e;
}

// --------------------------------------------------------------------------
// Small SVD of B (l x n) from B^H = Q_B R_B: one-sided Jacobi on C = R_B^H
// (l x l).  Column pairs are rotated in the round-robin order of the circle
// method, l/2 disjoint pairs per round, one pair per wavefront at a time.
// A pair (p, q) with Gram entries a = |c_p|^2, b = |c_q|^2, g = c_p^H c_q is
// rotated when |g| > tol sqrt(a b):  phi = arg g, zeta = (b - a) / (2|g|),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), cs = 1/sqrt(1+t^2), sn = t cs,
//   c_p <- cs c_p - sn e^{-i phi} c_q,  c_q <- sn c_p + cs e^{-i phi} c_q,
// which zeroes the (p, q) Gram entry.  The same rotation accumulates into J.
// At convergence C J = X Sigma with orthogonal columns, so
// B = X Sigma (Q_B J)^H: left vectors X (normalised columns), values Sigma,
// right vectors Q_B J (formed later).  Outputs are sorted descending.
// C and J live in LDS when 2 l^2 fits, else in global memory; a pair's
// columns are held in registers (l <= 64 * REGS) for the whole rotation.

// Rotation of a column pair with Gram entries a = |c_p|^2, b = |c_q|^2 and
// g = c_p^H c_q (given as gr + i gi): false when |g| <= tol sqrt(a b).
// Otherwise zeta = (b - a) / (2|g|), t = sign(zeta) / (|zeta| + sqrt(1 +
// zeta^2)), cs = 1 / sqrt(1 + t^2), sn = t cs, em = e^{-i arg g}, and
// ag = |g| (the carried norms move by t |g|).  Reciprocal square roots keep
// the chain of dependent operations short.
__device__ __forceinline__ bool jacobi_rotation(double gr, double gi, double a, double b,
                                                double tol, double& ag, double& t, double& cs,
                                                double& sn, zt& em) {
  const double g2 = gr * gr + gi * gi;
  if (!(g2 > tol * tol * (a * b)) || g2 == 0.0) return false;
  const double ig = rsqrt(g2);  // 1 / |g|
  ag = g2 * ig;
  const double zeta = 0.5 * (b - a) * ig;
  t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  cs = rsqrt(1.0 + t * t);
  sn = t * cs;
  em = make_double2(gr * ig, -gi * ig);
  return true;
}

// Round-robin (circle method) pairing of lp players: position 0 stays, the
// others rotate by one place per round.  pos < lp and round < lp - 1, so
// one conditional subtraction reduces modulo lp - 1 (no integer division).
__device__ __forceinline__ int circle_player(int pos, int round, int lp) {
  if (pos == 0) return 0;
  const int x = pos - 1 + round;
  return 1 + (x >= lp - 1 ? x - (lp - 1) : x);
}


// Column norms are recomputed exactly at the start of every sweep and then
// carried through the rotations analytically (a' = a - t|g|, b' = b + t|g|),
// so each pair needs a single complex reduction, g = c_p^H c_q.
// A sweep whose rotations all turned by less than about 1e-7 rad (|g|^2 <=
// kSmallTurn a b) leaves the columns so close to orthogonal that the next
// sweep would likely rotate nothing; instead of running that sweep,
// pairs_below_tol tests every pair of the current C at once.
constexpr double kSmallTurn = 1e-14;

// True when no pair of columns of C (column c at C + c S) would be rotated:
// every |c_p^H c_q| <= tol |c_p| |c_q| with nrm[c] = |c_c|^2 recomputed and
// visible to the workgroup (the test of jacobi_rotation).  The verdict of a
// sweep that rotates nothing, from l (l - 1) / 2 independent dot products
// instead of l - 1 dependent rounds.  Whole workgroup (one barrier).
template <int NT>
__device__ __forceinline__ bool pairs_below_tol(const zt* C, int S, int l, double tol,
                                                const double* nrm) {
  // thread t: columns {2a, 2a + 1} x {2b, 2b + 1}, a <= b, four dot products
  // per pass over the rows (a missing last column repeats the one before)
  const int nh = (l + 1) / 2;
  int bad = 0;
  for (int t = threadIdx.x; t < nh * nh; t += NT) {
    const int a = t / nh, b = t - a * nh;
    if (a > b) continue;
    const int p0 = 2 * a, q0 = 2 * b;
    const int p1 = p0 + 1 < l ? p0 + 1 : p0, q1 = q0 + 1 < l ? q0 + 1 : q0;
    const zt* x0 = C + size_t(p0) * S;
    const zt* x1 = C + size_t(p1) * S;
    const zt* y0 = C + size_t(q0) * S;
    const zt* y1 = C + size_t(q1) * S;
    double g[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int r = 0; r < l; ++r) {
      const zt u0 = x0[r], u1 = x1[r], v0 = y0[r], v1 = y1[r];
      zdot_acc(u0, v0, g[0][0], g[0][1]);
      zdot_acc(u0, v1, g[1][0], g[1][1]);
      zdot_acc(u1, v0, g[2][0], g[2][1]);
      zdot_acc(u1, v1, g[3][0], g[3][1]);
    }
    const int ps[4] = {p0, p0, p1, p1}, qs[4] = {q0, q1, q0, q1};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double g2 = g[i][0] * g[i][0] + g[i][1] * g[i][1];
      if (ps[i] < qs[i] && g2 > tol * tol * (nrm[ps[i]] * nrm[qs[i]]) && g2 != 0.0) bad = 1;
    }
  }
  return __syncthreads_or(bad) == 0;
}

// One pair per wavefront at a time; ALL_PAIRS: after a sweep of small turns,
// pairs_below_tol may end the iteration without the sweep that rotates
// nothing.
template <int NT, int REGS, bool ALL_PAIRS>
__device__ __forceinline__ void jacobi_core(zt* C, zt* J, int l, int& converged_out,
                                            int* rotated, int* large, double* nrm) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lp = l + (l & 1);
  const double tol = DBL_EPSILON * sqrt(double(l));
  constexpr int kMaxSweeps = 40;
  bool converged = (l == 1);
  for (int sweep = 0; sweep < kMaxSweeps && !converged; ++sweep) {
    for (int c = wave; c < l; c += NW) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < REGS; ++i) {
        const int r = lane + 64 * i;
        if (r < l) s += zabs2(C[size_t(c) * l + r]);
      }
      s = wave_sum(s);
      if (lane == 0) nrm[c] = s;
    }
    if (tid == 0) {
      *rotated = 0;
      *large = 0;
    }
    __syncthreads();
    for (int round = 0; round < lp - 1; ++round) {
      for (int pr = wave; pr < lp / 2; pr += NW) {
        const int a = circle_player(pr, round, lp), b = circle_player(lp - 1 - pr, round, lp);
        const int p = a < b ? a : b, q = a < b ? b : a;
        if (q >= l) continue;
        zt* cp = C + size_t(p) * l;
        zt* cq = C + size_t(q) * l;
        zt xp[REGS], xq[REGS];
        double gr = 0.0, gi = 0.0;
#pragma unroll
        for (int i = 0; i < REGS; ++i) {
          const int r = lane + 64 * i;
          xp[i] = r < l ? cp[r] : make_double2(0.0, 0.0);
          xq[i] = r < l ? cq[r] : make_double2(0.0, 0.0);
          const zt t = zcmul(xp[i], xq[i]);
          gr += t.x;
          gi += t.y;
        }
        gr = wave_sum(gr);
        gi = wave_sum(gi);
        const double app = nrm[p], aqq = nrm[q];
        double ag, t, cs, sn;
        zt em;  // e^{-i phi}
        if (!jacobi_rotation(gr, gi, app, aqq, tol, ag, t, cs, sn, em)) continue;
#pragma unroll
        for (int i = 0; i < REGS; ++i) {
          const int r = lane + 64 * i;
          if (r < l) {
            const zt x = xp[i], y = zmul(em, xq[i]);
            cp[r] = zrot_lo(x, y, cs, sn);
            cq[r] = zrot_hi(x, y, cs, sn);
          }
        }
        zt* jp = J + size_t(p) * l;
        zt* jq = J + size_t(q) * l;
#pragma unroll
        for (int i = 0; i < REGS; ++i) {
          const int r = lane + 64 * i;
          if (r < l) {
            const zt x = jp[r], y = zmul(em, jq[r]);
            jp[r] = zrot_lo(x, y, cs, sn);
            jq[r] = zrot_hi(x, y, cs, sn);
          }
        }
        if (lane == 0) {
          nrm[p] = fmax(app - t * ag, 0.0);
          nrm[q] = aqq + t * ag;
          *rotated = 1;
          if (ag * ag > kSmallTurn * (app * aqq)) *large = 1;
        }
      }
      __syncthreads();
    }
    converged = (*rotated == 0);
    const bool turned_far = (*large != 0);
    __syncthreads();
    if (ALL_PAIRS && !converged && !turned_far) {
      for (int c = wave; c < l; c += NW) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < REGS; ++i) {
          const int r = lane + 64 * i;
          if (r < l) s += zabs2(C[size_t(c) * l + r]);
        }
        s = wave_sum(s);
        if (lane == 0) nrm[c] = s;
      }
      __syncthreads();
      converged = pairs_below_tol<NT>(C, l, l, tol, nrm);
    }
  }
  converged_out = converged ? 1 : 0;
}

// Column norms, descending order, and the sorted outputs X, W, sig.
template <int NT>
__device__ __forceinline__ void jacobi_finish(Prob& P, const zt* C, const zt* J, int l,
                                              double* sig_s, int* perm_s) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c = wave; c < l; c += NW) {
    double s = 0.0;
    for (int r = lane; r < l; r += 64) s += zabs2(C[size_t(c) * l + r]);
    s = wave_sum(s);
    if (lane == 0) sig_s[c] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < l; j += NT) {
    const double sj = sig_s[j];
    int rank = 0;
    for (int i = 0; i < l; ++i) {
      const double si = sig_s[i];
      rank += (si > sj) || (si == sj && i < j);
    }
    perm_s[rank] = j;
  }
  __syncthreads();
  for (int e = tid; e < l * l; e += NT) {
    const int c = e / l, r = e - c * l;
    const int src = perm_s[c];
    const double sv = sig_s[src];
    const zt x = C[size_t(src) * l + r];
    P.X[e] = sv > 0.0 ? zscale(x, 1.0 / sv) : make_double2(0.0, 0.0);
    P.W[e] = J[size_t(src) * l + r];
  }
  for (int c = tid; c < l; c += NT) P.sig[c] = sig_s[perm_s[c]];
}

// --------------------------------------------------------------------------
// Truncation: chi' = min(chi_max, smallest c with w(c) <= eps), where
// w(c) = (||A||_F^2 - sum_{j<=c} s_j^2) / ||A||_F^2; eps <= 0 keeps
// min(chi_max, l).  TEBD: lambda' = s / ||s_{1..chi'}|| and chi' are written
// into the MPS.  Run by the whole workgroup of the problem's small SVD after
// it (sorted(c): the c-th largest singular value, from LDS); the scans run
// on thread 0 so the summation order is fixed.  The global reads (partial
// sums, outer lambdas) are spread over the workgroup first: one thread
// reading them one after another waited for each.
constexpr int kTailChunk = 64;

template <int NT, class Sorted>
__device__ __forceinline__ void truncate_tail(Prob& P, int l, double eps, int tebd,
                                              int32_t* retry_count, Sorted sorted, double* scan) {
  __shared__ int chi_s, first_s;
  __shared__ double norm_s, frob_s;
  __shared__ double part_s[kTailChunk];
  const int tid = threadIdx.x;
  // ||A||_F^2 from the partial sums, the gate product's (TEBD) or k_frob's:
  // loaded kTailChunk at a time, added by thread 0 in index order
  const int npart =
      tebd ? gate_partials(P.dl * P.dr, P.gcol0, P.chi_l * P.chi_r) : kFrobSlices;
  __syncthreads();  // the singular values are in place
  // one round of global reads: the first chunk of partial sums, and whether
  // an outer lambda is at or below the floor (its inverse was taken as 0)
  if (tid < kTailChunk && tid < npart) part_s[tid] = P.part[tid];
  bool floor_hit = false;
  if (tebd) {
    if (P.lam_l)
      for (int a = tid; a < P.chi_l; a += NT) floor_hit |= !(P.lam_l[a] > P.lambda_floor);
    if (P.lam_r)
      for (int b = tid; b < P.chi_r; b += NT) floor_hit |= !(P.lam_r[b] > P.lambda_floor);
  }
  floor_hit = __syncthreads_or(floor_hit) != 0;
  double frob2 = 0.0;
  for (int i0 = 0; i0 < npart; i0 += kTailChunk) {
    if (i0 > 0) {
      __syncthreads();  // the previous chunk is summed
      if (tid < kTailChunk && i0 + tid < npart) part_s[tid] = P.part[i0 + tid];
      __syncthreads();
    }
    if (tid == 0) {
      const int n = npart - i0 < kTailChunk ? npart - i0 : kTailChunk;
      for (int i = 0; i < n; ++i) frob2 += part_s[i];
    }
  }
  // kept(c) = s_1^2 + ... + s_c^2 in index order (thread 0, into scan[c - 1]);
  // then every c at once: w(c) = (||A||_F^2 - kept(c)) / ||A||_F^2, and chi'
  // the smallest c <= cap with w(c) <= eps.  The same operations as one
  // thread scanning c = 1, 2, ..., without its chain of divisions.
  // A first stage that may still be retried only accepts a rank <= k1.
  const bool can_retry = P.l2 > P.l1;
  int cap = P.kcap < l ? P.kcap : l;
  if (can_retry && P.k1 < cap) cap = P.k1;
  if (tid == 0) {
    double kept = 0.0;
    for (int c = 0; c < l; ++c) {
      const double sv = sorted(c);
      kept += sv * sv;
      scan[c] = kept;
    }
    frob_s = frob2;
    first_s = INT32_MAX;
  }
  __syncthreads();
  const double fr = frob_s;
  int first = INT32_MAX;
  bool nonfinite = false;
  for (int c = tid + 1; c <= l; c += NT) {
    nonfinite |= !isfinite(sorted(c - 1));
    const double wc = fr > 0.0 ? (fr - scan[c - 1]) / fr : 0.0;
    if (eps > 0.0 && c <= cap && wc <= eps && c < first) first = c;
  }
  if (first != INT32_MAX) atomicMin(&first_s, first);
  nonfinite = __syncthreads_or(nonfinite) != 0;
  if (tid == 0) {
    int flags = P.flags;
    P.frob2 = frob2;
    const bool found = first_s != INT32_MAX;
    const int chi = found ? first_s : cap;
    // the discarded weight at chi' (or at cap when no c qualifies)
    double w = fr > 0.0 ? (fr - scan[chi - 1]) / fr : 0.0;
    const double nk = scan[chi - 1];  // the kept squares summed up to chi'
    const bool finite = isfinite(frob2) && !nonfinite;
    int out = chi;
    if (can_retry && !(eps > 0.0 && found)) {
      // stage 1 rejected: leave every output untouched, run stage 2
      P.retry = 1;
      if (retry_count) atomicAdd(retry_count, 1);
      out = -1;
    }
    if (eps > 0.0 && !found) flags |= TEBD_DEV_CHI_BOUND;
    if (!finite) flags |= TEBD_DEV_NONFINITE;
    if (w < 0.0) w = 0.0;
    if (floor_hit) flags |= TEBD_DEV_LAMBDA_FLOOR;
    if (out >= 0) {
      P.chi_new = chi;
      P.flags = flags;
      *P.disc = w;
      *P.status = flags;
      if (P.chi_out) *P.chi_out = chi;
    }
    chi_s = out;
    norm_s = sqrt(nk);
  }
  __syncthreads();
  const int chi = chi_s;
  if (chi < 0) return;
  if (tebd) {
    const double inv = norm_s > 0.0 ? 1.0 / norm_s : 0.0;
    for (int j = threadIdx.x; j < P.chi_cap; j += NT) P.lam_mid[j] = j < chi ? sorted(j) * inv : 0.0;
    if (threadIdx.x == 0) *P.chi_slot = chi;
  } else {
    for (int j = threadIdx.x; j < P.kcap; j += NT) P.S[j] = j < chi ? sorted(j) : 0.0;
  }
}

// Size classes of the small SVD, by l: 0 (l <= 32, 256 threads) and 1
// (l <= 64, 512 threads) rotate every pair of a round at once (k_svd_pairs);
// 2 (C and J in LDS) and 3 (global memory) rotate one pair per wavefront at
// a time (jacobi_core).
__host__ __device__ __forceinline__ int svd_class(int l) {
  if (l <= 32) return 0;
  if (l <= 64) return 1;
  if (2 * l * l <= kLdsElems) return 2;
  return 3;
}

// C and J in LDS with an odd column stride, and all l/2 pairs of a round
// rotated at once: G = NT / (l/2 rounded up to a power of two) lanes per
// pair, at most 16 (DPP sums only; for these two classes always 16).  Lane h
// of a pair loads every G-th row of both columns of C and J into
// registers, sums its part of g = c_p^H c_q, the group sum
// combines them, and the same lanes rotate the rows they hold and store
// them; one barrier per round.  Same rotation, tolerance, carried norms and
// sweep limit as jacobi_core.
constexpr int kPairGroupMax = 16;


template <int NT, int CLS>
__global__ __launch_bounds__(NT) void k_svd_pairs(Prob* probs, double eps, int tebd,
                                                  int32_t* retry_count) {
  extern __shared__ zt lds[];  // C, then J: l columns of stride l | 1 each
  __shared__ double nrm[64];
  __shared__ double sig_s[64];
  __shared__ double srt_s[64];  // singular values in descending order
  __shared__ int perm_s[64];
  Prob& P = probs[blockIdx.x];
  const int l = P.l;
  if (l == 0 || svd_class(l) != CLS) return;
  const int S = l | 1;
  zt* Cs = lds;
  zt* Js = lds + l * S;
  const int tid = threadIdx.x;
  const zt zero = make_double2(0.0, 0.0);  // value, never addressed
  for (int e = tid; e < l * l; e += NT) {
    const int c = e / l, r = e - c * l;
    Cs[c * S + r] = zconj(P.Rb[size_t(r) * l + c]);
    Js[c * S + r] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  const int lp = l + (l & 1);
  // lanes per pair: l/2 <= NT / 16 pairs in these classes, so 16 each
  constexpr int G = kPairGroupMax;
  static_assert(NT / (CLS == 0 ? 16 : 32) >= kPairGroupMax, "pairs of a round fit at 16 lanes");
  const int k = tid / G, h = tid - k * G;
  int lc2 = 1;
  while (lc2 < l) lc2 <<= 1;
  const int GN = NT / lc2 < kPairGroupMax ? NT / lc2 : kPairGroupMax;  // lanes per column
  const int cn = tid / GN, hn = tid - cn * GN;
  const double tol = DBL_EPSILON * sqrt(double(l));
  constexpr int kMaxSweeps = 40;
  bool converged = (l == 1);
  __syncthreads();
  for (int sweep = 0; sweep < kMaxSweeps && !converged; ++sweep) {
    double s = 0.0;
    if (cn < l) s = col_norm2(Cs + cn * S, hn, l, GN);
    s = group_sum(s, GN);
    if (cn < l && hn == 0) nrm[cn] = s;
    __syncthreads();
    int any = 0, large = 0;
    for (int round = 0; round < lp - 1; ++round) {
      int p = 0, q = 0;
      bool act = k < lp / 2;
      if (act) {
        const int a = circle_player(k, round, lp), b = circle_player(lp - 1 - k, round, lp);
        p = a < b ? a : b;
        q = a < b ? b : a;
        act = q < l;
      }
      // rows h, h + G, ... < l: G = 16 here (l/2 <= NT / 16), so at most
      // 32 / 16 or 64 / 16 of them
      constexpr int RPR = (CLS == 0 ? 32 : 64) / kPairGroupMax;
      zt x[RPR], y[RPR], xj[RPR], yj[RPR];
      zt* cp = Cs + p * S;
      zt* cq = Cs + q * S;
      zt* jp = Js + p * S;
      zt* jq = Js + q * S;
      double g0 = 0.0, g1 = 0.0;
#pragma unroll
      for (int i = 0; i < RPR; ++i) {
        const int r = h + G * i;
        const bool in = act && r < l;
        x[i] = zload_if(in, cp + r);
        y[i] = zload_if(in, cq + r);
        xj[i] = zload_if(in, jp + r);
        yj[i] = zload_if(in, jq + r);
        zdot_acc(x[i], y[i], g0, g1);
      }
      const double gr = group_sum(g0, G), gi = group_sum(g1, G);
      if (act) {
        const double app = nrm[p], aqq = nrm[q];
        double ag, t, cs, sn;
        zt em;  // e^{-i phi}
        if (jacobi_rotation(gr, gi, app, aqq, tol, ag, t, cs, sn, em)) {
#pragma unroll
          for (int i = 0; i < RPR; ++i) {
            const int r = h + G * i;
            if (r < l) {
              const zt ey = zmul(em, y[i]), eyj = zmul(em, yj[i]);
              cp[r] = zrot_lo(x[i], ey, cs, sn);
              cq[r] = zrot_hi(x[i], ey, cs, sn);
              jp[r] = zrot_lo(xj[i], eyj, cs, sn);
              jq[r] = zrot_hi(xj[i], eyj, cs, sn);
            }
          }
          if (h == 0) {
            nrm[p] = fmax(app - t * ag, 0.0);
            nrm[q] = aqq + t * ag;
          }
          any = 1;
          if (ag * ag > kSmallTurn * (app * aqq)) large = 1;
        }
      }
      __syncthreads();
    }
    const bool rotated = __syncthreads_or(any) != 0;
    const bool turned_far = __syncthreads_or(large) != 0;
    converged = !rotated;
    if (rotated && !turned_far) {
      double s2 = 0.0;
      if (cn < l) s2 = col_norm2(Cs + cn * S, hn, l, GN);
      s2 = group_sum(s2, GN);
      if (cn < l && hn == 0) nrm[cn] = s2;
      __syncthreads();
      converged = pairs_below_tol<NT>(Cs, S, l, tol, nrm);
    }
  }
  if (!converged && tid == 0) P.flags |= TEBD_DEV_JACOBI_NOCONV;
  // singular values, descending order, sorted outputs
  {
    double s = 0.0;
    if (cn < l) s = col_norm2(Cs + cn * S, hn, l, GN);
    s = group_sum(s, GN);
    if (cn < l && hn == 0) sig_s[cn] = sqrt(s);
  }
  __syncthreads();
  if (tid < l) {
    const double sj = sig_s[tid];
    int rank = 0;
    for (int i = 0; i < l; ++i) {
      const double si = sig_s[i];
      rank += (si > sj) || (si == sj && i < tid);
    }
    perm_s[rank] = tid;
  }
  __syncthreads();
  for (int e = tid; e < l * l; e += NT) {
    const int c = e / l, r = e - c * l;
    const int src = perm_s[c];
    const double sv = sig_s[src];
    const zt x = Cs[src * S + r];
    P.X[e] = sv > 0.0 ? zscale(x, 1.0 / sv) : zero;
    P.W[e] = Js[src * S + r];
  }
  if (tid < l) {
    const double v = sig_s[perm_s[tid]];
    srt_s[tid] = v;
    P.sig[tid] = v;
  }
  truncate_tail<NT>(P, l, eps, tebd, retry_count, [&](int c) { return srt_s[c]; }, nrm);
}

// Classes 2 and 3: one pair per wavefront at a time (jacobi_core), C and J
// in LDS (LDS_CJ) or in the problem's global scratch.
template <int NT, int REGS, bool LDS_CJ>
__global__ __launch_bounds__(NT) void k_small_svd(Prob* probs, double eps, int tebd,
                                                  int32_t* retry_count) {
  extern __shared__ zt lds[];
  __shared__ double sig_s[kMaxL];
  __shared__ int perm_s[kMaxL];
  __shared__ int rotated, large_turn;
  __shared__ double nrm[kMaxL];
  Prob& P = probs[blockIdx.x];
  const int l = P.l;
  if (l == 0 || svd_class(l) != (LDS_CJ ? 2 : 3)) return;
  zt* C = LDS_CJ ? lds : P.C;
  zt* J = LDS_CJ ? lds + l * l : P.J;
  for (int e = threadIdx.x; e < l * l; e += NT) {
    const int c = e / l, r = e - c * l;
    C[e] = zconj(P.Rb[size_t(r) * l + c]);
    J[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  int converged;
  // the all-pairs test only where C is in LDS (from global memory it costs
  // about the sweep it would save)
  jacobi_core<NT, REGS, LDS_CJ>(C, J, l, converged, &rotated, &large_turn, nrm);
  if (!converged && threadIdx.x == 0) P.flags |= TEBD_DEV_JACOBI_NOCONV;
  jacobi_finish<NT>(P, C, J, l, sig_s, perm_s);
  truncate_tail<NT>(P, l, eps, tebd, retry_count, [&](int c) { return sig_s[perm_s[c]]; }, nrm);
}

hipError_t launch_small_svd(Prob* probs, const Common& c, hipStream_t s) {
  static const hipError_t attr = []() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_svd<1024, 2, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(size_t(kLdsElems) * sizeof(zt)));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_svd_pairs<512, 1>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(2 * 64 * 65 * sizeof(zt)));
  }();
  if (attr != hipSuccess) return attr;
  typedef void (*Launch)(hipStream_t, Prob*, int, double, int, int32_t*);
  struct Item {
    Launch fn;
    Prob* probs;
    int nprob;
    double eps;
    int tebd;
    int32_t* retry;
    void operator()(hipStream_t t) const { fn(t, probs, nprob, eps, tebd, retry); }
  };
  const Launch fns[4] = {
      [](hipStream_t t, Prob* p, int np, double e, int tb, int32_t* rc) {
        TEBD_LAUNCH("k_svd_pairs<256, 0>", (k_svd_pairs<256, 0>), dim3(np), dim3(256),
                    2 * 32 * 33 * sizeof(zt), t, p, e, tb, rc);
      },
      [](hipStream_t t, Prob* p, int np, double e, int tb, int32_t* rc) {
        TEBD_LAUNCH("k_svd_pairs<512, 1>", (k_svd_pairs<512, 1>), dim3(np), dim3(512),
                    2 * 64 * 65 * sizeof(zt), t, p, e, tb, rc);
      },
      [](hipStream_t t, Prob* p, int np, double e, int tb, int32_t* rc) {
        TEBD_LAUNCH("k_small_svd<1024, 2, true>", (k_small_svd<1024, 2, true>), dim3(np), dim3(1024),
                    size_t(kLdsElems) * sizeof(zt), t, p, e, tb, rc);
      },
      [](hipStream_t t, Prob* p, int np, double e, int tb, int32_t* rc) {
        TEBD_LAUNCH("k_small_svd<1024, 4, false>", (k_small_svd<1024, 4, false>), dim3(np), dim3(1024), 0,
                    t, p, e, tb, rc);
      }};
  // the problem's l here is the rank the range finder revealed
  const int lo = svd_class(c.lmin < 1 ? 1 : c.lmin), hi = svd_class(c.lmax);
  Item items[4];
  int n = 0;
  int32_t* retry = c.pass2 ? nullptr : c.retry_count;
  for (int k = lo; k <= hi; ++k) items[n++] = {fns[k], probs, c.nprob, c.eps, c.tebd, retry};
  return fork_join(s, items, n, c);
}

// --------------------------------------------------------------------------
// Accuracy Check (Sec. IV, Alg. 2), one workgroup per problem still probing:
// with Q the current basis (columns 0..l-1 of Y) and B = A Omega_r in the
// next r columns, D = B - Q (Q^H B) and MAX = max_i ||d_i||.  Theorem 2 with
// Fact 1 bounds the Frobenius residual ||(I - QQ^H) A||_F by (10/3) pi MAX
// (with probability 1 - 10^-r), so MAX is compared with
// tol = sqrt(eps) ||A||_F / ((10/3) pi), eps the relative discarded weight.
// MAX > tol: the basis takes B's first min(r, cap - l) columns (its QR runs
// next, grow_only), or, with no room left, the check stops with
// TEBD_DEV_ACC_CAPPED.  The check goes on while MAX > tol and l <= n - r;
// problems still probing are counted in count[round & 1] for the host, and
// count[(round + 1) & 1] is cleared for the next round.
__global__ __launch_bounds__(256) void k_acc_resid(Prob* probs, double eps, int32_t* count,
                                                   int round) {
  Prob& P = probs[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (blockIdx.x == 0 && tid == 0) count[(round + 1) & 1] = 0;
  const int l = P.l, r = P.ac_r;
  if (l == 0 || r == 0) {
    if (tid == 0) P.ac_grow = 0;
    return;
  }
  const int m = P.m;
  const zt* Q = P.Y;
  const zt* B = P.Y + size_t(l) * m;
  __shared__ zt cs[kMaxL * kAccMaxR];  // C = Q^H B, l x r, column j of Q in row j
  __shared__ double part[4][kAccMaxR];
  // one wavefront per column of Q, its lanes over the rows
  for (int j = wave; j < l; j += 4) {
    double cr[kAccMaxR], ci[kAccMaxR];
#pragma unroll
    for (int i = 0; i < kAccMaxR; ++i) cr[i] = ci[i] = 0.0;
    const zt* qj = Q + size_t(j) * m;
    for (int row = lane; row < m; row += 64) {
      const zt q = qj[row];
#pragma unroll
      for (int i = 0; i < kAccMaxR; ++i)
        if (i < r) zdot_acc(q, B[size_t(i) * m + row], cr[i], ci[i]);
    }
#pragma unroll
    for (int i = 0; i < kAccMaxR; ++i) {
      if (i >= r) break;  // uniform
      const double xr = wave_sum(cr[i]), xi = wave_sum(ci[i]);
      if (lane == 0) cs[j * kAccMaxR + i] = make_double2(xr, xi);
    }
  }
  __syncthreads();
  double nrm[kAccMaxR];
#pragma unroll
  for (int i = 0; i < kAccMaxR; ++i) nrm[i] = 0.0;
  for (int row = tid; row < m; row += 256) {
    zt d[kAccMaxR];  // row `row` of B - Q C, every Q entry read once
#pragma unroll
    for (int i = 0; i < kAccMaxR; ++i)
      d[i] = i < r ? B[size_t(i) * m + row] : make_double2(0.0, 0.0);
    for (int j = 0; j < l; ++j) {
      const zt q = Q[size_t(j) * m + row];
#pragma unroll
      for (int i = 0; i < kAccMaxR; ++i)
        if (i < r) d[i] = zsub(d[i], zmul(q, cs[j * kAccMaxR + i]));
    }
#pragma unroll
    for (int i = 0; i < kAccMaxR; ++i)
      if (i < r) nrm[i] += zabs2(d[i]);
  }
#pragma unroll
  for (int i = 0; i < kAccMaxR; ++i) {
    const double v = wave_sum(nrm[i]);
    if (lane == 0) part[wave][i] = v;
  }
  __syncthreads();
  if (tid != 0) return;
  double mx = 0.0;
  bool finite = true;
  for (int i = 0; i < r; ++i) {
    const double v = (part[0][i] + part[1][i]) + (part[2][i] + part[3][i]);
    finite = finite && isfinite(v);
    mx = fmax(mx, sqrt(v));
  }
  double frob2 = 0.0;
  const int npart = gate_partials(P.dl * P.dr, P.gcol0, P.chi_l * P.chi_r);
  for (int i = 0; i < npart; ++i) frob2 += P.part[i];
  const double tol = sqrt(eps) * sqrt(frob2) / kAccConst;
  const bool grow = finite && mx > tol;
  int lnew = l;
  P.ac_grow = 0;
  if (!finite) P.flags |= TEBD_DEV_NONFINITE;
  if (grow) {
    const int w = P.ac_cap - l < r ? P.ac_cap - l : r;
    if (w <= 0) {
      P.flags |= TEBD_DEV_ACC_CAPPED;
      P.ac_r = 0;
      atomicMax(count + 2, P.l1);
      return;
    }
    lnew = l + w;
    P.l = lnew;
    if (P.l1 < lnew) P.l1 = lnew;
    P.ac_grow = 1;
  }
  P.ac_col += r;
  atomicMax(count + 2, P.l1);  // the widest pass so far (it sets the QR classes of later launches)
  if (grow && lnew <= P.n - r)
    atomicAdd(count + (round & 1), 1);
  else
    P.ac_r = 0;
}

hipError_t launch_acc_resid(Prob* probs, const Common& c, int round, hipStream_t s) {
  TEBD_LAUNCH("k_acc_resid", k_acc_resid, dim3(c.nprob), dim3(256), 0, s, probs, c.eps,
              c.acc_count, round);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Adaptive rank, between the passes: problems whose first stage was rejected
// get the fixed-rank width (and are marked), every other problem is skipped.
__global__ void k_stage2(Prob* probs, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  Prob& P = probs[p];
  if (P.retry) {
    P.l = P.l2;
    P.l1 = P.l2;
    P.k1 = P.kcap;
    P.ldom = P.l2;
    P.retry = 0;
    P.flags |= TEBD_DEV_RANK_RETRY;
  } else {
    P.l = 0;
  }
}

hipError_t launch_stage2(Prob* probs, const Common& c, hipStream_t s) {
  TEBD_LAUNCH("k_stage2", k_stage2, dim3((c.nprob + 63) / 64), dim3(64), 0, s, probs, c.nprob);
  return hipGetLastError();
}

}  // namespace tebd

extern "C" int32_t tebd_size_class(int32_t factorization, int32_t rows, int32_t l) {
  using namespace tebd;
  if (l < 1 || l > kMaxL) return -1;
  if (factorization == 0) return rows < 1 || rows > kMaxRows ? -1 : qr_class(rows, l);
  if (factorization == 1) return svd_class(l);
  return -1;
}
