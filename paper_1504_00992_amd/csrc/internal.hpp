// Internal declarations shared by the HIP translation units of the library.
//
// The library runs the two-site TEBD update with RRSVD truncation
// (Tamascelli, Rosenbach, Plenio, arXiv:1504.00992, Sec. II.B and Sec. IV)
// as a pipeline of batched kernels.  Every kernel reads its per-problem
// geometry from a device-resident descriptor (Prob), so problem sizes chosen
// on the device (bond dimensions after truncation) never travel to the host.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "tebd_rrsvd.h"

namespace tebd {

typedef double2 zt;  // complex128 as (re, im)

// ---------------------------------------------------------------------------
// Per-problem descriptor.  Written by the host (standalone RRSVD) or by the
// planning kernel (TEBD sweeps); a few fields are updated by later kernels.
struct Prob {
  // geometry
  int32_t m, n, l, kcap;             // rows, cols, sketch width, kept capacity (chi_max)
  int32_t chi_l, chi_m, chi_r;       // TEBD: left, middle (old), right bond dims
  int32_t dl, dr;                    // TEBD: local dims of the two sites
  int32_t pid;                       // Philox problem id
  int32_t chi_new;                   // written by the truncation kernel
  int32_t flags;                     // TEBD_DEV_* bits accumulated on the device
  int32_t npart;                     // number of Frobenius partial sums
  int32_t mixed;                     // 1: sketch / power products in complex FP32
  int32_t om_ext;                    // 1: Omega supplied by the caller
  int32_t k1;                        // kept-rank cap of the current stage
  int32_t l1;                        // sketch width this stage started with
  int32_t l2;                        // sketch width of the fixed-rank stage
  int32_t retry;                     // 1: stage 1 rejected, stage 2 pending
  int32_t gcol0;                     // TEBD: first column of this problem in its gate group
  // Accuracy Check (adaptive rank 3): probe width (0: check finished), next
  // probe column of the Gaussian stream, capacity of the basis, and 1 while
  // the basis grew this round (its QR runs)
  int32_t ac_r, ac_col, ac_cap, ac_grow;
  // Gram-based QR (CholeskyQR2) of the large problems: eligible in this
  // pipeline, and 1 while the current QR's Gram passes have succeeded
  int32_t chol, chol_ok;
  // Gate groups (TEBD): consecutive problems of one bond that share its gate
  // form one product G [Theta_1 | Theta_2 | ...] over all their columns.
  // gtot: the group's columns (every member), gn: members (the first member
  // only, else 0), gstride: the distance between the descriptors of
  // consecutive members
  int32_t gtot, gn, gstride;
  double frob2;                      // ||A||_F^2, written on the device
  // input matrix (row-major, leading dim lda) and test matrix (row-major n x l)
  zt* A;
  int64_t lda;
  const zt* om;
  int64_t ldom;
  // scratch (inside the caller's workspace)
  zt* T;         // TEBD: the gate group's Theta before the gate, [(i' j')][group column],
                 // leading dimension gtot; this problem's columns start at gcol0
  zt* Y;         // m x l column-major (ld m): sketch, then Q
  zt* Yt;        // n x l column-major (ld n): A^H Q, then Q~ / Q_B
  zt* Rb;        // l x l column-major: R factor of B^H
  zt* C;         // l x l column-major: Jacobi working matrix
  zt* J;         // l x l column-major: accumulated Jacobi rotations
  zt* X;         // l x l column-major: left vectors of the small SVD, sorted
  zt* W;         // l x l column-major: right rotation, sorted
  zt* qru;       // 2 max(m, n): reflectors of the global-memory QR beyond its LDS rows
  zt* Qc;        // max(m, n) x l column-major: Q of the Gram-based QR (then swapped with Y or Yt)
  double* sig;   // l: singular values sorted descending
  int32_t* piv;  // l: column order of the QR of B^H (B^H P = Q_B R_B; P = I unless pivoted)
  double* part;  // npart Frobenius partial sums
  float2* Af;    // mixed: complex64 copy of A (row-major, ld n), read by the FP32 products
  // outputs of the standalone RRSVD
  zt* U;
  int64_t ldu;
  double* S;
  zt* VH;
  int64_t ldvh;
  int32_t* chi_out;
  double* disc;
  int32_t* status;
  // TEBD state around the bond
  zt* gk;              // Gamma of site k   (padded [d_max][chi_cap][chi_cap])
  zt* gk1;             // Gamma of site k+1
  const double* lam_l; // lambda left of site k (nullptr: chain edge, 1)
  const double* lam_r; // lambda right of site k+1 (nullptr: chain edge, 1)
  double* lam_mid;     // lambda of the updated bond
  int32_t* chi_slot;   // chi entry of the updated bond
  const zt* gate;      // (dl dr) x (dl dr), leading dim gate_ld
  int32_t gate_ld;
  int32_t chi_cap;     // padding capacity of the MPS arrays
  double lambda_floor;
  // recording for the adjoint (nullptr: not recording)
  zt* tape_u;          // U of every computed triplet, m x l row-major (ld tape_ldu)
  zt* tape_vh;         // V^H of every computed triplet, l x n row-major (ld tape_ldvh)
  double* tape_sig;    // the l singular values
  int32_t* tape_hdr;   // TH_* fields
  int32_t tape_ldu, tape_ldvh;
};

constexpr int TK_COUNT_MAX = 16;  // tile kinds of the forward pipeline (enum below)

// Parameters of a launch sequence that are common to all problems.
struct Common {
  int32_t nprob;
  int32_t q;
  double eps;
  uint64_t seed;
  uint32_t stream_id;
  // capacities (grid sizing): max over problems
  int32_t mmax, nmax, lmax, kcap;
  int32_t mmin, nmin, lmin;  // smallest possible sizes (size-class launches)
  int32_t tebd;      // 1: TEBD problems (Theta/gate/reabsorb kernels run)
  int32_t dmax;      // TEBD: max local dim
  int32_t chimax;    // TEBD: chi capacity
  int32_t adaptive;  // two-stage adaptive rank (TEBD only)
  int32_t pass2;     // 1: second (fixed-rank) pass of the adaptive scheme
  int32_t mixed;     // 1: complex FP32 sketch and power-iteration products
  int32_t record;    // 1: write the adjoint's tape
  int32_t nsites;    // TEBD: sites per chain
  int32_t* retry_count;  // device: problems whose first stage was rejected (adaptive rank)
  int32_t* bounds_dev = nullptr;  // host-mapped pinned memory: k_schedule writes {min, max}
                                  // of m, n, l1 there, then the tile total of every kind
  int32_t ktiles[TK_COUNT_MAX] = {-1, -1, -1, -1, -1, -1, -1, -1,
                                  -1, -1, -1, -1, -1, -1, -1, -1};  // host copy of the totals (-1: unknown)
  int32_t* offs;     // device: per tile kind, exclusive prefix sums of tile counts [nprob + 1]
  int32_t grid;      // workgroups of the persistent contraction launches (multiple of 8)
  // TEBD sweeps: the capacity sizes (d_max chi_cap rows, the fixed-rank sketch
  // width) under which the sweep table of the autotune cache is read, the same
  // in every rank mode; 0 elsewhere (the launch's own bounds, table 0)
  int32_t tune_rows = 0, tune_width = 0;
  int32_t serial = 0;  // 1: size classes run in order on the caller's stream (no side streams)
  // device: Accuracy Check, two counters of problems still probing (the
  // rounds alternate), then the widest basis so far
  int32_t* acc_count = nullptr;
  int32_t acc_lcap = 0;          // Accuracy Check: largest basis width (QR classes)
  int32_t acc_r = 0;             // Accuracy Check: probe width
  int32_t retry_read = 0;        // enqueue the host read of *retry_count after the truncation
  int32_t chol = 0;              // 1: Gram-based QR (CholeskyQR2) for the large problems
};

// Kernel-level event timing for tebd_profile_enable / tebd_profile_read:
// while profiling is on, every launch goes through hipExtLaunchKernelGGL
// with a start and a stop event that the dispatch itself records (so the
// interval is the kernel's execution, as profiler tools report it), keyed
// by the kernel's name (a string literal naming the instantiation as those
// tools print it); otherwise it is a plain launch.  prof_kernel_events hands
// out the two events (false when profiling is off), prof_kernel_done files
// them under the name.
bool prof_kernel_events(hipEvent_t* start, hipEvent_t* stop);
void prof_kernel_done(const char* name, hipEvent_t start, hipEvent_t stop);

#define TEBD_LAUNCH(name, kern, grid, block, shmem, strm, ...)                              \
  do {                                                                                      \
    const hipStream_t tebd_launch_s_ = (strm);                                              \
    hipEvent_t tebd_ev_a_ = nullptr, tebd_ev_b_ = nullptr;                                  \
    if (::tebd::prof_kernel_events(&tebd_ev_a_, &tebd_ev_b_)) {                             \
      hipExtLaunchKernelGGL(kern, grid, block, shmem, tebd_launch_s_, tebd_ev_a_, tebd_ev_b_, \
                            0, __VA_ARGS__);                                                \
      ::tebd::prof_kernel_done(name, tebd_ev_a_, tebd_ev_b_);                               \
    } else {                                                                                \
      hipLaunchKernelGGL(kern, grid, block, shmem, tebd_launch_s_, __VA_ARGS__);            \
    }                                                                                       \
  } while (0)

// Accuracy Check: widest probe block, the constant of Theorem 2 with Fact 1
// ((10/3) pi, the larger of the paper's two printed forms), and the slot of
// its two round counters in the workspace's counter area.
constexpr int kAccMaxR = 16;
constexpr double kAccConst = 10.0 * 3.14159265358979323846 / 3.0;
constexpr int kAccCountSlot = 32;

// Contraction kinds scheduled through a global tile queue: every kind has
// its own prefix sum over problems of the number of 64 x 64 output tiles.
enum {
  TK_THETA = 0,  // Theta build: (dl chi_l) x (dr chi_r)
  TK_GATE = 1,   // gate: (dl dr) x (chi_l chi_r)
  TK_SKM = 2,    // m x l products (A Omega, A Q~)
  TK_SKN = 3,    // n x l products (A^H Q)
  TK_FORMU = 4,  // m x (kept capacity)
  TK_FORMV = 5,  // (kept capacity) x n
  TK_TAPEU = 6,  // recording: m x l, U of every computed triplet
  TK_TAPEV = 7,  // recording: l x n, V^H of every computed triplet
  TK_ACB = 8,    // Accuracy Check: m x r probe products A Omega_r
  TK_SKM_W = 9,  // TK_SKM on 64 x 64 tiles (the wide sketch variant)
  TK_SKN_W = 10, // TK_SKN on 64 x 64 tiles
  TK_GRAM = 11,  // Gram-based QR: l x l Gram matrices Y^H Y
  TK_QAPM = 12,  // Gram-based QR: m x l products Y R^-1
  TK_QAPN = 13,  // Gram-based QR: n x l products Yt R^-1
  TK_SKM_S = 14, // TK_SKM on 16 x 16 tiles (the split-depth sketch variant)
  TK_SKN_S = 15, // TK_SKN on 16 x 16 tiles
  TK_COUNT = 16
};

static_assert(TK_COUNT == TK_COUNT_MAX, "Common::ktiles holds one total per kind");

// Autotune cache: tile-shape variant of the sketch, power-iteration and
// projection products (0: 32 x 32 tiles, 1: 64 x 64, 2: split-depth 16 x 16)
// for a launch whose largest problem has max_rows rows and sketch width l;
// table 0 the FP64 products of independent matrices, 1 the FP32 products,
// 2 the FP64 products of TEBD sweeps (read under the MPS capacities)
// (contract.hip).
int sketch_variant(int table, int max_rows, int width);

// Output tiles of the gate product of a group, (dl dr) x (sum of chi_l chi_r
// over its members): 16 x 16, each tile's depth dl dr split over the four
// wavefronts of its workgroup.  The product is short and wide (dl dr rows,
// the members' columns), so small tiles give the launch enough workgroups
// and waste little FP64 matrix-core work on padding when most bonds have
// chi_l chi_r = 1.  Members of at most kGateGroup consecutive chains.
constexpr int kGateTileM = 16, kGateTileN = 16;
constexpr int kGateGroup = 32;

// Frobenius partial sums of one problem: one per (row tile, column tile
// that holds some of its columns) of its group's gate product, in row-tile
// major order.
__host__ __device__ inline int gate_partials(int rows, int col0, int cols) {
  if (rows <= 0 || cols <= 0) return 0;
  const int rt = (rows + kGateTileM - 1) / kGateTileM;
  return rt * ((col0 + cols - 1) / kGateTileN - col0 / kGateTileN + 1);
}
// Capacity: a member's columns start anywhere in a 16-wide tile.
__host__ __device__ inline int gate_partials_cap(int rows, int cols) {
  if (rows <= 0 || cols <= 0) return 0;
  return ((rows + kGateTileM - 1) / kGateTileM) * ((cols + kGateTileN - 1) / kGateTileN + 1);
}

inline size_t sched_bytes(int64_t nprob) { return size_t(TK_COUNT) * size_t(nprob + 1) * sizeof(int32_t); }

// Workgroups of a persistent launch over the tiles of `kind` (and of
// `kind2`, when two queues share the launch): their tile total when the host
// knows it, else the capacity-based c.grid; a multiple of 8 (the XCD-aware
// tile mapping), at least 8, at most c.grid.
inline int32_t grid_for(const Common& c, int kind, int kind2 = -1) {
  int32_t t = c.ktiles[kind];
  if (kind2 >= 0) t = (t < 0 || c.ktiles[kind2] < 0) ? -1 : t + c.ktiles[kind2];
  if (t < 0) return c.grid;
  int32_t g = (t + 7) / 8 * 8;
  if (g < 8) g = 8;
  return g < c.grid ? g : c.grid;
}


// Launchers (defined in the .hip files).  All enqueue on `s` and return the
// first HIP error met, or hipSuccess.
hipError_t launch_plan_sweep(Prob* probs, const Common& c, const tebd_mps& mps, const zt* gates,
                             int64_t gate_chain_stride, int32_t parity, int32_t single_chain,
                             int32_t single_bond, int32_t p_over, char* slab_base,
                             size_t slab_bytes, double* disc, int32_t* status, double lambda_floor,
                             int32_t mixed, int32_t adaptive, char* tape, size_t tape_stride,
                             int32_t* retry_count, int64_t lslab, char* theta_base,
                             size_t theta_stride, hipStream_t s);
hipError_t launch_stage2(Prob* probs, const Common& c, hipStream_t s);
hipError_t launch_schedule(Prob* probs, const Common& c, hipStream_t s);
hipError_t launch_theta_gate(Prob* probs, const Common& c, hipStream_t s);
// ||A||_F^2 of caller-supplied matrices: kFrobSlices partial sums per
// problem (row slices, one workgroup each) into part; the truncation adds
// them up in order.
constexpr int kFrobSlices = 32;
hipError_t launch_frob(Prob* probs, const Common& c, hipStream_t s);
hipError_t launch_omega(Prob* probs, const Common& c, hipStream_t s);
hipError_t launch_sketch(Prob* probs, const Common& c, int which, hipStream_t s);
hipError_t launch_sketch_f32(Prob* probs, const Common& c, int which, hipStream_t s);
// pivot: column pivoting with the rank tolerance (with want_r it would keep
// every column); 0: plain Householder in column order, every column kept
// gate 1: only the problems whose basis the Accuracy Check just grew;
// gate 2: only the problems the Gram-based QR did not finish.
hipError_t launch_qr(Prob* probs, const Common& c, int which, int want_r, int pivot, hipStream_t s,
                     int gate = 0);
// Gram-based QR (CholeskyQR2) of the large problems of a QR step (which: 0
// the m x l sketch Y, 1 the n x l sketch Yt), before launch_qr(..., gate 2).
// want_r: also R (into Rb, column order) for the QR of B^H.
hipError_t launch_chol_qr(Prob* probs, const Common& c, int which, hipStream_t s, int want_r = 0);
hipError_t launch_chol_mark(Prob* probs, const Common& c, hipStream_t s);
hipError_t launch_gram(Prob* probs, const Common& c, int which, int pass, hipStream_t s);
hipError_t launch_qapply(Prob* probs, const Common& c, int which, hipStream_t s);
// Accuracy Check round: B = A Omega_r into the columns after the basis, then
// the probe residual, the decision and the growth of the basis.
hipError_t launch_acc_probe(Prob* probs, const Common& c, hipStream_t s);
hipError_t launch_acc_resid(Prob* probs, const Common& c, int round, hipStream_t s);
// Small SVD of every problem, then its truncation (chi', lambda', w, status).
hipError_t launch_small_svd(Prob* probs, const Common& c, hipStream_t s);
hipError_t launch_form_uv(Prob* probs, const Common& c, hipStream_t s);
hipError_t launch_tape(Prob* probs, const Common& c, hipStream_t s);

// Sketch-product selectors for launch_sketch.
enum {
  SK_Y_FROM_OMEGA = 0,  // Y  = A Omega
  SK_YT_FROM_Y = 1,     // Yt = A^H Y
  SK_Y_FROM_YT = 2      // Y  = A Yt
};

// Workspace carving helpers (host and device).
__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes of one problem's scratch slab for the given capacities.
__host__ __device__ inline size_t slab_bytes(int64_t m, int64_t n, int64_t l, int tebd, int mixed,
                                             int64_t npart) {
  size_t b = 0;
  const size_t z = sizeof(zt);
  if (tebd) b += align256(m * n * z);  // A (a TEBD sweep keeps Theta in a region of its own)
  // with the Gram-based QR, Y, Yt and Qc trade places: each holds max(m, n) rows
  const int64_t rows_y = (!tebd || mixed) && n > m ? n : m;
  const int64_t rows_yt = (!tebd || mixed) && m > n ? m : n;
  b += align256(n * l * z);          // Omega
  b += align256(rows_y * l * z);     // Y
  b += align256(rows_yt * l * z);    // Yt
  b += 5 * align256(l * l * z);      // Rb, C, J, X, W
  b += align256(2 * (m > n ? m : n) * z);  // reflector staging of the global-memory QR
  if (!tebd || mixed) b += align256((m > n ? m : n) * l * z);  // Qc of the Gram-based QR
  b += align256(l * sizeof(double)); // sig
  b += align256(l * sizeof(int32_t));  // piv
  b += align256(npart * sizeof(double));
  if (mixed) b += align256(m * n * sizeof(float2));  // complex64 copy of A
  return b;
}

// Carve one slab into the scratch pointers of a descriptor.
__host__ __device__ inline void carve_slab(Prob& p, char* base, int64_t m, int64_t n, int64_t l,
                                           int tebd, int mixed, int64_t npart) {
  const size_t z = sizeof(zt);
  char* c = base;
  p.T = nullptr;
  if (tebd) {
    p.A = reinterpret_cast<zt*>(c);
    c += align256(m * n * z);
  }
  p.om = reinterpret_cast<const zt*>(c);
  c += align256(n * l * z);
  const int64_t rows_y = (!tebd || mixed) && n > m ? n : m;
  const int64_t rows_yt = (!tebd || mixed) && m > n ? m : n;
  p.Y = reinterpret_cast<zt*>(c);
  c += align256(rows_y * l * z);
  p.Yt = reinterpret_cast<zt*>(c);
  c += align256(rows_yt * l * z);
  p.Rb = reinterpret_cast<zt*>(c);
  c += align256(l * l * z);
  p.C = reinterpret_cast<zt*>(c);
  c += align256(l * l * z);
  p.J = reinterpret_cast<zt*>(c);
  c += align256(l * l * z);
  p.X = reinterpret_cast<zt*>(c);
  c += align256(l * l * z);
  p.W = reinterpret_cast<zt*>(c);
  c += align256(l * l * z);
  p.qru = reinterpret_cast<zt*>(c);
  c += align256(2 * (m > n ? m : n) * z);
  p.Qc = nullptr;
  if (!tebd || mixed) {
    p.Qc = reinterpret_cast<zt*>(c);
    c += align256((m > n ? m : n) * l * z);
  }
  p.sig = reinterpret_cast<double*>(c);
  c += align256(l * sizeof(double));
  p.piv = reinterpret_cast<int32_t*>(c);
  c += align256(l * sizeof(int32_t));
  p.part = reinterpret_cast<double*>(c);
  c += align256(npart * sizeof(double));
  p.Af = nullptr;
  if (mixed) {
    p.Af = reinterpret_cast<float2*>(c);
    c += align256(m * n * sizeof(float2));
  }
}

// ---------------------------------------------------------------------------
// Tape of one recorded sweep: one fixed-size slot per problem, in the order
// of the sweep's problems (chain-major, bonds of the parity ascending).
// Slot: 256-byte header of int32 TH_* fields, the l singular values, U
// (mcap x lcap row-major), V^H (lcap x ncap row-major).
enum {
  TH_VALID = 0,  // 1: the slot holds a finished bond update
  TH_L,          // triplets computed (sketch width after the range finder)
  TH_K,          // triplets kept (chi')
  TH_M,
  TH_N,
  TH_CHI_L,
  TH_CHI_M,      // bond dimension before the update
  TH_CHI_R,
  TH_DL,
  TH_DR,
  TH_CHAIN,
  TH_BOND,
  TH_LCAP,
  TH_COUNT
};

__host__ __device__ inline size_t tape_slot_bytes(int64_t mcap, int64_t ncap, int64_t lcap) {
  return 256 + align256(size_t(lcap) * sizeof(double)) + align256(size_t(mcap * lcap) * sizeof(zt)) +
         align256(size_t(lcap * ncap) * sizeof(zt));
}
__host__ __device__ inline void tape_slot(char* base, int64_t mcap, int64_t lcap, int32_t*& hdr,
                                          double*& sig, zt*& u, zt*& vh) {
  hdr = reinterpret_cast<int32_t*>(base);
  sig = reinterpret_cast<double*>(base + 256);
  u = reinterpret_cast<zt*>(base + 256 + align256(size_t(lcap) * sizeof(double)));
  vh = u + align256(size_t(mcap * lcap) * sizeof(zt)) / sizeof(zt);
}

// ---------------------------------------------------------------------------
// Adjoint of one bond update (reverse mode), per problem.
struct AdjProb {
  int32_t m, n, L, k;              // blocked matrix, triplets computed / kept
  int32_t chi_l, chi_m, chi_r, dl, dr;
  int32_t nchunk;                  // K-chunks of the gate cotangent product
  int32_t chain, bond;
  int32_t ldu, ldvh, ldl, chi_cap, gate_ld, dmax;
  double lambda_floor, eta;        // eta: broadening of 1/(s_j^2 - s_i^2)
  // tape of the recorded update
  const zt* U;                     // m x L (ld ldu)
  const zt* VH;                    // L x n (ld ldvh)
  const double* sig;               // L, descending
  // state before the update
  const zt* gk;
  const zt* gk1;
  const double* lam_l;             // nullptr at the chain edge (1)
  const double* lam_m;
  const double* lam_r;             // nullptr at the chain edge (1)
  const zt* gate;
  // cotangents (in: of the update's outputs; out: of its inputs)
  zt* gbk;
  zt* gbk1;
  double* lbar_m;
  zt* gate_bar;
  int32_t* status;
  // scratch
  double* sbar;                    // L
  double* sinv;                    // L
  double* lamL;                    // chi_l: contribution to the cotangent of lambda_l
  double* lamR;                    // chi_r
  zt* M1;                          // L x k: U^H Ubar        (ld ldl)
  zt* M2;                          // L x k: V^H Vbar        (ld ldl)
  zt* D;                           // L x L core matrix      (ld ldl)
  zt* X;                           // m x L: U D + Ubar S^-1 (ld ldl)
  zt* AbT;                         // Abar as [(i j)][(a c)]
  zt* T;                           // Theta as [(i j)][(a c)]
  zt* Thb;                         // Theta-bar, blocked [(i a)][(j c)]
  zt* R1;                          // m x chi_m (ld chi_cap)
  zt* R2;                          // chi_m x n (ld ldvh)
  zt* gpart;                       // nchunk x (dl dr)^2 partial gate cotangents
};

enum {
  TA_M1 = 0,     // L x k
  TA_M2 = 1,     // L x k
  TA_THETA = 2,  // (dl chi_l) x (dr chi_r)
  TA_X = 3,      // m x L
  TA_ABAR = 4,   // m x n
  TA_GADJ = 5,   // (dl dr) x (chi_l chi_r)
  TA_GBAR = 6,   // per K-chunk: (dl dr) x (dl dr), chunks stacked on 64-row boundaries
  TA_R1 = 7,     // m x chi_m
  TA_R2 = 8,     // chi_m x n
  TA_COUNT = 9
};
constexpr int kGateChunk = 1024;  // K-chunk of the gate cotangent product

struct AdjCommon {
  int32_t nprob;
  int32_t n_chains, n_sites, parity, nb;
  int64_t gate_chain_stride;
  int32_t* offs;
  int32_t grid;
};

__host__ __device__ inline size_t adj_slab_bytes(int64_t mcap, int64_t ncap, int64_t lcap,
                                                 int64_t chicap, int64_t d2, int64_t nchunk) {
  const size_t z = sizeof(zt), d = sizeof(double);
  return 2 * align256(lcap * d) + 2 * align256(chicap * d) + 3 * align256(lcap * lcap * z) +
         align256(mcap * lcap * z) + 3 * align256(mcap * ncap * z) + align256(mcap * chicap * z) +
         align256(chicap * ncap * z) + align256(nchunk * d2 * d2 * z);
}

hipError_t launch_adjoint(AdjProb* probs, const AdjCommon& c, const tebd_mps& mps_in,
                          const zt* gates, const char* tape, size_t slot_bytes, int64_t mcap,
                          int64_t lcap, zt* gamma_bar, double* lambda_bar, zt* gate_bar,
                          int32_t* status, double lambda_floor, char* slab_base, size_t slab_sz,
                          int64_t nchunk_cap, hipStream_t s);

// Largest l (sketch width) and m supported by the factorisation kernels.
constexpr int kMaxL = 256;
constexpr int kMaxRows = 8192;

}  // namespace tebd
