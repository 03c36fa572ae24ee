// Host side of the C interface declared in include/tebd_rrsvd.h: argument
// validation, workspace planning and the launch sequence of the bond update.
//
// Launch sequence of one batch (Tamascelli, Rosenbach, Plenio,
// arXiv:1504.00992): [TEBD: Theta build, Eq. deftheta, and gate,
// Eq. defupdatetheta] -> Omega -> Alg. 1 (Y0 = A Omega, QR; q times
// A^H Q, QR, A Q~, QR) -> B^H = A^H Q and its QR (Sec. IV step i) -> small
// SVD (step ii) -> truncation rule (Sec. II.C) -> U = Q X, V^H = (Q_B W)^H
// with lambda^-1 reabsorption (step iii and Sec. II.B).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"

using namespace tebd;

namespace {

thread_local char g_err[512] = "";

tebd_status fail(tebd_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

tebd_status ok() {
  g_err[0] = '\0';
  return TEBD_OK;
}

tebd_status check_params(const tebd_params* prm) {
  if (!prm) return fail(TEBD_ERR_ARG, "argument prm is NULL");
  if (prm->chi_max < 1) return fail(TEBD_ERR_ARG, "prm->chi_max = %d must be >= 1", prm->chi_max);
  if (prm->p < 0) return fail(TEBD_ERR_ARG, "prm->p = %d must be >= 0", prm->p);
  if (prm->q < 0 || prm->q > 64) return fail(TEBD_ERR_ARG, "prm->q = %d must be in [0, 64]", prm->q);
  if (prm->precision != 0 && prm->precision != 1)
    return fail(TEBD_ERR_ARG, "prm->precision = %d must be 0 or 1", prm->precision);
  if (!std::isfinite(prm->trunc_eps))
    return fail(TEBD_ERR_ARG, "prm->trunc_eps must be finite");
  if (!(prm->lambda_floor >= 0.0) || !std::isfinite(prm->lambda_floor))
    return fail(TEBD_ERR_ARG, "prm->lambda_floor must be finite and >= 0");
  if (prm->adaptive < 0 || prm->adaptive > 3)
    return fail(TEBD_ERR_ARG, "prm->adaptive = %d must be 0, 1, 2 or 3", prm->adaptive);
  if (prm->adaptive == 3 && prm->p < 1)
    return fail(TEBD_ERR_ARG, "prm->adaptive = 3 (Accuracy Check) needs prm->p >= 1");
  if (prm->adaptive && !(prm->trunc_eps > 0.0))
    return fail(TEBD_ERR_ARG, "prm->adaptive = %d needs prm->trunc_eps > 0", prm->adaptive);
  return TEBD_OK;
}

tebd_status check_mps(const tebd_mps* mps, const tebd_params* prm) {
  if (!mps) return fail(TEBD_ERR_ARG, "argument mps is NULL");
  if (mps->n_chains < 1) return fail(TEBD_ERR_SHAPE, "mps->n_chains = %d must be >= 1", mps->n_chains);
  if (mps->n_sites < 2) return fail(TEBD_ERR_SHAPE, "mps->n_sites = %d must be >= 2", mps->n_sites);
  if (mps->d_max < 1) return fail(TEBD_ERR_SHAPE, "mps->d_max = %d must be >= 1", mps->d_max);
  if (mps->chi_max < 1) return fail(TEBD_ERR_SHAPE, "mps->chi_max = %d must be >= 1", mps->chi_max);
  if (!mps->d) return fail(TEBD_ERR_ARG, "mps->d is NULL");
  if (!mps->gamma) return fail(TEBD_ERR_ARG, "mps->gamma is NULL");
  if (!mps->lambda) return fail(TEBD_ERR_ARG, "mps->lambda is NULL");
  if (!mps->chi) return fail(TEBD_ERR_ARG, "mps->chi is NULL");
  if (int64_t(mps->d_max) * mps->chi_max > kMaxRows)
    return fail(TEBD_ERR_SHAPE, "d_max * chi_max = %lld exceeds the supported %d",
                (long long)(int64_t(mps->d_max) * mps->chi_max), kMaxRows);
  if (prm && prm->chi_max > mps->chi_max)
    return fail(TEBD_ERR_SHAPE, "prm->chi_max = %d exceeds the MPS capacity mps->chi_max = %d",
                prm->chi_max, mps->chi_max);
  if (prm) {
    const int64_t mc = int64_t(mps->d_max) * mps->chi_max;
    const int64_t l = int64_t(prm->chi_max) + prm->p < mc ? int64_t(prm->chi_max) + prm->p : mc;
    if (l > kMaxL) return fail(TEBD_ERR_SHAPE, "sketch width %lld exceeds the supported %d", (long long)l, kMaxL);
  }
  return TEBD_OK;
}

int sketch_l(int64_t k, int64_t p, int64_t m, int64_t n) {
  int64_t l = k + p;
  if (l > m) l = m;
  if (l > n) l = n;
  return int(l);
}

// Workspace plan of a TEBD sweep: descriptors for the largest parity, then
// one capacity-sized slab per problem.
struct SweepPlan {
  int64_t pmax;
  int64_t mcap, lcap, lslab, npart;
  size_t desc_bytes, slab_sz;
  // Theta of the gate groups: one capacity-sized block per problem after the
  // slabs; a group's Theta spans the blocks of its members
  size_t theta_off, theta_sz;
  // reverse mode of a sweep (same workspace)
  int64_t nchunk;
  size_t adj_desc_bytes, adj_slab_sz;
  size_t tape_slot;
  size_t total;      // forward sweep
  size_t adj_total;  // adjoint sweep (and the recorded forward): max of both
};

SweepPlan plan_sweep(const tebd_mps& mps, const tebd_params& prm) {
  SweepPlan s;
  const int64_t nb = mps.n_sites / 2;  // bonds of parity 0 (the larger set)
  s.pmax = int64_t(mps.n_chains) * nb;
  s.mcap = int64_t(mps.d_max) * mps.chi_max;
  s.lcap = sketch_l(prm.chi_max, prm.p, s.mcap, s.mcap);
  // the Accuracy Check writes a probe block of up to p columns after the basis
  const int64_t lslab = prm.adaptive == 3 ? s.lcap + prm.p : s.lcap;
  s.npart = gate_partials_cap(mps.d_max * mps.d_max, mps.chi_max * mps.chi_max);
  // descriptors, tile-queue offsets, then 256 bytes of counters
  s.desc_bytes = align256(size_t(s.pmax) * sizeof(Prob)) + align256(sched_bytes(s.pmax)) + 256;
  s.lslab = lslab;
  s.slab_sz = slab_bytes(s.mcap, s.mcap, lslab, 1, prm.precision, s.npart);
  const int64_t cap = mps.chi_max, d2 = int64_t(mps.d_max) * mps.d_max;
  s.nchunk = (cap * cap + kGateChunk - 1) / kGateChunk;
  s.adj_desc_bytes = align256(size_t(s.pmax) * sizeof(AdjProb)) +
                     align256(size_t(TA_COUNT) * size_t(s.pmax + 1) * sizeof(int32_t));
  s.adj_slab_sz = adj_slab_bytes(s.mcap, s.mcap, s.lcap, cap, d2, s.nchunk);
  s.tape_slot = tape_slot_bytes(s.mcap, s.mcap, s.lcap);
  s.theta_sz = align256(size_t(s.mcap) * size_t(s.mcap) * sizeof(zt));
  s.theta_off = s.desc_bytes + size_t(s.pmax) * s.slab_sz;
  s.total = s.theta_off + size_t(s.pmax) * s.theta_sz;
  const size_t adj = s.adj_desc_bytes + size_t(s.pmax) * s.adj_slab_sz;
  s.adj_total = s.total > adj ? s.total : adj;
  return s;
}

// Pinned staging ring for descriptor uploads of the standalone RRSVD.  Each
// slot is reused only after the copy that last read it has completed.
struct Staging {
  std::mutex mu;
  static constexpr int kSlots = 4;
  char* buf[kSlots] = {nullptr, nullptr, nullptr, nullptr};
  size_t cap[kSlots] = {0, 0, 0, 0};
  hipEvent_t ev[kSlots] = {nullptr, nullptr, nullptr, nullptr};
  int next = 0;
};
Staging g_stage;

hipError_t upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_stage.mu);
  const int k = g_stage.next;
  g_stage.next = (k + 1) % Staging::kSlots;
  hipError_t e;
  if (g_stage.ev[k]) {
    e = hipEventSynchronize(g_stage.ev[k]);
    if (e != hipSuccess) return e;
  } else {
    e = hipEventCreateWithFlags(&g_stage.ev[k], hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  if (g_stage.cap[k] < bytes) {
    if (g_stage.buf[k]) {
      e = hipHostFree(g_stage.buf[k]);
      if (e != hipSuccess) return e;
      g_stage.buf[k] = nullptr;
      g_stage.cap[k] = 0;
    }
    size_t want = bytes < (1u << 16) ? (1u << 16) : bytes;
    e = hipHostMalloc(reinterpret_cast<void**>(&g_stage.buf[k]), want, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    g_stage.cap[k] = want;
  }
  std::memcpy(g_stage.buf[k], src, bytes);
  e = hipMemcpyAsync(dst, g_stage.buf[k], bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipEventRecord(g_stage.ev[k], s);
}

// Reads of small device counters through pinned host memory (one buffer per
// host thread): counters_async enqueues the copy of n <= 32 values on s,
// counters_wait blocks until it has landed.  One read at a time per thread.
// The size bounds and tile totals of a batch take another route: k_schedule
// stores them straight into slots kBoundsSlot.. of the same (coherent,
// device-mapped) buffer, and the host waits for an event after it.
struct PinnedCounters {
  int32_t* buf = nullptr;   // host view
  int32_t* dbuf = nullptr;  // device view of the same memory
  hipEvent_t done = nullptr;
  hipEvent_t bounds = nullptr;
};
constexpr int kBoundsSlot = 32;

PinnedCounters& pinned_counters() {
  static thread_local PinnedCounters pc;
  return pc;
}

hipError_t pinned_init(PinnedCounters& pc) {
  hipError_t e = hipSuccess;
  if (!pc.buf)
    e = hipHostMalloc(reinterpret_cast<void**>(&pc.buf), 256,
                      hipHostMallocMapped | hipHostMallocPortable | hipHostMallocCoherent);
  if (e == hipSuccess && !pc.dbuf) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&pc.dbuf), pc.buf, 0);
  if (e == hipSuccess && !pc.done) e = hipEventCreateWithFlags(&pc.done, hipEventDisableTiming);
  if (e == hipSuccess && !pc.bounds) e = hipEventCreateWithFlags(&pc.bounds, hipEventDisableTiming);
  return e;
}

hipError_t counters_async(const int32_t* dev, int n, hipStream_t s) {
  PinnedCounters& pc = pinned_counters();
  hipError_t e = pinned_init(pc);
  if (e == hipSuccess) e = hipMemcpyAsync(pc.buf, dev, size_t(n) * sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(pc.done, s);
  return e;
}

hipError_t counters_wait(int32_t* out, int n) {
  PinnedCounters& pc = pinned_counters();
  hipError_t e = hipEventSynchronize(pc.done);
  if (e == hipSuccess)
    for (int i = 0; i < n; ++i) out[i] = pc.buf[i];
  return e;
}

// Device address k_schedule writes the bounds to (host-mapped memory).
hipError_t bounds_target(int32_t** dev) {
  PinnedCounters& pc = pinned_counters();
  hipError_t e = pinned_init(pc);
  if (e == hipSuccess) *dev = pc.dbuf + kBoundsSlot;
  return e;
}

hipError_t bounds_ready(hipStream_t s) { return hipEventRecord(pinned_counters().bounds, s); }

hipError_t bounds_wait(int32_t* out, int n) {
  PinnedCounters& pc = pinned_counters();
  hipError_t e = hipEventSynchronize(pc.bounds);
  if (e == hipSuccess)
    for (int i = 0; i < n; ++i) out[i] = reinterpret_cast<volatile int32_t*>(pc.buf)[kBoundsSlot + i];
  return e;
}

// Blocking read of one device counter, ordered after everything on s.
hipError_t read_counter(const int32_t* dev, int32_t* out, hipStream_t s) {
  hipError_t e = counters_async(dev, 1, s);
  return e == hipSuccess ? counters_wait(out, 1) : e;
}

// Optional per-kernel event timing (tebd_profile_enable / tebd_profile_read).
enum ProfKind {
  PK_PLAN, PK_SCHEDULE, PK_THETA_GATE, PK_FROB, PK_OMEGA, PK_SKETCH_AOM, PK_SKETCH_AHQ,
  PK_SKETCH_AQT, PK_QR, PK_QR_R, PK_SMALL_SVD, PK_FORM_UV, PK_STAGE2, PK_TAPE,
  PK_ADJOINT, PK_ACC, PK_COUNT
};
const char* const kProfNames[PK_COUNT] = {
    "plan_sweep", "schedule",  "theta_gate", "frobenius",  "omega",    "sketch_A_Omega",
    "sketch_AH_Q", "sketch_A_Qt", "qr",       "qr_with_r", "small_svd",
    "form_u_vh", "stage2_prep", "tape", "adjoint_sweep", "accuracy_check"};

struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  // kernel-level brackets (prof_kernel_begin / prof_kernel_end)
  struct KRec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<KRec> krecs;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void recycle() {
    for (auto& r : recs) {
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
    for (auto& r : krecs) {
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    krecs.clear();
  }
};
Profiler g_prof;

// Run one launcher, bracketed by events when profiling is on.
// The profiler's lock is not held while `launch` runs: the kernel-level
// brackets inside it take the same lock.
template <class F>
hipError_t timed(int kind, hipStream_t s, F&& launch) {
  if (!g_prof.on) return launch();
  hipEvent_t a, b;
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    a = g_prof.get();
    b = g_prof.get();
  }
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (e != hipSuccess) {
    g_prof.pool.push_back(a);
    g_prof.pool.push_back(b);
    return e;
  }
  g_prof.recs.push_back({kind, a, b});
  return hipSuccess;
}

}  // namespace

namespace tebd {

bool prof_kernel_events(hipEvent_t* start, hipEvent_t* stop) {
  if (!g_prof.on) return false;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  *start = g_prof.get();
  *stop = g_prof.get();
  if (*start && *stop) return true;
  if (*start) g_prof.pool.push_back(*start);
  if (*stop) g_prof.pool.push_back(*stop);
  return false;
}

void prof_kernel_done(const char* name, hipEvent_t start, hipEvent_t stop) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (hipGetLastError() != hipSuccess) {
    g_prof.pool.push_back(start);
    g_prof.pool.push_back(stop);
    return;
  }
  g_prof.krecs.push_back({name, start, stop});
}

}  // namespace tebd

namespace {

// Workgroups of the persistent contraction launches: enough to fill the 256
// CUs a few times over, never more than the largest possible tile count.
// Workgroups beyond the tiles still cost dispatch time, so launches whose
// tile totals the host knows use those instead (grid_for).
int32_t persistent_grid(int64_t cap_tiles) {
  int64_t g = cap_tiles < 2048 ? cap_tiles : 2048;
  g = (g + 7) / 8 * 8;
  return int32_t(g < 8 ? 8 : g);
}

// With c.bounds_dev set, the size bounds that k_schedule writes are read back
// while Theta, the gate and Omega run, and replace c's bounds, so that the
// products take the tile variant and grid of the batch's real sizes and only
// the QR size classes the batch reaches are launched.
hipError_t run_pipeline(Prob* probs, Common& c, hipStream_t s) {
  hipError_t e;
#define TRY(x)                     \
  do {                             \
    e = (x);                       \
    if (e != hipSuccess) return e; \
  } while (0)
#define TIMED(kind, call) TRY(timed(kind, s, [&]() { return (call); }))
  // (the sweep planner marks the large problems of a sweep's first pass itself)
  if ((c.pass2 || !c.tebd) && c.chol && tebd_size_class(0, std::max(c.mmax, c.nmax), c.lmax) >= 2)
    TIMED(PK_SCHEDULE, launch_chol_mark(probs, c, s));
  TIMED(PK_SCHEDULE, launch_schedule(probs, c, s));
  if (c.bounds_dev) TRY(bounds_ready(s));
  if (c.tebd) {
    if (!c.pass2) TIMED(PK_THETA_GATE, launch_theta_gate(probs, c, s));
  } else {
    TIMED(PK_FROB, launch_frob(probs, c, s));
  }
  TIMED(PK_OMEGA, launch_omega(probs, c, s));
  // mixed precision: sketch and power-iteration products in complex FP32;
  // the QRs, the final projection and everything after stay FP64
  auto sketch = [&](int which) {
    return c.mixed ? launch_sketch_f32(probs, c, which, s) : launch_sketch(probs, c, which, s);
  };
  // the bounds arrive while Theta, the gate and Omega run: the first sketch
  // product already takes the tile variant and grid of the batch's real sizes
  if (c.bounds_dev) {
    int32_t b[6 + TK_COUNT];
    static_assert(kBoundsSlot + 6 + TK_COUNT <= 64, "bounds fit the pinned buffer");
    TRY(bounds_wait(b, 6 + TK_COUNT));
    c.mmin = b[0];
    c.mmax = b[1];
    c.nmin = b[2];
    c.nmax = b[3];
    c.lmin = b[4];
    c.lmax = b[5];
    for (int k = 0; k < TK_COUNT; ++k) c.ktiles[k] = b[6 + k];
  }
  TIMED(PK_SKETCH_AOM, sketch(SK_Y_FROM_OMEGA));
  // the first QR reveals the sketch's rank (column pivoting); the power
  // iterations keep that rank and orthonormalise without pivoting
  // The large problems may take the Gram-based QR first (when their sketch
  // is well conditioned every column is kept, as the pivoted QR would);
  // the Householder kernels then take every problem it did not finish.
  auto qr_step = [&](int which, int pivot) -> hipError_t {
    // no problem of the batch can reach the Gram path's size classes: skip it
    const int rows_max = which ? c.nmax : c.mmax;
    if (c.chol && tebd_size_class(0, rows_max, c.lmax) >= 2) {
      hipError_t er = timed(PK_QR, s, [&]() { return launch_chol_qr(probs, c, which, s); });
      if (er != hipSuccess) return er;
    }
    const int gate = c.chol && tebd_size_class(0, rows_max, c.lmax) >= 2 ? 2 : 0;
    return timed(PK_QR, s, [&]() { return launch_qr(probs, c, which, 0, pivot, s, gate); });
  };
  TRY(qr_step(0, 1));
  if (c.acc_count) {
    // Accuracy Check rounds: probe, decide, orthonormalise the grown bases;
    // the host reads how many problems still probe after each round, and
    // the widest basis, which bounds the QR classes of the next launches
    // (a round grows a basis by at most acc_r columns)
    Common ca = c;
    const int32_t cap = std::min(c.acc_lcap, std::min(c.mmax, c.nmax));
    int32_t widest = c.lmax;
    ca.lmin = 1;
    for (int round = 0;; ++round) {
      ca.lmax = std::min(cap, widest + c.acc_r);
      TIMED(PK_ACC, launch_acc_probe(probs, ca, s));
      TIMED(PK_ACC, launch_acc_resid(probs, ca, round, s));
      TIMED(PK_QR, launch_qr(probs, ca, 0, 0, 0, s, 1));
      int32_t cnt[3] = {0, 0, 0};
      TRY(counters_async(c.acc_count, 3, s));
      TRY(counters_wait(cnt, 3));
      widest = std::max(1, std::min(cap, cnt[2]));
      if (cnt[round & 1] == 0) break;
    }
    // the sketch widths changed: tile counts anew, QR classes up to the widest basis
    c.lmax = widest;
    c.lmin = 1;
    for (int k = 0; k < TK_COUNT; ++k) c.ktiles[k] = -1;
    Common cr = c;
    cr.bounds_dev = nullptr;
    TIMED(PK_SCHEDULE, launch_schedule(probs, cr, s));
  }
  for (int j = 0; j < c.q; ++j) {
    TIMED(PK_SKETCH_AHQ, sketch(SK_YT_FROM_Y));
    TRY(qr_step(1, 0));
    TIMED(PK_SKETCH_AQT, sketch(SK_Y_FROM_YT));
    TRY(qr_step(0, 0));
  }
  TIMED(PK_SKETCH_AHQ, launch_sketch(probs, c, SK_YT_FROM_Y, s));  // B^H = A^H Q
  // B^H = Q_B R_B in column order: the one-sided Jacobi on R_B^H that follows
  // converges in as many sweeps as after a pivoted QR, and the QR is cheaper.
  // The large problems try the Gram-based QR first (R_B = R_2 R_1).
  {
    const bool gram_r = c.chol && tebd_size_class(0, c.nmax, c.lmax) >= 2;
    if (gram_r) TIMED(PK_QR_R, launch_chol_qr(probs, c, 1, s, 1));
    TIMED(PK_QR_R, launch_qr(probs, c, 1, 1, 0, s, gram_r ? 2 : 0));
  }
  {
    // the small SVD works on the revealed rank, anywhere in [1, l1]; each
    // launch ends with the truncation of its problems
    Common cs = c;
    cs.lmin = 1;
    TIMED(PK_SMALL_SVD, launch_small_svd(probs, cs, s));
  }
  // the host's read of the rejected first stages lands while U and V^H form
  if (c.retry_read) TRY(counters_async(c.retry_count, 1, s));
  TIMED(PK_FORM_UV, launch_form_uv(probs, c, s));
  if (c.record) TIMED(PK_TAPE, launch_tape(probs, c, s));
#undef TIMED
#undef TRY
  return hipSuccess;
}

tebd_status enqueue_sweep(const tebd_mps* mps, const tebd_z* gates, int64_t gate_chain_stride,
                          int32_t parity, int32_t single_chain, int32_t single_bond,
                          const tebd_params* prm, double* disc, int32_t* status, void* ws,
                          size_t ws_bytes, void* stream, void* tape = nullptr) {
  const SweepPlan pl = plan_sweep(*mps, *prm);
  if (!ws) return fail(TEBD_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(TEBD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < pl.total)
    return fail(TEBD_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, pl.total);
  Common c;
  const int64_t nb = (mps->n_sites - parity) / 2;
  c.nprob = single_chain >= 0 ? 1 : int32_t(int64_t(mps->n_chains) * nb);
  c.q = prm->q;
  c.eps = prm->trunc_eps;
  c.seed = prm->seed;
  c.stream_id = prm->stream_id;
  c.mmax = int32_t(pl.mcap);
  c.nmax = int32_t(pl.mcap);
  c.lmax = int32_t(pl.lcap);
  c.mmin = c.nmin = c.lmin = 1;  // bond dimensions are only known on the device
  c.tune_rows = int32_t(pl.mcap);
  c.tune_width = int32_t(pl.lcap);
  c.kcap = prm->chi_max;
  c.tebd = 1;
  c.adaptive = prm->adaptive;
  c.pass2 = 0;
  c.mixed = prm->precision;
  c.chol = prm->precision == 1 ? 1 : 0;  // the FP32-product path uses CholeskyQR2 where it can
  c.record = tape != nullptr;
  c.nsites = mps->n_sites;
  c.retry_count = prm->adaptive
                      ? reinterpret_cast<int32_t*>(reinterpret_cast<char*>(ws) + pl.desc_bytes - 256)
                      : nullptr;
  c.dmax = mps->d_max;
  c.chimax = mps->chi_max;
  c.offs = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(ws) +
                                      align256(size_t(pl.pmax) * sizeof(Prob)));
  {
    const int64_t t = (pl.mcap + 63) / 64;
    const int64_t tq = gate_partials_cap(mps->d_max * mps->d_max, mps->chi_max * mps->chi_max);
    c.grid = persistent_grid(int64_t(c.nprob) * (t * t > tq ? t * t : tq));
  }
  if (c.nprob == 0) return ok();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Prob* probs = reinterpret_cast<Prob*>(ws);
  char* slabs = reinterpret_cast<char*>(ws) + pl.desc_bytes;
  // The host-synchronising adaptive mode also reads the batch's size bounds
  // and tile totals.  Until they arrive, the grids of the first contractions
  // follow the totals of the previous sweep of this parity on this host
  // thread, with a quarter of headroom: any grid covers every tile (the
  // launches are persistent), so the estimate only affects speed.
  static thread_local int32_t last_tiles[2][TK_COUNT] = {
      {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1},
      {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1}};
  static_assert(TK_COUNT == 16, "one -1 per tile kind above");
  if (c.adaptive == 3) {
    c.acc_count = c.retry_count + kAccCountSlot;
    c.acc_lcap = int32_t(pl.lcap);
    c.acc_r = std::max(1, std::min(prm->p, kAccMaxR));
  }
  if (c.adaptive == 2 || c.adaptive == 3) {
    if (bounds_target(&c.bounds_dev) != hipSuccess)
      return fail(TEBD_ERR_DEVICE, "cannot map the pinned buffer of the size bounds");
    for (int k = 0; k < TK_COUNT; ++k) {
      const int32_t t = last_tiles[parity & 1][k];
      c.ktiles[k] = t < 0 ? -1 : t + t / 4;
    }
  }
  hipError_t e = timed(PK_PLAN, s, [&]() {
    return launch_plan_sweep(probs, c, *mps, reinterpret_cast<const zt*>(gates), gate_chain_stride,
                             parity, single_chain, single_bond, prm->p, slabs, pl.slab_sz, disc,
                             status, prm->lambda_floor, prm->precision, prm->adaptive,
                             reinterpret_cast<char*>(tape), pl.tape_slot, c.retry_count,
                             pl.lslab, reinterpret_cast<char*>(ws) + pl.theta_off, pl.theta_sz,
                             s);
  });
  c.retry_read = c.adaptive == 2;
  if (e == hipSuccess) e = run_pipeline(probs, c, s);
  c.retry_read = 0;
  if (c.bounds_dev) {
    for (int k = 0; k < TK_COUNT; ++k) last_tiles[parity & 1][k] = c.ktiles[k];
    // the second pass runs the fixed-rank stage: width min(chi_max + p, m, n)
    const int32_t l2 = prm->chi_max + prm->p;
    c.lmin = std::min(l2, std::min(c.mmin, c.nmin));
    c.lmax = std::min(l2, std::min(c.mmax, c.nmax));
    c.bounds_dev = nullptr;
    for (int k = 0; k < TK_COUNT; ++k) c.ktiles[k] = -1;  // the second pass schedules anew
  }
  bool second = c.adaptive == 1 || c.adaptive == 2;
  if (e == hipSuccess && c.adaptive == 2) {
    // the number of rejected first stages (its copy was enqueued after the
    // truncation): an empty second pass is skipped
    int32_t n_retry = 0;
    e = counters_wait(&n_retry, 1);
    second = n_retry > 0;
  }
  if (e == hipSuccess && second) {
    // second pass: only problems whose first stage was rejected do any work
    e = timed(PK_STAGE2, s, [&]() { return launch_stage2(probs, c, s); });
    c.pass2 = 1;
    if (e == hipSuccess) e = run_pipeline(probs, c, s);
  }
  if (e != hipSuccess) return fail(TEBD_ERR_DEVICE, "HIP error while enqueuing: %s", hipGetErrorString(e));
  return ok();
}

// Static scratch of rrsvd_truncate_noalloc, one copy per device (the code
// object's global), used through the address hipGetSymbolAddress gives on
// each device: the array's name is not a device address in host code.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Descriptors of the standalone RRSVD written on the device from kernel
// arguments (by value, so no host buffer outlives the call): up to
// kDescPerLaunch problems per launch, one lane each, the same fields as
// the host-built descriptors of rrsvd_truncate.
constexpr int kDescPerLaunch = 48;
struct DescArgs {
  int32_t first, count, chi_max, oversample, precision, om_ext;
  int64_t ldu, ldvh;
  Prob* probs;
  int32_t* chi_out;
  double* disc;
  int32_t* status;
  struct One {
    int32_t m, n;
    int64_t lda;
    const zt* A;
    const zt* om;
    zt* U;
    double* S;
    zt* VH;
    char* slab;
  } prob[kDescPerLaunch];
};
static_assert(sizeof(DescArgs) <= 4096, "kernel arguments of k_noalloc_desc");

__global__ void k_noalloc_desc(DescArgs a) {
  const int i = threadIdx.x;
  if (i >= a.count) return;
  const DescArgs::One& o = a.prob[i];
  const int32_t b = a.first + i;
  Prob P{};
  int32_t l = a.chi_max + a.oversample;
  l = l < o.m ? l : o.m;
  l = l < o.n ? l : o.n;
  P.m = o.m;
  P.n = o.n;
  P.l = l;
  P.kcap = a.chi_max;
  P.k1 = a.chi_max;
  P.l1 = P.l2 = l;
  P.pid = b;
  P.mixed = a.precision;
  carve_slab(P, o.slab, o.m, o.n, l, 0, a.precision, kFrobSlices);
  P.A = const_cast<zt*>(o.A);
  P.lda = o.lda;
  if (a.om_ext) {
    P.om = o.om;
    P.om_ext = 1;
  }
  P.ldom = l;
  P.U = o.U;
  P.ldu = a.ldu;
  P.S = o.S;
  P.VH = o.VH;
  P.ldvh = a.ldvh;
  P.chi_out = a.chi_out + b;
  P.disc = a.disc + b;
  P.status = a.status + b;
  a.probs[b] = P;
}

// Validation, planning and launch sequence of rrsvd_truncate.  With
// noalloc set the workspace is the library's static scratch: the
// descriptors are written on the device from kernel arguments (no host
// staging buffer) and the size classes run in order on the caller's stream.
tebd_status rrsvd_enqueue(int64_t batch, const int64_t* m, const int64_t* n,
                          const tebd_z* const* A, const int64_t* lda, const tebd_z* const* omega,
                          const tebd_params* prm, tebd_z* const* U, int64_t ldu,
                          double* const* S, tebd_z* const* VH, int64_t ldvh, int32_t* chi_kept,
                          double* disc_weight, int32_t* dev_status, void* workspace,
                          size_t ws_bytes, void* stream, bool noalloc) {
  tebd_status st = check_params(prm);
  if (st != TEBD_OK) return st;
  if (prm->adaptive)
    return fail(TEBD_ERR_ARG, "prm->adaptive: the two-stage rank needs a bond dimension and is "
                              "available in the TEBD entry points only");
  if (batch < 1) return fail(TEBD_ERR_ARG, "argument 1 (batch) = %lld must be >= 1", (long long)batch);
  if (!m) return fail(TEBD_ERR_ARG, "argument 2 (m) is NULL");
  if (!n) return fail(TEBD_ERR_ARG, "argument 3 (n) is NULL");
  if (!A) return fail(TEBD_ERR_ARG, "argument 4 (A) is NULL");
  if (!lda) return fail(TEBD_ERR_ARG, "argument 5 (lda) is NULL");
  if (!U) return fail(TEBD_ERR_ARG, "argument 8 (U) is NULL");
  if (!S) return fail(TEBD_ERR_ARG, "argument 10 (S) is NULL");
  if (!VH) return fail(TEBD_ERR_ARG, "argument 11 (VH) is NULL");
  if (!chi_kept) return fail(TEBD_ERR_ARG, "argument 13 (chi_kept) is NULL");
  if (!disc_weight) return fail(TEBD_ERR_ARG, "argument 14 (disc_weight) is NULL");
  if (!dev_status) return fail(TEBD_ERR_ARG, "argument 15 (dev_status) is NULL");
  if (ldu < prm->chi_max)
    return fail(TEBD_ERR_SHAPE, "argument 9 (ldu) = %lld < chi_max = %d", (long long)ldu, prm->chi_max);
  int64_t nmax = 0;
  for (int64_t b = 0; b < batch; ++b) nmax = n[b] > nmax ? n[b] : nmax;
  if (ldvh < nmax)
    return fail(TEBD_ERR_SHAPE, "argument 12 (ldvh) = %lld < max n = %lld", (long long)ldvh, (long long)nmax);
  for (int64_t b = 0; b < batch; ++b) {
    if (m[b] < 1 || n[b] < 1 || m[b] > kMaxRows || n[b] > kMaxRows)
      return fail(TEBD_ERR_SHAPE, "problem %lld: m = %lld, n = %lld out of range [1, %d]",
                  (long long)b, (long long)m[b], (long long)n[b], kMaxRows);
    if (lda[b] < n[b])
      return fail(TEBD_ERR_SHAPE, "problem %lld: lda = %lld < n = %lld", (long long)b,
                  (long long)lda[b], (long long)n[b]);
    if (!A[b] || !U[b] || !S[b] || !VH[b])
      return fail(TEBD_ERR_ARG, "problem %lld: a device pointer in A/U/S/VH is NULL", (long long)b);
    if (omega && !omega[b])
      return fail(TEBD_ERR_ARG, "problem %lld: omega[b] is NULL", (long long)b);
  }
  size_t need = 0;
  st = tebd_workspace_size(nullptr, batch, m, n, prm, &need);
  if (st != TEBD_OK) return st;
  if (noalloc) {
    if (need > kScratchBytes)
      return fail(TEBD_ERR_WORKSPACE,
                  "the batch needs %zu bytes of scratch; rrsvd_truncate_noalloc has %zu "
                  "(use rrsvd_truncate with a workspace)", need, kScratchBytes);
    hipError_t e = scratch_address(&workspace);
    if (e != hipSuccess)
      return fail(TEBD_ERR_DEVICE, "static scratch address: %s", hipGetErrorString(e));
    ws_bytes = kScratchBytes;
  }
  if (!workspace) return fail(TEBD_ERR_WORKSPACE, "argument 16 (workspace) is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(TEBD_ERR_WORKSPACE, "argument 16 (workspace) must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(TEBD_ERR_WORKSPACE, "argument 17 (ws_bytes) = %zu < %zu needed", ws_bytes, need);

  std::vector<Prob> host(noalloc ? 0 : batch);
  char* base = reinterpret_cast<char*>(workspace);
  char* slab0 = base + align256(size_t(batch) * sizeof(Prob)) + align256(sched_bytes(batch));
  char* slab = slab0;
  Common c;
  c.nprob = int32_t(batch);
  c.q = prm->q;
  c.eps = prm->trunc_eps;
  c.seed = prm->seed;
  c.stream_id = prm->stream_id;
  c.mmax = c.nmax = c.lmax = 0;
  c.mmin = c.nmin = c.lmin = 1 << 30;
  c.kcap = prm->chi_max;
  c.tebd = 0;
  c.adaptive = 0;
  c.pass2 = 0;
  c.mixed = prm->precision;
  c.record = 0;
  c.nsites = 0;
  c.retry_count = nullptr;
  c.dmax = 0;
  c.chimax = 0;
  c.serial = noalloc ? 1 : 0;
  c.chol = 1;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  DescArgs da;
  da.first = 0;
  da.count = 0;
  da.chi_max = prm->chi_max;
  da.oversample = prm->p;
  da.precision = prm->precision;
  da.om_ext = omega ? 1 : 0;
  da.ldu = ldu;
  da.ldvh = ldvh;
  da.probs = reinterpret_cast<Prob*>(workspace);
  da.chi_out = chi_kept;
  da.disc = disc_weight;
  da.status = dev_status;
  int64_t tiles = 0;
  for (int64_t b = 0; b < batch; ++b) {
    {
      const int64_t tm = (m[b] + 63) / 64, tn = (n[b] + 63) / 64;
      const int64_t tk = (prm->chi_max + 63) / 64;
      tiles += (tm > tn ? tm : tn) * (tk > 3 ? tk : 3);
    }
    if (noalloc) {
      const int l = sketch_l(prm->chi_max, prm->p, m[b], n[b]);
      DescArgs::One& o = da.prob[da.count++];
      o.m = int32_t(m[b]);
      o.n = int32_t(n[b]);
      o.lda = lda[b];
      o.A = reinterpret_cast<const zt*>(A[b]);
      o.om = omega ? reinterpret_cast<const zt*>(omega[b]) : nullptr;
      o.U = reinterpret_cast<zt*>(U[b]);
      o.S = S[b];
      o.VH = reinterpret_cast<zt*>(VH[b]);
      o.slab = slab;
      slab += slab_bytes(m[b], n[b], l, 0, prm->precision, kFrobSlices);
      c.mmax = o.m > c.mmax ? o.m : c.mmax;
      c.nmax = o.n > c.nmax ? o.n : c.nmax;
      c.lmax = l > c.lmax ? l : c.lmax;
      c.mmin = o.m < c.mmin ? o.m : c.mmin;
      c.nmin = o.n < c.nmin ? o.n : c.nmin;
      c.lmin = l < c.lmin ? l : c.lmin;
      if (da.count == kDescPerLaunch || b + 1 == batch) {
        hipLaunchKernelGGL(k_noalloc_desc, dim3(1), dim3(64), 0, s, da);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
          return fail(TEBD_ERR_DEVICE, "HIP error while enqueuing: %s", hipGetErrorString(e));
        da.first = int32_t(b + 1);
        da.count = 0;
      }
      continue;
    }
    Prob& P = host[b];
    std::memset(&P, 0, sizeof(Prob));
    P.m = int32_t(m[b]);
    P.n = int32_t(n[b]);
    P.l = sketch_l(prm->chi_max, prm->p, m[b], n[b]);
    P.kcap = prm->chi_max;
    P.k1 = prm->chi_max;
    P.l1 = P.l2 = P.l;
    P.pid = int32_t(b);
    P.mixed = prm->precision;
    carve_slab(P, slab, m[b], n[b], P.l, 0, prm->precision, kFrobSlices);
    slab += slab_bytes(m[b], n[b], P.l, 0, prm->precision, kFrobSlices);
    P.A = const_cast<zt*>(reinterpret_cast<const zt*>(A[b]));
    P.lda = lda[b];
    if (omega) {
      P.om = reinterpret_cast<const zt*>(omega[b]);
      P.om_ext = 1;
    }
    P.ldom = P.l;
    P.U = reinterpret_cast<zt*>(U[b]);
    P.ldu = ldu;
    P.S = S[b];
    P.VH = reinterpret_cast<zt*>(VH[b]);
    P.ldvh = ldvh;
    P.chi_out = chi_kept + b;
    P.disc = disc_weight + b;
    P.status = dev_status + b;
    c.mmax = P.m > c.mmax ? P.m : c.mmax;
    c.nmax = P.n > c.nmax ? P.n : c.nmax;
    c.lmax = P.l > c.lmax ? P.l : c.lmax;
    c.mmin = P.m < c.mmin ? P.m : c.mmin;
    c.nmin = P.n < c.nmin ? P.n : c.nmin;
    c.lmin = P.l < c.lmin ? P.l : c.lmin;
  }
  c.offs = reinterpret_cast<int32_t*>(base + align256(size_t(batch) * sizeof(Prob)));
  c.grid = persistent_grid(tiles);
  hipError_t e = noalloc ? hipSuccess : upload(workspace, host.data(), host.size() * sizeof(Prob), s);
  if (e == hipSuccess) e = run_pipeline(reinterpret_cast<Prob*>(workspace), c, s);
  if (e != hipSuccess) return fail(TEBD_ERR_DEVICE, "HIP error while enqueuing: %s", hipGetErrorString(e));
  return ok();
}

}  // namespace

extern "C" {

const char* tebd_last_error(void) { return g_err; }

const char* tebd_version(void) { return "tebd_rrsvd 0.1 (gfx950, complex128)"; }

tebd_status tebd_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (auto& r : g_prof.recs) {
    (void)hipEventSynchronize(r.b);
  }
  g_prof.recycle();
  g_prof.on = on != 0;
  return ok();
}

tebd_status tebd_profile_read(int32_t capacity, const char** names, double* ms, int64_t* launches,
                              int32_t* count) {
  if (!names || !ms || !launches || !count)
    return fail(TEBD_ERR_ARG, "tebd_profile_read: output arrays must not be NULL");
  std::lock_guard<std::mutex> lk(g_prof.mu);
  double tot[PK_COUNT] = {0};
  int64_t cnt[PK_COUNT] = {0};
  for (auto& r : g_prof.recs) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return fail(TEBD_ERR_DEVICE, "event wait failed: %s", hipGetErrorString(e));
    float t = 0.0f;
    e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) return fail(TEBD_ERR_DEVICE, "event timing failed: %s", hipGetErrorString(e));
    tot[r.kind] += t;
    cnt[r.kind] += 1;
  }
  // kernel-level records, summed per kernel name in first-seen order
  std::vector<const char*> kname;
  std::vector<double> ktot;
  std::vector<int64_t> kcnt;
  for (auto& r : g_prof.krecs) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return fail(TEBD_ERR_DEVICE, "event wait failed: %s", hipGetErrorString(e));
    float t = 0.0f;
    e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) return fail(TEBD_ERR_DEVICE, "event timing failed: %s", hipGetErrorString(e));
    size_t i = 0;
    while (i < kname.size() && std::strcmp(kname[i], r.name) != 0) ++i;
    if (i == kname.size()) {
      kname.push_back(r.name);
      ktot.push_back(0.0);
      kcnt.push_back(0);
    }
    ktot[i] += t;
    kcnt[i] += 1;
  }
  g_prof.recycle();
  int32_t k = 0;
  for (int i = 0; i < PK_COUNT && k < capacity; ++i) {
    if (!cnt[i]) continue;
    names[k] = kProfNames[i];
    ms[k] = tot[i];
    launches[k] = cnt[i];
    ++k;
  }
  for (size_t i = 0; i < kname.size() && k < capacity; ++i) {
    names[k] = kname[i];
    ms[k] = ktot[i];
    launches[k] = kcnt[i];
    ++k;
  }
  *count = k;
  return ok();
}

tebd_status tebd_workspace_size(const tebd_mps* mps, int64_t batch, const int64_t* m,
                                const int64_t* n, const tebd_params* prm, size_t* bytes) {
  if (!bytes) return fail(TEBD_ERR_ARG, "argument bytes is NULL");
  tebd_status st = check_params(prm);
  if (st != TEBD_OK) return st;
  if (mps) {
    st = check_mps(mps, prm);
    if (st != TEBD_OK) return st;
    *bytes = plan_sweep(*mps, *prm).total;
    return ok();
  }
  if (batch < 1) return fail(TEBD_ERR_ARG, "batch = %lld must be >= 1", (long long)batch);
  if (!m || !n) return fail(TEBD_ERR_ARG, "m and n must be host arrays when mps is NULL");
  size_t total = align256(size_t(batch) * sizeof(Prob)) + align256(sched_bytes(batch));
  for (int64_t b = 0; b < batch; ++b) {
    if (m[b] < 1 || n[b] < 1 || m[b] > kMaxRows || n[b] > kMaxRows)
      return fail(TEBD_ERR_SHAPE, "problem %lld: m = %lld, n = %lld out of range [1, %d]",
                  (long long)b, (long long)m[b], (long long)n[b], kMaxRows);
    const int l = sketch_l(prm->chi_max, prm->p, m[b], n[b]);
    if (l > kMaxL) return fail(TEBD_ERR_SHAPE, "problem %lld: sketch width %d > %d", (long long)b, l, kMaxL);
    total += slab_bytes(m[b], n[b], l, 0, prm->precision, kFrobSlices);
  }
  *bytes = total;
  return ok();
}

tebd_status rrsvd_truncate(int64_t batch, const int64_t* m, const int64_t* n,
                           const tebd_z* const* A, const int64_t* lda,
                           const tebd_z* const* omega, const tebd_params* prm,
                           tebd_z* const* U, int64_t ldu, double* const* S,
                           tebd_z* const* VH, int64_t ldvh, int32_t* chi_kept,
                           double* disc_weight, int32_t* dev_status, void* workspace,
                           size_t ws_bytes, void* stream) {
  return rrsvd_enqueue(batch, m, n, A, lda, omega, prm, U, ldu, S, VH, ldvh, chi_kept,
                       disc_weight, dev_status, workspace, ws_bytes, stream, false);
}

tebd_status rrsvd_truncate_noalloc(int64_t batch, const int64_t* m, const int64_t* n,
                                   const tebd_z* const* A, const int64_t* lda,
                                   const tebd_z* const* omega, const tebd_params* prm,
                                   tebd_z* const* U, int64_t ldu, double* const* S,
                                   tebd_z* const* VH, int64_t ldvh, int32_t* chi_kept,
                                   double* disc_weight, int32_t* dev_status, void* stream) {
  return rrsvd_enqueue(batch, m, n, A, lda, omega, prm, U, ldu, S, VH, ldvh, chi_kept,
                       disc_weight, dev_status, nullptr, 0, stream, true);
}

tebd_status tebd_bond_update(const tebd_mps* mps, int32_t chain, int32_t bond,
                             const tebd_z* gate, const tebd_params* prm, double* disc_weight,
                             int32_t* dev_status, void* workspace, size_t ws_bytes,
                             void* stream) {
  tebd_status st = check_params(prm);
  if (st != TEBD_OK) return st;
  st = check_mps(mps, prm);
  if (st != TEBD_OK) return st;
  if (chain < 0 || chain >= mps->n_chains)
    return fail(TEBD_ERR_ARG, "argument 2 (chain) = %d out of range [0, %d)", chain, mps->n_chains);
  if (bond < 0 || bond >= mps->n_sites - 1)
    return fail(TEBD_ERR_ARG, "argument 3 (bond) = %d out of range [0, %d)", bond, mps->n_sites - 1);
  if (!gate) return fail(TEBD_ERR_ARG, "argument 4 (gate) is NULL");
  if (!disc_weight) return fail(TEBD_ERR_ARG, "argument 6 (disc_weight) is NULL");
  if (!dev_status) return fail(TEBD_ERR_ARG, "argument 7 (dev_status) is NULL");
  return enqueue_sweep(mps, gate, 0, bond & 1, chain, bond, prm, disc_weight, dev_status,
                       workspace, ws_bytes, stream);
}

tebd_status tebd_sweep(const tebd_mps* mps, const tebd_z* gates, int64_t gate_chain_stride,
                       int32_t parity, const tebd_params* prm, double* disc_weight,
                       int32_t* dev_status, void* workspace, size_t ws_bytes, void* stream) {
  tebd_status st = check_params(prm);
  if (st != TEBD_OK) return st;
  st = check_mps(mps, prm);
  if (st != TEBD_OK) return st;
  if (!gates) return fail(TEBD_ERR_ARG, "argument 2 (gates) is NULL");
  if (gate_chain_stride < 0)
    return fail(TEBD_ERR_ARG, "argument 3 (gate_chain_stride) = %lld must be >= 0",
                (long long)gate_chain_stride);
  if (parity != 0 && parity != 1)
    return fail(TEBD_ERR_ARG, "argument 4 (parity) = %d must be 0 or 1", parity);
  if (!disc_weight) return fail(TEBD_ERR_ARG, "argument 6 (disc_weight) is NULL");
  if (!dev_status) return fail(TEBD_ERR_ARG, "argument 7 (dev_status) is NULL");
  return enqueue_sweep(mps, gates, gate_chain_stride, parity, -1, -1, prm, disc_weight,
                       dev_status, workspace, ws_bytes, stream);
}

tebd_status tebd_adjoint_workspace_size(const tebd_mps* mps, const tebd_params* prm,
                                        size_t* bytes) {
  if (!bytes) return fail(TEBD_ERR_ARG, "argument 3 (bytes) is NULL");
  tebd_status st = check_params(prm);
  if (st != TEBD_OK) return st;
  st = check_mps(mps, prm);
  if (st != TEBD_OK) return st;
  *bytes = plan_sweep(*mps, *prm).adj_total;
  return ok();
}

tebd_status tebd_tape_size(const tebd_mps* mps, const tebd_params* prm, size_t* bytes) {
  if (!bytes) return fail(TEBD_ERR_ARG, "argument 3 (bytes) is NULL");
  tebd_status st = check_params(prm);
  if (st != TEBD_OK) return st;
  st = check_mps(mps, prm);
  if (st != TEBD_OK) return st;
  const SweepPlan pl = plan_sweep(*mps, *prm);
  *bytes = size_t(pl.pmax) * pl.tape_slot;
  return ok();
}

tebd_status tebd_sweep_record(const tebd_mps* mps, const tebd_z* gates, int64_t gate_chain_stride,
                              int32_t parity, const tebd_params* prm, double* disc_weight,
                              int32_t* dev_status, void* tape, size_t tape_bytes,
                              void* workspace, size_t ws_bytes, void* stream) {
  tebd_status st = check_params(prm);
  if (st != TEBD_OK) return st;
  st = check_mps(mps, prm);
  if (st != TEBD_OK) return st;
  if (!gates) return fail(TEBD_ERR_ARG, "argument 2 (gates) is NULL");
  if (gate_chain_stride < 0)
    return fail(TEBD_ERR_ARG, "argument 3 (gate_chain_stride) = %lld must be >= 0",
                (long long)gate_chain_stride);
  if (parity != 0 && parity != 1)
    return fail(TEBD_ERR_ARG, "argument 4 (parity) = %d must be 0 or 1", parity);
  if (!disc_weight) return fail(TEBD_ERR_ARG, "argument 6 (disc_weight) is NULL");
  if (!dev_status) return fail(TEBD_ERR_ARG, "argument 7 (dev_status) is NULL");
  if (!tape) return fail(TEBD_ERR_ARG, "argument 8 (tape) is NULL");
  if (reinterpret_cast<uintptr_t>(tape) % 256 != 0)
    return fail(TEBD_ERR_WORKSPACE, "argument 8 (tape) must be 256-byte aligned");
  const SweepPlan pl = plan_sweep(*mps, *prm);
  if (tape_bytes < size_t(pl.pmax) * pl.tape_slot)
    return fail(TEBD_ERR_WORKSPACE, "argument 9 (tape_bytes) = %zu < %zu needed", tape_bytes,
                size_t(pl.pmax) * pl.tape_slot);
  return enqueue_sweep(mps, gates, gate_chain_stride, parity, -1, -1, prm, disc_weight,
                       dev_status, workspace, ws_bytes, stream, tape);
}

tebd_status tebd_sweep_adjoint(const tebd_mps* mps_in, const tebd_z* gates,
                               int64_t gate_chain_stride, int32_t parity, const tebd_params* prm,
                               const void* tape, size_t tape_bytes, tebd_z* gamma_bar,
                               double* lambda_bar, tebd_z* gate_bar, int32_t* dev_status,
                               void* workspace, size_t ws_bytes, void* stream) {
  tebd_status st = check_params(prm);
  if (st != TEBD_OK) return st;
  st = check_mps(mps_in, prm);
  if (st != TEBD_OK) return st;
  if (!gates) return fail(TEBD_ERR_ARG, "argument 2 (gates) is NULL");
  if (gate_chain_stride < 0)
    return fail(TEBD_ERR_ARG, "argument 3 (gate_chain_stride) = %lld must be >= 0",
                (long long)gate_chain_stride);
  if (parity != 0 && parity != 1)
    return fail(TEBD_ERR_ARG, "argument 4 (parity) = %d must be 0 or 1", parity);
  if (!tape) return fail(TEBD_ERR_ARG, "argument 6 (tape) is NULL");
  if (!gamma_bar) return fail(TEBD_ERR_ARG, "argument 8 (gamma_bar) is NULL");
  if (!lambda_bar) return fail(TEBD_ERR_ARG, "argument 9 (lambda_bar) is NULL");
  if (!gate_bar) return fail(TEBD_ERR_ARG, "argument 10 (gate_bar) is NULL");
  if (!dev_status) return fail(TEBD_ERR_ARG, "argument 11 (dev_status) is NULL");
  const SweepPlan pl = plan_sweep(*mps_in, *prm);
  if (reinterpret_cast<uintptr_t>(tape) % 256 != 0)
    return fail(TEBD_ERR_WORKSPACE, "argument 6 (tape) must be 256-byte aligned");
  if (tape_bytes < size_t(pl.pmax) * pl.tape_slot)
    return fail(TEBD_ERR_WORKSPACE, "argument 7 (tape_bytes) = %zu < %zu needed", tape_bytes,
                size_t(pl.pmax) * pl.tape_slot);
  if (!workspace) return fail(TEBD_ERR_WORKSPACE, "argument 12 (workspace) is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(TEBD_ERR_WORKSPACE, "argument 12 (workspace) must be 256-byte aligned");
  if (ws_bytes < pl.adj_total)
    return fail(TEBD_ERR_WORKSPACE, "argument 13 (ws_bytes) = %zu < %zu needed", ws_bytes,
                pl.adj_total);
  AdjCommon c;
  c.n_chains = mps_in->n_chains;
  c.n_sites = mps_in->n_sites;
  c.parity = parity;
  c.nb = (mps_in->n_sites - parity) / 2;
  c.nprob = int32_t(int64_t(c.n_chains) * c.nb);
  c.gate_chain_stride = gate_chain_stride;
  char* base = reinterpret_cast<char*>(workspace);
  c.offs = reinterpret_cast<int32_t*>(base + align256(size_t(pl.pmax) * sizeof(AdjProb)));
  {
    const int64_t t = (pl.mcap + 63) / 64;
    c.grid = persistent_grid(int64_t(c.nprob) * t * t * 2);
  }
  if (c.nprob == 0) return ok();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = timed(PK_ADJOINT, s, [&]() {
    return launch_adjoint(reinterpret_cast<AdjProb*>(base), c, *mps_in,
                          reinterpret_cast<const zt*>(gates), reinterpret_cast<const char*>(tape),
                          pl.tape_slot, pl.mcap, pl.lcap, reinterpret_cast<zt*>(gamma_bar),
                          lambda_bar, reinterpret_cast<zt*>(gate_bar), dev_status,
                          prm->lambda_floor, base + pl.adj_desc_bytes, pl.adj_slab_sz, pl.nchunk,
                          s);
  });
  if (e != hipSuccess) return fail(TEBD_ERR_DEVICE, "HIP error while enqueuing: %s", hipGetErrorString(e));
  return ok();
}

}  // extern "C"
