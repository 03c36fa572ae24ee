// Persistent tile queues over batches of problems whose sizes live on the
// device.
//
// Every contraction kind k has, per batch, an exclusive prefix sum over
// problems of its output-tile counts (offs[k][p], offs[k][nprob] =
// total), built on the device by k_schedule.  A persistent launch then walks
// the global tile index t = vb, vb + G, ... where vb = (i mod 8) * G/8 + i / 8
// for workgroup i of G: consecutive tiles of one problem, which share
// operand rows, are taken by workgroups of the same XCD and hit its L2.
//
// A descriptor type PT plugs in through TileKinds<PT>:
//   static constexpr int count;   number of kinds
//   static __device__ void shape(int kind, const PT&, int flag, int& M, int& N);
// (M x N = 0 x 0 when the problem has no tiles of that kind),
//   static constexpr int tile_m(int kind), tile_n(int kind);   the kind's tile
// (64 x 64 unless a kind's shapes call for another),
//   static constexpr bool col_major(int kind);   tiles of a problem numbered
// down the columns (the row tiles of one column block consecutive) instead
// of along the rows, and, for
// k_schedule<PT, true>, static __device__ bool dims(const PT&, int d[3])
// (false for an inactive problem).
#pragma once

#include "zdev.hpp"

namespace tebd {

template <class PT>
struct TileKinds;

__host__ __device__ __forceinline__ int tiles_of(int M, int N, int tm = 64, int tn = 64) {
  return (M <= 0 || N <= 0) ? 0 : ((M + tm - 1) / tm) * ((N + tn - 1) / tn);
}

template <class PT>
__device__ __forceinline__ int kind_tiles(int kind, const PT& P, int flag) {
  int M, N;
  TileKinds<PT>::shape(kind, P, flag, M, N);
  return tiles_of(M, N, TileKinds<PT>::tile_m(kind), TileKinds<PT>::tile_n(kind));
}

// Exclusive prefix sums of tile counts for every kind (one workgroup of
// kScheduleThreads): thread t reads its contiguous chunk of problems once
// and sums the tiles of every kind; a block-wide scan per kind (DPP scan
// inside each wavefront, then one thread per kind scans the wavefront
// totals) gives every chunk its starts; a second pass writes the chunk's
// offsets (from the counts kept in registers when the chunk is one problem).
// With BOUNDS, the same pass also writes the smallest and largest sizes
// over the active problems, {min, max} of each of TileKinds<PT>::dims
// (three values), to bounds[0..6) (an empty batch gives {1, 1} each), and
// the tile total of every kind to bounds[6..6 + count).
constexpr int kScheduleThreads = 1024;

// The body, for a workgroup of kScheduleThreads threads (also run at the end
// of a kernel that has just written the descriptors, after a barrier).
template <class PT, bool BOUNDS = false>
__device__ __forceinline__ void schedule_body(const PT* probs, int nprob, int flag, int32_t* offs,
                                              int32_t* bounds) {
  constexpr int NK = TileKinds<PT>::count, NT = kScheduleThreads, NW = NT / 64;
  __shared__ int32_t wsum[NK][NW];
  __shared__ int32_t wext[6][NW];  // per-wavefront {min, max} of the three sizes
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int chunk = (nprob + NT - 1) / NT;
  const int p0 = min(nprob, tid * chunk), p1 = min(nprob, p0 + chunk);
  int32_t own[NK], incl[NK];
  int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < NK; ++k) own[k] = 0;
  for (int p = p0; p < p1; ++p) {
    const PT& P = probs[p];
#pragma unroll
    for (int k = 0; k < NK; ++k) own[k] += kind_tiles(k, P, flag);
    if constexpr (BOUNDS) {
      int d[3];
      if (TileKinds<PT>::dims(P, d))
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          lo[i] = min(lo[i], d[i]);
          hi[i] = max(hi[i], d[i]);
        }
    }
  }
  const auto add = [](int32_t a, int32_t b) { return a + b; };
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int32_t v = wave_scan_i32(own[k], 0, add);
    incl[k] = v;
    if (lane == 63) wsum[k][wave] = v;
  }
  if constexpr (BOUNDS) {  // wavefront minima and maxima (empty lanes: INT32_MAX, 0), in lane 63
    const auto mn = [](int32_t a, int32_t b) { return a < b ? a : b; };
    const auto mx = [](int32_t a, int32_t b) { return a > b ? a : b; };
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      lo[i] = wave_scan_i32(lo[i], INT32_MAX, mn);
      hi[i] = wave_scan_i32(hi[i], INT32_MIN, mx);
      if (lane == 63) {
        wext[2 * i][wave] = lo[i];
        wext[2 * i + 1][wave] = hi[i];
      }
    }
  }
  __syncthreads();
  if constexpr (BOUNDS) {
    if (tid >= 64 && tid < 67) {  // one thread per size, beside the scan of wavefront 0
      const int i = tid - 64;
      int32_t mn = INT32_MAX, mx = 0;
      for (int w = 0; w < NW; ++w) {
        mn = min(mn, wext[2 * i][w]);
        mx = max(mx, wext[2 * i + 1][w]);
      }
      bounds[2 * i] = mx > 0 ? mn : 1;
      bounds[2 * i + 1] = mx > 0 ? mx : 1;
    }
  }
  if (tid < NK) {  // exclusive scan of the wavefront totals, one thread per kind
    int32_t acc = 0;
    for (int w = 0; w < NW; ++w) {
      const int32_t ws = wsum[tid][w];
      wsum[tid][w] = acc;
      acc += ws;
    }
    offs[size_t(tid) * (nprob + 1) + nprob] = acc;
    if (BOUNDS) bounds[6 + tid] = acc;
  }
  __syncthreads();
  int32_t run[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) run[k] = wsum[k][wave] + incl[k] - own[k];
  if (chunk == 1) {
    if (p0 < p1)
#pragma unroll
      for (int k = 0; k < NK; ++k) offs[size_t(k) * (nprob + 1) + p0] = run[k];
    return;
  }
  for (int p = p0; p < p1; ++p) {
    const PT& P = probs[p];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      offs[size_t(k) * (nprob + 1) + p] = run[k];
      run[k] += kind_tiles(k, P, flag);
    }
  }
}

template <class PT, bool BOUNDS = false>
__global__ __launch_bounds__(kScheduleThreads) void k_schedule(const PT* probs, int nprob,
                                                               int flag, int32_t* offs,
                                                               int32_t* bounds = nullptr) {
  schedule_body<PT, BOUNDS>(probs, nprob, flag, offs, bounds);
}

// Problem owning global tile t: the largest p with off[p] <= t (off is
// non-decreasing, off[0] = 0).  A 64-way search per wavefront: every lane
// probes one point of the current range and a ballot narrows it, so a
// batch of up to 4096 problems takes two rounds of independent loads
// instead of a dozen dependent ones (each a cache miss on the first tiles of
// a launch, whose XCD has not seen the offsets yet).  Called by whole
// wavefronts with a uniform t.
__device__ __forceinline__ int find_problem(const int32_t* off, int nprob, int t) {
  const int lane = threadIdx.x & 63;
  int lo = 0, n = nprob;  // the answer lies in [lo, lo + n)
  while (n > 1) {
    const int step = (n + 63) >> 6;
    const int q = lo + lane * step;
    const bool ok = q < lo + n && off[q] <= t;  // a prefix of the lanes (off[lo] <= t)
    const int cnt = __popcll(__ballot(ok));
    const int nlo = lo + (cnt - 1) * step;
    const int end = lo + n;
    lo = nlo;
    n = end - nlo < step ? end - nlo : step;
  }
  return lo;
}

__device__ __forceinline__ int virtual_block() {
  const int g = gridDim.x, i = blockIdx.x;
  return (i & 7) * (g >> 3) + (i >> 3);
}

// Run global tile t of one kind: body(P, M, N, m0, n0, tile_index_within_problem).
template <int KIND, class PT, class Body>
__device__ __forceinline__ void run_tile(PT* probs, const int32_t* off, int nprob, int flag, int t,
                                         Body& body) {
  const int p = find_problem(off, nprob, t);
  PT& P = probs[p];
  int M, N;
  TileKinds<PT>::shape(KIND, P, flag, M, N);
  const int local = t - off[p];
  // a size may have shrunk since the queue was built (the range finder
  // lowers l): tiles of the old shape that now lie outside are skipped
  constexpr int TM = TileKinds<PT>::tile_m(KIND), TN = TileKinds<PT>::tile_n(KIND);
  if constexpr (TileKinds<PT>::col_major(KIND)) {
    const int tiles_m = (M + TM - 1) / TM;
    if (tiles_m == 0) return;
    const int tn = local / tiles_m, tm = local - tn * tiles_m;
    if (tn * TN >= N) return;
    body(P, M, N, tm * TM, tn * TN, local);
  } else {
    const int tiles_n = (N + TN - 1) / TN;
    if (tiles_n == 0) return;
    const int tm = local / tiles_n, tn = local - tm * tiles_n;
    if (tm * TM >= M) return;
    body(P, M, N, tm * TM, tn * TN, local);
  }
}

// Iterate over this workgroup's tiles of one kind.
template <int KIND, class PT, class Body>
__device__ __forceinline__ void for_each_tile(PT* probs, const int32_t* offs, int nprob, int flag,
                                              Body body) {
  const int32_t* off = offs + size_t(KIND) * (nprob + 1);
  const int total = off[nprob];
  for (int t = virtual_block(); t < total; t += gridDim.x)
    run_tile<KIND>(probs, off, nprob, flag, t, body);
}

// Two independent kinds as one queue: the tiles of K1, then those of K2.
template <int K1, int K2, class PT, class B1, class B2>
__device__ __forceinline__ void for_each_tile2(PT* probs, const int32_t* offs, int nprob, int flag,
                                               B1 body1, B2 body2) {
  const int32_t* off1 = offs + size_t(K1) * (nprob + 1);
  const int32_t* off2 = offs + size_t(K2) * (nprob + 1);
  const int total1 = off1[nprob], total = total1 + off2[nprob];
  for (int t = virtual_block(); t < total; t += gridDim.x) {
    if (t < total1)
      run_tile<K1>(probs, off1, nprob, flag, t, body1);
    else
      run_tile<K2>(probs, off2, nprob, flag, t - total1, body2);
  }
}

}  // namespace tebd
