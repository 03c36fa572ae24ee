// Output tiles of every contraction kind of the forward pipeline: the
// TileKinds<Prob> trait that the tile queues (tilequeue.hpp) build on, shared
// by the kernels that schedule (k_schedule, the sweep planner) and those
// that walk the queues.
#pragma once

#include "tilequeue.hpp"

namespace tebd {

// Sketch and power-iteration products (m x l, n x l): the sketch width l is
// a few dozen in a TEBD sweep, so 32-wide tiles halve the FP64 matrix-core
// work spent on padding (FP64 MFMA runs at the vector rate on this chip).
// 32 x 32 tiles (one 16 x 16 block per wavefront): the largest problems of a
// batch set the duration of the launch, and their K loop over the full
// contraction depth is the critical path, so smaller tiles spread it over
// more compute units.
constexpr int kSketchTileM = 32, kSketchTileN = 32;
// The split-depth variant: 16 x 16 tiles, each computed by the four
// wavefronts of a workgroup over a quarter of the contraction depth, so
// that a tile's chain of matrix-core steps is four times shorter and the
// largest problems spread over four times as many compute units.
constexpr int kSketchTileS = 16;

// Extent of the updated bond index that a TEBD update writes in Gamma^[k]
// (columns) and Gamma^[k+1] (rows): the new dimension chi' <= min(l, chi_max)
// and, cleared to zero, the old one chi_m; beyond both the arrays are
// already zero, so the padding up to the capacity is not rewritten.
__device__ __forceinline__ int updated_bond_extent(const Prob& P) {
  const int kept = P.l < P.kcap ? P.l : P.kcap;
  const int e = kept > P.chi_m ? kept : P.chi_m;
  return e < P.chi_cap ? e : P.chi_cap;
}

// Output shape of each contraction kind for problem P (0 x 0 when skipped).
template <>
struct TileKinds<Prob> {
  static constexpr int count = TK_COUNT;
  static constexpr bool small_tiles(int kind) {
    return kind == TK_SKM || kind == TK_SKN || kind == TK_FORMU || kind == TK_FORMV ||
           kind == TK_THETA || kind == TK_ACB || kind == TK_GRAM || kind == TK_QAPM ||
           kind == TK_QAPN;
  }
  static constexpr int tile_m(int kind) {
    return kind == TK_GATE                      ? kGateTileM
           : kind == TK_SKM_S || kind == TK_SKN_S ? kSketchTileS
           : small_tiles(kind)                    ? kSketchTileM
                                                  : 64;
  }
  // TK_SKM_W / TK_SKN_W: the same products on 64 x 64 tiles
  static constexpr int tile_n(int kind) {
    return kind == TK_GATE                        ? kGateTileN
           : kind == TK_SKM_S || kind == TK_SKN_S ? kSketchTileS
           : small_tiles(kind)                    ? kSketchTileN
                                                  : 64;
  }
  // The gate product is short and wide (d_l d_r rows): the row tiles of a
  // column block run one after another, on one XCD, and share its Theta
  // columns in that XCD's L2; the whole gate matrix stays there too.
  static constexpr bool col_major(int kind) { return kind == TK_GATE; }
  __device__ static __forceinline__ void shape(int kind, const Prob& P, int tebd, int& M, int& N) {
    M = N = 0;
    if (kind == TK_GATE) {
      // the group's tiles belong to its first member, whatever its own state
      if (tebd && P.gn > 0 && P.gtot > 0) {
        M = P.dl * P.dr;
        N = P.gtot;
      }
      return;
    }
    if (P.l == 0) return;
    switch (kind) {
      case TK_THETA:
        if (tebd) {
          M = P.dl * P.chi_l;
          N = P.dr * P.chi_r;
        }
        break;
      case TK_SKM:
      case TK_SKM_W:
      case TK_SKM_S:
        M = P.m;
        N = P.l;
        break;
      case TK_SKN:
      case TK_SKN_W:
      case TK_SKN_S:
        M = P.n;
        N = P.l;
        break;
      case TK_FORMU:  // TEBD: the new bond's columns, and the old ones beyond it (cleared)
        M = P.m;
        N = tebd ? updated_bond_extent(P) : P.kcap;
        break;
      case TK_FORMV:
        M = tebd ? updated_bond_extent(P) : P.kcap;
        N = P.n;
        break;
      case TK_TAPEU:
        if (P.tape_u) {
          M = P.m;
          N = P.l;
        }
        break;
      case TK_TAPEV:
        if (P.tape_u) {
          M = P.l;
          N = P.n;
        }
        break;
      case TK_ACB:
        if (P.ac_r > 0) {
          M = P.m;
          N = P.ac_r;
        }
        break;
      case TK_GRAM:
        if (P.chol) M = N = P.l;
        break;
      case TK_QAPM:
        if (P.chol & 1) {
          M = P.m;
          N = P.l;
        }
        break;
      case TK_QAPN:
        if (P.chol & 2) {
          M = P.n;
          N = P.l;
        }
        break;
      default:
        break;
    }
  }
  // rows of the two sketches and the width of the pass (the QR size classes)
  __device__ static __forceinline__ bool dims(const Prob& P, int d[3]) {
    d[0] = P.m;
    d[1] = P.n;
    d[2] = P.l1;
    return P.l > 0;
  }
};

}  // namespace tebd
