// Tile shapes and block edges shared by the host planner and the kernels.
#pragma once

#include "device_common.hpp"

namespace sie {

constexpr int kOrb = 8;       // virtual block edge of the epilogue orbits
constexpr int kWWaves = 4;               // waves per work-group

// Tile shapes of the float64 build: BLK blocks per wave, TR x TC 16-wide
// MFMA tiles per wave along rows x cols, the occupancy target BPC
// (work-groups per CU), and how the 4 waves of a work-group tile it: WR x WC
// waves along rows x cols (then all waves share the BLK blocks), or, with
// WR = WC = 1, 4 waves along the blocks (4 BLK blocks per work-group).  Waves
// that share blocks share the per-block operand rows, which the work-group
// then reads from L2 once for more output columns (or rows).  Shapes with
// lay = 3 use the three-layout build (k_build_w3_f64), TR and TC then
// counting tiles of the per-block and of the shared side.  Variant 0 is the
// default; a tile table (sie_set_tile_table) picks one per fragment by n_v.
struct WShape {
  int blk, tr, tc, bpc, wr, wc;
  int lay;     // 2: two-layout build (k_build_w_f64); 3: k_build_w3_f64 with tr = P
               // (per-block side tiles) and tc = S (shared side tiles)
  int ks;      // k-steps per K-chunk: 2 (chunks of 8) or 4 (16: a 128-byte line per row)
};
constexpr int kWVariants = 15;
__host__ __device__ inline WShape wshape(int v) {
  switch (v) {
    case 1: return WShape{4, 2, 2, 1, 1, 1, 2, 2};
    case 2: return WShape{2, 2, 2, 2, 1, 1, 2, 2};
    case 3: return WShape{8, 1, 1, 2, 1, 1, 2, 2};
    case 4: return WShape{4, 4, 2, 1, 1, 1, 2, 2};
    case 5: return WShape{4, 2, 4, 1, 1, 1, 2, 2};
    case 6: return WShape{4, 2, 2, 2, 2, 2, 2, 2};
    case 7: return WShape{4, 2, 2, 2, 1, 4, 2, 2};
    case 8: return WShape{4, 2, 2, 2, 4, 1, 2, 2};
    case 9: return WShape{1, 1, 13, 2, 1, 1, 3, 2};
    case 10: return WShape{1, 2, 7, 2, 1, 1, 3, 2};
    case 11: return WShape{2, 1, 7, 2, 1, 1, 3, 2};
    case 12: return WShape{1, 1, 10, 2, 1, 1, 3, 2};
    case 13: return WShape{1, 2, 10, 1, 1, 1, 3, 2};
    case 14: return WShape{1, 2, 4, 2, 1, 1, 3, 2};
    default: return WShape{4, 2, 2, 2, 1, 1, 2, 2};
  }
}

// Work-group tile (blocks, rows, cols) of a shape.
__host__ __device__ inline void wtile(const WShape& w, int& bb, int& er, int& ec) {
  const bool grid = w.wr * w.wc > 1;
  bb = grid ? w.blk : kWWaves * w.blk;
  er = 16 * w.tr * (grid ? w.wr : 1);
  ec = 16 * w.tc * (grid ? w.wc : 1);
}

// Build work-groups of one layout of one unit for a fragment of n_v
// virtuals: the work-group tiles of the variant's shape over the cube.
__host__ __device__ inline int64_t wbuild_tiles(int nv, int variant) {
  int bb, er, ec;
  wtile(wshape(variant), bb, er, ec);
  return int64_t((nv + bb - 1) / bb) * ((nv + er - 1) / er) * ((nv + ec - 1) / ec);
}

constexpr int kKs = 32;       // K per bf16 MFMA step (and per LDS chunk)

// Tile shapes (TRW x TCW MFMA tiles per wave).
// wr x wc waves along rows x cols; wr = 2: the B cols go through LDS too
// (k_build_w_bf16x3_l).
struct SShape {
  int trw, tcw, wr, wc;
};
constexpr int kSShapes = 6;
__host__ __device__ constexpr SShape sshape(int s) {
  return s == 1 ? SShape{5, 5, 1, 4} : s == 2 ? SShape{7, 4, 1, 4} : s == 3 ? SShape{4, 4, 1, 4}
       : s == 4 ? SShape{5, 5, 2, 4} : s == 5 ? SShape{5, 5, 2, 2} : SShape{4, 2, 1, 4};
}
__host__ __device__ constexpr int split_rows(int s) { return 16 * sshape(s).trw * sshape(s).wr; }
__host__ __device__ constexpr int split_cols(int s) { return 16 * sshape(s).tcw * sshape(s).wc; }
__host__ __device__ inline int64_t split_tiles(int nv, int s) {
  const int R = split_rows(s), C = split_cols(s);
  return int64_t(nv) * ((nv + R - 1) / R) * ((nv + C - 1) / C);
}
// Shape of a fragment with n_v virtuals: among the shapes whose padded tile
// area is within 10% of the least, the first in the order of their measured
// speed at 32/320 (5, 4, 1, 2, 3, 0).
inline int split_shape_of(int nv) {
  int64_t best = -1;
  for (int s = 0; s < kSShapes; ++s) {
    const int64_t a = split_tiles(nv, s) / nv * split_rows(s) * split_cols(s);
    best = (best < 0 || a < best) ? a : best;
  }
  constexpr int kOrder[kSShapes] = {5, 4, 1, 2, 3, 0};
  for (int s : kOrder) {
    const int64_t a = split_tiles(nv, s) / nv * split_rows(s) * split_cols(s);
    if (10 * a <= 11 * best) return s;
  }
  return 0;
}

}  // namespace sie
