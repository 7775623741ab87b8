// Host-visible description of the adjoint's contraction lists: classes,
// output slices, list records and tile shapes (see k_adjoint.hpp).
#pragma once

#include "device_common.hpp"

namespace sie {

enum AdjClass {
  kAdjOvvv = 0,   // dE/d ovvv[x]       per-block tiles (block, row, col)
  kAdjT2oo = 1,   // dE/d t2[p][*] from the l-sums, per-block tiles
  kAdjT2vv = 2,   // dE/d t2[s1][s2] from the d-sums, summed-block tiles
  kAdjOoov = 3,   // dE/d ooov[m][*][n][*], summed-block tiles
  kAdjOvov = 4,   // dE/d ovov[p][*][q][*] from H
  kAdjT1 = 5,     // dE/d t1[p] from H
  kAdjClasses = 6
};

// Output slice (a0, a1) that term `kind` of class `cls` writes for the unit
// (i, j, k); a1 = 0 for classes with a single slice index.
template <typename T>
__host__ __device__ __forceinline__ T pick6(int q, T v0, T v1, T v2, T v3, T v4, T v5) {
  return q == 0 ? v0 : q == 1 ? v1 : q == 2 ? v2 : q == 3 ? v3 : q == 4 ? v4 : v5;
}

__host__ __device__ inline void adj_slice(int cls, int kind, int i, int j, int k, int& a0,
                                          int& a1) {
  a1 = 0;
  switch (cls) {
    case kAdjOvvv: a0 = pick6(kind, i, i, k, j, k, j); break;
    case kAdjT2oo: a0 = pick6(kind, i, i, k, k, j, j); break;
    case kAdjT2vv:
      a0 = pick6(kind, k, j, j, i, i, k);
      a1 = pick6(kind, j, k, i, k, j, i);
      break;
    case kAdjOoov:
      a0 = pick6(kind, k, j, i, j, k, i);
      a1 = pick6(kind, j, k, j, i, i, k);
      break;
    case kAdjOvov:
      a0 = pick6(kind, i, i, j, 0, 0, 0);
      a1 = pick6(kind, j, k, k, 0, 0, 0);
      break;
    default: a0 = pick6(kind, k, j, i, 0, 0, 0); break;   // kAdjT1
  }
}

__host__ __device__ inline int adj_kinds(int cls) { return cls >= kAdjOvov ? 3 : 6; }
// Summed-block classes split the first summed virtual index into groups of kABB.
__host__ __device__ inline bool adj_reduce(int cls) { return cls == kAdjT2vv || cls == kAdjOoov; }

struct AdjGroup {
  int frag;
  int a0, a1;          // output slice
  int rec_begin, rec_end;
  int pad;
  int64_t wg_end;      // inclusive prefix sum of work-groups over the launch
  int64_t part_off;    // summed-block classes: element offset of the partial slice it writes
};

// Output slice of a summed-block class and its nparts partial slices, at
// element offsets off0 + q * (slice elements), summed in that order into the
// gradient by k_adj_part_sum.
struct AdjSlice {
  int frag;
  int a0, a1;
  int nparts;
  int64_t off0;
};

// Partial slices of the summed-block classes, per fragment and round: at
// most kAdjParts n_o^2 (the workspace holds that many).  A slice's
// contributions are split over groups (work-group sets) of about equal
// length for parallelism, each writing a partial slice, then summed in a
// fixed order.
constexpr int kAdjParts = 4;

struct AdjRec {
  int item;            // index into the round's items
  int kind;            // term of the class
  int g;               // block group (summed-block classes), else 0
  int pad;
};

// Tiles of the G contractions (4 waves per work-group, operands loaded from
// L1/L2 straight into registers, two K-chunks of 8 in flight, the chunks of
// all of a group's records in one continuous stream):
//   per-block classes: wave w owns blocks 4w .. 4w + 3 of the work-group's
//     16 blocks, each TRW x TCW 16-wide MFMA tiles: 32 x 32 for ovvv, 32 x 16
//     for t2 from the l-sums (whose cols are the few occupied);
//   summed-block classes (t2 from the d-sums, ooov): the first summed
//     virtual runs in groups of kARB as the block index of both operands.
//     t2: 2 x 2 waves of 64 x 64, each over the whole stream.  ooov (cols:
//     the few occupied): all four waves compute the same 64 x 16 tile over
//     every fourth chunk of the stream, and their accumulators are added
//     through LDS in a fixed order.
constexpr int kABlk = 4;                 // blocks per wave, per-block classes
constexpr int kARB = 2;                  // summed-block group (blocks per wave) of the others
constexpr int kAT = 2;                   // 16-wide MFMA tiles per wave along rows and cols (ovvv)
constexpr int kAKc = 8;                  // K chunk
constexpr int kAThreads = 256;

// 16-wide MFMA tiles per wave along rows (trw) and cols (tcw) of a class,
// and the waves of a work-group along rows (wr) and cols (wc) of the output
// (per-block classes: 1 x 1, the waves take different blocks; ooov: 1 x 1,
// the waves take different chunks).
__host__ __device__ constexpr int adj_trw(int cls) { return cls == kAdjT2vv || cls == kAdjOoov ? 4 : kAT; }
__host__ __device__ constexpr int adj_tcw(int cls) {
  return cls == kAdjOvvv ? kAT : cls == kAdjT2vv ? 4 : 1;
}
__host__ __device__ constexpr int adj_wr(int cls) { return cls == kAdjT2vv ? 2 : 1; }
__host__ __device__ constexpr int adj_wc(int cls) { return cls == kAdjT2vv ? 2 : 1; }

// Work-group tile of a class: (blocks, rows, cols) per work-group.
__host__ __device__ inline void adj_tile_shape(int cls, int& tb, int& tr, int& tc) {
  const bool red = cls == kAdjT2vv || cls == kAdjOoov;
  tb = red ? 1 : 4 * kABlk;
  tr = 16 * adj_trw(cls) * adj_wr(cls);
  tc = 16 * adj_tcw(cls) * adj_wc(cls);
}

// Work-groups per output slice of a class for a fragment.
__host__ __device__ inline int64_t adj_tiles(int cls, int no, int nv) {
  if (cls == kAdjOvov) return (int64_t(nv) * nv + 255) / 256;
  if (cls == kAdjT1) return (nv + 63) / 64;
  int tb, tr, tc;
  adj_tile_shape(cls, tb, tr, tc);
  const int nb = (cls == kAdjT2vv || cls == kAdjOoov) ? 1 : nv;
  const int nc = (cls == kAdjT2oo || cls == kAdjOoov) ? no : nv;
  return int64_t((nb + tb - 1) / tb) * ((nv + tr - 1) / tr) * ((nc + tc - 1) / tc);
}

enum SymKind { kSymT2 = 0, kSymOvvv = 1, kSymOoov = 2, kSymOvov = 3 };

// Index of the twin of flat element e (same value for symmetric inputs):
//   t2[i][j][a][b] ~ t2[j][i][b][a], ovvv[i][a][b][d] ~ ovvv[i][a][d][b],
//   ooov[j][l][i][a] ~ ooov[l][j][i][a], ovov[i][a][j][b] ~ ovov[j][b][i][a].
__host__ __device__ inline int64_t twin_index(int kind, int64_t e, int64_t no, int64_t nv) {
  switch (kind) {
    case kSymT2: {
      const int64_t b = e % nv, a = (e / nv) % nv, j = (e / (nv * nv)) % no, i = e / (nv * nv * no);
      return ((j * no + i) * nv + b) * nv + a;
    }
    case kSymOvvv: {
      const int64_t d = e % nv, b = (e / nv) % nv, rest = e / (nv * nv);
      return (rest * nv + d) * nv + b;
    }
    case kSymOoov: {
      const int64_t a = e % nv, i = (e / nv) % no, l = (e / (nv * no)) % no, j = e / (nv * no * no);
      return ((l * no + j) * no + i) * nv + a;
    }
    default: {
      const int64_t b = e % nv, j = (e / nv) % no, a = (e / (nv * no)) % nv, i = e / (nv * no * nv);
      return ((j * nv + b) * no + i) * nv + a;
    }
  }
}

}  // namespace sie
