// Work description shared by the host runtime and the kernels.
//
// An evaluation covers one or more fragments.  Their occupied triples
// ("units", i >= j >= k, not all equal) are ordered longest-first by cost per
// unit and cut into rounds whose W-tilde cubes fit in the workspace arena.
// Each round is one build launch and one epilogue launch whose blocks are the
// concatenation of every item's blocks (item = one unit of one fragment):
// the hardware dispatcher hands blocks out in index order, so the round is a
// longest-job-first work queue over all fragments.
#pragma once

#include "device_common.hpp"
#include "shapes.hpp"

namespace sie {

struct FragDesc {
  // caller inputs: float64 (SIE_FP64) or float32 (SIE_SPLIT_BF16)
  const void* t1;
  const void* t2;
  const void* ovvv;
  const void* ooov;
  const void* ovov;
  // split copies in the workspace (SIE_SPLIT_BF16 only), see k_bf16.hpp
  const u4v* vS;
  const u4v* tS;
  const u4v* tT;
  const u4v* oT;
  const double* eps;      // [no + nv] workspace copy: eps_occ then eps_vir
  int no, nv;
  int Kv, Ko;             // padded contraction lengths of the split copies
  int vec;                // float64: rows may be read 16 bytes at a time
  int epv;                // epilogue: n_v even and ovov aligned to two elements, so
                          // pairs of adjacent c are read with one load
  int variant;            // float64: tile shape of the W-tilde build (see wshape)
  int pair;               // 1: pair units (two equal occupied indices) build only the
                          // first layout's cube (unit_triple); 0: both, as the adjoint needs
  int lay3;               // float64 energy: three-layout build (k_build_w3_f64), three
                          // partial cubes per unit (two for a pair unit)
  int blocked;            // partial cubes in 8^3-blocked order (energy), else row-major
                          // (the adjoint's cubes); see cube_at
  int n_part;             // epilogue partial slots per unit
  int64_t unit_base;      // first entry of this fragment in the per-unit arrays
  int64_t half;           // elements per partial cube (aligned)
  int64_t tiles;          // build work-groups of one layout of one unit
  // gradient outputs (float64, input shapes; backward only)
  double* g_t1;
  double* g_t2;
  double* g_ovvv;
  double* g_ooov;
  double* g_ovov;
  double* g_eo;           // [no]  orbital-energy gradients (backward only)
  double* g_ev;           // [nv]
};

// Element offset of (x, y, z) in a partial cube of edge n_v.  Energy
// evaluations store their cubes 8^3-blocked: the cube is cut into blocks of
// kOrb^3 elements (nb = ceil(n_v / kOrb) a side, the last ones padded), each
// block one contiguous run of 512 elements in (x, y, z) order, the blocks in
// (x, y, z) order too.  An orbit block of the epilogue is then whole 128-byte
// lines: with row-major cubes each of its 8-element rows pulled a full line
// from HBM of which it used a quarter (float32) or a half (float64).  The
// adjoint keeps row-major cubes ([x][y][z], n_v a side), which its
// contractions read with unit stride along rows.
__host__ __device__ __forceinline__ int64_t cube_at(bool blocked, int nv, int x, int y, int z) {
  if (!blocked) return ((int64_t)x * nv + y) * nv + z;
  const int nb = (nv + kOrb - 1) / kOrb;
  const int64_t blk = ((int64_t)(x >> 3) * nb + (y >> 3)) * nb + (z >> 3);
  return blk * (kOrb * kOrb * kOrb) + ((x & 7) << 6) + ((y & 7) << 3) + (z & 7);
}

// Elements of one blocked cube (nb^3 blocks of 512).
__host__ __device__ __forceinline__ int64_t cube_blocked_elems(int nv) {
  const int64_t nb = (nv + kOrb - 1) / kOrb;
  return nb * nb * nb * (kOrb * kOrb * kOrb);
}

struct Item {
  int frag;               // fragment index
  int unit;               // unit index u >= 0 within the fragment (tetrahedral order), or
                          // an ordered occupied triple (ordered_item, < 0)
  int64_t cube_off;       // element offset of the item's two partial cubes
  int64_t blk_end;        // inclusive end of the item's build blocks (prefix sum over the
                          // item's build segment: the round's items of one tile variant)
  int64_t part_end;       // inclusive end of the item's epilogue blocks (prefix sum)
};

// First item r with key(r) > x, for prefix-sum keys (blk_end or part_end).
template <bool BUILD>
__device__ __forceinline__ int find_item(const Item* __restrict__ items, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int64_t key = BUILD ? items[mid].blk_end : items[mid].part_end;
    if (key > x) hi = mid; else lo = mid + 1;
  }
  return lo;
}

}  // namespace sie
