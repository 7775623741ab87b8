// float64 (T) kernels for gfx950: the W-tilde build on the FP64 matrix cores
// and the R/D epilogue with the per-triple energy reduction.
//
// Work decomposition: the energy of the paper's in-situ (T) equation is a sum
// over unordered occupied triples i >= j >= k ("units"), each contributing
// 2 A_ijk sum_abc Wt^{abc}_{ijk} R'[Wt + Vt]^{abc}_{ijk} / D^{abc}_{ijk}, where
// A_ijk is the equal-index weight (1, 1/2, 1/6) and R' is the R operator of
// the paper moved from occupied to virtual indices using the simultaneous
// (occupied, virtual) pair symmetry of Wt and Vt:
//   R'[Y]^{abc} = 4 Y^{abc} + Y^{cab} + Y^{bca} - 2 Y^{cba} - 2 Y^{acb} - 2 Y^{bac}.
// Units with i = j = k contribute exactly zero (R' annihilates a function
// symmetric in abc) and are skipped.
//
// Per unit, Wt over the n_v^3 virtual cube is the sum of six permuted copies
// (the P operator) of
//   X^{abc}_{ijk} = sum_d (ia|bd) t_kj^cd - sum_l (ia|jl) t_lk^bc,
// i.e. 6 contractions over d (K = n_v) and 6 over l (K = n_occ).  A
// contraction maps onto 16x16xK matrix products only in a register layout
// whose block index is one of the indices its (ov|vv)-side operand carries;
// two layouts cover all twelve:
//   L1: block index a, MFMA rows b, MFMA cols c
//   L2: block index b, MFMA rows a, MFMA cols c
// The float64 build evaluates both layouts of a 16^3 tile in one work-group
// (the L2 half is added through LDS) and writes Wt[a][b][c] to the unit's
// cube.  The split build (k_bf16.hpp) evaluates each layout in its own
// work-groups over larger tiles and writes two partial cubes,
// Wt[a][b][c] = P1[a][b][c] + P2[b][a][c].  The epilogue kernel reads the
// cube(s) by symmetric orbits of 8 x 8 x 8 virtual blocks, so that every
// permuted element R' needs is in LDS, forms Vt and D on the fly and reduces
// in a fixed order.
#pragma once

#include "device_common.hpp"
#include "shapes.hpp"
#include "work.hpp"

namespace sie {


// ---------------------------------------------------------------------------
// float64 W-tilde build.  A work-group of 4 waves computes, for one unit and
// one register layout, the layout's six terms over 16 blocks x 32 rows x 32
// cols; wave w owns blocks 4w .. 4w + 3 and all 32 x 32 rows x cols, i.e. 16
// MFMA accumulators (4 blocks x 2 row tiles x 2 col tiles).  Each k-pair a
// lane loads feeds 8 MFMAs (per-block operand: 2 tiles of its side; shared
// operand: 4 blocks x 2 tiles), so a wave reads 160 bytes per lane per 32
// MFMAs.  Operands go straight from global memory (L1/L2) into registers in
// K-chunks of 8, two chunks in flight.  Each layout writes its own partial
// cube, Wt[a][b][c] = P1[a][b][c] + P2[b][a][c].
//   L1 (block a, rows b, cols c): d-sums of X^{abc}_{ijk}, X^{acb}_{ikj},
//       X^{cab}_{kij} and l-sums of X^{bca}_{jki}, X^{cba}_{kji}, X^{bac}_{jik}
//   L2 (block b, rows a, cols c): d-sums of X^{bca}_{jki}, X^{cba}_{kji},
//       X^{bac}_{jik} and l-sums of X^{abc}_{ijk}, X^{acb}_{ikj}, X^{cab}_{kij}
// with X^{abc}_{ijk} = sum_d (ia|bd) t_kj^cd - sum_l (ia|jl) t_lk^bc, (ia|jl)
// read as ooov[j][l][i][a] and t_ij^ab as t2[i][j][a][b] or its twin.
// ---------------------------------------------------------------------------

// Element (beta, x, k) of the per-block operand is bl[beta*bl_b + x*bl_x + k*bl_k];
// element (x, k) of the shared operand is scale * sh[x*sh_x + k*sh_k]; x is
// relative to the tile origin of the operand's MFMA side.
struct WTerm {
  const double* bl;
  int64_t bl_b, bl_x, bl_k;
  const double* sh;
  int64_t sh_x, sh_k;
  int nK;
  double scale;
};

// Term q (0..5) of layout L2 (or L1) for unit (i, j, k) and tile origin
// (blk0, row0, col0) in that layout's (block, row, col) naming; A_IS_BL
// tells which MFMA side the per-block operand is on (see wterm_a_is_bl).
template <bool L2, int Q>
__device__ __forceinline__ WTerm make_wterm(const double* __restrict__ t2,
                                            const double* __restrict__ ovvv,
                                            const double* __restrict__ ooov, int i, int j, int k,
                                            int no_, int nv_, int blk0, int row0, int col0) {
  const int64_t nv = nv_, no = no_, nv2 = nv * nv, nonv = no * nv;
  WTerm t;
  t.nK = nv_;
  t.scale = 1.0;
  if (!L2) {  // block a = blk0 + beta, row b = row0 + x, col c = col0 + x
    if (Q == 0) {         // X^{abc}_{ijk} d-sum: ovvv[i][a][b][d] * t2[k][j][c][d]
      t.bl = ovvv + ((i * nv + blk0) * nv + row0) * nv; t.bl_b = nv2; t.bl_x = nv; t.bl_k = 1;
      t.sh = t2 + ((k * no + j) * nv + col0) * nv; t.sh_x = nv; t.sh_k = 1;
    } else if (Q == 1) {  // X^{acb}_{ikj} d-sum: t2[j][k][b][d] * ovvv[i][a][c][d]
      t.sh = t2 + ((j * no + k) * nv + row0) * nv; t.sh_x = nv; t.sh_k = 1;
      t.bl = ovvv + ((i * nv + blk0) * nv + col0) * nv; t.bl_b = nv2; t.bl_x = nv; t.bl_k = 1;
    } else if (Q == 2) {  // X^{cab}_{kij} d-sum: t2[j][i][b][d] * ovvv[k][c][a][d]
      t.sh = t2 + ((j * no + i) * nv + row0) * nv; t.sh_x = nv; t.sh_k = 1;
      t.bl = ovvv + ((k * nv + col0) * nv + blk0) * nv; t.bl_b = nv; t.bl_x = nv2; t.bl_k = 1;
    } else if (Q == 3) {  // X^{bca}_{jki} l-sum: -ooov[k][l][j][b] * t2[i][l][a][c]
      t.sh = ooov + (k * no * no + j) * nv + row0; t.sh_x = 1; t.sh_k = nonv; t.scale = -1.0;
      t.bl = t2 + (i * no * nv + blk0) * nv + col0; t.bl_b = nv; t.bl_x = 1; t.bl_k = nv2;
      t.nK = no_;
    } else if (Q == 4) {  // X^{cba}_{kji} l-sum: t2[i][l][a][b] * -ooov[j][l][k][c]
      t.bl = t2 + (i * no * nv + blk0) * nv + row0; t.bl_b = nv; t.bl_x = 1; t.bl_k = nv2;
      t.sh = ooov + (j * no * no + k) * nv + col0; t.sh_x = 1; t.sh_k = nonv; t.scale = -1.0;
      t.nK = no_;
    } else {              // X^{bac}_{jik} l-sum: -ooov[i][l][j][b] * t2[l][k][a][c]
      t.sh = ooov + (i * no * no + j) * nv + row0; t.sh_x = 1; t.sh_k = nonv; t.scale = -1.0;
      t.bl = t2 + (k * nv + blk0) * nv + col0; t.bl_b = nv; t.bl_x = 1; t.bl_k = nonv * nv;
      t.nK = no_;
    }
  } else {    // block b = blk0 + beta, row a = row0 + x, col c = col0 + x
    if (Q == 0) {         // X^{bca}_{jki} d-sum: t2[i][k][a][d] * ovvv[j][b][c][d]
      t.sh = t2 + ((i * no + k) * nv + row0) * nv; t.sh_x = nv; t.sh_k = 1;
      t.bl = ovvv + ((j * nv + blk0) * nv + col0) * nv; t.bl_b = nv2; t.bl_x = nv; t.bl_k = 1;
    } else if (Q == 1) {  // X^{cba}_{kji} d-sum: t2[i][j][a][d] * ovvv[k][c][b][d]
      t.sh = t2 + ((i * no + j) * nv + row0) * nv; t.sh_x = nv; t.sh_k = 1;
      t.bl = ovvv + ((k * nv + col0) * nv + blk0) * nv; t.bl_b = nv; t.bl_x = nv2; t.bl_k = 1;
    } else if (Q == 2) {  // X^{bac}_{jik} d-sum: ovvv[j][b][a][d] * t2[k][i][c][d]
      t.bl = ovvv + ((j * nv + blk0) * nv + row0) * nv; t.bl_b = nv2; t.bl_x = nv; t.bl_k = 1;
      t.sh = t2 + ((k * no + i) * nv + col0) * nv; t.sh_x = nv; t.sh_k = 1;
    } else if (Q == 3) {  // X^{abc}_{ijk} l-sum: -ooov[j][l][i][a] * t2[l][k][b][c]
      t.sh = ooov + (j * no * no + i) * nv + row0; t.sh_x = 1; t.sh_k = nonv; t.scale = -1.0;
      t.bl = t2 + (k * nv + blk0) * nv + col0; t.bl_b = nv; t.bl_x = 1; t.bl_k = nonv * nv;
      t.nK = no_;
    } else if (Q == 4) {  // X^{acb}_{ikj} l-sum: -ooov[k][l][i][a] * t2[j][l][b][c]
      t.sh = ooov + (k * no * no + i) * nv + row0; t.sh_x = 1; t.sh_k = nonv; t.scale = -1.0;
      t.bl = t2 + (j * no * nv + blk0) * nv + col0; t.bl_b = nv; t.bl_x = 1; t.bl_k = nv2;
      t.nK = no_;
    } else {              // X^{cab}_{kij} l-sum: t2[l][j][a][b] * -ooov[i][l][k][c]
      t.bl = t2 + (j * nv + row0) * nv + blk0; t.bl_b = 1; t.bl_x = nv; t.bl_k = nonv * nv;
      t.sh = ooov + (i * no * no + k) * nv + col0; t.sh_x = 1; t.sh_k = nonv; t.scale = -1.0;
      t.nK = no_;
    }
  }
  return t;
}

// Per-block operand on the MFMA A side (rows)?  The d-sums read K contiguous
// (Q < 3); the l-sums read K with a stride.
template <bool L2, int Q>
__device__ __forceinline__ constexpr bool wterm_a_is_bl() {
  return L2 ? (Q == 2 || Q == 5) : (Q == 0 || Q == 4);
}

// Registers of one K-chunk: the per-block operand for BLK blocks x NB tiles
// of its MFMA side, the shared operand for NS tiles of the other side.  A
// chunk is 4 KS values of K; lane group g holds k = 4 KS c + KS g + s for
// s < KS (any bijection between lanes and k serves, as long as both operands
// use the same one).
template <int BLK, int NB, int NS, int KS>
struct WChunk {
  double bl[BLK][NB][KS];     // [block][tile][s]
  double sh[NS][KS];          // [tile][s], as loaded
  double m[KS];               // shared-operand factor per s: the term's scale, 0 past K
};

// Lane offsets of one term, in bytes from the term's (wave-uniform) operand
// bases: per-block rows (block 0) and shared rows of the lane's tiles,
// clamped into the valid range.  Uniform 64-bit bases plus 32-bit lane
// offsets keep the address registers of a chunk to one per row set (the
// host limits operand extents to 4 GiB, see check_fragment).
template <int NB, int NS>
struct WLane {
  uint32_t bl[NB];
  uint32_t sh[NS];
};

template <bool A_IS_BL, int NB, int NS>
__device__ __forceinline__ WLane<NB, NS> wlane(const WTerm& t, int r, int nrow, int ncol) {
  WLane<NB, NS> p;
  const int nb = A_IS_BL ? nrow : ncol;   // valid extent of the per-block side
  const int ns = A_IS_BL ? ncol : nrow;
#pragma unroll
  for (int q = 0; q < NB; ++q) p.bl[q] = uint32_t(min(16 * q + r, nb - 1) * t.bl_x * 8);
#pragma unroll
  for (int q = 0; q < NS; ++q) p.sh[q] = uint32_t(min(16 * q + r, ns - 1) * t.sh_x * 8);
  return p;
}

template <typename T>
__device__ __forceinline__ T ld_off(const double* base, uint32_t off) {
  return *(const SIE_GLOBAL T*)(gptr(reinterpret_cast<const char*>(base)) + off);
}

// Full chunk c of a term with K contiguous (16-byte aligned rows of even
// length), KS / 2 16-byte loads per row; blocks past `last` read block `last`.
template <int BLK, int NB, int NS, int KS>
__device__ __forceinline__ void load_wchunk_vec(const WTerm& t, const WLane<NB, NS>& p, int c,
                                                int last, int g,
                                                WChunk<BLK, NB, NS, KS>& x) {
  const uint32_t kb = uint32_t(4 * KS * c + KS * g) * 8u;
#pragma unroll
  for (int s = 0; s < KS; ++s) x.m[s] = t.scale;
#pragma unroll
  for (int q = 0; q < NS; ++q)
#pragma unroll
    for (int h = 0; h < KS / 2; ++h) {
      const d2v s0 = ld_off<d2v>(t.sh, p.sh[q] + kb + 16u * h);
      x.sh[q][2 * h] = s0.x;
      x.sh[q][2 * h + 1] = s0.y;
    }
#pragma unroll
  for (int beta = 0; beta < BLK; ++beta) {
    const double* b = t.bl + (int64_t)(beta < last ? beta : last) * t.bl_b;
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int h = 0; h < KS / 2; ++h) {
        const d2v u = ld_off<d2v>(b, p.bl[q] + kb + 16u * h);
        x.bl[beta][q][2 * h] = u.x;
        x.bl[beta][q][2 * h + 1] = u.y;
      }
  }
}

// Chunk c of a term, any K stride; k past K reads k = K - 1 (in bounds) and
// gets factor 0.  The loaded values are used as they arrive: the scale and
// the zeros are applied when the chunk is consumed (mma_wchunk), so issuing
// the next chunk's loads never waits for them.
template <int BLK, int NB, int NS, int KS>
__device__ __forceinline__ void load_wchunk_gen(const WTerm& t, const WLane<NB, NS>& p, int c,
                                                int last, int g,
                                                WChunk<BLK, NB, NS, KS>& x) {
  const int k0 = 4 * KS * c + KS * g;
  uint32_t ks[KS], kbl[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = k0 + s;
    const uint32_t kc = uint32_t(k < t.nK ? k : t.nK - 1);
    ks[s] = kc * uint32_t(t.sh_k * 8);
    kbl[s] = kc * uint32_t(t.bl_k * 8);
    x.m[s] = k < t.nK ? t.scale : 0.0;
  }
#pragma unroll
  for (int q = 0; q < NS; ++q)
#pragma unroll
    for (int s = 0; s < KS; ++s) x.sh[q][s] = ld_off<double>(t.sh, p.sh[q] + ks[s]);
#pragma unroll
  for (int beta = 0; beta < BLK; ++beta) {
    const double* b = t.bl + (int64_t)(beta < last ? beta : last) * t.bl_b;
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int s = 0; s < KS; ++s) x.bl[beta][q][s] = ld_off<double>(b, p.bl[q] + kbl[s]);
  }
}

// acc[beta][rt][ct]: rows 16 rt .., cols 16 ct .. of block beta.  Row / col
// tiles wholly outside the virtual range (uniform) are skipped.  SCALED: apply
// the chunk's per-k factors (general chunks; full 16-byte chunks are d-sums,
// whose factor is 1).
template <bool A_IS_BL, int BLK, int TR, int TC, int KS, bool SCALED>
__device__ __forceinline__ void mma_wchunk(
    const WChunk<BLK, (A_IS_BL ? TR : TC), (A_IS_BL ? TC : TR), KS>& x, int nrow, int ncol,
    d4 (&acc)[BLK][TR][TC]) {
  constexpr int NS = A_IS_BL ? TC : TR;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    double sh[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) sh[q] = SCALED ? x.sh[q][s] * x.m[s] : x.sh[q][s];
#pragma unroll
    for (int rt = 0; rt < TR; ++rt)
#pragma unroll
      for (int ct = 0; ct < TC; ++ct) {
        if ((rt > 0 && 16 * rt >= nrow) || (ct > 0 && 16 * ct >= ncol)) continue;
#pragma unroll
        for (int beta = 0; beta < BLK; ++beta)
          acc[beta][rt][ct] = A_IS_BL
              ? mfma16x16x4(x.bl[beta][rt][s], sh[ct], acc[beta][rt][ct])
              : mfma16x16x4(sh[rt], x.bl[beta][ct][s], acc[beta][rt][ct]);
      }
  }
}

// One term: two chunks in flight (loads of chunk c + 1 issued before the
// MFMAs of chunk c).  Chunks [0, nvec) use 16-byte loads, the rest (a ragged
// tail, or every chunk of a strided-K term) general loads; each loop body
// issues a fixed set of loads (the prefetch index is clamped, never
// skipped), so the wait before a chunk's MFMAs covers exactly that chunk.
// A: the per-block operand is on the MFMA A side (rows); V: 16-byte loads;
// KS: k-steps per chunk (chunks of 4 KS).
template <bool A, bool V, int BLK, int TR, int TC, int KS>
__device__ __forceinline__ void run_term(const WTerm& t, int nrow, int ncol, int last, int r,
                                         int g, d4 (&acc)[BLK][TR][TC]) {
  constexpr int NB = A ? TR : TC, NS = A ? TC : TR, KC = 4 * KS;
  const WLane<NB, NS> p = wlane<A, NB, NS>(t, r, nrow, ncol);
  const int nch = (t.nK + KC - 1) / KC;
  const int nvec = V ? t.nK / KC : 0;
  WChunk<BLK, NB, NS, KS> b0, b1;
  if (nvec > 0) {
    load_wchunk_vec(t, p, 0, last, g, b0);
    for (int c = 0;; c += 2) {
      load_wchunk_vec(t, p, min(c + 1, nvec - 1), last, g, b1);
      mma_wchunk<A, BLK, TR, TC, KS, false>(b0, nrow, ncol, acc);
      if (c + 1 >= nvec) break;
      load_wchunk_vec(t, p, min(c + 2, nvec - 1), last, g, b0);
      mma_wchunk<A, BLK, TR, TC, KS, false>(b1, nrow, ncol, acc);
      if (c + 2 >= nvec) break;
    }
  }
  if (nvec < nch) {
    load_wchunk_gen(t, p, nvec, last, g, b0);
    for (int c = nvec;; c += 2) {
      load_wchunk_gen(t, p, c + 1, last, g, b1);
      mma_wchunk<A, BLK, TR, TC, KS, true>(b0, nrow, ncol, acc);
      if (c + 1 >= nch) break;
      load_wchunk_gen(t, p, c + 2, last, g, b0);
      mma_wchunk<A, BLK, TR, TC, KS, true>(b1, nrow, ncol, acc);
      if (c + 2 >= nch) break;
    }
  }
}

template <bool L2, int Q, bool VEC, int BLK, int TR, int TC, int KS>
__device__ __forceinline__ void run_wterm(const double* t2, const double* ovvv,
                                          const double* ooov, int i, int j, int k, int no, int nv,
                                          int blk0, int row0, int col0, int nrow, int ncol,
                                          int last, int r, int g, d4 (&acc)[BLK][TR][TC]) {
  run_term<wterm_a_is_bl<L2, Q>(), VEC && Q < 3, BLK, TR, TC, KS>(
      make_wterm<L2, Q>(t2, ovvv, ooov, i, j, k, no, nv, blk0, row0, col0), nrow, ncol, last, r,
      g, acc);
}

template <bool L2, bool VEC, int BLK, int TR, int TC, int KS>
__device__ __forceinline__ void build_wtile(const double* t2, const double* ovvv,
                                            const double* ooov, int i, int j, int k, int no,
                                            int nv, int blk0, int row0, int col0, int nrow,
                                            int ncol, int last, int r, int g,
                                            d4 (&acc)[BLK][TR][TC]) {
#define SIE_WTERM(Q) \
  run_wterm<L2, Q, VEC, BLK, TR, TC, KS>(t2, ovvv, ooov, i, j, k, no, nv, blk0, row0, col0, \
                                         nrow, ncol, last, r, g, acc)
  SIE_WTERM(0);
  SIE_WTERM(1);
  SIE_WTERM(2);
  SIE_WTERM(3);
  SIE_WTERM(4);
  SIE_WTERM(5);
#undef SIE_WTERM
}

// ---------------------------------------------------------------------------
// Three-layout float64 build.  The twelve terms are regrouped by which MFMA
// side their per-block operand sits on, so that a work-group can span the
// whole shared side and read each per-block row once:
//   layout A, cube [a][b][c]: block a, per-block rows b, shared cols c
//     (X^abc_ijk and X^bac_jik d-sums, X^cba_kji and X^cab_kij l-sums);
//   layout B, cube [a][b][c]: block a, shared rows b, per-block cols c
//     (the first layout's other four terms);
//   layout C, cube [b][a][c]: block b, shared rows a, per-block cols c
//     (the second layout's other four terms);
// Wt[a][b][c] = A[a][b][c] + B[a][b][c] + C[b][a][c].  For a pair unit
// (i = j, see unit_triple) C equals B as an array, so only A and B are built.
// ---------------------------------------------------------------------------

// Layout-A terms of the second layout re-blocked on a: X^bac_jik d-sum
// ovvv[j][b][a][d] t2[k][i][c][d] and X^cab_kij l-sum
// -sum_l t2[l][j][a][b] ooov[i][l][k][c]; block a, rows b, cols c.
template <int Q>
__device__ __forceinline__ WTerm make_wterm_a(const double* __restrict__ t2,
                                              const double* __restrict__ ovvv,
                                              const double* __restrict__ ooov, int i, int j,
                                              int k, int no_, int nv_, int blk0, int row0,
                                              int col0) {
  const int64_t nv = nv_, no = no_, nv2 = nv * nv, nonv = no * nv;
  WTerm t;
  t.nK = nv_;
  t.scale = 1.0;
  if (Q == 0) {
    t.bl = ovvv + ((j * nv + row0) * nv + blk0) * nv; t.bl_b = nv; t.bl_x = nv2; t.bl_k = 1;
    t.sh = t2 + ((k * no + i) * nv + col0) * nv; t.sh_x = nv; t.sh_k = 1;
  } else {
    t.bl = t2 + (j * nv + blk0) * nv + row0; t.bl_b = nv; t.bl_x = 1; t.bl_k = nonv * nv;
    t.sh = ooov + (i * no * no + k) * nv + col0; t.sh_x = 1; t.sh_k = nonv; t.scale = -1.0;
    t.nK = no_;
  }
  return t;
}

// All terms of layout LAY into acc: layout A (LAY 0) has the per-block
// operand on the rows (acc[BLK][P][S]); B and C (LAY 1, 2) on the cols
// (acc[BLK][S][P]).
template <int LAY, bool VEC, int BLK, int TR, int TC, int KS>
__device__ __forceinline__ void build_wtile3(const double* t2, const double* ovvv,
                                             const double* ooov, int i, int j, int k, int no,
                                             int nv, int blk0, int row0, int col0, int nrow,
                                             int ncol, int last, int r, int g,
                                             d4 (&acc)[BLK][TR][TC]) {
  if (LAY == 0) {
    run_wterm<false, 0, VEC, BLK, TR, TC, KS>(t2, ovvv, ooov, i, j, k, no, nv, blk0, row0,
                                              col0, nrow, ncol, last, r, g, acc);
    run_term<true, VEC, BLK, TR, TC, KS>(
        make_wterm_a<0>(t2, ovvv, ooov, i, j, k, no, nv, blk0, row0, col0), nrow, ncol, last, r,
        g, acc);
    run_wterm<false, 4, VEC, BLK, TR, TC, KS>(t2, ovvv, ooov, i, j, k, no, nv, blk0, row0,
                                              col0, nrow, ncol, last, r, g, acc);
    run_term<true, false, BLK, TR, TC, KS>(
        make_wterm_a<1>(t2, ovvv, ooov, i, j, k, no, nv, blk0, row0, col0), nrow, ncol, last, r,
        g, acc);
  } else {
    constexpr bool L2 = LAY == 2;
#define SIE_WTERM(Q) \
  run_wterm<L2, Q, VEC, BLK, TR, TC, KS>(t2, ovvv, ooov, i, j, k, no, nv, blk0, row0, col0, \
                                         nrow, ncol, last, r, g, acc)
    if (L2) {
      SIE_WTERM(0);
      SIE_WTERM(1);
      SIE_WTERM(3);
      SIE_WTERM(4);
    } else {
      SIE_WTERM(1);
      SIE_WTERM(2);
      SIE_WTERM(3);
      SIE_WTERM(5);
    }
#undef SIE_WTERM
  }
}

// Store a wave's accumulators into a cube (block, row, col) of edge n_v, in
// the layout cube_at gives: element v of lane (g, r) in acc[beta][rt][ct]
// holds P[blk0 + beta][row0 + 16 rt + 4 v + g][col0 + 16 ct + r].
template <int BLK, int TR, int TC>
__device__ __forceinline__ void store_wtile(double* __restrict__ out, bool blocked, int nv,
                                            int blk0, int row0, int col0, int r, int g,
                                            const d4 (&acc)[BLK][TR][TC]) {
#pragma unroll
  for (int beta = 0; beta < BLK; ++beta) {
    const int blk = blk0 + beta;
#pragma unroll
    for (int rt = 0; rt < TR; ++rt)
#pragma unroll
      for (int ct = 0; ct < TC; ++ct) {
        const int col = col0 + 16 * ct + r;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + 16 * rt + 4 * v + g;
          if (blk < nv && row < nv && col < nv)
            gptr_w(out)[cube_at(blocked, nv, blk, row, col)] = acc[beta][rt][ct][v];
        }
      }
  }
}

template <int BLK, int TR, int TC>
__device__ __forceinline__ void zero_acc(d4 (&acc)[BLK][TR][TC]) {
#pragma unroll
  for (int b = 0; b < BLK; ++b)
#pragma unroll
    for (int p = 0; p < TR; ++p)
#pragma unroll
      for (int q = 0; q < TC; ++q) acc[b][p][q] = d4{0.0, 0.0, 0.0, 0.0};
}

// Map a linear block index to a tile so that the blocks the hardware places
// on one XCD (block index mod 8) cover a contiguous range of tiles and share
// their operand rows in that XCD's L2.
#ifndef SIE_XCD_MAP
#define SIE_XCD_MAP 1
#endif
__device__ __forceinline__ int xcd_tile(int bid, int n) {
  if (!SIE_XCD_MAP) return bid;
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd;
  const int xcd = bid % kXcd, local = bid / kXcd;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Partial cube of one layout over one tile of one unit, written to the
// unit's first (L1) or second (L2) cube in (block, row, col) order.  Grid:
// the concatenated build work-groups of the round's items (all of one tile
// variant): two layouts per unit, one for a pair unit (unit_triple).  Block:
// 256 threads.  VEC (FragDesc::vec): n_v is even and the t2 / ovvv bases are
// 16-byte aligned, so d-rows are read 16 bytes at a time.  KS: k-steps per
// K-chunk (chunks of 8 or 16).
template <int BLK, int TR, int TC, int BPC, int WR = 1, int WC = 1, int KS = 2>
__global__ __launch_bounds__(256, BPC) void k_build_w_f64(const FragDesc* __restrict__ descs,
                                                          const Item* __restrict__ items,
                                                          int n_items,
                                                          double* __restrict__ arena) {
  constexpr bool GRID = WR * WC > 1;
  static_assert(!GRID || WR * WC == kWWaves, "wave grid covers the work-group");
  constexpr int BB = GRID ? BLK : kWWaves * BLK;
  constexpr int ER = 16 * TR * (GRID ? WR : 1), EC = 16 * TC * (GRID ? WC : 1);
  const int ri = find_item<true>(items, n_items, blockIdx.x);
  const int64_t start = ri ? items[ri - 1].blk_end : 0;
  const Item it = items[ri];
  const FragDesc fd = descs[it.frag];
  int i, j, k;
  bool one;
  if (!item_triple(it.unit, fd.no, fd.pair, i, j, k, one)) return;
  const int nv = fd.nv;
  const int nbt = (nv + BB - 1) / BB, nrt = (nv + ER - 1) / ER, nct = (nv + EC - 1) / EC;
  const int per = nbt * nrt * nct;
  int t = xcd_tile(int(int64_t(blockIdx.x) - start), one ? per : 2 * per);
  const bool l2 = t >= per;
  if (l2) t -= per;
  const int tb = t / (nrt * nct);
  t -= tb * nrt * nct;
  const int tr = t / nct, tc = t - tr * nct;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int r = lane & 15, g = lane >> 4;
  const int blk0 = tb * BB + (GRID ? 0 : wave * BLK);
  const int row0 = tr * ER + (GRID ? (wave % WR) * 16 * TR : 0);
  const int col0 = tc * EC + (GRID ? (wave / WR) * 16 * TC : 0);
  if (blk0 >= nv || row0 >= nv || col0 >= nv) return;   // no barrier follows: waves may leave
  const int nrow = min(16 * TR, nv - row0), ncol = min(16 * TC, nv - col0);
  const int last = min(BLK, nv - blk0) - 1;
  const double* t2 = static_cast<const double*>(fd.t2);
  const double* ovvv = static_cast<const double*>(fd.ovvv);
  const double* ooov = static_cast<const double*>(fd.ooov);

  d4 acc[BLK][TR][TC];
  zero_acc(acc);

#define SIE_WTILE(L, V) \
  build_wtile<L, V, BLK, TR, TC, KS>(t2, ovvv, ooov, i, j, k, fd.no, nv, blk0, row0, col0, nrow, \
                                 ncol, last, r, g, acc)
  if (l2) {
    if (fd.vec) SIE_WTILE(true, true);
    else SIE_WTILE(true, false);
  } else {
    if (fd.vec) SIE_WTILE(false, true);
    else SIE_WTILE(false, false);
  }
#undef SIE_WTILE

  store_wtile(arena + it.cube_off + (l2 ? fd.half : 0), fd.blocked != 0, nv, blk0, row0, col0,
              r, g, acc);
}

// Three-layout build (build_wtile3): partial cubes A, B, C of one tile of
// one unit.  A work-group is 4 waves along the blocks (4 BLK blocks) x 16 P
// rows or cols of the per-block side x 16 S of the shared side, so with
// 16 S >= n_v it spans the shared side and each per-block operand row is
// read by one work-group only.  Grid: the concatenated work-groups of the
// round's items, three layouts per unit, two (A, B) for a pair unit.
template <int BLK, int P, int S, int BPC, int KS = 2>
__global__ __launch_bounds__(256, BPC) void k_build_w3_f64(const FragDesc* __restrict__ descs,
                                                           const Item* __restrict__ items,
                                                           int n_items,
                                                           double* __restrict__ arena) {
  constexpr int BB = kWWaves * BLK, EP = 16 * P, ES = 16 * S;
  const int ri = find_item<true>(items, n_items, blockIdx.x);
  const int64_t start = ri ? items[ri - 1].blk_end : 0;
  const Item it = items[ri];
  const FragDesc fd = descs[it.frag];
  int i, j, k;
  bool one;
  if (!item_triple(it.unit, fd.no, fd.pair, i, j, k, one)) return;
  const int nv = fd.nv;
  const int nbt = (nv + BB - 1) / BB, npt = (nv + EP - 1) / EP, nst = (nv + ES - 1) / ES;
  const int per = nbt * npt * nst;
  int t = xcd_tile(int(int64_t(blockIdx.x) - start), (one ? 2 : 3) * per);
  const int lay = t / per;
  t -= lay * per;
  const int tb = t / (npt * nst);
  t -= tb * npt * nst;
  const int tp = t / nst, ts = t - tp * nst;   // work-groups sharing per-block rows are adjacent
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int r = lane & 15, g = lane >> 4;
  const int blk0 = tb * BB + wave * BLK;
  if (blk0 >= nv) return;   // no barrier follows: waves may leave
  const int p0 = tp * EP, s0 = ts * ES;
  const int np = min(EP, nv - p0), ns = min(ES, nv - s0);
  const int last = min(BLK, nv - blk0) - 1;
  const double* t2 = static_cast<const double*>(fd.t2);
  const double* ovvv = static_cast<const double*>(fd.ovvv);
  const double* ooov = static_cast<const double*>(fd.ooov);
  double* __restrict__ out = arena + it.cube_off + lay * fd.half;
  if (lay == 0) {   // per-block rows, shared cols
    d4 acc[BLK][P][S];
    zero_acc(acc);
    if (fd.vec)
      build_wtile3<0, true, BLK, P, S, KS>(t2, ovvv, ooov, i, j, k, fd.no, nv, blk0, p0, s0, np, ns, last, r, g,
                            acc);
    else
      build_wtile3<0, false, BLK, P, S, KS>(t2, ovvv, ooov, i, j, k, fd.no, nv, blk0, p0, s0, np, ns, last, r,
                             g, acc);
    store_wtile(out, fd.blocked != 0, nv, blk0, p0, s0, r, g, acc);
  } else {          // shared rows, per-block cols
    d4 acc[BLK][S][P];
    zero_acc(acc);
#define SIE_W3(L, V) \
  build_wtile3<L, V, BLK, S, P, KS>(t2, ovvv, ooov, i, j, k, fd.no, nv, blk0, s0, p0, ns, np, \
                                    last, r, g, acc)
    if (lay == 1) {
      if (fd.vec) SIE_W3(1, true);
      else SIE_W3(1, false);
    } else {
      if (fd.vec) SIE_W3(2, true);
      else SIE_W3(2, false);
    }
#undef SIE_W3
    store_wtile(out, fd.blocked != 0, nv, blk0, s0, p0, r, g, acc);
  }
}

// LDS position of in-block offset (x, y, z) of an 8^3 orbit block, padded so
// that the six permuted reads of a wave (x fixed, y and z over the lanes)
// spread over the 16 double-wide banks (at most 5 lanes per bank instead of
// up to 32 without padding).
constexpr int kOrbPlane = 72, kOrbRow = 9;
constexpr int kOrbSlot = kOrb * kOrbPlane;
__device__ __forceinline__ int orb_lds(int x, int y, int z) {
  return x * kOrbPlane + y * kOrbRow + z;
}

// In-block offset e = x*64 + y*8 + z of element l (0 <= l < 512, in the
// order idx = threadIdx.x + 256 h of a 256-thread loop over one slot): thread
// t takes (t / 32, (t / 4) % 8, 2 (t % 4) + h), the element mapping of the
// epilogue, with which the permuted LDS reads of a wave spread over the banks
// (consecutive z across the lanes would put lanes a 72-double row apart into
// the same banks).
__device__ __forceinline__ int orb_elem(int l) {
  const int t = l & 255, h = l >> 8;
  return ((t >> 5) << 6) | (((t >> 2) & 7) << 3) | ((t & 3) << 1) | h;
}

// Orbit slots enumerate the position permutations (0,1,2) (0,2,1) (1,0,2)
// (1,2,0) (2,0,1) (2,1,0) of a block triple.
__device__ __forceinline__ int orbit_slot(int p, int q, int r) {
  return 2 * p + (q > r ? 1 : 0);
}
__device__ __forceinline__ void slot_perm(int s, int& p0, int& p1, int& p2) {
  p0 = s >> 1;
  const int o1 = p0 == 0 ? 1 : 0;
  const int o2 = p0 == 2 ? 1 : 2;
  p1 = (s & 1) ? o2 : o1;
  p2 = (s & 1) ? o1 : o2;
}
__device__ __forceinline__ int pick3(int p, int t0, int t1, int t2) {
  return p == 0 ? t0 : (p == 1 ? t1 : t2);
}

__device__ __forceinline__ double block_sum_256(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return s;
}

// Elements (row, c0) and (row, c0 + 1) of a row-major array with rows of
// stride `rs` and n columns: one two-element load (PV: n even, so an in-range
// even c0 has c0 + 1 < n and the pair is aligned), or two loads with each
// column clamped to n - 1 (callers mask columns past n).
template <typename T, bool PV>
__device__ __forceinline__ void ld_pair(const T* p, int64_t row, int64_t rs, int c0, int n,
                                        double (&v)[2]) {
  if (PV) {
    typedef typename std::conditional<sizeof(T) == 8, d2v, f2v>::type V2;
    const V2 u = *(const SIE_GLOBAL V2*)(gptr(p) + row * rs + min(c0, n - 2));
    v[0] = (double)u.x;
    v[1] = (double)u.y;
  } else {
    v[0] = (double)gptr(p)[row * rs + min(c0, n - 1)];
    v[1] = (double)gptr(p)[row * rs + min(c0 + 1, n - 1)];
  }
}

// Element of type T at byte offset `off` from a base that is the same in
// every lane of the wave (read from the first lane, so that the load takes
// the base from scalar registers and only the 32-bit offset per lane).
// (readfirstlane moves 32 bits: the two halves of the address go separately)
template <typename T, typename B>
__device__ __forceinline__ T ld_at(const B* base, uint32_t off) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(a))));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(a >> 32))));
  const uint64_t b = (uint64_t(hi) << 32) | lo;
  return *(const SIE_GLOBAL T*)(reinterpret_cast<const SIE_GLOBAL char*>(b) + off);
}

// Element mapping of the epilogue: thread t holds, in every slot s of the
// orbit, the two elements at in-block offsets (t / 32, (t / 4) % 8,
// 2 (t % 4) + h), h = 0, 1 (adjacent along c), i.e. elements 2t and 2t + 1
// of the slot's 8^3 block of a blocked cube (cube_at).  The cube pairs of
// those 12 elements from two-layout cubes: w1[a][b][c] (u) and w3[b][a][c]
// (w), as loaded (the caller sums them once every load of the orbit is in
// flight); every block of the padded cube exists, so nothing is clamped (the
// caller masks elements past n_v).
template <typename CubeT, typename V2>
__device__ __forceinline__ void epi_issue_w(const CubeT* __restrict__ w1,
                                            const CubeT* __restrict__ w3, int nb, int t0,
                                            int t1b, int t2b, V2 (&u)[6], V2 (&w)[6]) {
  constexpr int kB = kOrb * kOrb * kOrb;
  const int x = threadIdx.x >> 5, y = (threadIdx.x >> 2) & 7, z0 = 2 * (threadIdx.x & 3);
  // wave-uniform block bases, 32-bit lane offsets inside a block
  const uint32_t in_xy = uint32_t(x * 64 + y * 8 + z0) * sizeof(CubeT);
  const uint32_t in_yx = uint32_t(y * 64 + x * 8 + z0) * sizeof(CubeT);
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    int p0, p1, p2;
    slot_perm(s, p0, p1, p2);
    const int P0 = pick3(p0, t0, t1b, t2b), P1 = pick3(p1, t0, t1b, t2b);
    const int P2 = pick3(p2, t0, t1b, t2b);
    const int64_t o1 = ((int64_t(P0) * nb + P1) * nb + P2) * kB;
    const int64_t o3 = ((int64_t(P1) * nb + P0) * nb + P2) * kB;
    u[s] = ld_at<V2>(w1 + o1, in_xy);
    w[s] = ld_at<V2>(w3 + o3, in_yx);
  }
}

// Wt of the same 12 elements, summed as the loads arrive (float64 cubes,
// whose raw pairs would take twice the registers): w1[a][b][c] (+ w2[a][b][c], three layouts) + w3[b][a][c]; every
// block of the padded cube exists, so nothing is clamped (the caller masks
// elements past n_v); all loads are issued before any is summed.
template <bool L3, typename CubeT>
__device__ __forceinline__ void epi_load_w(const CubeT* __restrict__ w1,
                                           const CubeT* __restrict__ w2,
                                           const CubeT* __restrict__ w3, int nb, int t0, int t1b,
                                           int t2b, double (&wreg)[12]) {
  typedef typename std::conditional<sizeof(CubeT) == 8, d2v, f2v>::type V2;
  constexpr int kB = kOrb * kOrb * kOrb;
  const int x = threadIdx.x >> 5, y = (threadIdx.x >> 2) & 7, z0 = 2 * (threadIdx.x & 3);
  const int in_xy = x * 64 + y * 8 + z0, in_yx = y * 64 + x * 8 + z0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    int p0, p1, p2;
    slot_perm(s, p0, p1, p2);
    const int P0 = pick3(p0, t0, t1b, t2b), P1 = pick3(p1, t0, t1b, t2b);
    const int P2 = pick3(p2, t0, t1b, t2b);
    const int64_t o1 = ((int64_t(P0) * nb + P1) * nb + P2) * kB + in_xy;
    const int64_t o3 = ((int64_t(P1) * nb + P0) * nb + P2) * kB + in_yx;
    const V2 u = *(const SIE_GLOBAL V2*)(gptr(w1) + o1);
    V2 v{};
    if (L3) v = *(const SIE_GLOBAL V2*)(gptr(w2) + o1);
    const V2 w = *(const SIE_GLOBAL V2*)(gptr(w3) + o3);
    wreg[2 * s] = (double)u.x + (L3 ? (double)v.x : 0.0) + (double)w.x;
    wreg[2 * s + 1] = (double)u.y + (L3 ? (double)v.y : 0.0) + (double)w.y;
  }
}

// Z = Wt + V-tilde of slot s of the orbit (t0, t1b, t2b) at this thread's
// two elements, to LDS; elements past n_v get Z = 0 and Wt = 0.  rij, rik,
// rjk: the slot's (ia|jb), (ia|kc), (jb|kc) elements; V: the orbit's vectors.
template <typename InT>
__device__ __forceinline__ void epi_z_slot(int s, int t0, int t1b, int t2b, int x, int y, int z0,
                                           int nv, InT rij, const InT (&rik)[2],
                                           const InT (&rjk)[2], const double* V,
                                           double (&wreg)[12], double (*sz)[kOrbSlot]) {
  int p0, p1, p2;
  slot_perm(s, p0, p1, p2);
  const int a = kOrb * pick3(p0, t0, t1b, t2b) + x;
  const int b = kOrb * pick3(p1, t0, t1b, t2b) + y;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int zz = z0 + h;
    double z = 0.0;
    if (a < nv && b < nv && zz + kOrb * pick3(p2, t0, t1b, t2b) < nv) {
      const double vt = (double)rij * V[(9 + p2) * kOrb + zz] +
                        (double)rik[h] * V[(6 + p1) * kOrb + y] +
                        (double)rjk[h] * V[(3 + p0) * kOrb + x];
      z = wreg[2 * s + h] + vt;
    } else {
      wreg[2 * s + h] = 0.0;
    }
    sz[s][orb_lds(x, y, zz)] = z;
  }
}

// Sum over this thread's elements of the orbit of Wt R'[Z] / D, Z read from
// the six slots in LDS.  A slot whose block triple repeats an earlier slot's
// is not summed twice (only when two of the sorted block indices are equal).
__device__ __forceinline__ double epi_rprime(int t0, int t1b, int t2b, int x, int y, int z0,
                                             int nv, double eijk, const double* V,
                                             const double (&wreg)[12],
                                             const double (*sz)[kOrbSlot]) {
  unsigned primary = 63u;
  if (t0 == t1b || t1b == t2b) {
    primary = 0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      int p0, p1, p2;
      slot_perm(s, p0, p1, p2);
      bool dup = false;
#pragma unroll
      for (int s2 = 0; s2 < s; ++s2) {
        int q0, q1, q2;
        slot_perm(s2, q0, q1, q2);
        dup |= pick3(p0, t0, t1b, t2b) == pick3(q0, t0, t1b, t2b) &&
               pick3(p1, t0, t1b, t2b) == pick3(q1, t0, t1b, t2b) &&
               pick3(p2, t0, t1b, t2b) == pick3(q2, t0, t1b, t2b);
      }
      if (!dup) primary |= 1u << s;
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    if (!((primary >> s) & 1u)) continue;
    int p0, p1, p2;
    slot_perm(s, p0, p1, p2);
    const int a = kOrb * pick3(p0, t0, t1b, t2b) + x;
    const int b = kOrb * pick3(p1, t0, t1b, t2b) + y;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int zz = z0 + h;
      const int c = kOrb * pick3(p2, t0, t1b, t2b) + zz;
      if (a >= nv || b >= nv || c >= nv) continue;
      // Z at the five permuted virtual triples, found in the slot holding
      // the permuted block triple at the permuted in-block offsets
      const double zabc = sz[s][orb_lds(x, y, zz)];
      const double zcab = sz[orbit_slot(p2, p0, p1)][orb_lds(zz, x, y)];
      const double zbca = sz[orbit_slot(p1, p2, p0)][orb_lds(y, zz, x)];
      const double zcba = sz[orbit_slot(p2, p1, p0)][orb_lds(zz, y, x)];
      const double zacb = sz[orbit_slot(p0, p2, p1)][orb_lds(x, zz, y)];
      const double zbac = sz[orbit_slot(p1, p0, p2)][orb_lds(y, x, zz)];
      const double rz = 4.0 * zabc + zcab + zbca - 2.0 * (zcba + zacb + zbac);
      const double d = eijk - V[p0 * kOrb + x] - V[p1 * kOrb + y] - V[p2 * kOrb + zz];
      acc += wreg[2 * s + h] * rz * recip(d);
    }
  }
  return acc;
}

// Energy of this thread's virtual triples (a, b, c_h), h = 0, 1, of an orbit
// with all six orderings of each (float32 inputs): Wt of the orderings from
// the six slots in LDS (the first from wreg), V-tilde of each ordering from
// the ovov elements o_pq (slices (i,j), (i,k), (j,k)) and the orbit's t1
// vectors in V, Z = Wt + V-tilde.  With the cyclic orderings (abc, bca, cab)
// as even and the others as odd, R'[Z] of an even ordering is
// 3 Z + S_e - 2 S_o (S_e, S_o: the sums of Z over the even and the odd
// orderings), and of an odd one 3 Z + S_o - 2 S_e, so the six terms of
// Wt R'[Z] / D (one D for all six) add up to
//   (3 sum Wt Z + (S_e - 2 S_o) W_e + (S_o - 2 S_e) W_o) / D.
// Orbits with equal block indices repeat slots: there only triples with
// a >= b (first two blocks equal) or b >= c (last two) count, those with a
// repeated index at half weight (their six orderings hold each triple
// twice), and a = b = c not at all (R' annihilates it).
template <typename InT>
__device__ __forceinline__ double epi_triple_orbits(
    int t0, int t1b, int t2b, int x, int y, int z0, int ar, int br, int c0, int nv, double eijk,
    const double* V, const double (&wreg)[12], const double (*sz)[kOrbSlot],
    const InT (&o_ab)[3], const InT (&o_ba)[3], const InT (&o_ac)[3][2],
    const InT (&o_bc)[3][2], const InT (&o_ca)[3][2], const InT (&o_cb)[3][2]) {
  const bool e01 = t0 == t1b, e12 = t1b == t2b;
  // V[(3 q + p) kOrb + o]: e_vir (q = 0), t1[i], t1[j], t1[k] at block position p
  const double ea = V[x], eb = V[kOrb + y];
  const double ia = V[3 * kOrb + x], ib = V[4 * kOrb + y];
  const double ja = V[6 * kOrb + x], jb = V[7 * kOrb + y];
  const double ka = V[9 * kOrb + x], kb = V[10 * kOrb + y];
  // q = 0: (i|j), 1: (i|k), 2: (j|k)
  const double ij_ab = o_ab[0], ik_ab = o_ab[1], jk_ab = o_ab[2];
  const double ij_ba = o_ba[0], ik_ba = o_ba[1], jk_ba = o_ba[2];
  double acc = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int zz = z0 + h;
    const double ec = V[2 * kOrb + zz];
    const double ic = V[5 * kOrb + zz], jc = V[8 * kOrb + zz], kc = V[11 * kOrb + zz];
    const double ij_ac = o_ac[0][h], ik_ac = o_ac[1][h], jk_ac = o_ac[2][h];
    const double ij_bc = o_bc[0][h], ik_bc = o_bc[1][h], jk_bc = o_bc[2][h];
    const double ij_ca = o_ca[0][h], ik_ca = o_ca[1][h], jk_ca = o_ca[2][h];
    const double ij_cb = o_cb[0][h], ik_cb = o_cb[1][h], jk_cb = o_cb[2][h];
    // Wt of the orderings abc, bca, cab (even) and acb, bac, cba (odd)
    const double w_abc = wreg[h];
    const double w_bca = sz[3][orb_lds(y, zz, x)];
    const double w_cab = sz[4][orb_lds(zz, x, y)];
    const double w_acb = sz[1][orb_lds(x, zz, y)];
    const double w_bac = sz[2][orb_lds(y, x, zz)];
    const double w_cba = sz[5][orb_lds(zz, y, x)];
    // V-tilde(pqr) = (ip|jq) t1[k][r] + (ip|kr) t1[j][q] + (jq|kr) t1[i][p]
    const double z_abc = w_abc + (ij_ab * kc + ik_ac * jb + jk_bc * ia);
    const double z_bca = w_bca + (ij_bc * ka + ik_ba * jc + jk_ca * ib);
    const double z_cab = w_cab + (ij_ca * kb + ik_cb * ja + jk_ab * ic);
    const double z_acb = w_acb + (ij_ac * kb + ik_ab * jc + jk_cb * ia);
    const double z_bac = w_bac + (ij_ba * kc + ik_bc * ja + jk_ac * ib);
    const double z_cba = w_cba + (ij_cb * ka + ik_ca * jb + jk_ba * ic);
    const double se = (z_abc + z_bca) + z_cab, so = (z_acb + z_bac) + z_cba;
    const double we = (w_abc + w_bca) + w_cab, wo = (w_acb + w_bac) + w_cba;
    const double swz = w_abc * z_abc + w_bca * z_bca + w_cab * z_cab + w_acb * z_acb +
                       w_bac * z_bac + w_cba * z_cba;
    const double num = 3.0 * swz + (se - 2.0 * so) * we + (so - 2.0 * se) * wo;
    const int cr = c0 + h;
    // which triples of a degenerate orbit count, and at what weight (in-block
    // offsets x, y, zz)
    double wgt = 1.0;
    if (e01 && e12) {
      wgt = (x > y && y > zz) ? 1.0 : ((x >= y && y >= zz && !(x == y && y == zz)) ? 0.5 : 0.0);
    } else if (e01) {
      wgt = x > y ? 1.0 : (x == y ? 0.5 : 0.0);
    } else if (e12) {
      wgt = y > zz ? 1.0 : (y == zz ? 0.5 : 0.0);
    }
    const double d = eijk - ea - eb - ec;
    const double term = wgt * num * recip(d);
    acc += (ar < nv && br < nv && cr < nv && wgt != 0.0) ? term : 0.0;
  }
  return acc;
}

// Per-unit partial sums of Wt R'[Wt + Vt] / D over symmetric orbits of
// 8 x 8 x 8 virtual blocks (A >= B >= C and their permuted images).
// Wt[a][b][c] = P1[a][b][c] + P2[b][a][c] from the two-layout builds, or
// A[a][b][c] + B[a][b][c] + C[b][a][c] from the three-layout build
// (FragDesc::lay3), float64 or float32 cubes; V-tilde from t1 and ovov
// (float64 or float32 inputs), all arithmetic in float64.  Grid: the concatenated
// epilogue blocks of the round's items (n_part per item; block p of an item
// takes orbits p, p + n_part, ...).  At most 128 registers a lane (four
// waves a SIMD).
//
// Float32 cubes and inputs (the split form, whose build writes two layouts):
// every load of an orbit is issued before any is used (the V entries, the
// cube pairs and the ovov elements of each thread's triples), so that the
// orbit waits on memory once; Wt goes to LDS and each thread sums its
// triples with all six orderings (epi_triple_orbits).  Float64 (twice the
// registers): the cube pairs are summed as they arrive, each slot's ovov
// elements are loaded just before the slot, Z goes to LDS and every element
// is summed by the thread that holds it (epi_z_slot, epi_rprime).
template <typename CubeT, typename InT>
__global__ __launch_bounds__(256, 4) void k_epilogue(const FragDesc* __restrict__ descs,
                                                  const Item* __restrict__ items, int n_items,
                                                  const CubeT* __restrict__ arena,
                                                  double* __restrict__ partials, int pstride) {
  const int r = find_item<false>(items, n_items, blockIdx.x);
  const int64_t start = r ? items[r - 1].part_end : 0;
  const Item it = items[r];
  const FragDesc fd = descs[it.frag];
  const int slot = int(int64_t(blockIdx.x) - start);
  int i, j, k;
  const bool one = unit_triple(it.unit, fd.no, fd.pair, i, j, k);
  __shared__ double sz[6][kOrbSlot];   // the six slots' Wt (float32) or Z (float64)
  // per orbit, for its three block positions: e_vir, t1[i], t1[j], t1[k]
  __shared__ double sv[4 * 3 * kOrb];
  __shared__ double red[4];
  __shared__ int sorb[256];   // float32 path: packed orbit block triples
  double* out = partials + (fd.unit_base + it.unit) * pstride + slot;
  if (i == k) {
    if (threadIdx.x == 0) *out = 0.0;
    return;
  }
  const InT* __restrict__ t1 = static_cast<const InT*>(fd.t1);
  const InT* __restrict__ ovov = static_cast<const InT*>(fd.ovov);
  const double* __restrict__ eps = fd.eps;
  const int no_ = fd.no, nv_ = fd.nv;
  const int no = no_, nv = nv_;
  const int nb = (nv + kOrb - 1) / kOrb;
  const int64_t n_orb = tetra(nb);
  const double* __restrict__ ev = eps + no;
  const double eijk = gptr(eps)[i] + gptr(eps)[j] + gptr(eps)[k];
  // Wt = w1[a][b][c] (+ w2[a][b][c], three layouts) + w3[b][a][c]; a pair unit
  // has P2 = P1 (two layouts) or C = B (three layouts)
  const bool l3 = fd.lay3;
  const CubeT* __restrict__ w1 = arena + it.cube_off;
  const CubeT* __restrict__ w2 = w1 + fd.half;
  const CubeT* __restrict__ w3 = l3 ? (one ? w2 : w2 + fd.half) : (one ? w1 : w2);
  const int64_t nonv = (int64_t)no * nv;
  const InT* ov_ij = ovov + (int64_t)i * nv * nonv + (int64_t)j * nv;   // (ia|jb) = ov_ij[a*nonv + b]
  const InT* ov_ik = ovov + (int64_t)i * nv * nonv + (int64_t)k * nv;
  const InT* ov_jk = ovov + (int64_t)j * nv * nonv + (int64_t)k * nv;
  const InT* t1i = t1 + (int64_t)i * nv;
  const InT* t1j = t1 + (int64_t)j * nv;
  const InT* t1k = t1 + (int64_t)k * nv;

  const double* V = sv;   // V[(3 q + p) kOrb + x]: vector q at block position p
  const int x = threadIdx.x >> 5, y = (threadIdx.x >> 2) & 7, z0 = 2 * (threadIdx.x & 3);
  // V entry of this thread (threads below 3 x 4 x kOrb keep theirs): vector
  // vq at block position vp
  const int vq = threadIdx.x / (3 * kOrb), vp = (threadIdx.x / kOrb) % 3;

  // the slot's (ia|jb), (ia|kc), (jb|kc) elements at this thread's elements
  // (pv: fd.epv, as a constant or not)
  auto ov_load = [&](auto pv, int s, int t0, int t1b, int t2b, InT& rij, InT (&rik)[2],
                     InT (&rjk)[2]) {
    int p0, p1, p2;
    slot_perm(s, p0, p1, p2);
    const int ac = min(kOrb * pick3(p0, t0, t1b, t2b) + x, nv - 1);
    const int bc = min(kOrb * pick3(p1, t0, t1b, t2b) + y, nv - 1);
    const int c0 = kOrb * pick3(p2, t0, t1b, t2b) + z0;
    // byte offsets inside one (i, j) slice of ovov, below 2^32 (the host
    // limits s n_occ^2 n_vir^2)
    constexpr uint32_t es = sizeof(InT);
    const uint32_t ra = uint32_t(ac) * uint32_t(nonv), rb = uint32_t(bc) * uint32_t(nonv);
    rij = ld_at<InT>(ov_ij, (ra + uint32_t(bc)) * es);
    if (pv) {
      // nv even and the rows aligned to two elements: an in-range even c0
      // has c0 + 1 < nv, so the pair is one aligned load
      typedef typename std::conditional<sizeof(InT) == 8, d2v, f2v>::type IV2;
      const uint32_t cc = uint32_t(min(c0, nv - 2));
      const IV2 pk = ld_at<IV2>(ov_ik, (ra + cc) * es);
      const IV2 pj = ld_at<IV2>(ov_jk, (rb + cc) * es);
      rik[0] = pk.x;
      rik[1] = pk.y;
      rjk[0] = pj.x;
      rjk[1] = pj.y;
    } else {
      const uint32_t c1 = uint32_t(min(c0, nv - 1)), c2 = uint32_t(min(c0 + 1, nv - 1));
      rik[0] = ld_at<InT>(ov_ik, (ra + c1) * es);
      rik[1] = ld_at<InT>(ov_ik, (ra + c2) * es);
      rjk[0] = ld_at<InT>(ov_jk, (rb + c1) * es);
      rjk[1] = ld_at<InT>(ov_jk, (rb + c2) * es);
    }
  };

  double acc = 0.0;
  if constexpr (sizeof(CubeT) == 4 && sizeof(InT) == 4) {
    // n_v even with aligned ovov rows or not: a constant in the loop (the
    // loads are then free of branches, and none waits for another)
    auto orbits = [&](auto pvtag) {
      // this work-group's orbits slot + m n_part, decoded 256 at a time by
      // the threads in parallel into sorb (three 10-bit block indices;
      // n_v <= 2048 gives at most 256 blocks), then read as wave-uniform
      // values
      const int64_t n_mine = (n_orb - slot + fd.n_part - 1) / fd.n_part;
      for (int64_t m0 = 0; m0 < n_mine; m0 += 256) {
        if (m0 + threadIdx.x < n_mine) {
          int a, b, c;
          decode_sorted_triple(slot + (m0 + threadIdx.x) * fd.n_part, nb, a, b, c);
          sorb[threadIdx.x] = a | (b << 10) | (c << 20);
        }
        __syncthreads();
        const int cnt = int(n_mine - m0 < 256 ? n_mine - m0 : 256);
        for (int m = 0; m < cnt; ++m) {
          const int pk = __builtin_amdgcn_readfirstlane(sorb[m]);
          const int t0 = pk & 1023, t1b = (pk >> 10) & 1023, t2b = pk >> 20;
          // both candidate V loads are in bounds for every thread
          const int vv = min(kOrb * pick3(vp, t0, t1b, t2b) + int(threadIdx.x % kOrb), nv - 1);
          const double ve = gptr(ev)[vv];
          const InT vt = gptr(vq == 1 ? t1i : (vq == 2 ? t1j : t1k))[vv];
          f2v cu[6], cw[6];
          epi_issue_w(w1, w3, nb, t0, t1b, t2b, cu, cw);
          // This thread's virtual triples (a, b, c_h) of the first slot,
          // c_h = c0 + h, and the ovov elements of all six orderings of each:
          // (p|q) for the ordered pairs of {a, b, c_h} in the (i, j), (i, k)
          // and (j, k) slices (indices clamped in range; results past n_v are
          // not used).
          const int ar = kOrb * t0 + x, br = kOrb * t1b + y, c0 = kOrb * t2b + z0;
          const uint32_t ua = uint32_t(min(ar, nv - 1)), ub = uint32_t(min(br, nv - 1));
          const uint32_t nov = uint32_t(nonv);
          constexpr uint32_t es = sizeof(InT);
          const InT* const sl[3] = {ov_ij, ov_ik, ov_jk};
          InT o_ab[3], o_ba[3], o_ac[3][2], o_bc[3][2], o_ca[3][2], o_cb[3][2];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            o_ab[q] = ld_at<InT>(sl[q], (ua * nov + ub) * es);
            o_ba[q] = ld_at<InT>(sl[q], (ub * nov + ua) * es);
            if (decltype(pvtag)::value) {
              // n_v even, rows aligned to two elements: (c0, c0 + 1) in range
              // is one aligned pair
              const uint32_t cc = uint32_t(min(c0, nv - 2));
              const f2v pa = ld_at<f2v>(sl[q], (ua * nov + cc) * es);
              const f2v pb = ld_at<f2v>(sl[q], (ub * nov + cc) * es);
              o_ac[q][0] = pa.x;
              o_ac[q][1] = pa.y;
              o_bc[q][0] = pb.x;
              o_bc[q][1] = pb.y;
            } else {
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const uint32_t uc = uint32_t(min(c0 + h, nv - 1));
                o_ac[q][h] = ld_at<InT>(sl[q], (ua * nov + uc) * es);
                o_bc[q][h] = ld_at<InT>(sl[q], (ub * nov + uc) * es);
              }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const uint32_t uc = uint32_t(min(c0 + h, nv - 1));
              o_ca[q][h] = ld_at<InT>(sl[q], (uc * nov + ua) * es);
              o_cb[q][h] = ld_at<InT>(sl[q], (uc * nov + ub) * es);
            }
          }
          double wreg[12];
#pragma unroll
          for (int s = 0; s < 6; ++s) {
            wreg[2 * s] = (double)cu[s].x + (double)cw[s].x;
            wreg[2 * s + 1] = (double)cu[s].y + (double)cw[s].y;
          }
          // (the previous orbit's last barrier freed sv and sz)
          if (threadIdx.x < 4 * 3 * kOrb) sv[threadIdx.x] = vq == 0 ? ve : (double)vt;
#pragma unroll
          for (int s = 0; s < 6; ++s) {
            sz[s][orb_lds(x, y, z0)] = wreg[2 * s];
            sz[s][orb_lds(x, y, z0 + 1)] = wreg[2 * s + 1];
          }
          __syncthreads();   // Wt of the orbit and its vectors in LDS
          acc += epi_triple_orbits(t0, t1b, t2b, x, y, z0, ar, br, c0, nv, eijk, V, wreg, sz,
                                   o_ab, o_ba, o_ac, o_bc, o_ca, o_cb);
          __syncthreads();   // (also orders this chunk's reads of sorb before the next chunk's writes)
        }
      }
    };
    if (fd.epv) orbits(std::true_type{});
    else orbits(std::false_type{});
  } else {
    for (int64_t o = slot; o < n_orb; o += fd.n_part) {
      int t0, t1b, t2b;
      decode_sorted_triple(o, nb, t0, t1b, t2b);
      if (threadIdx.x < 4 * 3 * kOrb) {   // (the previous orbit's last barrier freed sv)
        const int v = min(kOrb * pick3(vp, t0, t1b, t2b) + int(threadIdx.x % kOrb), nv - 1);
        double xv;
        if (vq == 0) xv = gptr(ev)[v];
        else if (vq == 1) xv = (double)gptr(t1i)[v];
        else if (vq == 2) xv = (double)gptr(t1j)[v];
        else xv = (double)gptr(t1k)[v];
        sv[threadIdx.x] = xv;
      }
      double wreg[12];
      if (l3) epi_load_w<true>(w1, w2, w3, nb, t0, t1b, t2b, wreg);
      else epi_load_w<false>(w1, w2, w3, nb, t0, t1b, t2b, wreg);
      __syncthreads();   // sv filled
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        InT rij, rik[2], rjk[2];
        ov_load(fd.epv != 0, s, t0, t1b, t2b, rij, rik, rjk);
        epi_z_slot(s, t0, t1b, t2b, x, y, z0, nv, rij, rik, rjk, V, wreg, sz);
      }
      __syncthreads();
      acc += epi_rprime(t0, t1b, t2b, x, y, z0, nv, eijk, V, wreg, sz);
      __syncthreads();
    }
  }
  const double s = block_sum_256(acc, red);
  if (threadIdx.x == 0) *out = s;
}

}  // namespace sie
