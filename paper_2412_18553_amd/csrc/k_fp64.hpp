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
// i.e. 6 contractions over d (K = n_v) and 6 over l (K = n_occ).  The build
// kernel evaluates them for one 16 x 16 x 16 tile of (a, b, c) with two
// waves: each wave owns a register tile in one of two MFMA layouts
//   L1: block index a, MFMA rows b, MFMA cols c
//   L2: block index b, MFMA rows a, MFMA cols c
// (a term can be evaluated as a 16x16xK matrix product only in a layout whose
// block index is one of the indices its (ov|vv)-side operand carries).  The L2
// tile is passed through LDS, added to the L1 tile and written to the
// workspace cube.  The epilogue kernel then reads the cube by symmetric
// orbits of 8 x 8 x 8 virtual blocks, so that every permuted element R' needs
// is in LDS, forms Vt and D on the fly and reduces in a fixed order.
#pragma once

#include "device_common.hpp"

namespace sie {

struct FragDev {
  const double* t1;     // [no][nv]
  const double* t2;     // [no][no][nv][nv]
  const double* ovvv;   // [no][nv][nv][nv]
  const double* ooov;   // [no][no][no][nv]
  const double* ovov;   // [no][nv][no][nv]
  const double* eps;    // [no + nv]: eps_occ then eps_vir (workspace copy)
  int no, nv;
};

constexpr int kTile = 16;     // virtual tile edge of the build kernel
constexpr int kOrb = 8;       // virtual block edge of the epilogue orbits

#ifndef SIE_BUILD_BLOCKS_PER_CU
#define SIE_BUILD_BLOCKS_PER_CU 2   // occupancy target of the build kernel
#endif

// One contraction term of the build kernel for one wave:
//   acc[beta] += sum_{k < nK} A_beta[row][k] * B_beta[k][col],  beta < kBlk,
// where one operand ("per-block") depends on the block index beta and the
// other ("shared") does not.  For the lane's row (A) or column (B):
//   per-block element (beta, k) = bl[beta * bstride + k * bl_k]
//   shared element k            = scale * sh[k * sh_k]
// K runs in chunks of kChunk = 8: in chunk c, k-step s (0, 1) of lane group g
// covers k = 8 c + 2 g + s, so a lane reads two consecutive k per row.
// Rows of lanes outside the virtual range, and blocks past the range, are
// clamped to valid rows: they only feed output entries that are never
// stored.  K past nK is zeroed on the shared operand.
constexpr int kChunk = 8;
constexpr int kBlk = 8;       // blocks per wave (two waves per layout)

struct Term {
  const double* bl;
  const double* sh;
  int64_t bstride, bl_k, sh_k;
  int nK;
  double scale;
};

struct Chunk {
  double bl[kBlk][2];
  double sh[2];
};

template <bool VEC>
__device__ __forceinline__ void load_chunk(const Term& t, int c, int last, int g, Chunk& x) {
  const int k0 = kChunk * c + 2 * g;
  if (VEC && kChunk * c + kChunk <= t.nK) {
    // contiguous 16-byte aligned rows (even row length, aligned bases)
    const double2 s0 = *reinterpret_cast<const double2*>(t.sh + k0);
    x.sh[0] = s0.x;
    x.sh[1] = s0.y;
#pragma unroll
    for (int beta = 0; beta < kBlk; ++beta) {
      const double2 u = *reinterpret_cast<const double2*>(
          t.bl + (int64_t)(beta < last ? beta : last) * t.bstride + k0);
      x.bl[beta][0] = u.x;
      x.bl[beta][1] = u.y;
    }
  } else {
    int kc[2];
    double m[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int k = k0 + s;
      kc[s] = k < t.nK ? k : t.nK - 1;
      m[s] = k < t.nK ? t.scale : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) x.sh[s] = m[s] * t.sh[(int64_t)kc[s] * t.sh_k];
#pragma unroll
    for (int beta = 0; beta < kBlk; ++beta) {
      const double* p = t.bl + (int64_t)(beta < last ? beta : last) * t.bstride;
#pragma unroll
      for (int s = 0; s < 2; ++s) x.bl[beta][s] = p[(int64_t)kc[s] * t.bl_k];
    }
  }
}

template <bool A_IS_BL>
__device__ __forceinline__ void mma_chunk(const Chunk& x, d4 (&acc)[kBlk]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int beta = 0; beta < kBlk; ++beta)
      acc[beta] = A_IS_BL ? mfma16x16x4(x.bl[beta][s], x.sh[s], acc[beta])
                          : mfma16x16x4(x.sh[s], x.bl[beta][s], acc[beta]);
}

// One term as a three-stage register pipeline: the loads of chunks c+1 and
// c+2 are in flight while the 8 x 2 MFMAs of chunk c run.  Loads of chunks
// past the end read clamped, zero-masked data and are never consumed.
// `last` is the last block index (relative to this wave's first block) that
// lies inside the virtual range.
template <bool A_IS_BL, bool VEC>
__device__ __forceinline__ void run_term(const Term& t, int last, int g, d4 (&acc)[kBlk]) {
  const int nch = (t.nK + kChunk - 1) / kChunk;
  Chunk b0, b1, b2;
  load_chunk<VEC>(t, 0, last, g, b0);
  load_chunk<VEC>(t, 1, last, g, b1);
  for (int c = 0;; c += 3) {
    load_chunk<VEC>(t, c + 2, last, g, b2);
    mma_chunk<A_IS_BL>(b0, acc);
    if (c + 1 >= nch) break;
    load_chunk<VEC>(t, c + 3, last, g, b0);
    mma_chunk<A_IS_BL>(b1, acc);
    if (c + 2 >= nch) break;
    load_chunk<VEC>(t, c + 4, last, g, b1);
    mma_chunk<A_IS_BL>(b2, acc);
    if (c + 3 >= nch) break;
  }
}

// Wt for one 16^3 virtual tile (a0.., b0.., c0..) of one unit (i, j, k) is
// the sum of the six permuted copies (the P operator) of
//   X^{abc}_{ijk} = sum_d (ia|bd) t_kj^cd - sum_l (ia|jl) t_lk^bc,
// each split into its d-sum (K = n_v) and its l-sum (K = n_occ); (ia|jl) is
// read as ooov[j][l][i][a] and t_ij^ab as t2[i][j][a][b] or its twin
// t2[j][i][b][a].  Twelve terms, six per layout:
//   L2 (block b, rows a, cols c): X^{bca}_{jki}, X^{cba}_{kji}, X^{bac}_{jik}
//       d-sums and X^{abc}_{ijk}, X^{acb}_{ikj}, X^{cab}_{kij} l-sums;
//   L1 (block a, rows b, cols c): X^{abc}_{ijk}, X^{acb}_{ikj}, X^{cab}_{kij}
//       d-sums and X^{bca}_{jki}, X^{cba}_{kji}, X^{bac}_{jik} l-sums.
// A wave owns blocks blk0 .. blk0 + 7 of its layout's block index.
template <bool VEC>
__device__ __forceinline__ void build_tile(const double* __restrict__ t2,
                                           const double* __restrict__ ovvv,
                                           const double* __restrict__ ooov, int i, int j, int k,
                                           int no_, int nv_, int a0, int b0, int c0, bool l1,
                                           int blk0, int r, int g, d4 (&acc)[kBlk]) {
  const int64_t nv = nv_, no = no_, nv2 = nv * nv, nonv = no * nv;
  const int64_t arc = min(a0 + r, nv_ - 1), brc = min(b0 + r, nv_ - 1),
                crc = min(c0 + r, nv_ - 1);
  Term t;
  if (!l1) {
    const int bb = b0 + blk0;                     // first block (b) of this wave
    const int last = min(kBlk, nv_ - bb) - 1;
    // X^{bca}_{jki}: sum_d t2[i][k][a][d] * ovvv[j][b][c][d]
    t = Term{ovvv + ((j * nv + bb) * nv + crc) * nv, t2 + ((i * no + k) * nv + arc) * nv,
             nv2, 1, 1, nv_, 1.0};
    run_term<false, VEC>(t, last, g, acc);
    // X^{cba}_{kji}: sum_d t2[i][j][a][d] * ovvv[k][c][b][d]
    t = Term{ovvv + ((k * nv + crc) * nv + bb) * nv, t2 + ((i * no + j) * nv + arc) * nv,
             nv, 1, 1, nv_, 1.0};
    run_term<false, VEC>(t, last, g, acc);
    // X^{bac}_{jik}: sum_d ovvv[j][b][a][d] * t2[k][i][c][d]
    t = Term{ovvv + ((j * nv + bb) * nv + arc) * nv, t2 + ((k * no + i) * nv + crc) * nv,
             nv2, 1, 1, nv_, 1.0};
    run_term<true, VEC>(t, last, g, acc);
    // X^{abc}_{ijk}: -sum_l ooov[j][l][i][a] * t2[l][k][b][c]
    t = Term{t2 + (k * nv + bb) * nv + crc, ooov + (j * no * no + i) * nv + arc,
             nv, nonv * nv, nonv, no_, -1.0};
    run_term<false, false>(t, last, g, acc);
    // X^{acb}_{ikj}: -sum_l ooov[k][l][i][a] * t2[j][l][b][c]
    t = Term{t2 + (j * no * nv + bb) * nv + crc, ooov + (k * no * no + i) * nv + arc,
             nv, nv2, nonv, no_, -1.0};
    run_term<false, false>(t, last, g, acc);
    // X^{cab}_{kij}: -sum_l t2[l][j][a][b] * ooov[i][l][k][c]
    t = Term{t2 + (j * nv + arc) * nv + bb, ooov + (i * no * no + k) * nv + crc,
             1, nonv * nv, nonv, no_, -1.0};
    run_term<true, false>(t, last, g, acc);
  } else {
    const int aa = a0 + blk0;                     // first block (a) of this wave
    const int last = min(kBlk, nv_ - aa) - 1;
    // X^{abc}_{ijk}: sum_d ovvv[i][a][b][d] * t2[k][j][c][d]
    t = Term{ovvv + ((i * nv + aa) * nv + brc) * nv, t2 + ((k * no + j) * nv + crc) * nv,
             nv2, 1, 1, nv_, 1.0};
    run_term<true, VEC>(t, last, g, acc);
    // X^{acb}_{ikj}: sum_d t2[j][k][b][d] * ovvv[i][a][c][d]
    t = Term{ovvv + ((i * nv + aa) * nv + crc) * nv, t2 + ((j * no + k) * nv + brc) * nv,
             nv2, 1, 1, nv_, 1.0};
    run_term<false, VEC>(t, last, g, acc);
    // X^{cab}_{kij}: sum_d t2[j][i][b][d] * ovvv[k][c][a][d]
    t = Term{ovvv + ((k * nv + crc) * nv + aa) * nv, t2 + ((j * no + i) * nv + brc) * nv,
             nv, 1, 1, nv_, 1.0};
    run_term<false, VEC>(t, last, g, acc);
    // X^{bca}_{jki}: -sum_l ooov[k][l][j][b] * t2[i][l][a][c]
    t = Term{t2 + (i * no * nv + aa) * nv + crc, ooov + (k * no * no + j) * nv + brc,
             nv, nv2, nonv, no_, -1.0};
    run_term<false, false>(t, last, g, acc);
    // X^{cba}_{kji}: -sum_l t2[i][l][a][b] * ooov[j][l][k][c]
    t = Term{t2 + (i * no * nv + aa) * nv + brc, ooov + (j * no * no + k) * nv + crc,
             nv, nv2, nonv, no_, -1.0};
    run_term<true, false>(t, last, g, acc);
    // X^{bac}_{jik}: -sum_l ooov[i][l][j][b] * t2[l][k][a][c]
    t = Term{t2 + (k * nv + aa) * nv + crc, ooov + (i * no * no + j) * nv + brc,
             nv, nonv * nv, nonv, no_, -1.0};
    run_term<false, false>(t, last, g, acc);
  }
}

// Map a linear block index to a tile so that the blocks the hardware places
// on one XCD (block index mod 8) cover a contiguous range of tiles and share
// their operand rows in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd;
  const int xcd = bid % kXcd, local = bid / kXcd;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Wt for one 16^3 virtual tile of one unit, written to the unit's cube
// cube[a][b][c] (n_v^3 doubles, row-major).  Grid: x = tile (ta, tb, tc),
// y = unit within the launch.  Block: 256 threads; waves 0-1 build layout
// L2 (blocks b 0-7 / 8-15), waves 2-3 layout L1 (blocks a 0-7 / 8-15).  The
// L2 half goes through LDS and is added by the L1 waves, which store the
// tile.  VEC: n_v is even and every input base is 16-byte aligned, so
// d-rows can be read 16 bytes at a time.
template <bool VEC>
__global__ __launch_bounds__(256, SIE_BUILD_BLOCKS_PER_CU) void k_build_w_f64(FragDev f, int64_t u0,
                                                        int64_t n_units,
                                                        double* __restrict__ cube,
                                                        int64_t cube_stride) {
  const int64_t u = u0 + blockIdx.y;
  if (u >= n_units) return;
  int i, j, k;
  decode_sorted_triple(u, f.no, i, j, k);
  if (i == k) return;
  const int nv = f.nv;
  const int nbk = (nv + kTile - 1) / kTile;
  int t = xcd_tile(blockIdx.x, nbk * nbk * nbk);
  const int ta = t / (nbk * nbk);
  t -= ta * nbk * nbk;
  const int tb = t / nbk;
  const int tc = t - tb * nbk;
  const int a0 = ta * kTile, b0 = tb * kTile, c0 = tc * kTile;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const bool l1 = wave >= 2;
  const int blk0 = (wave & 1) * kBlk;

  __shared__ double xbuf[kTile * kTile * kTile];

  d4 acc[kBlk];
#pragma unroll
  for (int q = 0; q < kBlk; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};

  build_tile<VEC>(f.t2, f.ovvv, f.ooov, i, j, k, f.no, nv, a0, b0, c0, l1, blk0, r, g, acc);

  if (!l1) {
    // element v of lane (g, r) in block q holds Wt[a0 + 4v + g][b0 + blk0 + q][c0 + r]
#pragma unroll
    for (int q = 0; q < kBlk; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        xbuf[((blk0 + q) * kTile + 4 * v + g) * kTile + r] = acc[q][v];
  }
  __syncthreads();
  if (l1) {
    // element v of lane (g, r) in block q holds Wt[a0 + blk0 + q][b0 + 4v + g][c0 + r]
    double* __restrict__ out = cube + (int64_t)blockIdx.y * cube_stride;
    const int c = c0 + r;
#pragma unroll
    for (int q = 0; q < kBlk; ++q) {
      const int a = a0 + blk0 + q;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int bl = 4 * v + g;
        const int b = b0 + bl;
        const double w = acc[q][v] + xbuf[(bl * kTile + blk0 + q) * kTile + r];
        if (a < nv && b < nv && c < nv) out[((int64_t)a * nv + b) * nv + c] = w;
      }
    }
  }
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

// Per-unit partial sums of Wt R'[Wt + Vt] / D over symmetric orbits of
// 8 x 8 x 8 virtual blocks (A >= B >= C and their permuted images).
// Grid: x = partial slot (strides over orbits), y = unit within the launch.
__global__ __launch_bounds__(256) void k_epilogue_f64(FragDev f, int64_t u0,
                                                      int64_t n_units,
                                                      const double* __restrict__ cube,
                                                      int64_t cube_stride,
                                                      double* __restrict__ partials,
                                                      int n_part) {
  const int64_t u = u0 + blockIdx.y;
  if (u >= n_units) return;
  int i, j, k;
  decode_sorted_triple(u, f.no, i, j, k);
  __shared__ double sw[6][kOrb * kOrb * kOrb];
  __shared__ double sz[6][kOrb * kOrb * kOrb];
  __shared__ double red[4];
  double* out = partials + u * n_part + blockIdx.x;
  if (i == k) {
    if (threadIdx.x == 0) *out = 0.0;
    return;
  }
  const int no = f.no, nv = f.nv;
  const int nb = (nv + kOrb - 1) / kOrb;
  const int64_t n_orb = tetra(nb);
  const double* __restrict__ ev = f.eps + no;
  const double eijk = f.eps[i] + f.eps[j] + f.eps[k];
  const double* __restrict__ w3 = cube + (int64_t)blockIdx.y * cube_stride;
  const double* __restrict__ ovov = f.ovov;
  const double* __restrict__ t1 = f.t1;
  const int64_t nonv = (int64_t)no * nv;
  const double* ov_ij = ovov + (int64_t)i * nv * nonv + (int64_t)j * nv;   // (ia|jb) = ov_ij[a*nonv + b]
  const double* ov_ik = ovov + (int64_t)i * nv * nonv + (int64_t)k * nv;
  const double* ov_jk = ovov + (int64_t)j * nv * nonv + (int64_t)k * nv;
  const double* t1i = t1 + (int64_t)i * nv;
  const double* t1j = t1 + (int64_t)j * nv;
  const double* t1k = t1 + (int64_t)k * nv;

  constexpr int E = kOrb * kOrb * kOrb;

  double acc = 0.0;
  for (int64_t o = blockIdx.x; o < n_orb; o += gridDim.x) {
    int t0, t1b, t2b;
    decode_sorted_triple(o, nb, t0, t1b, t2b);
    for (int idx = threadIdx.x; idx < 6 * E; idx += 256) {
      const int s = idx / E, e = idx - s * E;
      int p0, p1, p2;
      slot_perm(s, p0, p1, p2);
      const int a = kOrb * pick3(p0, t0, t1b, t2b) + (e >> 6);
      const int b = kOrb * pick3(p1, t0, t1b, t2b) + ((e >> 3) & 7);
      const int c = kOrb * pick3(p2, t0, t1b, t2b) + (e & 7);
      double w = 0.0, z = 0.0;
      if (a < nv && b < nv && c < nv) {
        w = w3[((int64_t)a * nv + b) * nv + c];
        const double vt = ov_ij[(int64_t)a * nonv + b] * t1k[c] +
                          ov_ik[(int64_t)a * nonv + c] * t1j[b] +
                          ov_jk[(int64_t)b * nonv + c] * t1i[a];
        z = w + vt;
      }
      sw[s][e] = w;
      sz[s][e] = z;
    }
    __syncthreads();
    // a slot whose block triple repeats an earlier slot's is not summed twice
    unsigned primary = 0;
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
    for (int idx = threadIdx.x; idx < 6 * E; idx += 256) {
      const int s = idx / E, e = idx - s * E;
      if (!((primary >> s) & 1u)) continue;
      int p0, p1, p2;
      slot_perm(s, p0, p1, p2);
      const int x = e >> 6, y = (e >> 3) & 7, zz = e & 7;
      const int a = kOrb * pick3(p0, t0, t1b, t2b) + x;
      const int b = kOrb * pick3(p1, t0, t1b, t2b) + y;
      const int c = kOrb * pick3(p2, t0, t1b, t2b) + zz;
      if (a >= nv || b >= nv || c >= nv) continue;
      // Z at the five permuted virtual triples, found in the slot holding
      // the permuted block triple at the permuted in-block offsets
      const double zabc = sz[s][e];
      const double zcab = sz[orbit_slot(p2, p0, p1)][(zz << 6) | (x << 3) | y];
      const double zbca = sz[orbit_slot(p1, p2, p0)][(y << 6) | (zz << 3) | x];
      const double zcba = sz[orbit_slot(p2, p1, p0)][(zz << 6) | (y << 3) | x];
      const double zacb = sz[orbit_slot(p0, p2, p1)][(x << 6) | (zz << 3) | y];
      const double zbac = sz[orbit_slot(p1, p0, p2)][(y << 6) | (x << 3) | zz];
      const double rz = 4.0 * zabc + zcab + zbca - 2.0 * (zcba + zacb + zbac);
      const double d = eijk - ev[a] - ev[b] - ev[c];
      acc += sw[s][e] * rz / d;
    }
    __syncthreads();
  }
  const double s = block_sum_256(acc, red);
  if (threadIdx.x == 0) *out = s;
}

}  // namespace sie
