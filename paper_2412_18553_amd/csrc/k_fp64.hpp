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

// acc[beta] += sum_{d < nv} A_beta[row][d] * B_beta[d][col], beta < nblk.
// One operand is per block (row pointer + beta * blk_stride), the other is
// shared by all blocks.  `pa`/`pb` point at the lane's contiguous d-row (the
// row of A for lane % 16, the column of B for lane % 16); a_ok/b_ok mark lanes
// whose row/column lies inside the virtual range (their pointer is clamped to
// a valid row).  In each 16-wide chunk, k-step s of lane group g reads
// d = d0 + 4 g + s, so each lane reads four consecutive doubles per row.
template <bool A_PER_BLOCK>
__device__ __forceinline__ void vv_term(d4 (&acc)[kTile], int nblk, int nv, int g,
                                        const double* __restrict__ pa, bool a_ok,
                                        const double* __restrict__ pb, bool b_ok,
                                        int64_t blk_stride) {
  const double* psh = A_PER_BLOCK ? pb : pa;
  const double* pbl = A_PER_BLOCK ? pa : pb;
  const bool sh_ok = A_PER_BLOCK ? b_ok : a_ok;
  const bool bl_ok = A_PER_BLOCK ? a_ok : b_ok;
  const int last = nblk - 1;
  for (int d0 = 0; d0 < nv; d0 += 16) {
    const int dl = d0 + 4 * g;
    double sh[4];
    bool dok[4];
    int dc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      dok[s] = dl + s < nv;
      dc[s] = dok[s] ? dl + s : nv - 1;
      const double v = psh[dc[s]];
      sh[s] = (sh_ok && dok[s]) ? v : 0.0;
    }
#pragma unroll
    for (int beta = 0; beta < kTile; ++beta) {
      const double* p = pbl + (int64_t)(beta < last ? beta : last) * blk_stride;
      double x[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double v = p[dc[s]];
        x[s] = (bl_ok && dok[s]) ? v : 0.0;
      }
      if (beta < nblk) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
          acc[beta] = A_PER_BLOCK ? mfma16x16x4(x[s], sh[s], acc[beta])
                                  : mfma16x16x4(sh[s], x[s], acc[beta]);
      }
    }
  }
}

// acc[beta] += sum_{l < no} A_beta[row][l] * B_beta[l][col], beta < nblk.
// Element (lane, l, beta) of A is pa[l * a_ls + beta * a_bs] (B likewise);
// `a_scale` multiplies A (it carries the minus sign of the occupied term).
__device__ __forceinline__ void oo_term(d4 (&acc)[kTile], int nblk, int no, int g,
                                        const double* __restrict__ pa, bool a_ok,
                                        int64_t a_ls, int64_t a_bs, double a_scale,
                                        const double* __restrict__ pb, bool b_ok,
                                        int64_t b_ls, int64_t b_bs) {
  const int last = nblk - 1;
  for (int l0 = 0; l0 < no; l0 += 4) {
    const int l = l0 + g;
    const bool lok = l < no;
    const int lc = lok ? l : no - 1;
#pragma unroll
    for (int beta = 0; beta < kTile; ++beta) {
      const int bc = beta < last ? beta : last;
      const double va = pa[(int64_t)lc * a_ls + (int64_t)bc * a_bs];
      const double vb = pb[(int64_t)lc * b_ls + (int64_t)bc * b_bs];
      const double xa = (a_ok && lok) ? a_scale * va : 0.0;
      const double xb = (b_ok && lok) ? vb : 0.0;
      if (beta < nblk) acc[beta] = mfma16x16x4(xa, xb, acc[beta]);
    }
  }
}

// Wt for one 16^3 virtual tile of one unit, written to the unit's cube
// cube[a][b][c] (n_v^3 doubles, row-major).  Grid: x = tile (ta, tb, tc),
// y = unit within the launch.  Block: 128 threads (wave 0: layout L2,
// wave 1: layout L1).
__global__ __launch_bounds__(128) void k_build_w_f64(FragDev f, int64_t u0,
                                                     int64_t n_units,
                                                     double* __restrict__ cube,
                                                     int64_t cube_stride) {
  const int64_t u = u0 + blockIdx.y;
  if (u >= n_units) return;
  int i, j, k;
  decode_sorted_triple(u, f.no, i, j, k);
  if (i == k) return;
  const int no = f.no, nv = f.nv;
  const int nbk = (nv + kTile - 1) / kTile;
  int t = blockIdx.x;
  const int ta = t / (nbk * nbk);
  t -= ta * nbk * nbk;
  const int tb = t / nbk;
  const int tc = t - tb * nbk;
  const int a0 = ta * kTile, b0 = tb * kTile, c0 = tc * kTile;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t nv2 = (int64_t)nv * nv;
  const int64_t nonv = (int64_t)no * nv;

  __shared__ double xbuf[kTile * kTile * kTile];

  d4 acc[kTile];
#pragma unroll
  for (int q = 0; q < kTile; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};

  const double* __restrict__ t2 = f.t2;
  const double* __restrict__ ovvv = f.ovvv;
  const double* __restrict__ ooov = f.ooov;

  // lane row/column indices (clamped into range, flagged when outside)
  const int ar = a0 + r, br = b0 + r, cr = c0 + r;
  const bool a_ok = ar < nv, b_ok = br < nv, c_ok = cr < nv;
  const int arc = a_ok ? ar : nv - 1, brc = b_ok ? br : nv - 1, crc = c_ok ? cr : nv - 1;

  if (wave == 0) {
    // ---- layout L2: block b, rows a, cols c ----
    const int nblk = min(kTile, nv - b0);
    // T2 = X^{bca}_{jki}: sum_d t2[i][k][a][d] * ovvv[j][b][c][d]
    vv_term<false>(acc, nblk, nv, g,
                   t2 + (((int64_t)i * no + k) * nv + arc) * nv, a_ok,
                   ovvv + (((int64_t)j * nv + b0) * nv + crc) * nv, c_ok, nv2);
    // T5 = X^{cba}_{kji}: sum_d t2[i][j][a][d] * ovvv[k][c][b][d]
    vv_term<false>(acc, nblk, nv, g,
                   t2 + (((int64_t)i * no + j) * nv + arc) * nv, a_ok,
                   ovvv + (((int64_t)k * nv + crc) * nv + b0) * nv, c_ok, nv);
    // T6 = X^{bac}_{jik}: sum_d ovvv[j][b][a][d] * t2[k][i][c][d]
    vv_term<true>(acc, nblk, nv, g,
                  ovvv + (((int64_t)j * nv + b0) * nv + arc) * nv, a_ok,
                  t2 + (((int64_t)k * no + i) * nv + crc) * nv, c_ok, nv2);
    // O1 = X^{abc}_{ijk}: -sum_l ooov[j][l][i][a] * t2[l][k][b][c]
    oo_term(acc, nblk, no, g,
            ooov + ((int64_t)j * no * no + i) * nv + arc, a_ok, nonv, 0, -1.0,
            t2 + ((int64_t)k * nv + b0) * nv + crc, c_ok, nonv * nv, nv);
    // O4 = X^{acb}_{ikj}: -sum_l ooov[k][l][i][a] * t2[j][l][b][c]
    oo_term(acc, nblk, no, g,
            ooov + ((int64_t)k * no * no + i) * nv + arc, a_ok, nonv, 0, -1.0,
            t2 + ((int64_t)j * no * nv + b0) * nv + crc, c_ok, nv2, nv);
    // O3 = X^{cab}_{kij}: -sum_l t2[l][j][a][b] * ooov[i][l][k][c]
    oo_term(acc, nblk, no, g,
            t2 + ((int64_t)j * nv + arc) * nv + b0, a_ok, nonv * nv, 1, -1.0,
            ooov + ((int64_t)i * no * no + k) * nv + crc, c_ok, nonv, 0);
    // hand the tile to wave 1: xbuf[b][a][c]
#pragma unroll
    for (int q = 0; q < kTile; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        xbuf[(q * kTile + 4 * v + g) * kTile + r] = acc[q][v];
  } else {
    // ---- layout L1: block a, rows b, cols c ----
    const int nblk = min(kTile, nv - a0);
    // T1 = X^{abc}_{ijk}: sum_d ovvv[i][a][b][d] * t2[k][j][c][d]
    vv_term<true>(acc, nblk, nv, g,
                  ovvv + (((int64_t)i * nv + a0) * nv + brc) * nv, b_ok,
                  t2 + (((int64_t)k * no + j) * nv + crc) * nv, c_ok, nv2);
    // T4 = X^{acb}_{ikj}: sum_d t2[j][k][b][d] * ovvv[i][a][c][d]
    vv_term<false>(acc, nblk, nv, g,
                   t2 + (((int64_t)j * no + k) * nv + brc) * nv, b_ok,
                   ovvv + (((int64_t)i * nv + a0) * nv + crc) * nv, c_ok, nv2);
    // T3 = X^{cab}_{kij}: sum_d t2[j][i][b][d] * ovvv[k][c][a][d]
    vv_term<false>(acc, nblk, nv, g,
                   t2 + (((int64_t)j * no + i) * nv + brc) * nv, b_ok,
                   ovvv + (((int64_t)k * nv + crc) * nv + a0) * nv, c_ok, nv);
    // O2 = X^{bca}_{jki}: -sum_l ooov[k][l][j][b] * t2[i][l][a][c]
    oo_term(acc, nblk, no, g,
            ooov + ((int64_t)k * no * no + j) * nv + brc, b_ok, nonv, 0, -1.0,
            t2 + ((int64_t)i * no * nv + a0) * nv + crc, c_ok, nv2, nv);
    // O5 = X^{cba}_{kji}: -sum_l t2[i][l][a][b] * ooov[j][l][k][c]
    oo_term(acc, nblk, no, g,
            t2 + ((int64_t)i * no * nv + a0) * nv + brc, b_ok, nv2, nv, -1.0,
            ooov + ((int64_t)j * no * no + k) * nv + crc, c_ok, nonv, 0);
    // O6 = X^{bac}_{jik}: -sum_l ooov[i][l][j][b] * t2[l][k][a][c]
    oo_term(acc, nblk, no, g,
            ooov + ((int64_t)i * no * no + j) * nv + brc, b_ok, nonv, 0, -1.0,
            t2 + ((int64_t)k * nv + a0) * nv + crc, c_ok, nonv * nv, nv);
  }
  __syncthreads();
  if (wave == 1) {
    double* __restrict__ out = cube + (int64_t)blockIdx.y * cube_stride;
    const int c = c0 + r;
#pragma unroll
    for (int q = 0; q < kTile; ++q) {
      const int a = a0 + q;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int b = b0 + 4 * v + g;
        const double w = acc[q][v] + xbuf[(b - b0) * kTile * kTile + q * kTile + r];
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
