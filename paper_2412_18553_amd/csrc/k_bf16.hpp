// Split-precision (T) kernels for gfx950.
//
// Every float32 amplitude and integral that enters the W-tilde contractions
// is stored as two bfloat16 numbers, hi = bf16_rne(x) and lo = bf16_rne(x - hi)
// (x - hi is exact in float32).  Each product of the contractions is formed on
// the bf16 matrix cores as hi*hi + hi*lo + lo*hi (lo*lo dropped) with float32
// accumulation; D, V-tilde, R' and the energy sums stay in float64 in the
// epilogue.  The term structure is the float64 build's (see k_fp64.hpp).
//
// Operand copies (made once per evaluation, "split staging"): every copy has
// its contraction index K contiguous and padded with zeros to a multiple of
// kKs = 32, in groups of 8: [row][K/8][hi 8 | lo 8] (bfloat16 bit patterns).
//   vS  [o][v][v][Kv]   from ovvv (K = d)
//   tS  [o][o][v][Kv]   from t2   (K = d)
//   tT  [o][v][v][Ko]   tT[p][x][y][l] = t2[p][l][x][y]  (K = l)
//   oT  [o][o][v][Ko]   oT[x][y][v][l] = ooov[x][l][y][v] (K = l)
// Zero padding makes every K chunk full: no masking in the build kernel.
#pragma once

#include "k_fp64.hpp"

namespace sie {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kKs = 32;       // K per bf16 MFMA step (and per LDS chunk)

// D(16x16, f32) += A(16x32) * B(32x16) on the bf16 matrix cores.
__device__ __forceinline__ f4 mfma_bf16(const u4v& a, const u4v& b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// bf16 bit pattern nearest to a finite float (ties to even).
__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return b >> 16;
}

// Split copy of a float32 array viewed as rows (p, x, y) of a contraction
// index k: source element (p, x, y, k) = src[p*sp + x*sx + y*sy + k*sk],
// k < K; destination row r = (p*X + x)*Y + y holds Kpad/8 groups of
// [hi 8 | lo 8] bf16 (zeros for k >= K).  One thread per (row, group):
// kfast selects group-fastest thread order (contiguous k in the source) or
// y-fastest order (strided k, contiguous y in the source).
__global__ __launch_bounds__(256) void k_split_bf16(const float* __restrict__ src, int P, int X,
                                                    int Y, int64_t sp, int64_t sx, int64_t sy,
                                                    int64_t sk, int K, int Kpad, bool kfast,
                                                    u4v* __restrict__ dst) {
  const int64_t ng = Kpad / 8;
  const int64_t rows = (int64_t)P * X * Y;
  const int64_t total = rows * ng;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t row, grp;
    if (kfast) {
      grp = t % ng;
      row = t / ng;
    } else {
      const int64_t xy = (int64_t)X * Y;
      const int64_t y = t % Y;
      const int64_t rest = t / Y;            // = grp * (P * X) + p * X + x
      const int64_t px = rest % ((int64_t)P * X);
      grp = rest / ((int64_t)P * X);
      row = px * Y + y;
      (void)xy;
    }
    const int64_t y = row % Y;
    const int64_t px = row / Y;
    const int64_t x = px % X;
    const int64_t p = px / X;
    const float* s = src + p * sp + x * sx + y * sy;
    uint32_t hi[8], lo[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = int(grp) * 8 + e;
      const float v = k < K ? gptr(s)[(int64_t)k * sk] : 0.0f;
      const uint32_t h = bf16_rne_bits(v);
      hi[e] = h;
      lo[e] = bf16_rne_bits(v - __uint_as_float(h << 16));
    }
    u4v oh, ol;
    oh.x = hi[0] | (hi[1] << 16); oh.y = hi[2] | (hi[3] << 16);
    oh.z = hi[4] | (hi[5] << 16); oh.w = hi[6] | (hi[7] << 16);
    ol.x = lo[0] | (lo[1] << 16); ol.y = lo[2] | (lo[3] << 16);
    ol.z = lo[4] | (lo[5] << 16); ol.w = lo[6] | (lo[7] << 16);
    SIE_GLOBAL u4v* d = gptr_w(dst + (row * ng + grp) * 2);
    d[0] = oh;
    d[1] = ol;
  }
}

// One term of the split build: element (beta, x, group G) of the per-block
// operand is the u4v pair at bl + (beta*bl_b + x*bl_x + G) * 2 (hi, then lo);
// the shared operand likewise with sh, sh_x.  `neg` flips the sign of the
// shared operand (the minus of the occupied sums); nG = groups of K.
struct TermS {
  const u4v* bl;
  int64_t bl_b, bl_x;
  const u4v* sh;
  int64_t sh_x;
  int nG;
  bool neg;
  bool a_is_bl;
};

// Term q (0..5) of layout `l2`, in the same order and with the same operand
// roles as make_term (k_fp64.hpp); row strides are those of the split copies.
__device__ __forceinline__ TermS make_term_split(bool l2, int q, const FragDesc& f, int i,
                                                 int j, int k, int blk0, int row0, int col0) {
  const int64_t nv = f.nv, no = f.no;
  const int64_t gv = f.Kv / 8, go = f.Ko / 8;          // groups per row
  const int64_t rv = gv, ro = go;                      // row stride in groups
  TermS t;
  t.nG = int(gv);
  t.neg = false;
  // vS row (x, p, q) = (x*nv + p)*nv + q ; tS row (p, q, x) = (p*no + q)*nv + x
  // tT row (p, x, y) = (p*nv + x)*nv + y ; oT row (x, y, v) = (x*no + y)*nv + v
  if (!l2) {
    switch (q) {
      case 0:  // ovvv[i][a][b][d] * t2[k][j][c][d]
        t.bl = f.vS + ((i * nv + blk0) * nv + row0) * rv * 2; t.bl_b = nv * rv; t.bl_x = rv;
        t.sh = f.tS + ((k * no + j) * nv + col0) * rv * 2; t.sh_x = rv;
        t.a_is_bl = true; break;
      case 1:  // t2[j][k][b][d] * ovvv[i][a][c][d]
        t.sh = f.tS + ((j * no + k) * nv + row0) * rv * 2; t.sh_x = rv;
        t.bl = f.vS + ((i * nv + blk0) * nv + col0) * rv * 2; t.bl_b = nv * rv; t.bl_x = rv;
        t.a_is_bl = false; break;
      case 2:  // t2[j][i][b][d] * ovvv[k][c][a][d]
        t.sh = f.tS + ((j * no + i) * nv + row0) * rv * 2; t.sh_x = rv;
        t.bl = f.vS + ((k * nv + col0) * nv + blk0) * rv * 2; t.bl_b = rv; t.bl_x = nv * rv;
        t.a_is_bl = false; break;
      case 3:  // -ooov[k][l][j][b] * t2[i][l][a][c]:  oT[k][j][b][l], tT[i][a][c][l]
        t.sh = f.oT + ((k * no + j) * nv + row0) * ro * 2; t.sh_x = ro; t.neg = true;
        t.bl = f.tT + ((i * nv + blk0) * nv + col0) * ro * 2; t.bl_b = nv * ro; t.bl_x = ro;
        t.nG = int(go); t.a_is_bl = false; break;
      case 4:  // t2[i][l][a][b] * -ooov[j][l][k][c]:  tT[i][a][b][l], oT[j][k][c][l]
        t.bl = f.tT + ((i * nv + blk0) * nv + row0) * ro * 2; t.bl_b = nv * ro; t.bl_x = ro;
        t.sh = f.oT + ((j * no + k) * nv + col0) * ro * 2; t.sh_x = ro; t.neg = true;
        t.nG = int(go); t.a_is_bl = true; break;
      default:  // -ooov[i][l][j][b] * t2[l][k][a][c] (= t2[k][l][c][a]):  oT[i][j][b][l], tT[k][c][a][l]
        t.sh = f.oT + ((i * no + j) * nv + row0) * ro * 2; t.sh_x = ro; t.neg = true;
        t.bl = f.tT + ((k * nv + col0) * nv + blk0) * ro * 2; t.bl_b = ro; t.bl_x = nv * ro;
        t.nG = int(go); t.a_is_bl = false; break;
    }
  } else {
    switch (q) {
      case 0:  // t2[i][k][a][d] * ovvv[j][b][c][d]
        t.sh = f.tS + ((i * no + k) * nv + row0) * rv * 2; t.sh_x = rv;
        t.bl = f.vS + ((j * nv + blk0) * nv + col0) * rv * 2; t.bl_b = nv * rv; t.bl_x = rv;
        t.a_is_bl = false; break;
      case 1:  // t2[i][j][a][d] * ovvv[k][c][b][d]
        t.sh = f.tS + ((i * no + j) * nv + row0) * rv * 2; t.sh_x = rv;
        t.bl = f.vS + ((k * nv + col0) * nv + blk0) * rv * 2; t.bl_b = rv; t.bl_x = nv * rv;
        t.a_is_bl = false; break;
      case 2:  // ovvv[j][b][a][d] * t2[k][i][c][d]
        t.bl = f.vS + ((j * nv + blk0) * nv + row0) * rv * 2; t.bl_b = nv * rv; t.bl_x = rv;
        t.sh = f.tS + ((k * no + i) * nv + col0) * rv * 2; t.sh_x = rv;
        t.a_is_bl = true; break;
      case 3:  // -ooov[j][l][i][a] * t2[l][k][b][c] (= t2[k][l][c][b]):  oT[j][i][a][l], tT[k][c][b][l]
        t.sh = f.oT + ((j * no + i) * nv + row0) * ro * 2; t.sh_x = ro; t.neg = true;
        t.bl = f.tT + ((k * nv + col0) * nv + blk0) * ro * 2; t.bl_b = ro; t.bl_x = nv * ro;
        t.nG = int(go); t.a_is_bl = false; break;
      case 4:  // -ooov[k][l][i][a] * t2[j][l][b][c]:  oT[k][i][a][l], tT[j][b][c][l]
        t.sh = f.oT + ((k * no + i) * nv + row0) * ro * 2; t.sh_x = ro; t.neg = true;
        t.bl = f.tT + ((j * nv + blk0) * nv + col0) * ro * 2; t.bl_b = nv * ro; t.bl_x = ro;
        t.nG = int(go); t.a_is_bl = false; break;
      default:  // t2[l][j][a][b] (= t2[j][l][b][a]) * -ooov[i][l][k][c]:  tT[j][b][a][l], oT[i][k][c][l]
        t.bl = f.tT + ((j * nv + blk0) * nv + row0) * ro * 2; t.bl_b = nv * ro; t.bl_x = ro;
        t.sh = f.oT + ((i * no + k) * nv + col0) * ro * 2; t.sh_x = ro; t.neg = true;
        t.nG = int(go); t.a_is_bl = true; break;
    }
  }
  return t;
}

// Per-thread staging registers for one K chunk (kKs = 4 groups): per-block
// units kBB * kRows * 4 over kThreads threads, one shared unit at most.
constexpr int kBlUnitsS = (kBB * kRows * (kKs / 8) + kThreads - 1) / kThreads;

struct StageS {
  u4v blh[kBlUnitsS], bll[kBlUnitsS];
  u4v shh, shl;
};

__device__ __forceinline__ void stage_load_s(const TermS& t, int c, const TileDims& d, int tid,
                                             StageS& st) {
  const int Xb = t.a_is_bl ? kRows : kCols;
  const int Xs = t.a_is_bl ? kCols : kRows;
  const int xbmax = (t.a_is_bl ? d.nrow : d.ncol) - 1;
  const int xsmax = (t.a_is_bl ? d.ncol : d.nrow) - 1;
  const int nbl = kBB * Xb * 4;
  const int g0 = c * (kKs / 8);
  // every thread loads a valid (clamped) unit for every slot; only the stores
  // of slots past the operand's extent are skipped
#pragma unroll
  for (int m = 0; m < kBlUnitsS; ++m) {
    int u = tid + m * kThreads;
    u = u < nbl ? u : nbl - 1;
    const int gq = u & 3, rr = u >> 2;
    int beta = rr / Xb, x = rr - (rr / Xb) * Xb;
    beta = beta < d.nblk ? beta : d.nblk - 1;
    x = x < xbmax ? x : xbmax;
    const SIE_GLOBAL u4v* p =
        gptr(t.bl + ((int64_t)beta * t.bl_b + (int64_t)x * t.bl_x + g0 + gq) * 2);
    st.blh[m] = p[0];
    st.bll[m] = p[1];
  }
  int u = tid;
  const int nsh = Xs * 4;
  u = u < nsh ? u : nsh - 1;
  const int gq = u & 3;
  int x = u >> 2;
  x = x < xsmax ? x : xsmax;
  const SIE_GLOBAL u4v* p = gptr(t.sh + ((int64_t)x * t.sh_x + g0 + gq) * 2);
  // loaded values are left untouched until stage_store_s (after the chunk's
  // MFMAs), so the loads stay in flight across them
  st.shh = p[0];
  st.shl = p[1];
}

// LDS: [group in chunk (4)][hi, lo][row] of u4v (8 bf16).
__device__ __forceinline__ void stage_store_s(const TermS& t, int tid, const StageS& st,
                                              u4v (*buf)[2][kLdsRows]) {
  const int Xb = t.a_is_bl ? kRows : kCols;
  const int Xs = t.a_is_bl ? kCols : kRows;
  const int nbl = kBB * Xb * 4;
#pragma unroll
  for (int m = 0; m < kBlUnitsS; ++m) {
    const int u = tid + m * kThreads;
    if (u < nbl) {
      const int gq = u & 3, rr = u >> 2;
      buf[gq][0][rr] = st.blh[m];
      buf[gq][1][rr] = st.bll[m];
    }
  }
  const int u = tid;
  if (u < Xs * 4) {
    const int gq = u & 3, x = u >> 2;
    const uint32_t flip = t.neg ? 0x80008000u : 0u;   // sign of the occupied sums
    buf[gq][0][kShBase + x] = st.shh ^ flip;
    buf[gq][1][kShBase + x] = st.shl ^ flip;
  }
}

__device__ __forceinline__ void mma_chunk_s(bool a_is_bl, const u4v (*buf)[2][kLdsRows], int g,
                                            int rrow, int rcol, f4 (&acc)[kBB]) {
  // the three products of each block in turn over all blocks: consecutive
  // MFMAs never feed each other
  u4v vh[kBB], vl[kBB];
  if (a_is_bl) {
    const u4v sh = buf[g][0][kShBase + rcol], sl = buf[g][1][kShBase + rcol];
#pragma unroll
    for (int beta = 0; beta < kBB; ++beta) {
      vh[beta] = buf[g][0][beta * kRows + rrow];
      vl[beta] = buf[g][1][beta * kRows + rrow];
    }
#pragma unroll
    for (int beta = 0; beta < kBB; ++beta) acc[beta] = mfma_bf16(vl[beta], sh, acc[beta]);
#pragma unroll
    for (int beta = 0; beta < kBB; ++beta) acc[beta] = mfma_bf16(vh[beta], sl, acc[beta]);
#pragma unroll
    for (int beta = 0; beta < kBB; ++beta) acc[beta] = mfma_bf16(vh[beta], sh, acc[beta]);
  } else {
    const u4v sh = buf[g][0][kShBase + rrow], sl = buf[g][1][kShBase + rrow];
#pragma unroll
    for (int beta = 0; beta < kBB; ++beta) {
      vh[beta] = buf[g][0][beta * kCols + rcol];
      vl[beta] = buf[g][1][beta * kCols + rcol];
    }
#pragma unroll
    for (int beta = 0; beta < kBB; ++beta) acc[beta] = mfma_bf16(sl, vh[beta], acc[beta]);
#pragma unroll
    for (int beta = 0; beta < kBB; ++beta) acc[beta] = mfma_bf16(sh, vl[beta], acc[beta]);
#pragma unroll
    for (int beta = 0; beta < kBB; ++beta) acc[beta] = mfma_bf16(sh, vh[beta], acc[beta]);
  }
}

#ifndef SIE_BF16_DROW
// Result layout of the f32 16x16x32 bf16 MFMA: element v of lane (g, r) is
// D row SIE_BF16_DROW(v, g), col r.
#define SIE_BF16_DROW(v, g) (4 * (g) + (v))
#endif

// Split-precision partial cubes (float32) of one layout for one tile of one
// unit; same grid, tiles and term order as k_build_w_f64.
__global__ __launch_bounds__(kThreads, 1) void k_build_w_bf16x3(const FragDesc* __restrict__ descs,
                                                                const Item* __restrict__ items,
                                                                int n_items,
                                                                float* __restrict__ arena) {
  const int ri = find_item<true>(items, n_items, blockIdx.x);
  const int64_t start = ri ? items[ri - 1].blk_end : 0;
  const FragDesc fd = descs[items[ri].frag];
  int i, j, k;
  const bool one = unit_triple(items[ri].unit, fd.no, fd.pair, i, j, k);
  if (i == k) return;
  const BlockWork w = block_work(fd, items, ri, int64_t(blockIdx.x) - start, one);
  const int nv = fd.nv;
  const bool l2 = w.l2;
  const int blk0 = w.blk0, row0 = w.row0, col0 = w.col0;
  TileDims dims;
  dims.nblk = min(kBB, nv - blk0);
  dims.nrow = min(kRows, nv - row0);
  dims.ncol = min(kCols, nv - col0);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int rq = wave % (kRows / 16), ch = wave / (kRows / 16);
  const int rrow = rq * 16 + r, rcol = ch * 16 + r;

  __shared__ u4v lds[2][kKs / 8][2][kLdsRows];

  f4 acc[kBB];
#pragma unroll
  for (int q = 0; q < kBB; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};

  int q = 0, c = 0;
  TermS tcur = make_term_split(l2, 0, fd, i, j, k, blk0, row0, col0);
  StageS st;
  stage_load_s(tcur, 0, dims, tid, st);
  stage_store_s(tcur, tid, st, lds[0]);
  __syncthreads();
  int buf = 0;
  while (true) {
    int qn = q, cn = c + 1;
    TermS tn = tcur;
    bool more = true;
    if (cn * (kKs / 8) >= tcur.nG) {
      if (q == 5) {
        more = false;
      } else {
        qn = q + 1;
        cn = 0;
        tn = make_term_split(l2, qn, fd, i, j, k, blk0, row0, col0);
      }
    }
    if (more) stage_load_s(tn, cn, dims, tid, st);
    mma_chunk_s(tcur.a_is_bl, lds[buf], g, rrow, rcol, acc);
    if (!more) break;
    stage_store_s(tn, tid, st, lds[buf ^ 1]);
    __syncthreads();
    buf ^= 1;
    q = qn;
    c = cn;
    tcur = tn;
  }

  float* __restrict__ out = arena + w.it.cube_off + (l2 ? fd.half : 0);
  const int col = col0 + rcol;
#pragma unroll
  for (int beta = 0; beta < kBB; ++beta) {
    const int blk = blk0 + beta;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + rq * 16 + SIE_BF16_DROW(v, g);
      if (blk < nv && row < nv && col < nv)
        gptr_w(out)[((int64_t)blk * nv + row) * nv + col] = acc[beta][v];
    }
  }
}

}  // namespace sie
