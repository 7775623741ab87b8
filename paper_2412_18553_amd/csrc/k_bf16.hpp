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
#include "shapes.hpp"

namespace sie {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));


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
// the shared operand likewise with sh, sh_x.  `neg`: the term carries the
// minus of the occupied sums (the build flips the sign bits of its A
// operand); nG = groups of K; a_is_bl: the per-block operand is the MFMA's A
// side (rows), else its B side (cols).
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
// roles as make_wterm (k_fp64.hpp); row strides are those of the split copies.
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

// ---------------------------------------------------------------------------
// Split build.  A work-group computes, for one unit, one layout and one
// block, the six terms over a tile of 16 TRW rows x 64 TCW cols; its four
// waves sit side by side along the cols, wave w owning cols
// 16 TCW w .. 16 TCW (w + 1) - 1 of the tile.  Each term is
//   tile[row][col] += sum_K A[row][K] * B[col][K]
// with A and B two row-major split copies (one of them the per-block
// operand).  The A rows of a K chunk are read by all four waves, so they are
// staged through LDS (double-buffered, one barrier per chunk); each wave's B
// cols are its own and go straight from memory into registers, one chunk
// ahead.  Per chunk a wave issues 3 TRW TCW MFMAs for 2 TRW LDS reads and
// 2 TCW loads of 16 bytes per lane.
// ---------------------------------------------------------------------------

// One term's operands for a work-group: wave-uniform bases at row 0 / col 0
// of the tile and K group 0, row strides in bytes, K chunks, and the sign
// bits xor'ed into A (the minus of the occupied sums).
struct SOp {
  const char* a;
  const char* b;
  uint32_t sa, sb;
  int nch;
  uint32_t flip;
};

__device__ __forceinline__ SOp split_op(bool l2, int q, const FragDesc& f, int i, int j, int k,
                                        int blk, int row0, int col0) {
  const TermS t = make_term_split(l2, q, f, i, j, k, blk, row0, col0);
  SOp o;
  const char* bl = reinterpret_cast<const char*>(t.bl);
  const char* sh = reinterpret_cast<const char*>(t.sh);
  const uint32_t sbl = uint32_t(t.bl_x) * 32u, ssh = uint32_t(t.sh_x) * 32u;
  o.a = t.a_is_bl ? bl : sh;
  o.sa = t.a_is_bl ? sbl : ssh;
  o.b = t.a_is_bl ? sh : bl;
  o.sb = t.a_is_bl ? ssh : sbl;
  o.nch = t.nG / (kKs / 8);
  o.flip = t.neg ? 0x80008000u : 0u;
  return o;
}

__device__ __forceinline__ u4v ld_u4(const char* base, uint32_t off) {
  return *(const SIE_GLOBAL u4v*)(gptr(base) + off);
}

// Lane offsets of one term: A staging slots and this lane's B cols.
template <int NA, int TCW>
struct SLane {
  uint32_t a[NA];
  uint32_t b[TCW];
};

template <int TRW, int TCW, int NA>
__device__ __forceinline__ void split_lane(const SOp& o, int tid, int wave, int r, int g,
                                           int xa_max, int xb_max, SLane<NA, TCW>& L) {
  constexpr int R = 16 * TRW;
#pragma unroll
  for (int m = 0; m < NA; ++m) {
    int u = tid + 256 * m;
    u = u < 4 * R ? u : 4 * R - 1;
    const int x = min(u >> 2, xa_max);
    L.a[m] = uint32_t(x) * o.sa + uint32_t(u & 3) * 32u;
  }
#pragma unroll
  for (int ct = 0; ct < TCW; ++ct) {
    const int x = min(wave * 16 * TCW + 16 * ct + r, xb_max);
    L.b[ct] = uint32_t(x) * o.sb + uint32_t(g) * 32u;
  }
}

template <int NA, int TCW>
struct SRegs {
  u4v ah[NA], al[NA];     // A staging (hi, lo) for the LDS
  u4v bh[TCW], bl[TCW];   // B fragments (hi, lo)
};

template <int NA, int TCW>
__device__ __forceinline__ void split_load(const SOp& o, int c, const SLane<NA, TCW>& L,
                                           SRegs<NA, TCW>& x) {
  const char* a = o.a + c * 128;
  const char* b = o.b + c * 128;
#pragma unroll
  for (int m = 0; m < NA; ++m) {
    x.ah[m] = ld_u4(a, L.a[m]);
    x.al[m] = ld_u4(a, L.a[m] + 16u);
  }
#pragma unroll
  for (int ct = 0; ct < TCW; ++ct) {
    x.bh[ct] = ld_u4(b, L.b[ct]);
    x.bl[ct] = ld_u4(b, L.b[ct] + 16u);
  }
}

// LDS rows of K group g are stored xor-swizzled, row ^ lds_swz(g) (a
// permutation inside each aligned block of 16 rows): the four group planes
// lie a multiple of 256 bytes apart, so without it the staging stores of
// the four lanes that write one row (one lane per group) meet in the same
// banks.  With it every 8 (and every 16) consecutive lanes of a store reach
// distinct 16-byte bank groups, and the MFMA reads (16 lanes of one group,
// 16 consecutive rows) stay conflict-free.
__device__ __forceinline__ int lds_swz(int g) { return (0xAC60 >> (4 * g)) & 15; }

// LDS chunk: [K group (4)][hi, lo][row] of u4v.
template <int R, int NA, int TCW>
__device__ __forceinline__ void split_stage(const SRegs<NA, TCW>& x, uint32_t flip, int tid,
                                            u4v (*buf)[2][R]) {
#pragma unroll
  for (int m = 0; m < NA; ++m) {
    const int u = tid + 256 * m;
    if (u < 4 * R) {
      const int row = (u >> 2) ^ lds_swz(u & 3);
      buf[u & 3][0][row] = x.ah[m] ^ flip;
      buf[u & 3][1][row] = x.al[m] ^ flip;
    }
  }
}

// The three products of every tile, ordered so that MFMAs into one
// accumulator are TCW apart.
template <int TRW, int TCW, int NX>
__device__ __forceinline__ void split_mma(const u4v (*buf)[2][NX], int g, int r, int ra,
                                          const u4v (&bh)[TCW], const u4v (&bl)[TCW],
                                          f4 (&acc)[TRW][TCW]) {
#pragma unroll
  for (int rt = 0; rt < TRW; ++rt) {
    const u4v ah = buf[g][0][ra + 16 * rt + r], al = buf[g][1][ra + 16 * rt + r];
#pragma unroll
    for (int ct = 0; ct < TCW; ++ct) acc[rt][ct] = mfma_bf16(al, bh[ct], acc[rt][ct]);
#pragma unroll
    for (int ct = 0; ct < TCW; ++ct) acc[rt][ct] = mfma_bf16(ah, bl[ct], acc[rt][ct]);
#pragma unroll
    for (int ct = 0; ct < TCW; ++ct) acc[rt][ct] = mfma_bf16(ah, bh[ct], acc[rt][ct]);
  }
}

#ifndef SIE_BF16_DROW
// Result layout of the f32 16x16x32 bf16 MFMA: element v of lane (g, r) is
// D row SIE_BF16_DROW(v, g), col r.
#define SIE_BF16_DROW(v, g) (4 * (g) + (v))
#endif

// Split-precision partial cubes (float32): grid = the items' tiles, one
// layout (pair units) or two per unit, split_tiles(n_v, shape) per layout.
// Two work-groups per CU (at most 256 registers a lane): while one waits at
// its barrier or on its loads, the other keeps the matrix cores busy.
template <int TRW, int TCW>
__global__ __launch_bounds__(256, 2) void k_build_w_bf16x3(const FragDesc* __restrict__ descs,
                                                           const Item* __restrict__ items,
                                                           int n_items,
                                                           float* __restrict__ arena) {
  constexpr int R = 16 * TRW, C = 64 * TCW;
  constexpr int NA = (4 * R + 255) / 256;
  const int ri = find_item<true>(items, n_items, blockIdx.x);
  const int64_t start = ri ? items[ri - 1].blk_end : 0;
  const Item it = items[ri];
  const FragDesc fd = descs[it.frag];
  int i, j, k;
  bool one;
  if (!item_triple(it.unit, fd.no, fd.pair, i, j, k, one)) return;
  const int nv = fd.nv;
  const int nrt = (nv + R - 1) / R, nct = (nv + C - 1) / C;
  const int per = nv * nrt * nct;
  int t = xcd_tile(int(int64_t(blockIdx.x) - start), one ? per : 2 * per);
  const bool l2 = t >= per;
  if (l2) t -= per;
  const int blk = t / (nrt * nct);
  t -= blk * nrt * nct;
  const int tr = t / nct, tc = t - tr * nct;
  const int row0 = tr * R, col0 = tc * C;
  const int xa_max = min(R, nv - row0) - 1, xb_max = nv - 1 - col0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r = lane & 15, g = lane >> 4;

  __shared__ u4v lds[2][kKs / 8][2][R];

  f4 acc[TRW][TCW];
#pragma unroll
  for (int a = 0; a < TRW; ++a)
#pragma unroll
    for (int b = 0; b < TCW; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  int q = 0, c = 0;
  SOp cur = split_op(l2, 0, fd, i, j, k, blk, row0, col0);
  SLane<NA, TCW> L;
  split_lane<TRW, TCW, NA>(cur, tid, wave, r, g, xa_max, xb_max, L);
  SRegs<NA, TCW> x;
  split_load(cur, 0, L, x);
  u4v bh[TCW], bl[TCW];
  split_stage<R>(x, cur.flip, tid, lds[0]);
#pragma unroll
  for (int ct = 0; ct < TCW; ++ct) {
    bh[ct] = x.bh[ct];
    bl[ct] = x.bl[ct];
  }
  __syncthreads();
  int buf = 0;
  while (true) {
    int cn = c + 1;
    bool more = true;
    SOp nxt = cur;
    if (cn >= cur.nch) {
      if (q == 5) {
        more = false;
      } else {
        ++q;
        cn = 0;
        nxt = split_op(l2, q, fd, i, j, k, blk, row0, col0);
        split_lane<TRW, TCW, NA>(nxt, tid, wave, r, g, xa_max, xb_max, L);
      }
    }
    if (more) split_load(nxt, cn, L, x);
    split_mma<TRW, TCW>(lds[buf], g, r ^ lds_swz(g), 0, bh, bl, acc);
    if (!more) break;
    split_stage<R>(x, nxt.flip, tid, lds[buf ^ 1]);
#pragma unroll
    for (int ct = 0; ct < TCW; ++ct) {
      bh[ct] = x.bh[ct];
      bl[ct] = x.bl[ct];
    }
    __syncthreads();
    buf ^= 1;
    c = cn;
    cur = nxt;
  }

  float* __restrict__ out = arena + it.cube_off + (l2 ? fd.half : 0);
  const bool blocked = fd.blocked != 0;
#pragma unroll
  for (int ct = 0; ct < TCW; ++ct) {
    const int col = col0 + wave * 16 * TCW + 16 * ct + r;
#pragma unroll
    for (int rt = 0; rt < TRW; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + 16 * rt + SIE_BF16_DROW(v, g);
        if (row < nv && col < nv)
          gptr_w(out)[cube_at(blocked, nv, blk, row, col)] = acc[rt][ct][v];
      }
  }
}

// Split build with 2 x WC waves: 32 TRW rows x 16 TCW WC cols of one block,
// wave w at rows 16 TRW (w / WC) and cols 16 TCW (w % WC) of the tile.  Both
// operands of a K chunk are staged through LDS ([K group][hi, lo][A rows,
// then B cols]): each A row is read by WC waves and each B col by two, so a
// work-group reads (R + C) rows from memory per chunk for R x C outputs.
// WC = 4 (eight waves, 160 x 320 at TRW = TCW = 5) fills a CU with one
// work-group; WC = 2 (four waves, 160 x 160) needs half the LDS, so two
// work-groups share a CU and one's barrier waits overlap the other's work.
template <int TRW, int TCW, int WC>
__global__ __launch_bounds__(128 * WC, WC == 4 ? 1 : 2) void k_build_w_bf16x3_l(
    const FragDesc* __restrict__ descs, const Item* __restrict__ items, int n_items,
    float* __restrict__ arena) {
  constexpr int NT = 128 * WC;                   // threads
  constexpr int R = 32 * TRW, C = 16 * TCW * WC, X = R + C;
  constexpr int NU = (4 * X + NT - 1) / NT;      // staging units (32 bytes) per thread
  const int ri = find_item<true>(items, n_items, blockIdx.x);
  const int64_t start = ri ? items[ri - 1].blk_end : 0;
  const Item it = items[ri];
  const FragDesc fd = descs[it.frag];
  int i, j, k;
  bool one;
  if (!item_triple(it.unit, fd.no, fd.pair, i, j, k, one)) return;
  const int nv = fd.nv;
  const int nrt = (nv + R - 1) / R, nct = (nv + C - 1) / C;
  const int per = nv * nrt * nct;
  int t = xcd_tile(int(int64_t(blockIdx.x) - start), one ? per : 2 * per);
  const bool l2 = t >= per;
  if (l2) t -= per;
  const int blk = t / (nrt * nct);
  t -= blk * nrt * nct;
  const int tr = t / nct, tc = t - tr * nct;
  const int row0 = tr * R, col0 = tc * C;
  const int xa_max = min(R, nv - row0) - 1, xb_max = min(C, nv - col0) - 1;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r = lane & 15, g = lane >> 4;
  const int ra = (wave / WC) * 16 * TRW;          // this wave's first row in the A region
  const int cb = R + (wave % WC) * 16 * TCW;      // ... first col in the B region
  const int rx = r ^ lds_swz(g);                  // swizzled row within a 16-row block

  __shared__ u4v lds[2][kKs / 8][2][X];

  f4 acc[TRW][TCW];
#pragma unroll
  for (int a = 0; a < TRW; ++a)
#pragma unroll
    for (int b = 0; b < TCW; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  // staging unit u = tid + NT m: LDS row x = u / 4 (A row x, or B col x - R),
  // K group u % 4; lane addresses are rebuilt per term
  const char* src[NU];
  uint32_t flip_a = 0;
  auto lanes = [&](const SOp& o) {
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      int u = tid + NT * m;
      u = u < 4 * X ? u : 4 * X - 1;
      const int x = u >> 2;
      const uint32_t gq = uint32_t(u & 3) * 32u;
      src[m] = x < R ? o.a + (uint32_t(min(x, xa_max)) * o.sa + gq)
                     : o.b + (uint32_t(min(x - R, xb_max)) * o.sb + gq);
    }
    flip_a = o.flip;
  };
  u4v sh[NU], sl[NU];
  auto load = [&](int c) {
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const SIE_GLOBAL u4v* p = (const SIE_GLOBAL u4v*)(gptr(src[m] + c * 128));
      sh[m] = p[0];
      sl[m] = p[1];
    }
  };
  auto stage = [&](int b) {
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int u = tid + NT * m;
      if (u < 4 * X) {
        const uint32_t f = (u >> 2) < R ? flip_a : 0u;
        const int row = (u >> 2) ^ lds_swz(u & 3);
        lds[b][u & 3][0][row] = sh[m] ^ f;
        lds[b][u & 3][1][row] = sl[m] ^ f;
      }
    }
  };

  int q = 0, c = 0;
  SOp cur = split_op(l2, 0, fd, i, j, k, blk, row0, col0);
  lanes(cur);
  load(0);
  stage(0);
  __syncthreads();
  int buf = 0;
  while (true) {
    int cn = c + 1;
    bool more = true;
    if (cn >= cur.nch) {
      if (q == 5) {
        more = false;
      } else {
        ++q;
        cn = 0;
        cur = split_op(l2, q, fd, i, j, k, blk, row0, col0);
        lanes(cur);
      }
    }
    if (more) load(cn);
    {
      u4v bh[TCW], bl[TCW];
#pragma unroll
      for (int ct = 0; ct < TCW; ++ct) {
        bh[ct] = lds[buf][g][0][cb + 16 * ct + rx];
        bl[ct] = lds[buf][g][1][cb + 16 * ct + rx];
      }
      split_mma<TRW, TCW>(lds[buf], g, rx, ra, bh, bl, acc);
    }
    if (!more) break;
    stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    c = cn;
  }

  float* __restrict__ out = arena + it.cube_off + (l2 ? fd.half : 0);
  const bool blocked = fd.blocked != 0;
#pragma unroll
  for (int ct = 0; ct < TCW; ++ct) {
    const int col = col0 + (wave % WC) * 16 * TCW + 16 * ct + r;
#pragma unroll
    for (int rt = 0; rt < TRW; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + ra + 16 * rt + SIE_BF16_DROW(v, g);
        if (row < nv && col < nv)
          gptr_w(out)[cube_at(blocked, nv, blk, row, col)] = acc[rt][ct][v];
      }
  }
}

}  // namespace sie
