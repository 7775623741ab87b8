// MP2 energy, amplitudes and 1-RDM blocks of a cluster from density-fitting
// factors, on the float64 matrix cores of gfx950.
//
// The paper's embedding workflow (SI section "Systematically Improvable
// Quantum Embedding Workflow") ranks bath natural orbitals by the MP2 1-RDM
// of a subspace and corrects the bath truncation with MP2 energies:
//   t_ij^ab  = -(ia|jb) / D_ij^ab,   D_ij^ab = e_a + e_b - e_i - e_j,
//   E        = sum_ijab t_ij^ab [2 (ia|jb) - (ib|ja)],
//   gamma_ab = 2 sum_ij sum_c t_ij^ac (2 t_ij^bc - t_ij^cb),
//   gamma_ij = 2 delta_ij - 2 sum_k sum_ab t_ik^ab (2 t_jk^ab - t_jk^ba),
// with (ia|jb) = sum_P L[i][a][P] L[j][b][P] (factors row-major, P fastest).
//
// k_mp2_pair: one work-group per (occupied pair i >= j, virtual tile pair
// A <= B of 64 x 64).  It forms K_ij[a][b] = (ia|jb) and K_ij[b][a] = (ib|ja)
// for a in A, b in B as two products of factor rows on the matrix cores
// (both land in the same register layout: rows a, cols b), then in registers
// the amplitudes, the energy terms of (a, b) and, for A != B, of (b, a), and
// optionally writes t_ij^ab, t_ij^ba and their twins t_ji^ba, t_ji^ab.  The
// pair (j, i) contributes what (i, j) does, so pairs i > j count twice.
//
// k_mp2_gram: sums over a batch range of products A_q (alpha B1_q + beta
// B2_q)^T with rows contiguous along the contraction, into one partial slice
// per work-group group; with the amplitudes t2 stored,
//   gamma_vv: q = (i, j), A_q = B1_q = t_ij (rows a, K = c), B2_q = t_ji
//             (t_ij^cb = t_ji^bc), alpha = 2, beta = -1, then x 2;
//   gamma_oo: q = k, A_q[i] = t_ik (K = ab), B1_q[j] = t_jk, B2_q[j] = t_kj
//             (t_jk^ba = t_kj^ab), alpha = 2, beta = -1, then 2 delta - 2 x.
// k_mp2_gram_sum adds the slices in a fixed order.
#pragma once

#include "device_common.hpp"

namespace sie {

constexpr int kMp2Tile = 64;   // virtual tile edge of k_mp2_pair (2 x 2 waves of 32 x 32)
// Wave tiles (16-wide MFMA tiles, rows x cols) of the Gram products: gamma_vv
// (n_v x n_v outputs, K = n_v per batch entry) and gamma_oo (n_o x n_o, few
// outputs: small tiles keep enough work-groups).
constexpr int kGramVvM = 4, kGramVvN = 2, kGramOoM = 2, kGramOoN = 2;

// Two consecutive float64 values along the contraction of row `row` at
// column k0 (k0 even), zero past K; `even`: rows start 16-byte aligned.
__device__ __forceinline__ d2v mp2_ld2(const double* base, int64_t row, int64_t stride, int k0,
                                       int K, bool even) {
  const double* p = base + row * stride + k0;
  if (even && k0 + 1 < K) return *(const SIE_GLOBAL d2v*)gptr(p);
  d2v x;
  x.x = k0 < K ? gptr(p)[0] : 0.0;
  x.y = k0 + 1 < K ? gptr(p)[1] : 0.0;
  return x;
}

// Grid: (tile pairs) x (occupied pairs), 256 threads.  eps: e_occ then
// e_vir.  e_part[blockIdx.y * gridDim.x + blockIdx.x]: the work-group's
// energy terms (pair weight included).  t2: [o][o][v][v] or NULL.
__global__ __launch_bounds__(256, 2) void k_mp2_pair(const double* __restrict__ L,
                                                     const double* __restrict__ eps, int no,
                                                     int nv, int np, double* __restrict__ t2,
                                                     double* __restrict__ e_part) {
  int i, j, A, B;
  {
    int64_t q = blockIdx.y;   // i >= j, lexicographic
    i = int(0.5 * (sqrt(8.0 * double(q) + 1.0) - 1.0));
    while (tri(i) > q) --i;
    while (tri(i + 1) <= q) ++i;
    j = int(q - tri(i));
    int64_t t = blockIdx.x;   // B >= A
    B = int(0.5 * (sqrt(8.0 * double(t) + 1.0) - 1.0));
    while (tri(B) > t) --B;
    while (tri(B + 1) <= t) ++B;
    A = int(t - tri(B));
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;
  const int wr = wave >> 1, wc = wave & 1;
  const int a0 = A * kMp2Tile + 32 * wr, b0 = B * kMp2Tile + 32 * wc;
  const bool even = (np % 2) == 0;
  const int64_t rs = np;                                   // row stride of L
  const double* Li = L + (int64_t)i * nv * np;
  const double* Lj = L + (int64_t)j * nv * np;
  int ra[2], rb[2];                                          // clamped rows of this lane
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    ra[t] = min(a0 + 16 * t + r, nv - 1);
    rb[t] = min(b0 + 16 * t + r, nv - 1);
  }
  d4 k1[2][2], k2[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) k1[p][q] = k2[p][q] = d4{0.0, 0.0, 0.0, 0.0};

  // chunk of 8 along P: lane group g holds k = 8c + 2g, 8c + 2g + 1; the
  // first values of all lanes make one K = 4 product, the second another
  d2v xi[2], xj[2], yj[2], yi[2];
  auto load = [&](int c, d2v (&ai)[2], d2v (&bj)[2], d2v (&aj)[2], d2v (&bi)[2]) {
    const int k0 = 8 * c + 2 * g;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      ai[t] = mp2_ld2(Li, ra[t], rs, k0, np, even);
      bj[t] = mp2_ld2(Lj, rb[t], rs, k0, np, even);
      aj[t] = mp2_ld2(Lj, ra[t], rs, k0, np, even);
      bi[t] = mp2_ld2(Li, rb[t], rs, k0, np, even);
    }
  };
  const int nch = (np + 7) / 8;
  load(0, xi, xj, yj, yi);
  for (int c = 0; c < nch; ++c) {
    d2v ni[2], nj[2], mj[2], mi[2];
    const bool more = c + 1 < nch;
    if (more) load(c + 1, ni, nj, mj, mi);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        k1[p][q] = mfma16x16x4(xi[p].x, xj[q].x, k1[p][q]);   // (ia|jb)
        k1[p][q] = mfma16x16x4(xi[p].y, xj[q].y, k1[p][q]);
        k2[p][q] = mfma16x16x4(yj[p].x, yi[q].x, k2[p][q]);   // (ib|ja) at [a][b]
        k2[p][q] = mfma16x16x4(yj[p].y, yi[q].y, k2[p][q]);
      }
    if (more) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        xi[t] = ni[t];
        xj[t] = nj[t];
        yj[t] = mj[t];
        yi[t] = mi[t];
      }
    }
  }

  const double ei = gptr(eps)[i], ej = gptr(eps)[j];
  const double* ev = eps + no;
  const bool off = A != B;
  const int64_t nv2 = (int64_t)nv * nv;
  double* tij = t2 ? t2 + ((int64_t)i * no + j) * nv2 : nullptr;
  double* tji = t2 ? t2 + ((int64_t)j * no + i) * nv2 : nullptr;
  double e = 0.0;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = a0 + 16 * p + 4 * u + g, b = b0 + 16 * q + r;
        if (a >= nv || b >= nv) continue;
        const double kab = k1[p][q][u], kba = k2[p][q][u];
        const double id = recip(gptr(ev)[a] + gptr(ev)[b] - ei - ej);
        const double tab = -kab * id, tba = -kba * id;
        e += tab * (2.0 * kab - kba);
        if (off) e += tba * (2.0 * kba - kab);
        if (tij) {   // t_ji^ba = t_ij^ab; for i = j the block is its own twin
          gptr_w(tij)[(int64_t)a * nv + b] = tab;
          if (off) gptr_w(tij)[(int64_t)b * nv + a] = tba;
          if (i != j) {
            gptr_w(tji)[(int64_t)b * nv + a] = tab;
            if (off) gptr_w(tji)[(int64_t)a * nv + b] = tba;
          }
        }
      }
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) e += __shfl_down(e, o, 64);
  if (lane == 0) red[wave] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double s = ((red[0] + red[1]) + red[2]) + red[3];
    e_part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (i == j ? 1.0 : 2.0) * s;
  }
}

// Batched sums of products for the density blocks (see the file comment).
// Output tile 32 x 32 per work-group (2 x 2 waves of 16 rows x 16 cols); grid (ceil(N / 32), ceil(M / 32), groups); group s
// sums batches q in [s * per, min((s + 1) * per, nq)) in order and writes
// part[s][m][n].  PAIRT: B2's batch is the transposed occupied pair of q
// (q = i * no + j -> j * no + i, gamma_vv); else B2 batch offset q * sB2q.
// Batch entry q of a launch is (entry q / ks, contraction split q % ks):
// with ks > 1 each entry's contraction of Ktot elements is cut into ks runs
// of K (the last one shorter), so that products with few outputs and a long
// contraction (gamma_oo) still give enough work-groups.
struct GramArgs {
  const double* a;
  const double* b1;
  const double* b2;
  int64_t sAq, sAm, sB1q, sB1n, sB2q, sB2n;
  int M, N, K, nq, per, no;
  double alpha, beta;
  double* part;
  int ks;
  int64_t Ktot;
};

// Wave tile of the Gram products: TM x TN 16-wide MFMA tiles; work-group:
// 2 x 2 waves, (32 TM) x (32 TN) outputs.  A work-group runs the chunks of
// its batch range as one stream with two chunks in flight.
template <bool PAIRT, int TM, int TN>
__global__ __launch_bounds__(256, 2) void k_mp2_gram(GramArgs ga) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;
  const int m0 = blockIdx.y * 32 * TM + 16 * TM * (wave >> 1);
  const int n0 = blockIdx.x * 32 * TN + 16 * TN * (wave & 1);
  int rm[TM], rn[TN];
#pragma unroll
  for (int t = 0; t < TM; ++t) rm[t] = min(m0 + 16 * t + r, ga.M - 1);
#pragma unroll
  for (int t = 0; t < TN; ++t) rn[t] = min(n0 + 16 * t + r, ga.N - 1);
  const bool even = (ga.K % 2) == 0 && (ga.Ktot % 2) == 0 && (ga.sAm % 2) == 0 &&
                    (ga.sB1n % 2) == 0 &&
                    (ga.sB2n % 2) == 0 && (ga.sAq % 2) == 0 && (ga.sB1q % 2) == 0 &&
                    (ga.sB2q % 2) == 0;
  const int q0 = blockIdx.z * ga.per, q1 = min(q0 + ga.per, ga.nq);
  d4 acc[TM][TN];
#pragma unroll
  for (int u = 0; u < TM; ++u)
#pragma unroll
    for (int v = 0; v < TN; ++v) acc[u][v] = d4{0.0, 0.0, 0.0, 0.0};
  const int nch = (ga.K + 7) / 8;
  struct Chunk {
    d2v x[TM], y1[TN], y2[TN];
  };
  auto load = [&](int q, int c, Chunk& ch) {
    const int qe = q / ga.ks;
    const int64_t koff = int64_t(q - qe * ga.ks) * ga.K;
    const int klim = int(min(int64_t(ga.K), ga.Ktot - koff));
    const int q2 = PAIRT ? (qe % ga.no) * ga.no + qe / ga.no : qe;
    const double* pa = ga.a + (int64_t)qe * ga.sAq + koff;
    const double* p1 = ga.b1 + (int64_t)qe * ga.sB1q + koff;
    const double* p2 = ga.b2 + (int64_t)q2 * ga.sB2q + koff;
    const int k0 = 8 * c + 2 * g;
#pragma unroll
    for (int t = 0; t < TM; ++t) ch.x[t] = mp2_ld2(pa, rm[t], ga.sAm, k0, klim, even);
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      ch.y1[t] = mp2_ld2(p1, rn[t], ga.sB1n, k0, klim, even);
      ch.y2[t] = mp2_ld2(p2, rn[t], ga.sB2n, k0, klim, even);
    }
  };
  auto mma = [&](const Chunk& ch) {
    double yx[TN], yy[TN];
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      yx[t] = ga.alpha * ch.y1[t].x + ga.beta * ch.y2[t].x;
      yy[t] = ga.alpha * ch.y1[t].y + ga.beta * ch.y2[t].y;
    }
#pragma unroll
    for (int u = 0; u < TM; ++u)
#pragma unroll
      for (int v = 0; v < TN; ++v) {
        acc[u][v] = mfma16x16x4(ch.x[u].x, yx[v], acc[u][v]);
        acc[u][v] = mfma16x16x4(ch.x[u].y, yy[v], acc[u][v]);
      }
  };
  auto next = [&](int& q, int& c) {
    if (++c == nch) {
      c = 0;
      ++q;
    }
  };
  if (q0 < q1) {
    int q = q0, c = 0;
    Chunk b0, b1;
    load(q, c, b0);
    for (;;) {
      next(q, c);
      const bool h1 = q < q1;
      if (h1) load(q, c, b1);
      mma(b0);
      if (!h1) break;
      next(q, c);
      const bool h0 = q < q1;
      if (h0) load(q, c, b0);
      mma(b1);
      if (!h0) break;
    }
  }
  double* out = ga.part + (int64_t)blockIdx.z * ga.M * ga.N;
#pragma unroll
  for (int u = 0; u < TM; ++u)
#pragma unroll
    for (int v = 0; v < TN; ++v)
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int m = m0 + 16 * u + 4 * w + g, n = n0 + 16 * v + r;
        if (m < ga.M && n < ga.N) gptr_w(out)[(int64_t)m * ga.N + n] = acc[u][v][w];
      }
}

// out[m][n] = diag * delta_mn + scale * sum_{s < groups} part[s][m][n], the
// slices added in order.
__global__ __launch_bounds__(256) void k_mp2_gram_sum(const double* __restrict__ part, int groups,
                                                      int M, int N, double scale, double diag,
                                                      double* __restrict__ out) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t mn = (int64_t)M * N;
  if (x >= mn) return;
  double s = 0.0;
  for (int q = 0; q < groups; ++q) s += part[(int64_t)q * mn + x];
  const int m = int(x / N), n = int(x % N);
  out[x] = (m == n ? diag : 0.0) + scale * s;
}

// out[0] = sum_{q < n} x[q] in a fixed order (one block: strided partial
// sums, then a fixed binary tree).
__global__ __launch_bounds__(256) void k_mp2_sum(const double* __restrict__ x, int64_t n,
                                                 double* __restrict__ out) {
  __shared__ double buf[256];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < n; q += 256) s += x[q];
  buf[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = buf[0];
}

}  // namespace sie
