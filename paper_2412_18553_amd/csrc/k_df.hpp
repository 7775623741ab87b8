// Integral blocks of a fragment formed from its density-fitting factors on
// the float64 matrix cores: C[m][n] = sum_P X_P[m] Y_P[n] with
//   X_P[m] = b[P][xr(m)][xc(m)],  Y_P[n] = b[P][yr(n)][yc(n)],
// b [n_aux][n][n] (n = n_occ + n_vir, occupied orbitals first, symmetric in
// its last two indices), and each index a pair (m / div, m % div) mapped to
// a row and column of b by strides.  Every block the (T) energy reads is
// such a product: (ia|bc), (jl|ia), (ia|jb).  The sum runs over P in order
// (fixed), in float64; the output is float64, or float32 rounded to nearest.
#pragma once

#include "device_common.hpp"

namespace sie {

struct DfMap {
  int64_t base;        // element offset of index 0 in one P plane of b
  int div;             // m = (m / div, m % div)
  int64_t s1, s2;      // strides of the two parts
};

struct DfArgs {
  const double* b;
  int64_t plane;       // n * n
  int naux;
  int M, N;
  DfMap x, y;
  int64_t ldc;         // row stride of the output
};

constexpr int kDfTM = 2, kDfTN = 4;   // 16-wide MFMA tiles per wave (rows x cols)

__device__ __forceinline__ int64_t df_at(const DfMap& m, int idx) {
  const int q = idx / m.div;
  return m.base + int64_t(q) * m.s1 + int64_t(idx - q * m.div) * m.s2;
}

// Grid: (ceil(N / (32 kDfTN)), ceil(M / (32 kDfTM))), 256 threads: 2 x 2
// waves of (16 kDfTM) x (16 kDfTN).  Lane (r, g) of an MFMA holds row r of
// the A side at P = p0 + g and col r of the B side at the same P; two steps
// of four P in flight.
template <typename OutT>
__global__ __launch_bounds__(256, 2) void k_df_form(DfArgs a, OutT* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;
  const int m0 = blockIdx.y * 32 * kDfTM + 16 * kDfTM * (wave >> 1);
  const int n0 = blockIdx.x * 32 * kDfTN + 16 * kDfTN * (wave & 1);
  int64_t xo[kDfTM], yo[kDfTN];
#pragma unroll
  for (int t = 0; t < kDfTM; ++t) xo[t] = df_at(a.x, min(m0 + 16 * t + r, a.M - 1));
#pragma unroll
  for (int t = 0; t < kDfTN; ++t) yo[t] = df_at(a.y, min(n0 + 16 * t + r, a.N - 1));
  d4 acc[kDfTM][kDfTN];
#pragma unroll
  for (int u = 0; u < kDfTM; ++u)
#pragma unroll
    for (int v = 0; v < kDfTN; ++v) acc[u][v] = d4{0.0, 0.0, 0.0, 0.0};
  struct Step {
    double x[kDfTM], y[kDfTN];
  };
  auto load = [&](int p0, Step& st) {
    const int p = p0 + g;
    const bool in = p < a.naux;
    const SIE_GLOBAL double* pl = gptr(a.b) + int64_t(in ? p : 0) * a.plane;
#pragma unroll
    for (int t = 0; t < kDfTM; ++t) st.x[t] = in ? pl[xo[t]] : 0.0;
#pragma unroll
    for (int t = 0; t < kDfTN; ++t) st.y[t] = in ? pl[yo[t]] : 0.0;
  };
  auto mma = [&](const Step& st) {
#pragma unroll
    for (int u = 0; u < kDfTM; ++u)
#pragma unroll
      for (int v = 0; v < kDfTN; ++v) acc[u][v] = mfma16x16x4(st.x[u], st.y[v], acc[u][v]);
  };
  Step s0, s1;
  load(0, s0);
  for (int p0 = 0;; p0 += 8) {
    const bool h1 = p0 + 4 < a.naux;
    if (h1) load(p0 + 4, s1);
    mma(s0);
    if (!h1) break;
    const bool h0 = p0 + 8 < a.naux;
    if (h0) load(p0 + 8, s0);
    mma(s1);
    if (!h0) break;
  }
  // acc[u][v][w] = C[m0 + 16 u + 4 w + g][n0 + 16 v + r]
#pragma unroll
  for (int u = 0; u < kDfTM; ++u)
#pragma unroll
    for (int v = 0; v < kDfTN; ++v)
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int m = m0 + 16 * u + 4 * w + g, n = n0 + 16 * v + r;
        if (m < a.M && n < a.N) gptr_w(out)[int64_t(m) * a.ldc + n] = OutT(acc[u][v][w]);
      }
}

}  // namespace sie
