// Fixed-order float64 reductions: per-unit partials -> per-unit energies ->
// fragment energy.  No atomics: the same inputs give bitwise the same sums.
#pragma once

#include "device_common.hpp"

namespace sie {

// e_units[u] = 2 A_ijk * sum_{p < n_part} partials[u][p]  (u in [0, n_units)),
// A_ijk the equal-index weight of the unordered occupied triple (i, j, k).
__global__ __launch_bounds__(256) void k_unit_energy(int no, int64_t n_units,
                                                     const double* __restrict__ partials,
                                                     int n_part,
                                                     double* __restrict__ e_units) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n_units) return;
  int i, j, k;
  decode_sorted_triple(u, no, i, j, k);
  if (i == k) {
    e_units[u] = 0.0;
    return;
  }
  const double* p = partials + u * n_part;
  double s = 0.0;
  for (int q = 0; q < n_part; ++q) s += p[q];
  const double weight = (i == j || j == k) ? 1.0 : 2.0;   // 2 A_ijk
  e_units[u] = weight * s;
}

// out[0] = sum_{q < n} x[q] in a fixed order (one block of 256 threads:
// strided partial sums, then a fixed binary tree).
__global__ __launch_bounds__(256) void k_sum_fixed(const double* __restrict__ x,
                                                   int64_t n, double* __restrict__ out) {
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
