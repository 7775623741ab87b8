// Fixed-order float64 reductions: per-unit partials -> per-unit energies ->
// fragment energy.  No atomics: the same inputs give bitwise the same sums.
#pragma once

#include "device_common.hpp"
#include "work.hpp"

namespace sie {

// e_units[unit_base + u] = 2 A_ijk * sum_{p < n_part} partials[(unit_base + u) * pstride + p]
// for every unit u of fragment blockIdx.y, A_ijk the equal-index weight of
// the unordered occupied triple (i, j, k); units with i = j = k are 0.
__global__ __launch_bounds__(256) void k_unit_energy(const FragDesc* __restrict__ descs,
                                                     const double* __restrict__ partials,
                                                     int pstride, double* __restrict__ e_units) {
  const FragDesc fd = descs[blockIdx.y];
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= tetra(fd.no)) return;
  int i, j, k;
  decode_sorted_triple(u, fd.no, i, j, k);
  double* out = e_units + fd.unit_base + u;
  if (i == k) {
    *out = 0.0;
    return;
  }
  const double* p = partials + (fd.unit_base + u) * pstride;
  double s = 0.0;
  for (int q = 0; q < fd.n_part; ++q) s += p[q];
  const double weight = (i == j || j == k) ? 1.0 : 2.0;   // 2 A_ijk
  *out = weight * s;
}

__device__ __forceinline__ double block_sum_fixed(double s, double* buf) {
  buf[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
    __syncthreads();
  }
  return buf[0];
}

// e_frag[f] = sum of fragment f's per-unit energies, in a fixed order
// (one block of 256 threads per fragment).
__global__ __launch_bounds__(256) void k_frag_energy(const FragDesc* __restrict__ descs,
                                                     const double* __restrict__ e_units,
                                                     double* __restrict__ e_frag) {
  __shared__ double buf[256];
  const FragDesc fd = descs[blockIdx.x];
  const int64_t n = tetra(fd.no);
  const double* x = e_units + fd.unit_base;
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < n; q += 256) s += x[q];
  const double t = block_sum_fixed(s, buf);
  if (threadIdx.x == 0) e_frag[blockIdx.x] = t;
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

// flags[slot] = 1 if any of x[0 .. n) is not finite (NaN or +-inf), else
// unchanged (zeroed by the caller).  Every finding thread stores the same
// value, so the stores need no ordering.
template <typename T>
__global__ __launch_bounds__(256) void k_nonfinite(const T* __restrict__ x, int64_t n,
                                                   int* __restrict__ flags, int slot) {
  bool bad = false;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    bad |= !__builtin_isfinite(gptr(x)[q]);
  if (bad) gptr_w(flags)[slot] = 1;
}

// flags[0 .. n) = 0.
__global__ __launch_bounds__(256) void k_zero_flags(int* __restrict__ flags, int n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) flags[q] = 0;
}

}  // namespace sie
