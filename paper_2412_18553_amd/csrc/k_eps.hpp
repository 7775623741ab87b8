// Fixed-order reductions of the orbital-energy gradient (see k_hat in
// k_adjoint.hpp): the work-group rows of a backward round into per-item rows
// and those into the virtual gradient, and the per-unit occupied sums into
// the occupied gradient.  No atomics: bitwise reproducible.
#pragma once

#include "device_common.hpp"
#include "work.hpp"

namespace sie {

// ev_item[r * ev_stride + x] = sum over the round's work-group rows of item r
// (slots 0 .. n_part - 1 in order).  Grid: (ceil(ev_stride / 256), items).
__global__ __launch_bounds__(256) void k_eps_vir_items(const FragDesc* __restrict__ descs,
                                                       const Item* __restrict__ items,
                                                       const double* __restrict__ ev_part,
                                                       int pstride, int ev_stride,
                                                       double* __restrict__ ev_item) {
  const int r = blockIdx.y;
  const FragDesc fd = descs[items[r].frag];
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= fd.nv) return;
  const double* p = ev_part + (int64_t)r * pstride * ev_stride + x;
  double s = 0.0;
  for (int q = 0; q < fd.n_part; ++q) s += p[(int64_t)q * ev_stride];
  ev_item[(int64_t)r * ev_stride + x] = s;
}

// g_ev[x] += sum over the round's items of fragment blockIdx.y, in item order.
// Grid: (ceil(nv_max / 256), fragments).
__global__ __launch_bounds__(256) void k_eps_vir_add(const FragDesc* __restrict__ descs,
                                                     const Item* __restrict__ items, int n_items,
                                                     const double* __restrict__ ev_item,
                                                     int ev_stride) {
  const int f = blockIdx.y;
  const FragDesc fd = descs[f];
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (!fd.g_ev || x >= fd.nv) return;
  double s = 0.0;
  for (int r = 0; r < n_items; ++r)
    if (items[r].frag == f) s += ev_item[(int64_t)r * ev_stride + x];
  fd.g_ev[x] += s;
}

// eo_units[unit_base + u] = sum_{p < n_part} eo_part[(unit_base + u) * pstride + p]
// (0 for the units i = j = k, which contribute nothing).
// Grid: (ceil(max units / 256), fragments).
__global__ __launch_bounds__(256) void k_eps_occ_units(const FragDesc* __restrict__ descs,
                                                       const double* __restrict__ eo_part,
                                                       int pstride, double* __restrict__ eo_units) {
  const FragDesc fd = descs[blockIdx.y];
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= tetra(fd.no)) return;
  int i, j, k;
  decode_sorted_triple(u, fd.no, i, j, k);
  double s = 0.0;
  if (i != k) {   // units i = j = k are never evaluated: their partials are not written
    const double* p = eo_part + (fd.unit_base + u) * pstride;
    for (int q = 0; q < fd.n_part; ++q) s += p[q];
  }
  eo_units[fd.unit_base + u] = s;
}

// g_eo[p] = -sum_u count_p(u) eo_units[u] over the units u = (i, j, k),
// i >= j >= k, of fragment blockIdx.y in index order.  Grid: (ceil(no / 256),
// fragments).
__global__ __launch_bounds__(256) void k_eps_occ(const FragDesc* __restrict__ descs,
                                                 const double* __restrict__ eo_units) {
  const FragDesc fd = descs[blockIdx.y];
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (!fd.g_eo || p >= fd.no) return;
  const double* q = eo_units + fd.unit_base;
  double s = 0.0;
  int64_t u = 0;
  for (int i = 0; i < fd.no; ++i)
    for (int j = 0; j <= i; ++j)
      for (int k = 0; k <= j; ++k, ++u) {
        const int cnt = (i == p) + (j == p) + (k == p);
        if (cnt) s += double(cnt) * q[u];
      }
  fd.g_eo[p] = -s;
}

}  // namespace sie
