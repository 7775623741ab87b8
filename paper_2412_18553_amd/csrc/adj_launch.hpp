// Launch sequence of one backward round's G and H contractions, shared by
// the float64 and the split-precision adjoint translation units.
#pragma once

#include "k_adjoint.hpp"
#include "launch.hpp"

namespace sie {

template <typename CubeT>
void launch_adj_round(const AdjLaunch* L, const AdjArgs& a, const CubeT* arena, hipStream_t s) {
  using InT = CubeT;
  auto contract = [&](auto kernel, const AdjLaunch& l) {
    if (l.n_wg)
      hipLaunchKernelGGL(kernel, dim3(unsigned(l.n_wg)), dim3(kAThreads), 0, s, a.desc, a.items,
                         a.groups + l.group_off, l.n_groups, a.recs, arena, a.parts);
  };
  auto part_sum = [&](auto kernel, const AdjLaunch& l) {   // after the class's contraction
    if (l.n_slices)
      hipLaunchKernelGGL(kernel, dim3(unsigned((l.max_slice + 255) / 256), unsigned(l.n_slices)),
                         dim3(256), 0, s, a.desc, a.slices + l.slice_off,
                         static_cast<const double*>(a.parts));
  };
  contract(k_adj_contract<kAdjOvvv, CubeT, InT>, L[kAdjOvvv]);
  contract(k_adj_contract<kAdjT2vv, CubeT, InT>, L[kAdjT2vv]);
  part_sum(k_adj_part_sum<kAdjT2vv>, L[kAdjT2vv]);
  contract(k_adj_contract<kAdjT2oo, CubeT, InT>, L[kAdjT2oo]);
  contract(k_adj_contract<kAdjOoov, CubeT, InT>, L[kAdjOoov]);
  part_sum(k_adj_part_sum<kAdjOoov>, L[kAdjOoov]);
  const AdjLaunch& lp = L[kAdjOvov];
  if (lp.n_wg)
    hipLaunchKernelGGL((k_adj_ovov<CubeT, InT>), dim3(unsigned(lp.n_wg)), dim3(256), 0, s,
                       a.desc, a.items, a.groups + lp.group_off, lp.n_groups, a.recs, arena);
  const AdjLaunch& l1 = L[kAdjT1];
  if (l1.n_groups) {
    const int r0 = l1.rec_begin, r1 = l1.rec_end;
    for (int b0 = r0; b0 < r1; b0 += a.t1_batch) {
      const int b1 = b0 + a.t1_batch < r1 ? b0 + a.t1_batch : r1;
      hipLaunchKernelGGL((k_adj_t1_part<CubeT, InT>), dim3(unsigned(b1 - b0)), dim3(256), 0, s,
                         a.desc, a.items, a.recs, b0, arena, a.t1_part, a.nv_max);
      hipLaunchKernelGGL(k_adj_t1_sum<>,
                         dim3(unsigned((a.nv_max + 255) / 256), unsigned(l1.n_groups)),
                         dim3(256), 0, s, a.desc, a.groups + l1.group_off, b0, b1, a.t1_part,
                         a.nv_max);
    }
  }
}

}  // namespace sie
