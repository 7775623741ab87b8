// float64 adjoint kernels (see k_adjoint.hpp).
#include "adj_launch.hpp"
#include "k_eps.hpp"

namespace sie {

void launch_hat_f64(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                    int n_items, double* arena, double* partials, int pstride,
                    const double* grad_e, double* eo_part, double* ev_part, int ev_stride) {
  hipLaunchKernelGGL((k_hat<double, double>), dim3(grid), dim3(256), 0, s, desc, items, n_items,
                     arena, partials, pstride, grad_e, eo_part, ev_part, ev_stride);
}

void launch_eps_vir(hipStream_t s, const FragDesc* desc, const Item* items, int n_items,
                    int n_frag, const double* ev_part, int pstride, int ev_stride,
                    double* ev_item) {
  const unsigned gx = unsigned((ev_stride + 255) / 256);
  hipLaunchKernelGGL(k_eps_vir_items, dim3(gx, unsigned(n_items)), dim3(256), 0, s, desc, items,
                     ev_part, pstride, ev_stride, ev_item);
  hipLaunchKernelGGL(k_eps_vir_add, dim3(gx, unsigned(n_frag)), dim3(256), 0, s, desc, items,
                     n_items, ev_item, ev_stride);
}

void launch_eps_occ(hipStream_t s, const FragDesc* desc, int n_frag, int64_t max_units,
                    int max_no, const double* eo_part, int pstride, double* eo_units) {
  hipLaunchKernelGGL(k_eps_occ_units, dim3(unsigned((max_units + 255) / 256), unsigned(n_frag)),
                     dim3(256), 0, s, desc, eo_part, pstride, eo_units);
  hipLaunchKernelGGL(k_eps_occ, dim3(unsigned((max_no + 255) / 256), unsigned(n_frag)),
                     dim3(256), 0, s, desc, eo_units);
}

void launch_adj_f64(const AdjLaunch* L, const AdjArgs& a, const double* arena, hipStream_t s) {
  launch_adj_round<double>(L, a, arena, s);
}

}  // namespace sie
