// float64 adjoint kernels (see k_adjoint.hpp).
#include "adj_launch.hpp"

namespace sie {

void launch_hat_f64(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                    int n_items, double* arena, double* partials, int pstride,
                    const double* grad_e) {
  hipLaunchKernelGGL((k_hat<double, double>), dim3(grid), dim3(256), 0, s, desc, items, n_items,
                     arena, partials, pstride, grad_e);
}

void launch_adj_f64(const AdjLaunch* L, const AdjArgs& a, const double* arena, hipStream_t s) {
  launch_adj_round<double>(L, a, arena, s);
}

}  // namespace sie
