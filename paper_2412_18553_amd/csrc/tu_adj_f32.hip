// Split-precision adjoint kernels: float32 G and H cubes and inputs, float64
// contractions and gradients (see k_adjoint.hpp).
#include "adj_launch.hpp"

namespace sie {

void launch_hat_f32(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                    int n_items, float* arena, double* partials, int pstride,
                    const double* grad_e, double* eo_part, double* ev_part, int ev_stride) {
  hipLaunchKernelGGL((k_hat<float, float>), dim3(grid), dim3(256), 0, s, desc, items, n_items,
                     arena, partials, pstride, grad_e, eo_part, ev_part, ev_stride);
}

void launch_adj_f32(const AdjLaunch* L, const AdjArgs& a, const float* arena, hipStream_t s) {
  launch_adj_round<float>(L, a, arena, s);
}

}  // namespace sie
