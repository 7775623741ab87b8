// float64 W-tilde build, two-layout tile variants (see k_fp64.hpp).
#include "k_fp64.hpp"
#include "launch.hpp"

namespace sie {

void launch_build_f64_l2(int variant, unsigned grid, hipStream_t s, const FragDesc* desc,
                         const Item* items, int n_items, double* arena) {
#define SIE_L2(V, ...)                                                                   \
  case V:                                                                                \
    hipLaunchKernelGGL((k_build_w_f64<__VA_ARGS__>), dim3(grid), dim3(256), 0, s, desc,  \
                       items, n_items, arena);                                           \
    break;
  switch (variant) {
    SIE_L2(1, 4, 2, 2, 1)
    SIE_L2(2, 2, 2, 2, 2)
    SIE_L2(3, 8, 1, 1, 2)
    SIE_L2(4, 4, 4, 2, 1)
    SIE_L2(5, 4, 2, 4, 1)
    SIE_L2(6, 4, 2, 2, 2, 2, 2)
    SIE_L2(7, 4, 2, 2, 2, 1, 4)
    SIE_L2(8, 4, 2, 2, 2, 4, 1)
    default:
      hipLaunchKernelGGL((k_build_w_f64<4, 2, 2, 2>), dim3(grid), dim3(256), 0, s, desc, items,
                         n_items, arena);
      break;
  }
#undef SIE_L2
}

}  // namespace sie
