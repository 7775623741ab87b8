// float64 W-tilde build, three-layout tile variants (see k_fp64.hpp).
#include "k_fp64.hpp"
#include "launch.hpp"

namespace sie {

void launch_build_f64_l3(int variant, unsigned grid, hipStream_t s, const FragDesc* desc,
                         const Item* items, int n_items, double* arena) {
#define SIE_L3(V, ...)                                                                    \
  case V:                                                                                 \
    hipLaunchKernelGGL((k_build_w3_f64<__VA_ARGS__>), dim3(grid), dim3(256), 0, s, desc,  \
                       items, n_items, arena);                                            \
    break;
  switch (variant) {
    SIE_L3(9, 1, 1, 13, 2)
    SIE_L3(10, 1, 2, 7, 2)
    SIE_L3(11, 2, 1, 7, 2)
    SIE_L3(12, 1, 1, 10, 2)
    SIE_L3(13, 1, 2, 10, 1)
    SIE_L3(14, 1, 2, 4, 2)
    default:
      break;
  }
#undef SIE_L3
}

}  // namespace sie
