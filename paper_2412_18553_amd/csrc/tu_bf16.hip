// Split-precision staging and W-tilde build (see k_bf16.hpp).
#include "k_bf16.hpp"
#include "launch.hpp"

namespace sie {

void launch_build_split(int shape, unsigned grid, hipStream_t s, const FragDesc* desc,
                        const Item* items, int n_items, float* arena) {
  switch (shape) {
#define SIE_SPLIT_CASE(S)                                                                   \
  case S:                                                                                   \
    hipLaunchKernelGGL((k_build_w_bf16x3<sshape(S).trw, sshape(S).tcw>), dim3(grid),        \
                       dim3(256), 0, s, desc, items, n_items, arena);                       \
    break;
    SIE_SPLIT_CASE(0)
    SIE_SPLIT_CASE(1)
    SIE_SPLIT_CASE(2)
    SIE_SPLIT_CASE(3)
#undef SIE_SPLIT_CASE
#define SIE_SPLIT_CASE_L(S)                                                                 \
  case S:                                                                                   \
    hipLaunchKernelGGL((k_build_w_bf16x3_l<sshape(S).trw, sshape(S).tcw, sshape(S).wc>),    \
                       dim3(grid), dim3(128 * sshape(S).wc), 0, s, desc, items, n_items,    \
                       arena);                                                              \
    break;
    SIE_SPLIT_CASE_L(4)
    SIE_SPLIT_CASE_L(5)
#undef SIE_SPLIT_CASE_L
    default:
      break;
  }
}
static_assert(kSShapes == 6 && sshape(3).wr == 1 && sshape(4).wr == 2 && sshape(5).wr == 2,
              "one launch case per split shape");

void launch_split_bf16(unsigned grid, hipStream_t s, const float* src, int P, int X, int Y,
                       int64_t sp, int64_t sx, int64_t sy, int64_t sk, int K, int Kpad,
                       bool kfast, u4v* dst) {
  hipLaunchKernelGGL(k_split_bf16, dim3(grid), dim3(256), 0, s, src, P, X, Y, sp, sx, sy, sk, K,
                     Kpad, kfast, dst);
}

}  // namespace sie
