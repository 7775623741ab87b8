// Integral blocks from density-fitting factors (see k_df.hpp).
#include "k_df.hpp"
#include "launch.hpp"

namespace sie {

namespace {
template <typename OutT>
void launch_df(hipStream_t s, const DfArgs& a, OutT* out) {
  const dim3 grid(unsigned((a.N + 32 * kDfTN - 1) / (32 * kDfTN)),
                  unsigned((a.M + 32 * kDfTM - 1) / (32 * kDfTM)));
  hipLaunchKernelGGL(k_df_form<OutT>, grid, dim3(256), 0, s, a, out);
}
}  // namespace

void launch_df_form_f64(hipStream_t s, const DfArgs& a, double* out) { launch_df(s, a, out); }
void launch_df_form_f32(hipStream_t s, const DfArgs& a, float* out) { launch_df(s, a, out); }

}  // namespace sie
