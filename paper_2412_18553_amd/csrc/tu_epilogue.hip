// R/D epilogue, fixed-order reductions, fill and symmetrize (see k_fp64.hpp,
// k_reduce.hpp, k_adjoint.hpp).
#include "k_adjoint.hpp"
#include "k_fp64.hpp"
#include "k_proj.hpp"
#include "k_reduce.hpp"
#include "launch.hpp"

namespace sie {

void launch_epilogue_f64(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                         int n_items, const double* arena, double* partials, int pstride) {
  hipLaunchKernelGGL((k_epilogue<double, double>), dim3(grid), dim3(256), 0, s, desc, items,
                     n_items, arena, partials, pstride);
}

void launch_epilogue_f32(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                         int n_items, const float* arena, double* partials, int pstride) {
  hipLaunchKernelGGL((k_epilogue<float, float>), dim3(grid), dim3(256), 0, s, desc, items,
                     n_items, arena, partials, pstride);
}

void launch_proj_wq_f64(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                        int n_items, double* arena) {
  hipLaunchKernelGGL((k_proj_wq<double, double>), dim3(grid), dim3(256), 0, s, desc, items,
                     n_items, arena);
}

void launch_proj_wq_f32(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                        int n_items, float* arena) {
  hipLaunchKernelGGL((k_proj_wq<float, float>), dim3(grid), dim3(256), 0, s, desc, items,
                     n_items, arena);
}

void launch_proj_m_f64(hipStream_t s, const double* wt, const double* q, int64_t stride, int no,
                       int64_t K, int64_t chunk, int chunks, double* part) {
  const unsigned t = unsigned((no + 31) / 32);
  hipLaunchKernelGGL(k_proj_m<double>, dim3(t, t, unsigned(chunks)), dim3(256), 0, s, wt, q,
                     stride, no, K, chunk, part);
}

void launch_proj_m_f32(hipStream_t s, const float* wt, const float* q, int64_t stride, int no,
                       int64_t K, int64_t chunk, int chunks, double* part) {
  const unsigned t = unsigned((no + 31) / 32);
  hipLaunchKernelGGL(k_proj_m<float>, dim3(t, t, unsigned(chunks)), dim3(256), 0, s, wt, q,
                     stride, no, K, chunk, part);
}

void launch_proj_msum(hipStream_t s, const double* part, int chunks, int no, double weight,
                      double* m) {
  const int64_t n = int64_t(no) * no;
  hipLaunchKernelGGL(k_proj_msum, dim3(unsigned((n + 15) / 16)), dim3(256), 0, s, part, chunks,
                     no, weight, m);
}

void launch_proj_energy(hipStream_t s, const double* c, const double* m, int64_t n, double* out) {
  hipLaunchKernelGGL(k_proj_energy, dim3(1), dim3(256), 0, s, c, m, n, out);
}

void launch_unit_energy(dim3 grid, hipStream_t s, const FragDesc* desc, const double* partials,
                        int pstride, double* e_units) {
  hipLaunchKernelGGL(k_unit_energy, grid, dim3(256), 0, s, desc, partials, pstride, e_units);
}

void launch_frag_energy(unsigned grid, hipStream_t s, const FragDesc* desc,
                        const double* e_units, double* e_frag) {
  hipLaunchKernelGGL(k_frag_energy, dim3(grid), dim3(256), 0, s, desc, e_units, e_frag);
}

void launch_sum_fixed(hipStream_t s, const double* x, int64_t n, double* out) {
  hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, x, n, out);
}

void launch_fill_zero(unsigned grid, hipStream_t s, double* p, int64_t n) {
  hipLaunchKernelGGL(k_fill_zero<>, dim3(grid), dim3(256), 0, s, p, n);
}

void launch_symmetrize(unsigned grid, hipStream_t s, double* g, int kind, int no, int nv,
                       int64_t n) {
  hipLaunchKernelGGL(k_symmetrize<>, dim3(grid), dim3(256), 0, s, g, kind, no, nv, n);
}

void launch_zero_flags(hipStream_t s, int* flags, int n) {
  hipLaunchKernelGGL(k_zero_flags, dim3((n + 255) / 256), dim3(256), 0, s, flags, n);
}

void launch_nonfinite(hipStream_t s, const void* x, bool f64, int64_t n, int* flags, int slot) {
  const int64_t nb = (n + 255) / 256;
  const unsigned grid = unsigned(nb < 8192 ? (nb > 0 ? nb : 1) : 8192);
  if (f64)
    hipLaunchKernelGGL(k_nonfinite<double>, dim3(grid), dim3(256), 0, s,
                       static_cast<const double*>(x), n, flags, slot);
  else
    hipLaunchKernelGGL(k_nonfinite<float>, dim3(grid), dim3(256), 0, s,
                       static_cast<const float*>(x), n, flags, slot);
}

}  // namespace sie
