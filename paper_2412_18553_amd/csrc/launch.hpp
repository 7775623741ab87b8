// Launch wrappers of the (T) kernels.  Each kernel family lives in its own
// translation unit (tu_*.hip) so that the library's device code compiles in
// parallel; the host runtime (sie_triples.hip) sees only these plain
// functions.  Every wrapper enqueues on stream `s` and returns without
// waiting; grids, items and contraction lists are described in work.hpp and
// adj_plan.hpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adj_plan.hpp"
#include "shapes.hpp"
#include "work.hpp"

namespace sie {

// ---- W-tilde build, float64 (tile variants of shapes.hpp) ----
// tu_build_f64.hip: two-layout variants; tu_build_f64_l3.hip: three-layout.
void launch_build_f64_l2(int variant, unsigned grid, hipStream_t s, const FragDesc* desc,
                         const Item* items, int n_items, double* arena);
void launch_build_f64_l3(int variant, unsigned grid, hipStream_t s, const FragDesc* desc,
                         const Item* items, int n_items, double* arena);
inline void launch_build_f64(int variant, unsigned grid, hipStream_t s, const FragDesc* desc,
                             const Item* items, int n_items, double* arena) {
  if (wshape(variant).lay == 3)
    launch_build_f64_l3(variant, grid, s, desc, items, n_items, arena);
  else
    launch_build_f64_l2(variant, grid, s, desc, items, n_items, arena);
}

// ---- split precision (tu_bf16.hip) ----
void launch_build_split(int shape, unsigned grid, hipStream_t s, const FragDesc* desc,
                        const Item* items, int n_items, float* arena);
void launch_split_bf16(unsigned grid, hipStream_t s, const float* src, int P, int X, int Y,
                       int64_t sp, int64_t sx, int64_t sy, int64_t sk, int K, int Kpad,
                       bool kfast, u4v* dst);

// ---- integral blocks from density-fitting factors (tu_df.hip) ----
struct DfArgs;
void launch_df_form_f64(hipStream_t s, const DfArgs& a, double* out);
void launch_df_form_f32(hipStream_t s, const DfArgs& a, float* out);

// ---- epilogue and reductions (tu_epilogue.hip) ----
void launch_epilogue_f64(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                         int n_items, const double* arena, double* partials, int pstride);
void launch_epilogue_f32(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                         int n_items, const float* arena, double* partials, int pstride);
void launch_unit_energy(dim3 grid, hipStream_t s, const FragDesc* desc, const double* partials,
                        int pstride, double* e_units);
void launch_frag_energy(unsigned grid, hipStream_t s, const FragDesc* desc,
                        const double* e_units, double* e_frag);
void launch_sum_fixed(hipStream_t s, const double* x, int64_t n, double* out);
void launch_fill_zero(unsigned grid, hipStream_t s, double* p, int64_t n);
void launch_symmetrize(unsigned grid, hipStream_t s, double* g, int kind, int no, int nv,
                       int64_t n);
// flags[slot] = 1 if x[0 .. n) holds a non-finite value (float64 or float32
// elements); launch_zero_flags clears flags[0 .. n) first.
void launch_zero_flags(hipStream_t s, int* flags, int n);
void launch_nonfinite(hipStream_t s, const void* x, bool f64, int64_t n, int* flags, int slot);

// ---- fragment projector (k_proj.hpp, in tu_epilogue.hip) ----
void launch_proj_wq_f64(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                        int n_items, double* arena);
void launch_proj_wq_f32(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                        int n_items, float* arena);
void launch_proj_m_f64(hipStream_t s, const double* wt, const double* q, int64_t stride, int no,
                       int64_t K, int64_t chunk, int chunks, double* part);
void launch_proj_m_f32(hipStream_t s, const float* wt, const float* q, int64_t stride, int no,
                       int64_t K, int64_t chunk, int chunks, double* part);
void launch_proj_msum(hipStream_t s, const double* part, int chunks, int no, double weight,
                      double* m);
void launch_proj_energy(hipStream_t s, const double* c, const double* m, int64_t n, double* out);

// ---- adjoint (tu_adj_f64.hip, tu_adj_f32.hip) ----
// Contraction lists of one class in one backward round (host tables uploaded
// to the workspace): the class's groups and records, and for the
// summed-block classes its output slices and partial-slice extent.
struct AdjLaunch {
  size_t group_off = 0;   // first group in the uploaded group table
  int n_groups = 0;
  int64_t n_wg = 0;
  int rec_begin = 0, rec_end = 0;   // the class's records in the uploaded record table
  size_t slice_off = 0;   // summed-block classes: output slices in the slice table
  int n_slices = 0;
  int64_t max_slice = 0;  // largest slice (elements): the partial-sum grid
  int64_t part_elems = 0; // partial-slice elements the class writes
};

struct AdjArgs {
  const FragDesc* desc;   // device descriptors
  const Item* items;      // the round's items (device)
  int n_items;
  const AdjGroup* groups; // device tables
  const AdjRec* recs;
  const AdjSlice* slices;
  double* parts;          // partial slices of the summed-block classes
  double* t1_part;        // t1 partial rows
  int nv_max;             // row stride of t1_part
  int t1_batch;           // t1 records per partial-sum batch
};

// G and H over the round's partial cubes (and the unit energy partials).
void launch_hat_f64(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                    int n_items, double* arena, double* partials, int pstride,
                    const double* grad_e, double* eo_part, double* ev_part, int ev_stride);
void launch_hat_f32(unsigned grid, hipStream_t s, const FragDesc* desc, const Item* items,
                    int n_items, float* arena, double* partials, int pstride,
                    const double* grad_e, double* eo_part, double* ev_part, int ev_stride);
// Orbital-energy gradient reductions (k_adjoint.hpp): per round, the
// work-group rows into per-item rows and those into g_ev; after the last
// round, the per-unit sums and g_eo.
void launch_eps_vir(hipStream_t s, const FragDesc* desc, const Item* items, int n_items,
                    int n_frag, const double* ev_part, int pstride, int ev_stride,
                    double* ev_item);
void launch_eps_occ(hipStream_t s, const FragDesc* desc, int n_frag, int64_t max_units,
                    int max_no, const double* eo_part, int pstride, double* eo_units);
// Every G and H contraction of one round (L: kAdjClasses entries).
void launch_adj_f64(const AdjLaunch* L, const AdjArgs& a, const double* arena, hipStream_t s);
void launch_adj_f32(const AdjLaunch* L, const AdjArgs& a, const float* arena, hipStream_t s);

}  // namespace sie
