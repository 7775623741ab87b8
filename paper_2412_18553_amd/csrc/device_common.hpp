// Device helpers shared by the (T) kernels (gfx950, wave64).
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sie {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));   // 8 bf16 or 16 bytes

// Global-address-space views of generic pointers: loads through them are
// global (vmcnt only), not flat (which also counts against the LDS counter
// and would make every LDS wait also wait for in-flight prefetches).
#define SIE_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const SIE_GLOBAL T* gptr(const T* p) {
  return (const SIE_GLOBAL T*)(p);
}
template <typename T>
__device__ __forceinline__ SIE_GLOBAL T* gptr_w(T* p) {
  return (SIE_GLOBAL T*)(p);
}

// D(16x16, f64) += A(16x4) * B(4x16) on the matrix cores.
// Operand layout (one f64 per lane): A[row = lane % 16][k = lane / 16],
// B[k = lane / 16][col = lane % 16]; result lane l, element v holds
// D[4 * v + l / 16][l % 16] (measured on gfx950).
__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 1 / d for a normal float64 d: the hardware reciprocal estimate refined by
// two Newton-Raphson steps r <- r + r (1 - d r) (each squares the relative
// error), within an ulp or two of the rounded quotient, at a fraction of the
// cost of an IEEE division.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
  return r;
}

__host__ __device__ __forceinline__ int64_t tetra(int64_t n) {   // n(n+1)(n+2)/6
  return n * (n + 1) * (n + 2) / 6;
}
__host__ __device__ __forceinline__ int64_t tri(int64_t n) {     // n(n+1)/2
  return n * (n + 1) / 2;
}

// Linear index u of a sorted triple p >= q >= r (lexicographic in (p, q, r))
// back to (p, q, r).  `bound` is an upper bound on p.  p is the largest value
// below `bound` with tetra(p) <= u and q the largest value <= p with
// tri(q) <= u - tetra(p): both start from the real-valued inverse (cube and
// square root) and are then corrected with exact integer comparisons, so the
// result does not depend on the rounding of the estimates.
__host__ __device__ __forceinline__ void decode_sorted_triple(int64_t u, int bound,
                                                     int& p, int& q, int& r) {
  int pp = int(cbrt(6.0 * double(u)));
  pp = pp < 0 ? 0 : (pp > bound - 1 ? bound - 1 : pp);
  while (pp > 0 && tetra(pp) > u) --pp;
  while (pp + 1 < bound && tetra(pp + 1) <= u) ++pp;
  const int64_t rem = u - tetra(pp);
  int qq = int(0.5 * (sqrt(8.0 * double(rem) + 1.0) - 1.0));
  qq = qq < 0 ? 0 : (qq > pp ? pp : qq);
  while (qq > 0 && tri(qq) > rem) --qq;
  while (qq + 1 <= pp && tri(qq + 1) <= rem) ++qq;
  p = pp;
  q = qq;
  r = (int)(rem - tri(qq));
}

// Occupied triple (i, j, k) with which unit u (sorted p >= q >= r) is
// evaluated.  With `pair` set, a unit p > q = r is evaluated as (q, q, p):
// the unit energy sum_abc Wt R'[Wt + Vt] / D is unchanged by a simultaneous
// permutation of the occupied and the virtual indices (Wt, Vt and D are
// invariant under it and R' commutes with it), and with the two equal
// indices first, Wt[a][b][c] = Wt[b][a][c], so the second layout's partial
// cube equals the first's (P2[x][y][z] = P1[x][y][z]): only the first layout
// is built.  Returns whether the unit is such a pair unit.
__host__ __device__ __forceinline__ bool unit_triple(int64_t u, int bound, bool pair, int& i,
                                                     int& j, int& k) {
  decode_sorted_triple(u, bound, i, j, k);
  if (!pair || i == k) return false;
  if (j == k) {
    k = i;
    i = j;
  }
  return i == j;
}

// Occupied triple of a work item.  u >= 0: the unordered triple u as above
// (unit_triple); returns false for i = j = k, whose energy contribution is
// exactly zero.  u < 0: the ordered triple (i, j, k) with
// -1 - u = (i n_occ + j) n_occ + k (the projector evaluation, which needs
// W-tilde of every ordered triple, i = j = k included); `one` is then false.
__host__ __device__ __forceinline__ bool item_triple(int64_t u, int bound, bool pair, int& i,
                                                     int& j, int& k, bool& one) {
  if (u >= 0) {
    one = unit_triple(u, bound, pair, i, j, k);
    return i != k;
  }
  const int64_t x = -1 - u;
  k = int(x % bound);
  j = int((x / bound) % bound);
  i = int(x / (int64_t(bound) * bound));
  one = false;
  return true;
}

// Item code of the ordered occupied triple (i, j, k).
__host__ __device__ __forceinline__ int ordered_item(int i, int j, int k, int bound) {
  return -1 - int((int64_t(i) * bound + j) * bound + k);
}

}  // namespace sie
