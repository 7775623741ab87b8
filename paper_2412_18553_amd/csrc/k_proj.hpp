// Fragment projector of the in-situ (T) energy (the C^f factor of equation
// E_corr_CCSD_T in the paper's in-situ (T) section).
//
// With C acting on the first occupied index of W-tilde (the reading that does
// not depend on how the virtual triples are ordered),
//   E_x(C) = (1/3) sum_{ijk abc} (C Wt)_{ijk} R[Wt + Vt]_{ijk} / D_{ijk}
//          = sum_{i i'} C_{i i'} M_{i i'},
//   M_{i i'} = (1/3) sum_{jk} sum_abc Wt^{abc}_{i'jk} Q^{abc}_{ijk},
//   Q = R[Wt + Vt] / D.
// M is independent of C, so one evaluation serves every projector of the
// cluster, and tr M is the unprojected energy.  M pairs W-tilde and Q of
// different occupied triples that share (j, k), so the GPU evaluates the
// ordered triples (i', j, k), i' = 0 .. n_o - 1, of one pair j >= k at a
// time (a "group"; (i', k, j) is the b <-> c image of (i', j, k), so a group
// with j > k counts twice): the build kernels write the two partial cubes of
// every ordered triple (8^3-blocked, cube_at), k_proj_wq replaces them by Wt
// and Q (R in its virtual form at the fixed ordered triple, as in the
// energy; zeros in the padding past n_v), and k_proj_m / k_proj_msum form the
// group's n_o x n_o product of Q and Wt cubes over every element of the
// blocked cube on the float64 matrix cores (split in chunks, summed in a
// fixed order) and add it into M.
#pragma once

#include "device_common.hpp"
#include "k_fp64.hpp"
#include "work.hpp"

namespace sie {

// Wt and Q in place of the two row-major partial cubes of each ordered
// triple of the round (same orbit traversal and in-place rule as k_hat: the
// work-group that reads an orbit's blocks of both cubes writes exactly those
// blocks).  Grid: the concatenated epilogue blocks of the round's items.
template <typename CubeT, typename InT>
__global__ __launch_bounds__(256) void k_proj_wq(const FragDesc* __restrict__ descs,
                                                 const Item* __restrict__ items, int n_items,
                                                 CubeT* __restrict__ arena) {
  const int r = find_item<false>(items, n_items, blockIdx.x);
  const int64_t start = r ? items[r - 1].part_end : 0;
  const Item it = items[r];
  const FragDesc fd = descs[it.frag];
  const int slot = int(int64_t(blockIdx.x) - start);
  int i, j, k;
  bool one;
  item_triple(it.unit, fd.no, false, i, j, k, one);
  __shared__ double sw[6][kOrbSlot];
  __shared__ double sz[6][kOrbSlot];
  const InT* __restrict__ t1 = static_cast<const InT*>(fd.t1);
  const InT* __restrict__ ovov = static_cast<const InT*>(fd.ovov);
  const double* __restrict__ eps = fd.eps;
  const int no = fd.no, nv = fd.nv;
  const int nb = (nv + kOrb - 1) / kOrb;
  const int64_t n_orb = tetra(nb);
  const double* __restrict__ ev = eps + no;
  const double eijk = gptr(eps)[i] + gptr(eps)[j] + gptr(eps)[k];
  CubeT* __restrict__ w1 = arena + it.cube_off;
  CubeT* __restrict__ w2 = w1 + fd.half;
  const int64_t nonv = (int64_t)no * nv;
  const InT* ov_ij = ovov + (int64_t)i * nv * nonv + (int64_t)j * nv;
  const InT* ov_ik = ovov + (int64_t)i * nv * nonv + (int64_t)k * nv;
  const InT* ov_jk = ovov + (int64_t)j * nv * nonv + (int64_t)k * nv;
  const InT* t1i = t1 + (int64_t)i * nv;
  const InT* t1j = t1 + (int64_t)j * nv;
  const InT* t1k = t1 + (int64_t)k * nv;
  constexpr int E = kOrb * kOrb * kOrb;

  for (int64_t o = slot; o < n_orb; o += fd.n_part) {
    int t0, t1b, t2b;
    decode_sorted_triple(o, nb, t0, t1b, t2b);
    for (int idx = threadIdx.x; idx < 6 * E; idx += 256) {
      const int s = idx / E, e = orb_elem(idx - s * E);
      int p0, p1, p2;
      slot_perm(s, p0, p1, p2);
      const int a = kOrb * pick3(p0, t0, t1b, t2b) + (e >> 6);
      const int b = kOrb * pick3(p1, t0, t1b, t2b) + ((e >> 3) & 7);
      const int c = kOrb * pick3(p2, t0, t1b, t2b) + (e & 7);
      double w = 0.0, z = 0.0;
      if (a < nv && b < nv && c < nv) {
        w = (double)gptr(w1)[cube_at(true, nv, a, b, c)] +
            (double)gptr(w2)[cube_at(true, nv, b, a, c)];
        const double vt = (double)gptr(ov_ij)[(int64_t)a * nonv + b] * (double)gptr(t1k)[c] +
                          (double)gptr(ov_ik)[(int64_t)a * nonv + c] * (double)gptr(t1j)[b] +
                          (double)gptr(ov_jk)[(int64_t)b * nonv + c] * (double)gptr(t1i)[a];
        z = w + vt;
      }
      sw[s][orb_lds(e >> 6, (e >> 3) & 7, e & 7)] = w;
      sz[s][orb_lds(e >> 6, (e >> 3) & 7, e & 7)] = z;
    }
    __syncthreads();
    unsigned primary = 0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      int p0, p1, p2;
      slot_perm(s, p0, p1, p2);
      bool dup = false;
#pragma unroll
      for (int s2 = 0; s2 < s; ++s2) {
        int q0, q1, q2;
        slot_perm(s2, q0, q1, q2);
        dup |= pick3(p0, t0, t1b, t2b) == pick3(q0, t0, t1b, t2b) &&
               pick3(p1, t0, t1b, t2b) == pick3(q1, t0, t1b, t2b) &&
               pick3(p2, t0, t1b, t2b) == pick3(q2, t0, t1b, t2b);
      }
      if (!dup) primary |= 1u << s;
    }
    for (int idx = threadIdx.x; idx < 6 * E; idx += 256) {
      const int s = idx / E, e = orb_elem(idx - s * E);
      if (!((primary >> s) & 1u)) continue;
      int p0, p1, p2;
      slot_perm(s, p0, p1, p2);
      const int x = e >> 6, y = (e >> 3) & 7, zz = e & 7;
      const int a = kOrb * pick3(p0, t0, t1b, t2b) + x;
      const int b = kOrb * pick3(p1, t0, t1b, t2b) + y;
      const int c = kOrb * pick3(p2, t0, t1b, t2b) + zz;
      const int64_t pos = cube_at(true, nv, a, b, c);
      if (a >= nv || b >= nv || c >= nv) {   // padding: zero in both cubes
        gptr_w(w1)[pos] = CubeT(0);
        gptr_w(w2)[pos] = CubeT(0);
        continue;
      }
      const double rz = 4.0 * sz[s][orb_lds(x, y, zz)] +
                        sz[orbit_slot(p2, p0, p1)][orb_lds(zz, x, y)] +
                        sz[orbit_slot(p1, p2, p0)][orb_lds(y, zz, x)] -
                        2.0 * (sz[orbit_slot(p2, p1, p0)][orb_lds(zz, y, x)] +
                               sz[orbit_slot(p0, p2, p1)][orb_lds(x, zz, y)] +
                               sz[orbit_slot(p1, p0, p2)][orb_lds(y, x, zz)]);
      const double id = recip(eijk - gptr(ev)[a] - gptr(ev)[b] - gptr(ev)[c]);
      gptr_w(w1)[pos] = CubeT(sw[s][orb_lds(x, y, zz)]);
      gptr_w(w2)[pos] = CubeT(rz * id);
    }
    __syncthreads();
  }
}

// part[z][m][n] = sum over the cube elements q in chunk z of
// Q_m[q] Wt_n[q], Q_m = cube 2 and Wt_n = cube 1 of the group's item m / n
// (items `stride` elements apart).  Grid (ceil(no / 32), ceil(no / 32),
// chunks), 2 x 2 waves of 16 x 16.
template <typename CubeT>
__global__ __launch_bounds__(256, 2) void k_proj_m(const CubeT* __restrict__ wt,
                                                   const CubeT* __restrict__ q, int64_t stride,
                                                   int no, int64_t K, int64_t chunk,
                                                   double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;
  const int m0 = blockIdx.y * 32 + 16 * (wave >> 1), n0 = blockIdx.x * 32 + 16 * (wave & 1);
  const int rm = min(m0 + r, no - 1), rn = min(n0 + r, no - 1);
  const int64_t k_begin = (int64_t)blockIdx.z * chunk;
  const int64_t k_end = min(k_begin + chunk, K);
  const CubeT* pa = q + (int64_t)rm * stride;
  const CubeT* pb = wt + (int64_t)rn * stride;
  d4 acc = d4{0.0, 0.0, 0.0, 0.0};
  // steps of 8 elements, the same trip count for every lane (the matrix
  // instructions run on the whole wave); lane group g takes elements
  // kb + 2g, kb + 2g + 1, zero past the chunk.  Chunk starts are even and the
  // cubes 8-aligned, so with even stride and K a full pair is one 2-element
  // load (`pair`).
  const bool pair = (stride % 2) == 0 && (K % 2) == 0 && (chunk % 2) == 0;
  typedef typename std::conditional<sizeof(CubeT) == 8, d2v, f2v>::type V2;
  for (int64_t kb = k_begin; kb < k_end; kb += 8) {
    const int64_t k0 = kb + 2 * g;
    double a0, a1, b0, b1;
    if (pair && k0 + 1 < k_end) {
      const V2 u = *(const SIE_GLOBAL V2*)(gptr(pa) + k0);
      const V2 w = *(const SIE_GLOBAL V2*)(gptr(pb) + k0);
      a0 = (double)u.x;
      a1 = (double)u.y;
      b0 = (double)w.x;
      b1 = (double)w.y;
    } else {
      a0 = k0 < k_end ? (double)gptr(pa)[k0] : 0.0;
      b0 = k0 < k_end ? (double)gptr(pb)[k0] : 0.0;
      a1 = k0 + 1 < k_end ? (double)gptr(pa)[k0 + 1] : 0.0;
      b1 = k0 + 1 < k_end ? (double)gptr(pb)[k0 + 1] : 0.0;
    }
    acc = mfma16x16x4(a0, b0, acc);
    acc = mfma16x16x4(a1, b1, acc);
  }
  double* out = part + (int64_t)blockIdx.z * no * no;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int m = m0 + 4 * u + g, n = n0 + r;
    if (m < no && n < no) gptr_w(out)[(int64_t)m * no + n] = acc[u];
  }
}

// M[m][n] += weight * sum_{z < chunks} part[z][m][n]: a work-group takes 16
// elements, lane q of an element sums chunks q, q + 16, ... in order, and
// the 16 lane sums are added by a fixed tree.
__global__ __launch_bounds__(256) void k_proj_msum(const double* __restrict__ part, int chunks,
                                                   int no, double weight,
                                                   double* __restrict__ m_out) {
  __shared__ double buf[16][17];
  const int e = threadIdx.x >> 4, q = threadIdx.x & 15;
  const int64_t x = (int64_t)blockIdx.x * 16 + e;
  const int64_t mn = (int64_t)no * no;
  double s = 0.0;
  if (x < mn)
    for (int z = q; z < chunks; z += 16) s += part[(int64_t)z * mn + x];
  buf[e][q] = s;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (q < w) buf[e][q] += buf[e][q + w];
    __syncthreads();
  }
  if (q == 0 && x < mn) m_out[x] += weight * buf[e][0];
}

// out[0] = sum_{m, n} c[m][n] M[m][n] in a fixed order (one block).
__global__ __launch_bounds__(256) void k_proj_energy(const double* __restrict__ c,
                                                     const double* __restrict__ m, int64_t n,
                                                     double* __restrict__ out) {
  __shared__ double buf[256];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < n; q += 256) s += c[q] * m[q];
  buf[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = buf[0];
}

}  // namespace sie
