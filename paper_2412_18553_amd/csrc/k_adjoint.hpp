// Adjoint (gradient) kernels of the float64 (T) energy.
//
// With the energy written per unordered occupied triple ("unit") u = (i, j, k),
//   E = sum_u w_u sum_abc Wt R'[Wt + Vt] / D,      w_u = 2 A_ijk,
// and R' symmetric under the abc inner product (its cyclic terms are each
// other's transposes, its transpositions their own) with D symmetric in abc,
//   dE = sum_u sum_abc G dWt + H dVt,
//   G = w_u (R'[Wt] + R'[Wt + Vt]) / D,     H = w_u R'[Wt] / D.
// Wt of a unit is the sum of the twelve contractions the forward build
// evaluates (six over d, six over l; see k_fp64.hpp); the gradient with
// respect to each contraction's two operands is a contraction of G with the
// other operand.  Vt = (ia|jb) t_k^c + (ia|kc) t_j^b + (jb|kc) t_i^a gives
// the t1 and ovov parts from H.
//
// Per round of units (cubes resident in the workspace arena):
//   k_hat            Wt partial cubes -> G, H in place (and the unit energies)
//   k_adj_contract   the 24 G contractions, grouped by output slice
//   k_adj_ovov/t1    the H contractions
// Every launch owns each output element it writes (the host groups all of a
// round's contributions to one output slice into one list, summed in a fixed
// order by the work-groups that own the slice's tiles), so the gradient is a
// plain read-modify-write sum without atomics and bitwise reproducible.
#pragma once

#include "sie_triples.h"

#include "device_common.hpp"
#include "k_fp64.hpp"
#include "adj_plan.hpp"
#include "work.hpp"

namespace sie {

// ---------------------------------------------------------------------------
// G and H, in place of the two partial cubes of each unit.
// ---------------------------------------------------------------------------

// Same orbit traversal as k_epilogue (partial cubes, Wt[a][b][c] =
// P1[a][b][c] + P2[b][a][c]): the work-group that reads an orbit's blocks of
// both cubes writes G[a][b][c] over the first and H[a][b][c] over the second
// at exactly those blocks, and G transposed (Gt[a][b][c] = G(c, b, a)) into
// the unit's third cube.  Also
// writes the unit's energy partials (as k_epilogue).  grad_e[frag] (or 1)
// scales G and H.
//
// Orbital-energy gradient (eo_part non-NULL): the energy depends on the
// orbital energies only through D, dE_u/dD = -w W R'[Z] / D^2 per element.
// Per tuple (the six orderings of a virtual triple, which share D; see
// k_epilogue) q = scale * weight * sum_m Wt_m R'[Z]_m / D^2, so
//   dL/de_p (occupied) = -sum_u count_p(u) sum_{tuples of u} q,
//   dL/de_x (virtual)  = +sum_u sum_{tuples of u} count_x(tuple) q.
// Each work-group writes its share of the first sum to eo_part (layout of
// `partials`) and its per-virtual sums, accumulated over its orbits in an LDS
// row, to ev_part[(r pstride + slot) ev_stride + x] (r: item index in the
// round).  All sums run in fixed orders (wave shuffles, then fixed lanes).
template <typename CubeT, typename InT>
__global__ __launch_bounds__(256, 2) void k_hat(const FragDesc* __restrict__ descs,
                                             const Item* __restrict__ items, int n_items,
                                             CubeT* __restrict__ arena,
                                             double* __restrict__ partials, int pstride,
                                             const double* __restrict__ grad_e,
                                             double* __restrict__ eo_part,
                                             double* __restrict__ ev_part, int ev_stride) {
  const int r = find_item<false>(items, n_items, blockIdx.x);
  const int64_t start = r ? items[r - 1].part_end : 0;
  const Item it = items[r];
  const FragDesc fd = descs[it.frag];
  const int slot = int(int64_t(blockIdx.x) - start);
  int i, j, k;
  decode_sorted_triple(it.unit, fd.no, i, j, k);
  __shared__ double sw[6][kOrbSlot];
  __shared__ double sz[6][kOrbSlot];
  __shared__ double red[4];
  __shared__ double sev[3 * kOrb];   // e_vir at the orbit's three blocks
  // orbital-energy gradient: virtual row of this work-group and the
  // cross-wave partials of one orbit's marginals
  __shared__ double dv[SIE_MAX_VIR];
  __shared__ double tp0[2][4], tp1[2][4][kOrb], tp2[2][4][kOrb];
  const bool want_eps = eo_part != nullptr;
  double* out = partials + (fd.unit_base + it.unit) * pstride + slot;
  double* ev_row = want_eps ? ev_part + ((int64_t)r * pstride + slot) * ev_stride : nullptr;
  if (i == k) {
    if (threadIdx.x == 0) *out = 0.0;
    if (want_eps) {
      if (threadIdx.x == 0) eo_part[(fd.unit_base + it.unit) * pstride + slot] = 0.0;
      for (int a = threadIdx.x; a < fd.nv; a += 256) ev_row[a] = 0.0;
    }
    return;
  }
  if (want_eps)
    for (int a = threadIdx.x; a < fd.nv; a += 256) dv[a] = 0.0;   // first read after barriers
  const InT* __restrict__ t1 = static_cast<const InT*>(fd.t1);
  const InT* __restrict__ ovov = static_cast<const InT*>(fd.ovov);
  const double* __restrict__ eps = fd.eps;
  const int no = fd.no, nv = fd.nv;
  const int nb = (nv + kOrb - 1) / kOrb;
  const int64_t n_orb = tetra(nb);
  const double* __restrict__ ev = eps + no;
  const double eijk = gptr(eps)[i] + gptr(eps)[j] + gptr(eps)[k];
  const double scale = ((i == j || j == k) ? 1.0 : 2.0) * (grad_e ? gptr(grad_e)[it.frag] : 1.0);
  CubeT* __restrict__ w1 = arena + it.cube_off;
  CubeT* __restrict__ w2 = w1 + fd.half;
  CubeT* __restrict__ w3 = w2 + fd.half;     // G transposed, Gt[a][b][c] = G(c, b, a)
  const int64_t nonv = (int64_t)no * nv;
  const InT* ov_ij = ovov + (int64_t)i * nv * nonv + (int64_t)j * nv;
  const InT* ov_ik = ovov + (int64_t)i * nv * nonv + (int64_t)k * nv;
  const InT* ov_jk = ovov + (int64_t)j * nv * nonv + (int64_t)k * nv;
  const InT* t1i = t1 + (int64_t)i * nv;
  const InT* t1j = t1 + (int64_t)j * nv;
  const InT* t1k = t1 + (int64_t)k * nv;
  constexpr int E = kOrb * kOrb * kOrb;

  double acc = 0.0, eacc = 0.0;
  for (int64_t o = slot; o < n_orb; o += fd.n_part) {
    int t0, t1b, t2b;
    decode_sorted_triple(o, nb, t0, t1b, t2b);
    // Wt and Z of the orbit's 6 x 512 elements, 12 per thread, in batches
    // (all 12 with float32 values, 6 with float64: registers): every load
    // of a batch (indices clamped in range, results past n_v masked) is
    // issued before any is used
    // (the previous orbit's last barrier freed sev)
    if (threadIdx.x < 3 * kOrb)
      sev[threadIdx.x] = gptr(ev)[min(kOrb * pick3(threadIdx.x / kOrb, t0, t1b, t2b) +
                                         int(threadIdx.x % kOrb), nv - 1)];
    typedef typename std::conditional<sizeof(CubeT) == 8, d2v, f2v>::type CV2;
    typedef typename std::conditional<sizeof(InT) == 8, d2v, f2v>::type IV2;
    const bool even_nv = (nv & 1) == 0;
    constexpr int kPer = 6 * E / 256;
    constexpr int kBatch = sizeof(CubeT) == 4 && sizeof(InT) == 4 ? kPer : kPer / 2;
#pragma unroll
    for (int m0 = 0; m0 < kPer; m0 += kBatch) {
      CubeT lw1[kBatch], lw2[kBatch];
      InT lij[kBatch], lik[kBatch], ljk[kBatch], lti[kBatch], ltj[kBatch], ltk[kBatch];
      // elements 2q and 2q + 1 of a batch are this thread's (x, y, z0) and
      // (x, y, z0 + 1) of one slot, adjacent along c: with n_v even their
      // cube values are one two-element load each (an in-range even c0 has
      // c0 + 1 < n_v), and so are (ia|kc), (jb|kc) with aligned ovov rows
#pragma unroll
      for (int q = 0; q < kBatch / 2; ++q) {
        const int m = 2 * q;
        const int idx = threadIdx.x + 256 * (m0 + m);
        const int s = idx / E, e = orb_elem(idx - s * E);
        int p0, p1, p2;
        slot_perm(s, p0, p1, p2);
        const int64_t a = min(kOrb * pick3(p0, t0, t1b, t2b) + (e >> 6), nv - 1);
        const int64_t b = min(kOrb * pick3(p1, t0, t1b, t2b) + ((e >> 3) & 7), nv - 1);
        const int cr = kOrb * pick3(p2, t0, t1b, t2b) + (e & 7);   // even
        lij[m] = lij[m + 1] = gptr(ov_ij)[a * nonv + b];
        lti[m] = lti[m + 1] = gptr(t1i)[a];
        ltj[m] = ltj[m + 1] = gptr(t1j)[b];
#pragma unroll
        for (int h = 0; h < 2; ++h) ltk[m + h] = gptr(t1k)[min(cr + h, nv - 1)];
        if (even_nv) {
          const int64_t c = min(cr, nv - 2);
          const CV2 u = *(const SIE_GLOBAL CV2*)(gptr(w1) + (a * nv + b) * nv + c);
          const CV2 v = *(const SIE_GLOBAL CV2*)(gptr(w2) + (b * nv + a) * nv + c);
          lw1[m] = u.x;
          lw1[m + 1] = u.y;
          lw2[m] = v.x;
          lw2[m + 1] = v.y;
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int64_t c = min(cr + h, nv - 1);
            lw1[m + h] = gptr(w1)[(a * nv + b) * nv + c];
            lw2[m + h] = gptr(w2)[(b * nv + a) * nv + c];
          }
        }
        if (fd.epv) {
          const int64_t c = min(cr, nv - 2);
          const IV2 u = *(const SIE_GLOBAL IV2*)(gptr(ov_ik) + a * nonv + c);
          const IV2 v = *(const SIE_GLOBAL IV2*)(gptr(ov_jk) + b * nonv + c);
          lik[m] = u.x;
          lik[m + 1] = u.y;
          ljk[m] = v.x;
          ljk[m + 1] = v.y;
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int64_t c = min(cr + h, nv - 1);
            lik[m + h] = gptr(ov_ik)[a * nonv + c];
            ljk[m + h] = gptr(ov_jk)[b * nonv + c];
          }
        }
      }
#pragma unroll
      for (int m = 0; m < kBatch; ++m) {
        const int idx = threadIdx.x + 256 * (m0 + m);
        const int s = idx / E, e = orb_elem(idx - s * E);
        int p0, p1, p2;
        slot_perm(s, p0, p1, p2);
        const int a = kOrb * pick3(p0, t0, t1b, t2b) + (e >> 6);
        const int b = kOrb * pick3(p1, t0, t1b, t2b) + ((e >> 3) & 7);
        const int c = kOrb * pick3(p2, t0, t1b, t2b) + (e & 7);
        double w = 0.0, z = 0.0;
        if (a < nv && b < nv && c < nv) {
          w = (double)lw1[m] + (double)lw2[m];
          const double vt = (double)lij[m] * (double)ltk[m] + (double)lik[m] * (double)ltj[m] +
                            (double)ljk[m] * (double)lti[m];
          z = w + vt;
        }
        sw[s][orb_lds(e >> 6, (e >> 3) & 7, e & 7)] = w;
        sz[s][orb_lds(e >> 6, (e >> 3) & 7, e & 7)] = z;
      }
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
    // G, H and Gt of this thread's two elements (x, y, z0 + h), h = 0, 1, of
    // each slot (the elements of iterations 2s and 2s + 1 of the loads
    // above), adjacent along c: with n_v even each cube takes one
    // two-element store
    const int x = threadIdx.x >> 5, y = (threadIdx.x >> 2) & 7, z0 = 2 * (threadIdx.x & 3);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      if (!((primary >> s) & 1u)) continue;
      int p0, p1, p2;
      slot_perm(s, p0, p1, p2);
      const int a = kOrb * pick3(p0, t0, t1b, t2b) + x;
      const int b = kOrb * pick3(p1, t0, t1b, t2b) + y;
      const int c0 = kOrb * pick3(p2, t0, t1b, t2b) + z0;
      if (a >= nv || b >= nv || c0 >= nv) continue;
      const int s_cab = orbit_slot(p2, p0, p1), s_bca = orbit_slot(p1, p2, p0);
      const int s_cba = orbit_slot(p2, p1, p0), s_acb = orbit_slot(p0, p2, p1);
      const int s_bac = orbit_slot(p1, p0, p2);
      CubeT vg[2], vh[2], vt[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int zz = z0 + h;
        const int e_abc = orb_lds(x, y, zz);
        const int e_cab = orb_lds(zz, x, y), e_bca = orb_lds(y, zz, x);
        const int e_cba = orb_lds(zz, y, x), e_acb = orb_lds(x, zz, y);
        const int e_bac = orb_lds(y, x, zz);
        const double rz = 4.0 * sz[s][e_abc] + sz[s_cab][e_cab] + sz[s_bca][e_bca] -
                          2.0 * (sz[s_cba][e_cba] + sz[s_acb][e_acb] + sz[s_bac][e_bac]);
        const double rw = 4.0 * sw[s][e_abc] + sw[s_cab][e_cab] + sw[s_bca][e_bca] -
                          2.0 * (sw[s_cba][e_cba] + sw[s_acb][e_acb] + sw[s_bac][e_bac]);
        const double id =
            recip(eijk - sev[p0 * kOrb + x] - sev[p1 * kOrb + y] - sev[p2 * kOrb + zz]);   // 1 / D
        if (c0 + h < nv) acc += sw[s][e_abc] * rz * id;
        vg[h] = CubeT(scale * (rw + rz) * id);
        vh[h] = CubeT(scale * rw * id);
        // G at (c, b, a), stored at this thread's (a, b, c) of the transposed
        // cube (contiguous across the wave); R' at (c, b, a) combines the same
        // six permuted values with the roles of (abc, cba), (cab, acb) and
        // (bca, bac) exchanged.
        const double rz_t = 4.0 * sz[s_cba][e_cba] + sz[s_acb][e_acb] + sz[s_bac][e_bac] -
                            2.0 * (sz[s][e_abc] + sz[s_cab][e_cab] + sz[s_bca][e_bca]);
        const double rw_t = 4.0 * sw[s_cba][e_cba] + sw[s_acb][e_acb] + sw[s_bac][e_bac] -
                            2.0 * (sw[s][e_abc] + sw[s_cab][e_cab] + sw[s_bca][e_bca]);
        vt[h] = CubeT(scale * (rw_t + rz_t) * id);
      }
      const int64_t pos = ((int64_t)a * nv + b) * nv + c0;
      if (even_nv) {
        *(SIE_GLOBAL CV2*)(gptr_w(w1) + pos) = CV2{vg[0], vg[1]};
        *(SIE_GLOBAL CV2*)(gptr_w(w2) + pos) = CV2{vh[0], vh[1]};
        *(SIE_GLOBAL CV2*)(gptr_w(w3) + pos) = CV2{vt[0], vt[1]};
      } else {
        gptr_w(w1)[pos] = vg[0];
        gptr_w(w2)[pos] = vh[0];
        gptr_w(w3)[pos] = vt[0];
        if (c0 + 1 < nv) {
          gptr_w(w1)[pos + 1] = vg[1];
          gptr_w(w2)[pos + 1] = vh[1];
          gptr_w(w3)[pos + 1] = vt[1];
        }
      }
    }
    if (want_eps) {
      // tuples: threads t and t + 256 take slot-0 offsets e = x*64 + y*8 + z
      // (x = wave + 4 m, so position 0's marginal is a whole-wave sum)
      const bool eqAB = t0 == t1b, eqBC = t1b == t2b;
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int e = threadIdx.x + 256 * m;
        const int ox = e >> 6, oy = (e >> 3) & 7, oz = e & 7;
        const int a = kOrb * t0 + ox, b = kOrb * t1b + oy, c = kOrb * t2b + oz;
        double q = 0.0;
        if (!((eqAB && ox < oy) || (eqBC && oy < oz)) && a < nv && b < nv && c < nv) {
          const int s0 = orbit_slot(0, 1, 2), e0 = orb_lds(ox, oy, oz);
          const int s1 = orbit_slot(1, 2, 0), e1 = orb_lds(oy, oz, ox);
          const int s2 = orbit_slot(2, 0, 1), e2 = orb_lds(oz, ox, oy);
          const int s3 = orbit_slot(0, 2, 1), e3 = orb_lds(ox, oz, oy);
          const int s4 = orbit_slot(1, 0, 2), e4 = orb_lds(oy, ox, oz);
          const int s5 = orbit_slot(2, 1, 0), e5 = orb_lds(oz, oy, ox);
          const double w0 = sw[s0][e0], w1v = sw[s1][e1], w2v = sw[s2][e2];
          const double w3v = sw[s3][e3], w4 = sw[s4][e4], w5 = sw[s5][e5];
          const double z0 = sz[s0][e0], z1 = sz[s1][e1], z2 = sz[s2][e2];
          const double z3 = sz[s3][e3], z4 = sz[s4][e4], z5 = sz[s5][e5];
          const double wz = w0 * z0 + w1v * z1 + w2v * z2 + w3v * z3 + w4 * z4 + w5 * z5;
          const double we = w0 + w1v + w2v, wo = w3v + w4 + w5;
          const double ze = z0 + z1 + z2, zo = z3 + z4 + z5;
          const double f = 3.0 * wz - 0.5 * (we + wo) * (ze + zo) + 1.5 * (we - wo) * (ze - zo);
          const int eq = (a == b) + (b == c) + (a == c);
          const double wt = eq == 0 ? 1.0 : (eq == 1 ? 0.5 : 1.0 / 6.0);
          const double id = recip(eijk - sev[ox] - sev[kOrb + oy] - sev[2 * kOrb + oz]);
          q = scale * wt * f * id * id;
        }
        eacc += q;
        double s0v = q, s1v = q, s2v = q;
        for (int off = 32; off > 0; off >>= 1) s0v += __shfl_xor(s0v, off, 64);   // all lanes
        for (int off = 1; off < 8; off <<= 1) s1v += __shfl_xor(s1v, off, 64);   // same oy
        for (int off = 8; off < 64; off <<= 1) s2v += __shfl_xor(s2v, off, 64);  // same oz
        if (lane == 0) tp0[m][wave] = s0v;
        if ((lane & 7) == 0) tp1[m][wave][lane >> 3] = s1v;
        if (lane < 8) tp2[m][wave][lane] = s2v;
      }
      __syncthreads();
      if (threadIdx.x < kOrb) {
        const int o = threadIdx.x;
        const double p0 = tp0[o >> 2][o & 3];
        double p1 = 0.0, p2 = 0.0;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            p1 += tp1[m][w][o];
            p2 += tp2[m][w][o];
          }
        // one thread per offset adds the three positions in order, so equal
        // blocks (t0 = t1b or t1b = t2b) add into one entry one after another
        const int a = kOrb * t0 + o, b = kOrb * t1b + o, c = kOrb * t2b + o;
        if (a < nv) dv[a] += p0;
        if (b < nv) dv[b] += p1;
        if (c < nv) dv[c] += p2;
      }
    }
    __syncthreads();
  }
  const double s = block_sum_256(acc, red);
  if (threadIdx.x == 0) *out = s;
  if (want_eps) {
    const double se = block_sum_256(eacc, red);
    if (threadIdx.x == 0) eo_part[(fd.unit_base + it.unit) * pstride + slot] = se;
    for (int a = threadIdx.x; a < nv; a += 256) ev_row[a] = dv[a];
  }
}


// ---------------------------------------------------------------------------
// Contractions of G: output-stationary grouped products on the FP64 matrix
// cores.
// ---------------------------------------------------------------------------

// Element (beta, x, k) of the A side (rows, always G or its transpose) is
// a[beta*a_b + x*a_x + k*a_k]; of the B side (cols) b[beta*b_b + x*b_x +
// k*b_k] times `scale`, with b_b = 0 when the B side is shared by all blocks.
template <typename CubeT, typename InT>
struct ATerm {
  const CubeT* a;
  int64_t a_b, a_x, a_k;
  const InT* b;
  int64_t b_b, b_x, b_k;
  double scale;
  int nblk;            // valid blocks (summed-block classes)
};

// Term `kind` of class CLS for unit (i, j, k) at tile origin (blk0, row0,
// col0); block group g (summed-block classes).  G[a][b][c] has strides
// (nv^2, nv, 1), its transpose Gt[a][b][c] = G(c, b, a) has (1, nv, nv^2) in
// G's (a, b, c): for each kind the layout giving unit stride along the rows
// or K is used.
template <int CLS, typename CubeT, typename InT>
__device__ __forceinline__ ATerm<CubeT, InT> make_adj(int kind, int g, int i, int j, int k, int no_,
                                                      int nv_, const CubeT* G, const CubeT* Gt,
                                                      const InT* t2, const InT* ovvv,
                                                      const InT* ooov, int blk0, int row0,
                                                      int col0) {
  const int64_t nv = nv_, no = no_, nv2 = nv * nv;
  const int64_t sA = nv2, sB = nv, sC = 1;       // strides of a, b, c in G
  const int64_t tA = 1, tB = nv, tC = nv2;       // ... in Gt
  ATerm<CubeT, InT> t;
  t.scale = 1.0;
  t.nblk = kABlk;
  if (CLS == kAdjOvvv) {
    // dovvv[x][p][q][d] += sum_r Gperm[p][q][r] t2[s1][s2][r][d], t2 read as
    // its twin t2[s2][s1][d][r] (K contiguous)
    const bool tr = kind == 2 || kind == 4;
    const int64_t Sb = tr ? tC : pick6(kind, sA, sA, sC, sB, sC, sB);
    const int64_t Sx = tr ? pick6<int64_t>(kind, 0, 0, tA, 0, tB, 0) : pick6(kind, sB, sC, sA, sC, sB, sA);
    const int64_t Sk = tr ? pick6<int64_t>(kind, 0, 0, tB, 0, tA, 0) : pick6(kind, sC, sB, sB, sA, sA, sC);
    const int64_t s1 = pick6(kind, k, j, j, i, i, k), s2 = pick6(kind, j, k, i, k, j, i);
    t.a = (tr ? Gt : G) + blk0 * Sb + row0 * Sx;
    t.a_b = Sb; t.a_x = Sx; t.a_k = Sk;
    t.b = t2 + (s2 * no + s1) * nv2 + col0 * nv;
    t.b_b = 0; t.b_x = nv; t.b_k = 1;
  } else if (CLS == kAdjT2oo) {
    // dt2[p][l][y][z] += -sum_K Gperm[y][z][K] ooov[m][l][n][K]
    const bool tr = kind == 2 || kind == 3;
    const int64_t Sy = tr ? tC : pick6(kind, sA, sA, sC, sC, sB, sB);
    const int64_t Sz = tr ? pick6<int64_t>(kind, 0, 0, tA, tB, 0, 0) : pick6(kind, sC, sB, sA, sB, sC, sA);
    const int64_t SK = tr ? pick6<int64_t>(kind, 0, 0, tB, tA, 0, 0) : pick6(kind, sB, sC, sB, sA, sA, sC);
    const int64_t m = pick6(kind, k, j, i, j, k, i), n = pick6(kind, j, k, j, i, i, k);
    t.a = (tr ? Gt : G) + blk0 * Sy + row0 * Sz;
    t.a_b = Sy; t.a_x = Sz; t.a_k = SK;
    t.b = ooov + ((m * no + col0) * no + n) * nv;
    t.b_b = 0; t.b_x = no * nv; t.b_k = 1;
    t.scale = -1.0;
  } else if (CLS == kAdjT2vv) {
    // dt2[s1][s2][r][d] += sum_{k1, k2} Gperm[k1][r][k2] ovvv[x][..k1..k2..][d]
    const int64_t Ab = pick6(kind, sA, sA, sA, sB, sB, sA);
    const int64_t Ax = pick6(kind, sC, sB, sB, sA, sA, sC);
    const int64_t Ak = pick6(kind, sB, sC, sC, sC, sC, sB);
    const int64_t Bb = pick6(kind, nv2, nv2, nv, nv2, nv, nv);
    const int64_t Bk = pick6(kind, nv, nv, nv2, nv, nv2, nv2);
    const int64_t x = pick6(kind, i, i, k, j, k, j);
    const int64_t k10 = int64_t(g) * kARB;
    t.a = G + k10 * Ab + row0 * Ax;
    t.a_b = Ab; t.a_x = Ax; t.a_k = Ak;
    t.b = ovvv + x * nv2 * nv + k10 * Bb + col0;
    t.b_b = Bb; t.b_x = 1; t.b_k = Bk;
    t.nblk = nv_ - int(k10) < kARB ? nv_ - int(k10) : kARB;
  } else {   // kAdjOoov
    // dooov[m][l][n][x] += -sum_{k1, k2} Gperm[k1][x][k2] t2[..l..][k1][k2]
    const int64_t Ab = pick6(kind, sA, sA, sA, sB, sB, sA);
    const int64_t Ax = pick6(kind, sB, sC, sB, sA, sA, sC);
    const int64_t Ak = pick6(kind, sC, sB, sC, sC, sC, sB);
    const int64_t base = pick6(kind, i * no * nv2, i * no * nv2, k * nv2, k * nv2, j * no * nv2,
                               j * nv2);
    const int64_t Bl = pick6(kind, nv2, nv2, no * nv2, no * nv2, nv2, no * nv2);
    const int64_t k10 = int64_t(g) * kARB;
    t.a = G + k10 * Ab + row0 * Ax;
    t.a_b = Ab; t.a_x = Ax; t.a_k = Ak;
    t.b = t2 + base + col0 * Bl + k10 * nv;
    t.b_b = nv; t.b_x = Bl; t.b_k = 1;
    t.scale = -1.0;
    t.nblk = nv_ - int(k10) < kARB ? nv_ - int(k10) : kARB;
  }
  return t;
}

// Registers of one K-chunk for one wave: A side (G) for BLK blocks x TRW
// row tiles, B side for BLK blocks (or the shared row) x TCW col tiles, as
// loaded; m: the B-side factor per k of the pair (the term's scale, 0 past
// K), applied when the chunk is consumed so that issuing the next chunk's
// loads never waits for them (A needs no zeros: B's cancel it).
template <int BLK, int TRW, int TCW>
struct AChunk {
  double a[BLK][TRW][2];
  double b[BLK][TCW][2];
  double m[2];
};

// Element at byte offset `off` from a wave-uniform base (32-bit lane
// offsets; the host limits operand extents to 4 GiB, see check_fragment).
template <typename T>
__device__ __forceinline__ T aload(const void* base, uint32_t off) {
  return *(const SIE_GLOBAL T*)(gptr(reinterpret_cast<const char*>(base)) + off);
}

// The lane's k-pair (k, k+1) of one row (byte offset `row` from `base`, K
// stride ks elements), as loaded; k past nK reads nK - 1 (in bounds; the
// chunk's factor zeroes it).  `vec`: unit stride and 16-byte aligned pairs.
template <typename T>
__device__ __forceinline__ void apair(const T* base, uint32_t row, int64_t ks, int k, int nK,
                                      bool vec, double (&out)[2]) {
  if (vec && k + 1 < nK) {
    const uint32_t o = row + uint32_t(k) * uint32_t(sizeof(T));
    if (sizeof(T) == 8) {
      const d2v v = aload<d2v>(base, o);
      out[0] = v.x;
      out[1] = v.y;
    } else {
      out[0] = (double)aload<T>(base, o);
      out[1] = (double)aload<T>(base, o + uint32_t(sizeof(T)));
    }
  } else {
    const uint32_t kb = uint32_t(ks * int64_t(sizeof(T)));
    const uint32_t k0 = uint32_t(k < nK ? k : nK - 1);
    const uint32_t k1 = uint32_t(k + 1 < nK ? k + 1 : nK - 1);
    out[0] = (double)aload<T>(base, row + k0 * kb);
    out[1] = (double)aload<T>(base, row + k1 * kb);
  }
}

// Lane rows of one term: clamped A-side rows x_rt and B-side rows x_ct;
// blocks past nblk read block 0 (their results are not stored).
template <int BLK, int TRW, int TCW, typename CubeT, typename InT>
__device__ __forceinline__ void adj_load(const ATerm<CubeT, InT>& t, bool reduce, int c, int nK,
                                         int nrow, int ncol, int nblk, int r, int g, bool vec,
                                         AChunk<BLK, TRW, TCW>& x) {
  const int k = c * kAKc + 2 * g;
  const bool va = vec && t.a_k == 1, vb = vec && t.b_k == 1;
  x.m[0] = k < nK ? t.scale : 0.0;
  x.m[1] = k + 1 < nK ? t.scale : 0.0;
#pragma unroll
  for (int rt = 0; rt < TRW; ++rt) {
    const uint32_t xr = uint32_t(min(16 * rt + r, nrow - 1) * t.a_x * int64_t(sizeof(CubeT)));
#pragma unroll
    for (int beta = 0; beta < BLK; ++beta)
      apair(t.a + (beta < nblk ? beta : 0) * t.a_b, xr, t.a_k, k, nK, va, x.a[beta][rt]);
  }
#pragma unroll
  for (int ct = 0; ct < TCW; ++ct) {
    const uint32_t xc = uint32_t(min(16 * ct + r, ncol - 1) * t.b_x * int64_t(sizeof(InT)));
    if (reduce) {
#pragma unroll
      for (int beta = 0; beta < BLK; ++beta)
        apair(t.b + (beta < nblk ? beta : 0) * t.b_b, xc, t.b_k, k, nK, vb, x.b[beta][ct]);
    } else {
      apair(t.b, xc, t.b_k, k, nK, vb, x.b[0][ct]);
    }
  }
}

// acc[beta][rt][ct] += A[beta][rt] * B[beta or shared][ct] over the chunk;
// row / col tiles wholly outside the output (uniform) are skipped.
template <int BLK, int TRW, int TCW>
__device__ __forceinline__ void adj_mma(const AChunk<BLK, TRW, TCW>& x, bool reduce, int nrow,
                                        int ncol, d4 (&acc)[BLK][TRW][TCW]) {
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    double b[BLK][TCW];
#pragma unroll
    for (int beta = 0; beta < (reduce ? BLK : 1); ++beta)
#pragma unroll
      for (int ct = 0; ct < TCW; ++ct) b[beta][ct] = x.b[beta][ct][s] * x.m[s];
#pragma unroll
    for (int rt = 0; rt < TRW; ++rt)
#pragma unroll
      for (int ct = 0; ct < TCW; ++ct) {
        if ((rt > 0 && 16 * rt >= nrow) || (ct > 0 && 16 * ct >= ncol)) continue;
#pragma unroll
        for (int beta = 0; beta < BLK; ++beta)
          acc[beta][rt][ct] =
              mfma16x16x4(x.a[beta][rt][s], b[reduce ? beta : 0][ct], acc[beta][rt][ct]);
      }
  }
}

struct AdjOut {
  double* out;
  int64_t ob, orow, ocol;
  int nb, nr, nc;        // output extent: blocks, rows, cols
};

template <int CLS>
__device__ __forceinline__ AdjOut adj_out(const FragDesc& fd, const AdjGroup& gr) {
  const int64_t nv = fd.nv, no = fd.no, nv2 = nv * nv;
  AdjOut o;
  if (CLS == kAdjOvvv) {
    o.out = fd.g_ovvv + gr.a0 * nv2 * nv;
    o.ob = nv2; o.orow = nv; o.ocol = 1;
    o.nb = fd.nv; o.nr = fd.nv; o.nc = fd.nv;
  } else if (CLS == kAdjT2oo) {
    o.out = fd.g_t2 + gr.a0 * no * nv2;
    o.ob = nv; o.orow = 1; o.ocol = nv2;
    o.nb = fd.nv; o.nr = fd.nv; o.nc = fd.no;
  } else if (CLS == kAdjT2vv) {
    o.out = fd.g_t2 + (gr.a0 * no + gr.a1) * nv2;
    o.ob = 0; o.orow = nv; o.ocol = 1;
    o.nb = 1; o.nr = fd.nv; o.nc = fd.nv;
  } else {
    o.out = fd.g_ooov + (gr.a0 * no * no + gr.a1) * nv;
    o.ob = 0; o.orow = 1; o.ocol = no * nv;
    o.nb = 1; o.nr = fd.nv; o.nc = fd.no;
  }
  return o;
}

// Wave tile of a class: BLK blocks x TRW x TCW 16-wide MFMA tiles.  The
// summed-block classes run the summed virtual one block at a time through
// K (BLK = 1).
template <int CLS>
struct AdjWave {
  static constexpr bool kReduce = CLS == kAdjT2vv || CLS == kAdjOoov;
  static constexpr bool kKSplit = CLS == kAdjOoov;   // waves split the stream
  static constexpr int BLK = kReduce ? 1 : kABlk;
  static constexpr int TRW = adj_trw(CLS);
  static constexpr int TCW = adj_tcw(CLS);
};

__device__ __forceinline__ int find_group(const AdjGroup* __restrict__ gs, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (gs[mid].wg_end > x) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Position in a group's chunk stream: record `rec`, summed virtual `kb` of
// its block group (summed-block classes; 0 otherwise), K chunk `c`; `tm` is
// the record's term.
template <typename CubeT, typename InT>
struct AdjPos {
  int rec, kb, c;
  ATerm<CubeT, InT> tm;
};

// Grid: the concatenated tiles of the launch's groups.  Block: 256 threads.
// arena holds per unit G, H and Gt (cube_off, + half, + 2 half).  Per-block
// classes add their tile into the gradient (read-modify-write: a slice's
// groups run in separate launches of successive rounds only); summed-block
// classes store their tile of the group's partial slice into parts (at
// gr.part_off, o.nr x o.nc row-major), summed by k_adj_part_sum.
template <int CLS, typename CubeT, typename InT>
__global__ __launch_bounds__(kAThreads, CLS == kAdjT2vv ? 1 : 2) void k_adj_contract(
    const FragDesc* __restrict__ descs, const Item* __restrict__ items,
    const AdjGroup* __restrict__ groups, int n_groups, const AdjRec* __restrict__ recs,
    const CubeT* __restrict__ arena, double* __restrict__ parts) {
  using W = AdjWave<CLS>;
  constexpr bool kReduce = W::kReduce, kKSplit = W::kKSplit;
  constexpr int BLK = W::BLK, TRW = W::TRW, TCW = W::TCW;
  const int gi = find_group(groups, n_groups, blockIdx.x);
  const AdjGroup gr = groups[gi];
  const int64_t start = gi ? groups[gi - 1].wg_end : 0;
  const FragDesc fd = descs[gr.frag];
  const int no = fd.no, nv = fd.nv;
  const AdjOut o = adj_out<CLS>(fd, gr);
  int TB, TR, TC;
  adj_tile_shape(CLS, TB, TR, TC);
  const int nrt = (o.nr + TR - 1) / TR, nct = (o.nc + TC - 1) / TC;
  const int ntile = int(adj_tiles(CLS, no, nv));
  int t = xcd_tile(int(int64_t(blockIdx.x) - start), ntile);
  const int tb = t / (nrt * nct);
  t -= tb * nrt * nct;
  const int trow = t / nct, tcol = t - trow * nct;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int r = lane & 15, g = lane >> 4;
  // this wave's part of the tile: its own blocks (per-block classes), its
  // own sub-tile (t2 from the d-sums), or the whole tile and every fourth
  // chunk (ooov)
  const int blk0 = kReduce ? 0 : tb * TB + wave * kABlk;
  const int row0 = trow * TR + (adj_wr(CLS) > 1 ? (wave & 1) * 16 * TRW : 0);
  const int col0 = tcol * TC + (adj_wc(CLS) > 1 ? (wave >> 1) * 16 * TCW : 0);
  // work-group-uniform where the waves meet at barriers below (ooov)
  if ((!kReduce && blk0 >= o.nb) || row0 >= o.nr || col0 >= o.nc) return;
  const int nrow = min(16 * TRW, o.nr - row0), ncol = min(16 * TCW, o.nc - col0);
  const int nblk_tile = kReduce ? 1 : min(kABlk, o.nb - blk0);
  const bool vec = fd.vec != 0;

  d4 acc[BLK][TRW][TCW];
#pragma unroll
  for (int b = 0; b < BLK; ++b)
#pragma unroll
    for (int p = 0; p < TRW; ++p)
#pragma unroll
      for (int q = 0; q < TCW; ++q) acc[b][p][q] = d4{0.0, 0.0, 0.0, 0.0};

  const InT* t2p = static_cast<const InT*>(fd.t2);
  const InT* ovvvp = static_cast<const InT*>(fd.ovvv);
  const InT* ooovp = static_cast<const InT*>(fd.ooov);
  const int nchunk = (nv + kAKc - 1) / kAKc;

  auto term = [&](int rec) {
    const AdjRec rr = recs[rec];
    const Item it = items[rr.item];
    int i, j, k;
    decode_sorted_triple(it.unit, no, i, j, k);
    const CubeT* G = arena + it.cube_off;
    return make_adj<CLS, CubeT, InT>(rr.kind, rr.g, i, j, k, no, nv, G, G + 2 * fd.half, t2p,
                                     ovvvp, ooovp, blk0, row0, col0);
  };
  // advance a position by `step` chunks of the stream
  auto advance = [&](AdjPos<CubeT, InT>& p, int step) {
    p.c += step;
    while (p.c >= nchunk && p.rec < gr.rec_end) {
      p.c -= nchunk;
      if (kReduce && ++p.kb < p.tm.nblk) continue;
      p.kb = 0;
      if (++p.rec < gr.rec_end) p.tm = term(p.rec);
    }
  };
  auto load = [&](const AdjPos<CubeT, InT>& p, AChunk<BLK, TRW, TCW>& x) {
    if (kReduce) {
      ATerm<CubeT, InT> t1 = p.tm;
      t1.a += p.kb * p.tm.a_b;
      t1.b += p.kb * p.tm.b_b;
      adj_load(t1, true, p.c, nv, nrow, ncol, 1, r, g, vec, x);
    } else {
      adj_load(p.tm, false, p.c, nv, nrow, ncol, nblk_tile, r, g, vec, x);
    }
  };

  if (gr.rec_begin < gr.rec_end) {
    // one stream over the group's records with two chunks in flight
    AdjPos<CubeT, InT> p;
    p.rec = gr.rec_begin;
    p.kb = 0;
    p.c = 0;
    p.tm = term(p.rec);
    const int step = kKSplit ? 4 : 1;
    if (kKSplit) advance(p, wave);
    AChunk<BLK, TRW, TCW> b0, b1;
    bool have = p.rec < gr.rec_end;
    if (have) load(p, b0);
    while (have) {
      advance(p, step);
      const bool have1 = p.rec < gr.rec_end;
      if (have1) load(p, b1);
      adj_mma(b0, kReduce, nrow, ncol, acc);
      if (!have1) break;
      advance(p, step);
      have = p.rec < gr.rec_end;
      if (have) load(p, b0);
      adj_mma(b1, kReduce, nrow, ncol, acc);
    }
  }

  if (kKSplit) {
    // (acc0 + acc2) + (acc1 + acc3) through LDS, a fixed order
    constexpr int NV = kKSplit ? TRW * TCW * 4 : 1;
    __shared__ double red[2][NV][64];
    if (wave >= 2) {
#pragma unroll
      for (int rt = 0; rt < TRW; ++rt)
#pragma unroll
        for (int ct = 0; ct < TCW; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) red[wave - 2][(rt * TCW + ct) * 4 + v][lane] = acc[0][rt][ct][v];
    }
    __syncthreads();
    if (wave < 2) {
#pragma unroll
      for (int rt = 0; rt < TRW; ++rt)
#pragma unroll
        for (int ct = 0; ct < TCW; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[0][rt][ct][v] += red[wave][(rt * TCW + ct) * 4 + v][lane];
    }
    __syncthreads();
    if (wave == 1) {
#pragma unroll
      for (int rt = 0; rt < TRW; ++rt)
#pragma unroll
        for (int ct = 0; ct < TCW; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) red[0][(rt * TCW + ct) * 4 + v][lane] = acc[0][rt][ct][v];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int rt = 0; rt < TRW; ++rt)
#pragma unroll
      for (int ct = 0; ct < TCW; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[0][rt][ct][v] += red[0][(rt * TCW + ct) * 4 + v][lane];
  }

  // acc[beta][rt][ct][v] = out[blk0 + beta][row0 + 16 rt + 4 v + g][col0 + 16 ct + r]
#pragma unroll
  for (int rt = 0; rt < TRW; ++rt)
#pragma unroll
    for (int ct = 0; ct < TCW; ++ct) {
      const int col = col0 + 16 * ct + r;
      if (kReduce) {
        SIE_GLOBAL double* pp = gptr_w(parts) + gr.part_off;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + 16 * rt + 4 * v + g;
          if (row < o.nr && col < o.nc) pp[int64_t(row) * o.nc + col] = acc[0][rt][ct][v];
        }
      } else {
#pragma unroll
        for (int beta = 0; beta < BLK; ++beta) {
          const int blk = blk0 + beta;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = row0 + 16 * rt + 4 * v + g;
            if (blk < o.nb && row < o.nr && col < o.nc) {
              SIE_GLOBAL double* p = gptr_w(o.out) + blk * o.ob + row * o.orow + col * o.ocol;
              *p = *p + acc[beta][rt][ct][v];
            }
          }
        }
      }
    }
}

// gradient slice += sum of its partial slices, in slot order (fixed), for
// the summed-block classes.  Grid: (element chunks of 256, slices).
template <int CLS>
__global__ __launch_bounds__(256) void k_adj_part_sum(const FragDesc* __restrict__ descs,
                                                      const AdjSlice* __restrict__ slices,
                                                      const double* __restrict__ parts) {
  const AdjSlice sl = slices[blockIdx.y];
  const FragDesc fd = descs[sl.frag];
  AdjGroup gr{};
  gr.a0 = sl.a0;
  gr.a1 = sl.a1;
  const AdjOut o = adj_out<CLS>(fd, gr);
  const int64_t n = int64_t(o.nr) * o.nc;
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= n) return;
  double s = 0.0;
  for (int q = 0; q < sl.nparts; ++q) s += gptr(parts)[sl.off0 + int64_t(q) * n + e];
  const int row = int(e / o.nc), col = int(e - int64_t(row) * o.nc);
  SIE_GLOBAL double* p = gptr_w(o.out) + row * o.orow + col * o.ocol;
  *p = *p + s;
}

// ---------------------------------------------------------------------------
// Contractions of H (memory-bound; one output element per thread or per
// fixed-order block reduction).
// ---------------------------------------------------------------------------

// dovov[p][y][q][z] += sum over the third virtual of H t1.  Block: 256
// threads, one (y, z) element each.
template <typename CubeT, typename InT>
__global__ __launch_bounds__(256) void k_adj_ovov(const FragDesc* __restrict__ descs,
                                                  const Item* __restrict__ items,
                                                  const AdjGroup* __restrict__ groups,
                                                  int n_groups, const AdjRec* __restrict__ recs,
                                                  const CubeT* __restrict__ arena) {
  const int gi = find_group(groups, n_groups, blockIdx.x);
  const AdjGroup gr = groups[gi];
  const int64_t start = gi ? groups[gi - 1].wg_end : 0;
  const FragDesc fd = descs[gr.frag];
  const int no = fd.no, nv = fd.nv;
  const int64_t e = (int64_t(blockIdx.x) - start) * 256 + threadIdx.x;
  if (e >= int64_t(nv) * nv) return;
  const int y = int(e / nv), z = int(e - int64_t(y) * nv);
  const InT* t1 = static_cast<const InT*>(fd.t1);
  const int64_t nv2 = int64_t(nv) * nv;
  double s = 0.0;
  for (int q = gr.rec_begin; q < gr.rec_end; ++q) {
    const AdjRec rr = recs[q];
    const Item it = items[rr.item];
    int i, j, k;
    decode_sorted_triple(it.unit, no, i, j, k);
    const CubeT* H = arena + it.cube_off + fd.half;
    // (y, z) = (a, b): sum_c H[a][b][c] t1[k][c]; (a, c): sum_b H[a][b][c]
    // t1[j][b]; (b, c): sum_a H[a][b][c] t1[i][a] -- a dot product of
    // stride hs with a t1 row, in four interleaved partial sums (more loads
    // in flight) added in a fixed order
    const SIE_GLOBAL CubeT* h;
    const SIE_GLOBAL InT* tv;
    int64_t hs;
    if (rr.kind == 0) {
      h = gptr(H) + y * nv2 + int64_t(z) * nv;
      tv = gptr(t1) + int64_t(k) * nv;
      hs = 1;
    } else if (rr.kind == 1) {
      h = gptr(H) + y * nv2 + z;
      tv = gptr(t1) + int64_t(j) * nv;
      hs = nv;
    } else {
      h = gptr(H) + int64_t(y) * nv + z;
      tv = gptr(t1) + int64_t(i) * nv;
      hs = nv2;
    }
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
    int u = 0;
    if (hs == 1 && (nv & 1) == 0) {
      // kind 0, rows of even length: the row starts at an even element, so
      // (u, u + 1) is one two-element load (same products, same sums)
      typedef typename std::conditional<sizeof(CubeT) == 8, d2v, f2v>::type CV2;
      for (; u + 4 <= nv; u += 4) {
        const CV2 h01 = *(const SIE_GLOBAL CV2*)(h + u);
        const CV2 h23 = *(const SIE_GLOBAL CV2*)(h + u + 2);
        p0 += (double)h01.x * (double)tv[u];
        p1 += (double)h01.y * (double)tv[u + 1];
        p2 += (double)h23.x * (double)tv[u + 2];
        p3 += (double)h23.y * (double)tv[u + 3];
      }
    }
    for (; u + 4 <= nv; u += 4) {
      p0 += (double)h[int64_t(u) * hs] * (double)tv[u];
      p1 += (double)h[int64_t(u + 1) * hs] * (double)tv[u + 1];
      p2 += (double)h[int64_t(u + 2) * hs] * (double)tv[u + 2];
      p3 += (double)h[int64_t(u + 3) * hs] * (double)tv[u + 3];
    }
    for (; u < nv; ++u) p0 += (double)h[int64_t(u) * hs] * (double)tv[u];
    s += (p0 + p1) + (p2 + p3);
  }
  SIE_GLOBAL double* p = gptr_w(fd.g_ovov) + ((int64_t(gr.a0) * nv + y) * no + gr.a1) * nv + z;
  *p = *p + s;
}

__device__ __forceinline__ double block_sum_fixed256(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  const double s = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return s;
}

// dt1 in two passes over a batch of records [b0, b0 + gridDim.x).  Pass 1:
// one work-group per H record writes that record's contribution to all n_v
// entries of its t1 row into part[(rec - b0) * pstride + y]; pass 2 adds
// each group's records of the batch in list order.
//   kind 0: y = c, sum_{a,b} H[a][b][c] ovov[i][a][j][b]
//   kind 1: y = b, sum_{a,c} H[a][b][c] ovov[i][a][k][c]
//   kind 2: y = a, sum_{b,c} H[a][b][c] ovov[j][b][k][c]
// Lanes run along c (contiguous in H) in chunks of 64, so H streams once per
// record, coalesced.  Grid: the launch's T1 records.  Block: 256 threads.
template <typename CubeT, typename InT>
__global__ __launch_bounds__(256) void k_adj_t1_part(const FragDesc* __restrict__ descs,
                                                     const Item* __restrict__ items,
                                                     const AdjRec* __restrict__ recs, int b0,
                                                     const CubeT* __restrict__ arena,
                                                     double* __restrict__ part, int pstride) {
  __shared__ double red[4][64];
  const int q = b0 + blockIdx.x;
  const AdjRec rr = recs[q];
  const Item it = items[rr.item];
  const FragDesc fd = descs[it.frag];
  const int no = fd.no, nv = fd.nv;
  int i, j, k;
  decode_sorted_triple(it.unit, no, i, j, k);
  const SIE_GLOBAL CubeT* H = gptr(arena + it.cube_off + fd.half);
  const SIE_GLOBAL InT* ovov = gptr(static_cast<const InT*>(fd.ovov));
  const int64_t nv2 = int64_t(nv) * nv, onv = int64_t(no) * nv;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* out = part + int64_t(blockIdx.x) * pstride;
  if (rr.kind == 0) {
    const SIE_GLOBAL InT* m = ovov + int64_t(i) * nv * onv + int64_t(j) * nv;   // m[a*onv + b]
    for (int c0 = 0; c0 < nv; c0 += 64) {
      const int c = c0 + lane;
      double s = 0.0;
      if (c < nv) {   // four interleaved partial sums, added in a fixed order
        double p[4] = {0.0, 0.0, 0.0, 0.0};
        int64_t ab = wave;
        // (a, b) of ab = a nv + b, stepped along with ab (no division per term)
        int aa = wave / nv, bb = wave - aa * nv;
        auto step = [&](int d, int& a2, int& b2) {
          a2 = aa;
          b2 = bb + d;
          while (b2 >= nv) {
            b2 -= nv;
            ++a2;
          }
        };
        for (; ab + 12 < nv2; ab += 16) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            int a2, b2;
            step(4 * u, a2, b2);
            p[u] += (double)H[(ab + 4 * u) * nv + c] * (double)m[int64_t(a2) * onv + b2];
          }
          step(16, aa, bb);
        }
        for (; ab < nv2; ab += 4) {
          p[0] += (double)H[ab * nv + c] * (double)m[int64_t(aa) * onv + bb];
          step(4, aa, bb);
        }
        s = (p[0] + p[1]) + (p[2] + p[3]);
      }
      red[wave][lane] = s;
      __syncthreads();
      if (wave == 0 && c < nv)
        out[c] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
      __syncthreads();
    }
  } else {
    // kind 1: y = b, weight M[a][c] = ovov[i][a][k][c], H row (a, y)
    // kind 2: y = a, weight M[b][c] = ovov[j][b][k][c], H row (y, b)
    const SIE_GLOBAL InT* m = rr.kind == 1 ? ovov + int64_t(i) * nv * onv + int64_t(k) * nv
                                           : ovov + int64_t(j) * nv * onv + int64_t(k) * nv;
    for (int y = wave; y < nv; y += 4) {
      double tot = 0.0;
      for (int c0 = 0; c0 < nv; c0 += 64) {
        const int c = c0 + lane;
        double s = 0.0;
        if (c < nv) {   // four interleaved partial sums, added in a fixed order
          const int64_t h0 = rr.kind == 1 ? int64_t(y) * nv + c : int64_t(y) * nv2 + c;
          const int64_t hu = rr.kind == 1 ? nv2 : nv;
          double p[4] = {0.0, 0.0, 0.0, 0.0};
          int u = 0;
          for (; u + 4 <= nv; u += 4) {
#pragma unroll
            for (int w = 0; w < 4; ++w)
              p[w] += (double)H[h0 + int64_t(u + w) * hu] * (double)m[int64_t(u + w) * onv + c];
          }
          for (; u < nv; ++u) p[0] += (double)H[h0 + int64_t(u) * hu] * (double)m[int64_t(u) * onv + c];
          s = (p[0] + p[1]) + (p[2] + p[3]);
        }
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        tot += s;
      }
      if (lane == 0) out[y] = tot;
    }
  }
}

// dt1[p][y] += sum over the group's records in [b0, b1) (list order) of
// part[(rec - b0) * pstride + y].  Grid: ceil(max n_v / 256) x groups.
// Block: 256 threads.
template <int = 0>
__global__ __launch_bounds__(256) void k_adj_t1_sum(const FragDesc* __restrict__ descs,
                                                    const AdjGroup* __restrict__ groups, int b0,
                                                    int b1, const double* __restrict__ part,
                                                    int pstride) {
  const AdjGroup gr = groups[blockIdx.y];
  const FragDesc fd = descs[gr.frag];
  const int y = blockIdx.x * 256 + threadIdx.x;
  const int q0 = max(gr.rec_begin, b0), q1 = min(gr.rec_end, b1);
  if (y >= fd.nv || q0 >= q1) return;
  double s = 0.0;
  for (int q = q0; q < q1; ++q) s += part[int64_t(q - b0) * pstride + y];
  SIE_GLOBAL double* p = gptr_w(fd.g_t1) + int64_t(gr.a0) * fd.nv + y;
  *p = *p + s;
}

// ---------------------------------------------------------------------------
// Fill and symmetrize.
// ---------------------------------------------------------------------------

template <int = 0>
__global__ __launch_bounds__(256) void k_fill_zero(double* __restrict__ p, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n;
       e += int64_t(gridDim.x) * 256)
    gptr_w(p)[e] = 0.0;
}

// g[e] = g[twin(e)] = (g[e] + g[twin(e)]) / 2; the thread of the smaller
// index of each pair does both writes.
template <int = 0>
__global__ __launch_bounds__(256) void k_symmetrize(double* __restrict__ g, int kind, int no,
                                                    int nv, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n;
       e += int64_t(gridDim.x) * 256) {
    const int64_t t = twin_index(kind, e, no, nv);
    if (t <= e) continue;
    const double m = 0.5 * (gptr(g)[e] + gptr(g)[t]);
    gptr_w(g)[e] = m;
    gptr_w(g)[t] = m;
  }
}

}  // namespace sie
