// Host side of the MP2 entry points declared in include/sie_triples.h
// (sie_mp2_workspace_size, sie_mp2): argument checks, workspace layout and
// the launches of the kernels in k_mp2.hpp on the caller's stream.
#include "sie_triples.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "k_mp2.hpp"

namespace sie {
sie_status set_error(sie_status s, const std::string& msg);   // sie_triples.hip
}

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Work-group groups of the two density products: enough groups that a launch
// has a few thousand work-groups, and the slices they write.
struct Mp2Plan {
  int64_t pairs = 0, tile_pairs = 0;
  int g_vv = 1, per_vv = 1, g_oo = 1, per_oo = 1;
  int ks_oo = 1;            // contraction splits of gamma_oo (K = n_v^2 per entry)
  int64_t kc_oo = 0;        // their length (a multiple of 8)
  size_t off_eps = 0, off_epart = 0, off_t2 = 0, off_gram = 0, bytes = 0;
};

Mp2Plan mp2_plan(const sie_mp2_input& in, bool density, bool own_t2) {
  Mp2Plan p;
  const int64_t o = in.n_occ, v = in.n_vir;
  p.pairs = o * (o + 1) / 2;
  const int64_t nt = (v + sie::kMp2Tile - 1) / sie::kMp2Tile;
  p.tile_pairs = nt * (nt + 1) / 2;
  auto groups = [](int64_t nq, int64_t tiles, int& g, int& per) {
    int64_t want = (4096 + tiles - 1) / tiles;
    want = want < 1 ? 1 : (want > nq ? nq : want);
    per = int((nq + want - 1) / want);
    g = int((nq + per - 1) / per);
  };
  const int64_t tvm = (v + 32 * sie::kGramVvM - 1) / (32 * sie::kGramVvM);
  const int64_t tvn = (v + 32 * sie::kGramVvN - 1) / (32 * sie::kGramVvN);
  const int64_t tom = (o + 32 * sie::kGramOoM - 1) / (32 * sie::kGramOoM);
  const int64_t ton = (o + 32 * sie::kGramOoN - 1) / (32 * sie::kGramOoN);
  groups(o * o, tvm * tvn, p.g_vv, p.per_vv);
  // gamma_oo: n_o entries of n_v^2 each; split each contraction so that
  // entries x splits x tiles reach a few thousand work-groups
  {
    const int64_t want = (4096 + tom * ton - 1) / (tom * ton);
    int64_t ks = (want + o - 1) / o;
    const int64_t max_ks = (v * v + 7) / 8;
    ks = ks < 1 ? 1 : (ks > max_ks ? max_ks : ks);
    p.kc_oo = ((v * v + ks - 1) / ks + 7) / 8 * 8;
    p.ks_oo = int((v * v + p.kc_oo - 1) / p.kc_oo);
  }
  groups(o * int64_t(p.ks_oo), tom * ton, p.g_oo, p.per_oo);
  size_t off = 0;
  p.off_eps = off;
  off = align256(off + sizeof(double) * size_t(o + v));
  p.off_epart = off;
  off = align256(off + sizeof(double) * size_t(p.pairs * p.tile_pairs));
  p.off_t2 = off;
  if (density && own_t2) off = align256(off + sizeof(double) * size_t(o * o * v * v));
  p.off_gram = off;
  if (density) {
    const size_t vv = size_t(p.g_vv) * size_t(v * v), oo = size_t(p.g_oo) * size_t(o * o);
    off = align256(off + sizeof(double) * (vv > oo ? vv : oo));
  }
  p.bytes = off;
  return p;
}

sie_status check_mp2(const sie_mp2_input* in, const char* who) {
  const std::string w(who);
  if (!in) return sie::set_error(SIE_ERR_INVALID_ARG, w + ": input descriptor is NULL");
  if (in->n_occ < 1 || in->n_occ > SIE_MAX_OCC)
    return sie::set_error(SIE_ERR_INVALID_ARG, w + ": n_occ out of range [1, SIE_MAX_OCC]");
  if (in->n_vir < 1 || in->n_vir > SIE_MAX_VIR)
    return sie::set_error(SIE_ERR_INVALID_ARG, w + ": n_vir out of range [1, SIE_MAX_VIR]");
  if (in->n_aux < 1) return sie::set_error(SIE_ERR_INVALID_ARG, w + ": n_aux must be >= 1");
  if (!in->eps_occ || !in->eps_vir || !in->l_ov)
    return sie::set_error(SIE_ERR_INVALID_ARG, w + ": a pointer is NULL");
  if (reinterpret_cast<uintptr_t>(in->l_ov) % sizeof(double))
    return sie::set_error(SIE_ERR_INVALID_ARG, w + ": l_ov is not aligned to 8 bytes");
  double max_occ = -INFINITY, min_vir = INFINITY;
  for (int i = 0; i < in->n_occ; ++i) {
    if (!std::isfinite(in->eps_occ[i]))
      return sie::set_error(SIE_ERR_NONFINITE, w + ": eps_occ has a non-finite entry");
    max_occ = in->eps_occ[i] > max_occ ? in->eps_occ[i] : max_occ;
  }
  for (int a = 0; a < in->n_vir; ++a) {
    if (!std::isfinite(in->eps_vir[a]))
      return sie::set_error(SIE_ERR_NONFINITE, w + ": eps_vir has a non-finite entry");
    min_vir = in->eps_vir[a] < min_vir ? in->eps_vir[a] : min_vir;
  }
  if (!(max_occ < min_vir))
    return sie::set_error(SIE_ERR_INVALID_ARG,
                          w + ": max(eps_occ) >= min(eps_vir): a pair denominator would not be "
                              "positive");
  return SIE_OK;
}

sie_status hip_fail(hipError_t e, const std::string& what) {
  return sie::set_error(SIE_ERR_HIP, what + ": " + hipGetErrorString(e));
}

}  // namespace

extern "C" {

size_t sie_mp2_workspace_size(const sie_mp2_input* in, int32_t want_density) {
  if (check_mp2(in, "sie_mp2_workspace_size") != SIE_OK) return 0;
  return mp2_plan(*in, want_density != 0, true).bytes;
}

sie_status sie_mp2(const sie_mp2_input* in, double* e_out, double* t2, double* gamma_oo,
                   double* gamma_vv, void* ws, size_t ws_bytes, void* stream) {
  const char* who = "sie_mp2";
  const std::string w(who);
  sie_status st = check_mp2(in, who);
  if (st != SIE_OK) return st;
  for (const double* q : {static_cast<const double*>(e_out), static_cast<const double*>(t2),
                          static_cast<const double*>(gamma_oo),
                          static_cast<const double*>(gamma_vv)})
    if (q && reinterpret_cast<uintptr_t>(q) % sizeof(double))
      return sie::set_error(SIE_ERR_INVALID_ARG, w + ": an output is misaligned");
  if (!e_out) return sie::set_error(SIE_ERR_INVALID_ARG, w + ": e_out is NULL");
  const bool density = gamma_oo || gamma_vv;
  const Mp2Plan pl = mp2_plan(*in, density, t2 == nullptr);
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256)
    return sie::set_error(SIE_ERR_WORKSPACE, w + ": workspace is NULL or not 256-byte aligned");
  if (ws_bytes < pl.bytes)
    return sie::set_error(SIE_ERR_WORKSPACE,
                          w + ": workspace smaller than required (see sie_mp2_workspace_size)");
  if (pl.pairs > 65535 || pl.tile_pairs > 2147483647)
    return sie::set_error(SIE_ERR_UNSUPPORTED, w + ": too many occupied pairs for one launch");

  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const int o = in->n_occ, v = in->n_vir, np = in->n_aux;
  double* d_eps = reinterpret_cast<double*>(base + pl.off_eps);
  double* d_epart = reinterpret_cast<double*>(base + pl.off_epart);
  double* d_t2 = t2 ? t2 : (density ? reinterpret_cast<double*>(base + pl.off_t2) : nullptr);
  double* d_gram = reinterpret_cast<double*>(base + pl.off_gram);

  // the orbital energies: two small pageable copies (consumed before they return)
  hipError_t e = hipMemcpyAsync(d_eps, in->eps_occ, sizeof(double) * size_t(o),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_eps + o, in->eps_vir, sizeof(double) * size_t(v),
                       hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, w + ": upload orbital energies");

  hipLaunchKernelGGL(sie::k_mp2_pair, dim3(unsigned(pl.tile_pairs), unsigned(pl.pairs)),
                     dim3(256), 0, s, in->l_ov, d_eps, o, v, np, d_t2, d_epart);
  hipLaunchKernelGGL(sie::k_mp2_sum, dim3(1), dim3(256), 0, s, d_epart,
                     pl.pairs * pl.tile_pairs, e_out);
  if (density) {
    const int64_t nv2 = int64_t(v) * v;
    if (gamma_vv) {
      sie::GramArgs ga{d_t2, d_t2, d_t2, nv2, v, nv2, v, nv2, v, v, v, v, o * o, pl.per_vv, o,
                       2.0, -1.0, d_gram, 1, v};
      hipLaunchKernelGGL((sie::k_mp2_gram<true, sie::kGramVvM, sie::kGramVvN>),
                         dim3(unsigned((v + 32 * sie::kGramVvN - 1) / (32 * sie::kGramVvN)),
                              unsigned((v + 32 * sie::kGramVvM - 1) / (32 * sie::kGramVvM)),
                              unsigned(pl.g_vv)),
                         dim3(256), 0, s, ga);
      hipLaunchKernelGGL(sie::k_mp2_gram_sum, dim3(unsigned((nv2 + 255) / 256)), dim3(256), 0, s,
                         d_gram, pl.g_vv, v, v, 2.0, 0.0, gamma_vv);
    }
    if (gamma_oo) {
      const int64_t onv2 = int64_t(o) * nv2;
      sie::GramArgs ga{d_t2, d_t2, d_t2, nv2, onv2, nv2, onv2, onv2, nv2, o, o,
                       int(pl.kc_oo), o * pl.ks_oo, pl.per_oo, o, 2.0, -1.0, d_gram,
                       pl.ks_oo, nv2};
      hipLaunchKernelGGL((sie::k_mp2_gram<false, sie::kGramOoM, sie::kGramOoN>),
                         dim3(unsigned((o + 32 * sie::kGramOoN - 1) / (32 * sie::kGramOoN)),
                              unsigned((o + 32 * sie::kGramOoM - 1) / (32 * sie::kGramOoM)),
                              unsigned(pl.g_oo)),
                         dim3(256), 0, s, ga);
      hipLaunchKernelGGL(sie::k_mp2_gram_sum, dim3(unsigned((int64_t(o) * o + 255) / 256)),
                         dim3(256), 0, s, d_gram, pl.g_oo, o, o, -2.0, 2.0, gamma_oo);
    }
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, w + ": launch MP2 kernels");
  return SIE_OK;
}

}  // extern "C"
