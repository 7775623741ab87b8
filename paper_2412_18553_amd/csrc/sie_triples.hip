// Host side of the C ABI declared in include/sie_triples.h: argument checks,
// workspace planning and kernel launches on the caller's stream.
#include "sie_triples.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "k_fp64.hpp"
#include "k_reduce.hpp"

namespace {

thread_local std::string g_err;

sie_status fail(sie_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

constexpr size_t kDefaultCap = size_t(2) << 30;   // 2 GiB
constexpr int kMaxPartials = 256;                  // epilogue blocks per unit

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t default_cap() {
  const char* env = std::getenv("SIE_MAX_WORKSPACE_BYTES");
  if (env && *env) {
    char* end = nullptr;
    unsigned long long v = std::strtoull(env, &end, 10);
    if (end && *end == '\0' && v > 0) return size_t(v);
  }
  return kDefaultCap;
}

// Workspace layout of one energy evaluation:
//   [eps copy (no + nv)] [unit energies] [partials units x n_part] [cube x chunk]
struct Plan {
  int no = 0, nv = 0;
  int64_t n_units = 0;
  int n_part = 0;
  size_t off_eps = 0, off_units = 0, off_part = 0, off_cube = 0;
  size_t cube_bytes = 0;     // one unit's Wt cube
  size_t fixed_bytes = 0;    // everything but the cubes
};

Plan make_plan(int no, int nv) {
  Plan p;
  p.no = no;
  p.nv = nv;
  p.n_units = sie::tetra(no);
  const int64_t nb = (nv + sie::kOrb - 1) / sie::kOrb;
  const int64_t n_orb = sie::tetra(nb);
  p.n_part = int(n_orb < kMaxPartials ? n_orb : kMaxPartials);
  size_t off = 0;
  p.off_eps = off;
  off = align_up(off + sizeof(double) * size_t(no + nv), 256);
  p.off_units = off;
  off = align_up(off + sizeof(double) * size_t(p.n_units), 256);
  p.off_part = off;
  off = align_up(off + sizeof(double) * size_t(p.n_units) * size_t(p.n_part), 256);
  p.off_cube = off;
  p.fixed_bytes = off;
  p.cube_bytes = align_up(sizeof(double) * size_t(nv) * size_t(nv) * size_t(nv), 256);
  return p;
}

bool aligned(const void* ptr, size_t a) { return (reinterpret_cast<uintptr_t>(ptr) % a) == 0; }

sie_status check_fragment(const sie_fragment* f, sie_precision prec, const char* who) {
  std::string w(who);
  if (!f) return fail(SIE_ERR_INVALID_ARG, w + ": fragment descriptor is NULL");
  if (prec != SIE_FP64 && prec != SIE_SPLIT_BF16)
    return fail(SIE_ERR_INVALID_ARG, w + ": unknown precision");
  if (f->n_occ < 1 || f->n_occ > SIE_MAX_OCC)
    return fail(SIE_ERR_INVALID_ARG, w + ": n_occ out of range [1, SIE_MAX_OCC]");
  if (f->n_vir < 1 || f->n_vir > SIE_MAX_VIR)
    return fail(SIE_ERR_INVALID_ARG, w + ": n_vir out of range [1, SIE_MAX_VIR]");
  if (!f->eps_occ || !f->eps_vir)
    return fail(SIE_ERR_INVALID_ARG, w + ": eps_occ / eps_vir is NULL");
  if (!f->t1 || !f->t2 || !f->ovvv || !f->ooov || !f->ovov)
    return fail(SIE_ERR_INVALID_ARG, w + ": an amplitude or integral pointer is NULL");
  const size_t esz = prec == SIE_FP64 ? sizeof(double) : sizeof(float);
  if (!aligned(f->t1, esz) || !aligned(f->t2, esz) || !aligned(f->ovvv, esz) ||
      !aligned(f->ooov, esz) || !aligned(f->ovov, esz))
    return fail(SIE_ERR_INVALID_ARG, w + ": an input is not aligned to its element size");
  double max_occ = -INFINITY, min_vir = INFINITY;
  for (int i = 0; i < f->n_occ; ++i) {
    if (!std::isfinite(f->eps_occ[i]))
      return fail(SIE_ERR_INVALID_ARG, w + ": eps_occ has a non-finite entry");
    max_occ = f->eps_occ[i] > max_occ ? f->eps_occ[i] : max_occ;
  }
  for (int a = 0; a < f->n_vir; ++a) {
    if (!std::isfinite(f->eps_vir[a]))
      return fail(SIE_ERR_INVALID_ARG, w + ": eps_vir has a non-finite entry");
    min_vir = f->eps_vir[a] < min_vir ? f->eps_vir[a] : min_vir;
  }
  if (!(max_occ < min_vir))
    return fail(SIE_ERR_INVALID_ARG,
                w + ": max(eps_occ) >= min(eps_vir): a triples denominator would not be negative");
  if (f->frag_proj)
    return fail(SIE_ERR_UNSUPPORTED, w + ": fragment projector C^f is not supported by this build");
  if (prec == SIE_SPLIT_BF16)
    return fail(SIE_ERR_UNSUPPORTED, w + ": SIE_SPLIT_BF16 is not supported by this build");
  return SIE_OK;
}

sie_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return SIE_OK;
  return fail(SIE_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---- optional kernel timing ----
struct ProfRec {
  hipEvent_t start, stop;
  int kind;
};
thread_local bool g_prof_on = false;
thread_local std::vector<ProfRec> g_prof;

void prof_clear() {
  for (auto& r : g_prof) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  g_prof.clear();
}

// Brackets one launch with events when timing is enabled.
struct ProfScope {
  hipStream_t s;
  ProfRec rec{};
  bool on;
  ProfScope(hipStream_t st, int kind) : s(st), on(g_prof_on) {
    if (!on) return;
    rec.kind = kind;
    if (hipEventCreate(&rec.start) != hipSuccess) { on = false; return; }
    if (hipEventCreate(&rec.stop) != hipSuccess) { (void)hipEventDestroy(rec.start); on = false; return; }
    (void)hipEventRecord(rec.start, s);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(rec.stop, s);
    g_prof.push_back(rec);
  }
};

}  // namespace

extern "C" {

int sie_abi_version(void) { return SIE_ABI_VERSION; }

void sie_profile_enable(int on) {
  prof_clear();
  g_prof_on = on != 0;
}

sie_status sie_profile_collect(double* ms, int64_t* launches) {
  if (!ms || !launches) return fail(SIE_ERR_INVALID_ARG, "sie_profile_collect: NULL output");
  for (int c = 0; c < SIE_PROF_CLASSES; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  sie_status st = SIE_OK;
  for (auto& r : g_prof) {
    float t = 0.f;
    if (st == SIE_OK) st = hip_check(hipEventSynchronize(r.stop), "sie_profile_collect");
    if (st == SIE_OK) st = hip_check(hipEventElapsedTime(&t, r.start, r.stop), "sie_profile_collect");
    if (st == SIE_OK && r.kind >= 0 && r.kind < SIE_PROF_CLASSES) {
      ms[r.kind] += t;
      launches[r.kind] += 1;
    }
  }
  prof_clear();
  return st;
}

const char* sie_last_error(void) { return g_err.c_str(); }

int64_t sie_occupied_triples(int32_t n_occ) {
  return n_occ < 0 ? 0 : sie::tetra(n_occ);
}

size_t sie_triples_workspace_size(const sie_fragment* frags, int32_t n, sie_precision p,
                                  size_t max_bytes) {
  if (!frags || n < 1) {
    fail(SIE_ERR_INVALID_ARG, "sie_triples_workspace_size: need at least one fragment");
    return 0;
  }
  const size_t cap = max_bytes ? max_bytes : default_cap();
  size_t need = 0;
  for (int32_t x = 0; x < n; ++x) {
    if (check_fragment(&frags[x], p, "sie_triples_workspace_size") != SIE_OK) return 0;
    const Plan pl = make_plan(frags[x].n_occ, frags[x].n_vir);
    const size_t one = pl.fixed_bytes + pl.cube_bytes;
    if (one > cap) {
      fail(SIE_ERR_WORKSPACE, "sie_triples_workspace_size: cap below the minimum for one fragment");
      return 0;
    }
    int64_t chunk = int64_t((cap - pl.fixed_bytes) / pl.cube_bytes);
    if (chunk > pl.n_units) chunk = pl.n_units;
    const size_t bytes = pl.fixed_bytes + size_t(chunk) * pl.cube_bytes;
    need = bytes > need ? bytes : need;
  }
  return need;
}

sie_status sie_triples_energy(const sie_fragment* f, sie_precision p, double* e_out,
                              double* e_triples, void* ws, size_t ws_bytes, void* stream) {
  sie_status st = check_fragment(f, p, "sie_triples_energy");
  if (st != SIE_OK) return st;
  if (!e_out || !aligned(e_out, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, "sie_triples_energy: e_out is NULL or misaligned");
  if (e_triples && !aligned(e_triples, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, "sie_triples_energy: e_triples is misaligned");
  const Plan pl = make_plan(f->n_occ, f->n_vir);
  if (!ws || !aligned(ws, 256))
    return fail(SIE_ERR_WORKSPACE, "sie_triples_energy: workspace is NULL or not 256-byte aligned");
  if (ws_bytes < pl.fixed_bytes + pl.cube_bytes)
    return fail(SIE_ERR_WORKSPACE, "sie_triples_energy: workspace smaller than required (see "
                                   "sie_triples_workspace_size)");
  int64_t chunk = int64_t((ws_bytes - pl.fixed_bytes) / pl.cube_bytes);
  if (chunk > pl.n_units) chunk = pl.n_units;
  if (chunk > 65535) chunk = 65535;

  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  double* d_eps = reinterpret_cast<double*>(base + pl.off_eps);
  double* d_units = e_triples ? e_triples : reinterpret_cast<double*>(base + pl.off_units);
  double* d_part = reinterpret_cast<double*>(base + pl.off_part);
  double* d_cube = reinterpret_cast<double*>(base + pl.off_cube);

  const int no = pl.no, nv = pl.nv;
  st = hip_check(hipMemcpyAsync(d_eps, f->eps_occ, sizeof(double) * no, hipMemcpyHostToDevice, s),
                 "copy eps_occ");
  if (st != SIE_OK) return st;
  st = hip_check(hipMemcpyAsync(d_eps + no, f->eps_vir, sizeof(double) * nv,
                                hipMemcpyHostToDevice, s),
                 "copy eps_vir");
  if (st != SIE_OK) return st;

  sie::FragDev fd;
  fd.t1 = static_cast<const double*>(f->t1);
  fd.t2 = static_cast<const double*>(f->t2);
  fd.ovvv = static_cast<const double*>(f->ovvv);
  fd.ooov = static_cast<const double*>(f->ooov);
  fd.ovov = static_cast<const double*>(f->ovov);
  fd.eps = d_eps;
  fd.no = no;
  fd.nv = nv;

  const int nbk = (nv + sie::kTile - 1) / sie::kTile;
  const unsigned n_tiles = unsigned(nbk) * unsigned(nbk) * unsigned(nbk);
  const int64_t cube_stride = int64_t(pl.cube_bytes / sizeof(double));
  // 16-byte row reads need an even row length and 16-byte aligned bases
  const bool vec = (nv % 2 == 0) && aligned(f->t2, 16) && aligned(f->ovvv, 16);
  for (int64_t u0 = 0; u0 < pl.n_units; u0 += chunk) {
    const int64_t cnt = (pl.n_units - u0) < chunk ? (pl.n_units - u0) : chunk;
    {
      ProfScope ps(s, 0);
      if (vec)
        hipLaunchKernelGGL(sie::k_build_w_f64<true>, dim3(n_tiles, unsigned(cnt)), dim3(256), 0,
                           s, fd, u0, pl.n_units, d_cube, cube_stride);
      else
        hipLaunchKernelGGL(sie::k_build_w_f64<false>, dim3(n_tiles, unsigned(cnt)), dim3(256), 0,
                           s, fd, u0, pl.n_units, d_cube, cube_stride);
    }
    {
      ProfScope ps(s, 1);
      hipLaunchKernelGGL(sie::k_epilogue_f64, dim3(unsigned(pl.n_part), unsigned(cnt)),
                         dim3(256), 0, s, fd, u0, pl.n_units, d_cube, cube_stride, d_part,
                         pl.n_part);
    }
    st = hip_check(hipGetLastError(), "launch (T) kernels");
    if (st != SIE_OK) return st;
  }
  const unsigned ub = unsigned((pl.n_units + 255) / 256);
  {
    ProfScope ps(s, 2);
    hipLaunchKernelGGL(sie::k_unit_energy, dim3(ub), dim3(256), 0, s, no, pl.n_units, d_part,
                       pl.n_part, d_units);
    hipLaunchKernelGGL(sie::k_sum_fixed, dim3(1), dim3(256), 0, s, d_units, pl.n_units, e_out);
  }
  return hip_check(hipGetLastError(), "launch reductions");
}

}  // extern "C"
