// Host side of the C ABI declared in include/sie_triples.h: argument checks,
// workspace planning and kernel launches on the caller's stream.
#include "sie_triples.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <array>
#include <atomic>
#include <iterator>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "adj_plan.hpp"
#include "k_df.hpp"
#include "launch.hpp"
#include "shapes.hpp"
#include "staging.hpp"
#include "work.hpp"

namespace {

thread_local std::string g_err;

sie_status fail(sie_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

constexpr size_t kDefaultCap = size_t(16) << 30;  // 16 GiB of the 288 GB of HBM
constexpr int kMaxPartials = 256;                  // epilogue blocks per unit
constexpr int kMinOrbits = 16;                     // orbits per epilogue block, where there are enough

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

size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

// Page-locked staging of the per-call tables (see staging.hpp).
sie::Staging g_staging;

// Device scratch of sie_triples_energy_static: one copy per GPU, held from the
// library's load on that GPU until the process ends.  Host code never passes
// `scratch` itself to a kernel or a copy (in host code the name is only a
// stand-in); it uses the device address hipGetSymbolAddress returns for the
// current GPU, looked up once per device.
static __device__ __align__(256) unsigned char scratch[SIE_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

sie_status fail_hip(hipError_t e, const std::string& what);

sie_status static_scratch(void** out, const std::string& who) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, who + ": hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SIE_ERR_UNSUPPORTED, who + ": device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, who + ": hipGetSymbolAddress(scratch)");
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) % 256) != 0)
      return fail(SIE_ERR_HIP, who + ": scratch address is NULL or not 256-byte aligned");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SIE_OK;
}

// Optional scan of the device inputs for non-finite values (SIE_CHECK_FINITE).
std::atomic<int> g_check_finite{-1};

bool check_finite_on() {
  int v = g_check_finite.load();
  if (v < 0) {
    const char* env = std::getenv("SIE_CHECK_FINITE");
    v = (env && *env && std::string(env) != "0") ? 1 : 0;
    int expect = -1;
    g_check_finite.compare_exchange_strong(expect, v);
    v = g_check_finite.load();
  }
  return v == 1;
}

// Per-fragment sizes.
struct FragPlan {
  int no = 0, nv = 0;
  int Kv = 0, Ko = 0;
  int64_t n_units = 0;       // all i >= j >= k (per-unit arrays)
  int64_t work_units = 0;    // units that are not i = j = k
  int n_part = 0;
  size_t split_bytes = 0;    // vS + tS + tT + oT
  size_t half_bytes = 0;     // one partial cube (aligned)
  double unit_cost = 0.0;    // flops per unit (ordering key)
  int variant = 0;           // build tile shape (float64: sie::wshape; split: sie::sshape)
  bool lay3 = false;         // three-layout build (float64 energy only)
  int cubes = 2;             // partial cubes of a unit in flight
  int cubes_pair = 1;        // ... of a pair unit (sie::unit_triple)
};

FragPlan frag_plan(int no, int nv, bool split) {
  FragPlan p;
  p.no = no;
  p.nv = nv;
  p.n_units = sie::tetra(no);
  p.work_units = p.n_units - no;
  const int64_t nb = (nv + sie::kOrb - 1) / sie::kOrb;
  const int64_t n_orb = sie::tetra(nb);
  // each epilogue block takes at least kMinOrbits orbits (its set-up is paid
  // once per block), up to kMaxPartials blocks per unit
  const int64_t parts = (n_orb + kMinOrbits - 1) / kMinOrbits;
  p.n_part = int(parts < kMaxPartials ? parts : kMaxPartials);
  const size_t o = size_t(no), v = size_t(nv);
  if (split) {
    p.Kv = int(round_up(v, sie::kKs));
    p.Ko = int(round_up(o, sie::kKs));
    // 4 bytes (bf16 hi + lo) per padded element
    p.split_bytes = align_up(4 * o * v * v * size_t(p.Kv), 256) +
                    align_up(4 * o * o * v * size_t(p.Kv), 256) +
                    align_up(4 * o * v * v * size_t(p.Ko), 256) +
                    align_up(4 * o * o * v * size_t(p.Ko), 256);
  }
  p.half_bytes = align_up((split ? sizeof(float) : sizeof(double)) * v * v * v, 256);
  p.unit_cost = 12.0 * double(v) * v * v * v + 12.0 * double(o) * v * v * v;
  return p;
}

// Workspace layout of one evaluation of n fragments:
//   [descriptors] [eps copies] [per-unit energies] [per-unit partials]
//   [fragment energies] [items] [split copies] [cube arena]
struct Plan {
  bool split = false;
  std::vector<FragPlan> frags;
  int64_t total_units = 0, total_work = 0;
  int pstride = 0;
  size_t off_desc = 0, off_eps = 0, off_units = 0, off_part = 0, off_efrag = 0, off_items = 0;
  size_t off_flags = 0;      // non-finite scan flags: 5 per fragment
  size_t off_split = 0, off_adj = 0, off_t1 = 0, off_parts = 0, off_arena = 0;
  // orbital-energy gradient (backward only): occupied partials per (unit,
  // slot) and per unit; virtual rows per (round item, slot) and per item
  size_t off_eo = 0, off_eou = 0, off_evp = 0, off_evi = 0;
  int nv_max = 1;            // largest n_vir (row stride of the t1 partials)
  size_t adj_recs = 0;       // bound on the adjoint records (= groups) of all rounds
  size_t part_elems = 0;     // bound on the partial-slice elements of a summed-block class
  size_t fixed_bytes = 0;    // everything before the arena
  int cubes = 2;             // cubes per unit in flight (backward: G, H and G transposed)
  bool pair = false;         // pair units build one layout into one cube (energy only)
  bool blocked = false;      // 8^3-blocked cubes (energy only; see sie::cube_at)
  size_t min_arena = 0;      // the largest cube set of any fragment
  size_t all_arena = 0;      // every unit's cube set at once
};

// Records per unit of the backward pass: 6 + 6 per-block terms, 6 + 6 summed
// terms per block group of kARB virtuals, 3 + 3 H terms.
constexpr int kT1Batch = 4096;    // t1 records per partial-sum batch (backward)
// Items per backward round at most: bounds the per-work-group rows of the
// virtual orbital-energy gradient (items x epilogue slots x n_vir).
constexpr size_t kGradRoundItems = 256;

size_t adj_recs_per_unit(int nv) {
  return size_t(18) + size_t(12) * size_t((nv + sie::kARB - 1) / sie::kARB);
}

int tile_variant(int nv);
int split_shape(int nv);
bool aligned(const void* ptr, size_t a) { return (reinterpret_cast<uintptr_t>(ptr) % a) == 0; }

Plan make_plan(const sie_fragment* frags, int n, sie_precision prec, bool grad = false) {
  Plan p;
  p.cubes = grad ? 3 : 2;
  p.pair = !grad;
  p.blocked = !grad;
  p.split = prec == SIE_SPLIT_BF16;
  size_t eps_n = 0, split_bytes = 0;
  for (int x = 0; x < n; ++x) {
    FragPlan fp = frag_plan(frags[x].n_occ, frags[x].n_vir, p.split);
    // the adjoint rebuilds W-tilde with a two-layout shape (its G and H
    // cubes follow that layout); the energy takes the table's shape
    if (!p.split) {
      fp.variant = tile_variant(fp.nv);
      if (grad && sie::wshape(fp.variant).lay == 3) fp.variant = 0;
      fp.lay3 = sie::wshape(fp.variant).lay == 3;
    } else {
      fp.variant = split_shape(fp.nv);
    }
    if (p.blocked)   // the blocked cube pads its edge to a multiple of the orbit block
      fp.half_bytes = align_up((p.split ? sizeof(float) : sizeof(double)) *
                                   size_t(sie::cube_blocked_elems(fp.nv)), 256);
    fp.cubes = grad ? 3 : fp.lay3 ? 3 : 2;
    fp.cubes_pair = grad ? 3 : fp.lay3 ? 2 : 1;
    p.total_units += fp.n_units;
    p.total_work += fp.work_units;
    p.pstride = fp.n_part > p.pstride ? fp.n_part : p.pstride;
    eps_n += size_t(fp.no + fp.nv);
    split_bytes += fp.split_bytes;
    const size_t pair = size_t(fp.cubes) * fp.half_bytes;
    p.min_arena = fp.work_units > 0 && pair > p.min_arena ? pair : p.min_arena;
    // units with exactly two equal occupied indices: n_o (n_o - 1)
    const size_t n_pair = p.pair ? size_t(fp.no) * size_t(fp.no - 1) : 0;
    p.all_arena += pair * (size_t(fp.work_units) - n_pair) +
                   size_t(fp.cubes_pair) * fp.half_bytes * n_pair;
    if (grad) {
      p.adj_recs += size_t(fp.work_units) * adj_recs_per_unit(fp.nv);
      // a round's slices of a summed-block class are distinct occupied pairs
      // (at most n_o^2 per fragment), with kAdjParts n_o^2 partials in all
      const size_t slice = size_t(fp.nv) * size_t(fp.nv > fp.no ? fp.nv : fp.no);
      p.part_elems += size_t(sie::kAdjParts) * size_t(fp.no) * size_t(fp.no) * slice;
    }
    p.nv_max = fp.nv > p.nv_max ? fp.nv : p.nv_max;
    p.frags.push_back(fp);
  }
  size_t off = 0;
  p.off_desc = off;
  off = align_up(off + sizeof(sie::FragDesc) * size_t(n), 256);
  p.off_eps = off;
  off = align_up(off + sizeof(double) * eps_n, 256);
  p.off_units = off;
  off = align_up(off + sizeof(double) * size_t(p.total_units), 256);
  p.off_part = off;
  off = align_up(off + sizeof(double) * size_t(p.total_units) * size_t(p.pstride), 256);
  p.off_efrag = off;
  off = align_up(off + sizeof(double) * size_t(n), 256);
  p.off_flags = off;
  off = align_up(off + sizeof(int) * 5 * size_t(n), 256);
  p.off_items = off;
  off = align_up(off + sizeof(sie::Item) * size_t(p.total_work), 256);
  p.off_split = off;
  off = align_up(off + split_bytes, 256);
  p.off_adj = off;
  off = align_up(off + (sizeof(sie::AdjRec) + sizeof(sie::AdjGroup) + sizeof(sie::AdjSlice)) *
                           p.adj_recs + 512, 256);
  p.off_t1 = off;
  if (grad) off = align_up(off + sizeof(double) * size_t(kT1Batch) * size_t(p.nv_max), 256);
  p.off_parts = off;
  if (grad) off = align_up(off + sizeof(double) * p.part_elems, 256);
  if (grad) {
    p.off_eo = off;
    off = align_up(off + sizeof(double) * size_t(p.total_units) * size_t(p.pstride), 256);
    p.off_eou = off;
    off = align_up(off + sizeof(double) * size_t(p.total_units), 256);
    p.off_evp = off;
    off = align_up(off + sizeof(double) * kGradRoundItems * size_t(p.pstride) *
                             size_t(p.nv_max), 256);
    p.off_evi = off;
    off = align_up(off + sizeof(double) * kGradRoundItems * size_t(p.nv_max), 256);
  }
  p.off_arena = off;
  p.fixed_bytes = off;
  return p;
}


// allow_proj: the entry point evaluates the fragment projector C^f (the
// single-fragment energy and the projector matrix); elsewhere it is rejected.
sie_status check_fragment(const sie_fragment* f, sie_precision prec, const char* who,
                          bool allow_proj = false) {
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
      return fail(SIE_ERR_NONFINITE, w + ": eps_occ has a non-finite entry");
    max_occ = f->eps_occ[i] > max_occ ? f->eps_occ[i] : max_occ;
  }
  for (int a = 0; a < f->n_vir; ++a) {
    if (!std::isfinite(f->eps_vir[a]))
      return fail(SIE_ERR_NONFINITE, w + ": eps_vir has a non-finite entry");
    min_vir = f->eps_vir[a] < min_vir ? f->eps_vir[a] : min_vir;
  }
  if (!(max_occ < min_vir))
    return fail(SIE_ERR_INVALID_ARG,
                w + ": max(eps_occ) >= min(eps_vir): a triples denominator would not be negative");
  if (f->frag_proj) {
    if (!allow_proj)
      return fail(SIE_ERR_UNSUPPORTED,
                  w + ": the fragment projector C^f is supported by sie_triples_energy and "
                      "sie_triples_projector_matrix only");
    for (int64_t q = 0; q < int64_t(f->n_occ) * f->n_occ; ++q)
      if (!std::isfinite(f->frag_proj[q]))
        return fail(SIE_ERR_NONFINITE, w + ": frag_proj has a non-finite entry");
  }
  // the float64 build and the gradient contractions address each operand
  // with 32-bit byte offsets from a per-term base: the largest extent is an
  // l-sum's t2 pair block plus a row
  const double o = f->n_occ, v = f->n_vir;
  if (double(esz) * (o * o * v * v + v * v * v + v * v) >= 4294967296.0)
    return fail(SIE_ERR_UNSUPPORTED,
                w + ": (element size) x (n_occ^2 n_vir^2 + n_vir^3 + n_vir^2) must be below 2^32");
  // the split build's largest extent: a (K = d) split copy's i-slice, 4 bytes
  // per padded element
  const double kv = double(round_up(size_t(f->n_vir), sie::kKs));
  if (prec == SIE_SPLIT_BF16 && 4.0 * v * (v + 1) * kv >= 4294967296.0)
    return fail(SIE_ERR_UNSUPPORTED,
                w + ": split precision needs 4 n_vir (n_vir + 1) round_up(n_vir, 32) below 2^32");
  return SIE_OK;
}

}  // namespace

namespace sie {
// Error reporting for the other host translation units (sie_mp2.hip).
sie_status set_error(sie_status s, const std::string& msg) { return fail(s, msg); }
}  // namespace sie

namespace {

sie_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return SIE_OK;
  return fail(SIE_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

sie_status fail_hip(hipError_t e, const std::string& what) {
  return fail(SIE_ERR_HIP, what + ": " + hipGetErrorString(e));
}

// ---- float64 build tile table: (n_v upper bound, variant), ascending ----
// The built-in table comes from the autotuner (tile_table.inc); callers may
// install another with sie_set_tile_table.
struct TileEntry {
  int32_t nv_max, variant;
};
const TileEntry kBuiltinTiles[] = {
#include "tile_table.inc"
};
std::mutex g_tiles_mu;
std::vector<TileEntry> g_tiles(std::begin(kBuiltinTiles), std::end(kBuiltinTiles));

int tile_variant(int nv) {
  std::lock_guard<std::mutex> lock(g_tiles_mu);
  for (const TileEntry& e : g_tiles)
    if (nv <= e.nv_max) return e.variant;
  return 0;
}

// ---- split build tile shape: forced, else the tuned table (split_table.inc,
// or one installed by sie_set_split_table), else by padded area
// (sie::split_shape_of) ----
std::atomic<int> g_split_forced{-1};
const TileEntry kBuiltinSplit[] = {
#include "split_table.inc"
    {0, -1}};   // terminator (also keeps the array non-empty)
std::mutex g_split_mu;
std::vector<TileEntry> g_split(std::begin(kBuiltinSplit), std::end(kBuiltinSplit) - 1);

int split_shape(int nv) {
  const int f = g_split_forced.load();
  if (f >= 0) return f;
  {
    std::lock_guard<std::mutex> lock(g_split_mu);
    for (const TileEntry& e : g_split)
      if (nv <= e.nv_max) return e.variant;
  }
  return sie::split_shape_of(nv);
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

int32_t sie_tile_variants(void) { return sie::kWVariants; }

int32_t sie_tile_variant_of(int32_t n_vir) { return n_vir < 1 ? -1 : tile_variant(n_vir); }

sie_status sie_tile_variant_shape(int32_t variant, int32_t* shape) {
  if (variant < 0 || variant >= sie::kWVariants || !shape)
    return fail(SIE_ERR_INVALID_ARG, "sie_tile_variant_shape: bad variant or NULL output");
  const sie::WShape w = sie::wshape(variant);
  shape[0] = w.blk;
  shape[1] = w.tr;
  shape[2] = w.tc;
  shape[3] = w.bpc;
  shape[4] = w.wr;
  shape[5] = w.wc;
  shape[6] = w.lay;
  shape[7] = w.ks;
  return SIE_OK;
}

sie_status sie_set_tile_table(int32_t n, const int32_t* nv_max, const int32_t* variant) {
  std::vector<TileEntry> t;
  if (n < 0 || (n > 0 && (!nv_max || !variant)))
    return fail(SIE_ERR_INVALID_ARG, "sie_set_tile_table: bad count or NULL arrays");
  for (int32_t q = 0; q < n; ++q) {
    if (variant[q] < 0 || variant[q] >= sie::kWVariants)
      return fail(SIE_ERR_INVALID_ARG, "sie_set_tile_table: unknown variant");
    if (nv_max[q] < 1 || (q > 0 && nv_max[q] <= nv_max[q - 1]))
      return fail(SIE_ERR_INVALID_ARG, "sie_set_tile_table: bounds must be positive and ascending");
    t.push_back(TileEntry{nv_max[q], variant[q]});
  }
  if (n == 0) t.assign(std::begin(kBuiltinTiles), std::end(kBuiltinTiles));
  std::lock_guard<std::mutex> lock(g_tiles_mu);
  g_tiles.swap(t);
  return SIE_OK;
}

int32_t sie_split_shape_of(int32_t n_vir) { return n_vir < 1 ? -1 : split_shape(n_vir); }

sie_status sie_set_split_shape(int32_t shape) {
  if (shape < -1 || shape >= sie::kSShapes)
    return fail(SIE_ERR_INVALID_ARG, "sie_set_split_shape: shape out of range");
  g_split_forced.store(shape);
  return SIE_OK;
}
sie_status sie_set_split_table(int32_t n, const int32_t* nv_max, const int32_t* shape) {
  std::vector<TileEntry> t;
  if (n < 0 || (n > 0 && (!nv_max || !shape)))
    return fail(SIE_ERR_INVALID_ARG, "sie_set_split_table: bad count or NULL arrays");
  for (int32_t q = 0; q < n; ++q) {
    if (shape[q] < 0 || shape[q] >= sie::kSShapes)
      return fail(SIE_ERR_INVALID_ARG, "sie_set_split_table: unknown shape");
    if (nv_max[q] < 1 || (q > 0 && nv_max[q] <= nv_max[q - 1]))
      return fail(SIE_ERR_INVALID_ARG, "sie_set_split_table: bounds must be positive and ascending");
    t.push_back(TileEntry{nv_max[q], shape[q]});
  }
  if (n == 0) t.assign(std::begin(kBuiltinSplit), std::end(kBuiltinSplit) - 1);
  std::lock_guard<std::mutex> lock(g_split_mu);
  g_split.swap(t);
  return SIE_OK;
}
static_assert(SIE_SPLIT_SHAPES == sie::kSShapes, "header and kernels agree on the split shapes");

const char* sie_last_error(void) { return g_err.c_str(); }

void sie_set_check_finite(int on) { g_check_finite.store(on ? 1 : 0); }

int64_t sie_occupied_triples(int32_t n_occ) {
  return n_occ < 0 ? 0 : sie::tetra(n_occ);
}

}  // extern "C"

namespace {

size_t proj_workspace(const sie_fragment& f, sie_precision p, size_t max_bytes);

size_t workspace_size(const sie_fragment* frags, int32_t n, sie_precision p, size_t max_bytes,
                      bool grad, const char* who) {
  const std::string w(who);
  if (!frags || n < 1) {
    fail(SIE_ERR_INVALID_ARG, w + ": need at least one fragment");
    return 0;
  }
  if (!grad && n == 1 && frags[0].frag_proj) {   // the single-fragment projector energy
    if (check_fragment(&frags[0], p, who, true) != SIE_OK) return 0;
    return proj_workspace(frags[0], p, max_bytes);
  }
  for (int32_t x = 0; x < n; ++x)
    if (check_fragment(&frags[x], p, who) != SIE_OK) return 0;
  const size_t cap = max_bytes ? max_bytes : default_cap();
  const Plan pl = make_plan(frags, n, p, grad);
  const size_t need_min = pl.fixed_bytes + pl.min_arena;
  if (need_min > cap) {
    fail(SIE_ERR_WORKSPACE, w + ": cap below the minimum workspace");
    return 0;
  }
  size_t arena = cap - pl.fixed_bytes;
  if (arena > pl.all_arena) arena = pl.all_arena;
  if (arena < pl.min_arena) arena = pl.min_arena;
  return pl.fixed_bytes + arena;
}

}  // namespace

namespace {

// ---- density-fitting input (sie_triples_energy_df) ----
// Workspace: [formed blocks][the energy's workspace for the formed fragment].
// Formed blocks: float64 ovvv, ooov, ovov (SIE_FP64), or float32 ooov, ovov
// and one float32 (ia|bc) slice (SIE_SPLIT_BF16).
struct DfPlan {
  size_t off_ovvv = 0, off_ooov = 0, off_ovov = 0, off_slice = 0, bytes = 0;
};

DfPlan df_plan(const sie_fragment_df& f, sie_precision p) {
  DfPlan q;
  const size_t o = size_t(f.n_occ), v = size_t(f.n_vir);
  const size_t esz = p == SIE_FP64 ? sizeof(double) : sizeof(float);
  size_t off = 0;
  if (p == SIE_FP64) {
    q.off_ovvv = off;
    off = align_up(off + esz * o * v * v * v, 256);
  }
  q.off_ooov = off;
  off = align_up(off + esz * o * o * o * v, 256);
  q.off_ovov = off;
  off = align_up(off + esz * o * v * o * v, 256);
  if (p != SIE_FP64) {
    q.off_slice = off;
    off = align_up(off + sizeof(float) * v * v * v, 256);
  }
  q.bytes = off;
  return q;
}

sie_status check_df(const sie_fragment_df* f, sie_precision p, const std::string& w) {
  if (!f) return fail(SIE_ERR_INVALID_ARG, w + ": fragment descriptor is NULL");
  if (p != SIE_FP64 && p != SIE_SPLIT_BF16)
    return fail(SIE_ERR_INVALID_ARG, w + ": unknown precision");
  if (f->n_occ < 1 || f->n_occ > SIE_MAX_OCC || f->n_vir < 1 || f->n_vir > SIE_MAX_VIR)
    return fail(SIE_ERR_INVALID_ARG, w + ": n_occ or n_vir out of range");
  if (f->n_aux < 1) return fail(SIE_ERR_INVALID_ARG, w + ": n_aux must be >= 1");
  if (!f->b || !aligned(f->b, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, w + ": b is NULL or not aligned to 8 bytes");
  const double n = double(f->n_occ) + f->n_vir;
  if (8.0 * n * n * f->n_aux >= 9.2e18)
    return fail(SIE_ERR_INVALID_ARG, w + ": b is too large");
  return SIE_OK;
}

// The descriptor of the formed fragment: integral blocks in the formed-block
// region (for the split form ovvv points at the slice buffer; the split
// staging forms the (ia|bc) copy from the factors instead of reading it).
sie_fragment df_fragment(const sie_fragment_df& f, sie_precision p, char* region,
                         const DfPlan& q) {
  sie_fragment g{};
  g.n_occ = f.n_occ;
  g.n_vir = f.n_vir;
  g.eps_occ = f.eps_occ;
  g.eps_vir = f.eps_vir;
  g.t1 = f.t1;
  g.t2 = f.t2;
  g.ovvv = region + (p == SIE_FP64 ? q.off_ovvv : q.off_slice);
  g.ooov = region + q.off_ooov;
  g.ovov = region + q.off_ovov;
  g.frag_proj = nullptr;
  return g;
}

}  // namespace

extern "C" {

size_t sie_triples_workspace_size(const sie_fragment* frags, int32_t n, sie_precision p,
                                  size_t max_bytes) {
  return workspace_size(frags, n, p, max_bytes, false, "sie_triples_workspace_size");
}

size_t sie_triples_backward_workspace_size(const sie_fragment* frags, int32_t n,
                                           sie_precision p, size_t max_bytes) {
  return workspace_size(frags, n, p, max_bytes, true, "sie_triples_backward_workspace_size");
}

}  // extern "C"

namespace {

// Host tables of one evaluation: descriptors, orbital energies, and the
// work items (units of all fragments, longest first) cut into rounds whose
// cube pairs fit in the arena.
struct Tables {
  std::vector<sie::FragDesc> desc;
  std::vector<double> eps;
  std::vector<sie::Item> items;
  std::vector<size_t> round_begin;   // item index of each round's start, then the end
  struct Segment {
    size_t round, r0, r1;            // items [r0, r1) of the round share a tile variant
    int variant;
  };
  std::vector<Segment> segments;     // in round order
};

void make_tables(const sie_fragment* frags, int n, const Plan& pl, char* base,
                 size_t arena_bytes, const sie_fragment_grad* grads, Tables& T) {
  auto dev = [&](size_t off) { return base + off; };
  std::vector<sie::FragDesc>& desc = T.desc;
  std::vector<double>& eps = T.eps;
  desc.assign(static_cast<size_t>(n), sie::FragDesc{});
  eps.clear();
  int64_t unit_base = 0;
  size_t split_off = pl.off_split;
  for (int x = 0; x < n; ++x) {
    const sie_fragment& f = frags[x];
    const FragPlan& fp = pl.frags[size_t(x)];
    sie::FragDesc& d = desc[size_t(x)];
    d.t1 = f.t1; d.t2 = f.t2; d.ovvv = f.ovvv; d.ooov = f.ooov; d.ovov = f.ovov;
    d.eps = reinterpret_cast<const double*>(dev(pl.off_eps)) + eps.size();
    eps.insert(eps.end(), f.eps_occ, f.eps_occ + f.n_occ);
    eps.insert(eps.end(), f.eps_vir, f.eps_vir + f.n_vir);
    d.no = fp.no;
    d.nv = fp.nv;
    d.Kv = fp.Kv;
    d.Ko = fp.Ko;
    // 16-byte row reads need an even row length and 16-byte aligned bases
    d.vec = (!pl.split && fp.nv % 2 == 0 && aligned(f.t2, 16) && aligned(f.ovvv, 16)) ? 1 : 0;
    d.epv = (fp.nv % 2 == 0 && aligned(f.ovov, pl.split ? 8 : 16)) ? 1 : 0;
    d.n_part = fp.n_part;
    d.unit_base = unit_base;
    d.half = int64_t(fp.half_bytes / (pl.split ? sizeof(float) : sizeof(double)));
    // work-groups of one layout (split) or of one unit (float64)
    d.variant = fp.variant;
    d.pair = pl.pair ? 1 : 0;
    d.lay3 = fp.lay3 ? 1 : 0;
    d.blocked = pl.blocked ? 1 : 0;
    d.tiles = pl.split ? sie::split_tiles(fp.nv, d.variant)
                       : sie::wbuild_tiles(fp.nv, d.variant);
    d.vS = d.tS = d.tT = d.oT = nullptr;
    d.g_t1 = grads ? grads[x].t1 : nullptr;
    d.g_t2 = grads ? grads[x].t2 : nullptr;
    d.g_ovvv = grads ? grads[x].ovvv : nullptr;
    d.g_ooov = grads ? grads[x].ooov : nullptr;
    d.g_ovov = grads ? grads[x].ovov : nullptr;
    d.g_eo = grads ? grads[x].eps_occ : nullptr;
    d.g_ev = grads ? grads[x].eps_vir : nullptr;
    if (pl.split) {
      const size_t o = size_t(fp.no), v = size_t(fp.nv);
      d.vS = reinterpret_cast<const sie::u4v*>(dev(split_off));
      split_off += align_up(4 * o * v * v * size_t(fp.Kv), 256);
      d.tS = reinterpret_cast<const sie::u4v*>(dev(split_off));
      split_off += align_up(4 * o * o * v * size_t(fp.Kv), 256);
      d.tT = reinterpret_cast<const sie::u4v*>(dev(split_off));
      split_off += align_up(4 * o * v * v * size_t(fp.Ko), 256);
      d.oT = reinterpret_cast<const sie::u4v*>(dev(split_off));
      split_off += align_up(4 * o * o * v * size_t(fp.Ko), 256);
    }
    unit_base += fp.n_units;
  }

  // units that are not i = j = k, longest first (stable within a fragment);
  // a pair unit (sie::unit_triple) builds one layout and costs half
  struct Unit {
    int frag, unit;
    bool one;
    double cost;
  };
  std::vector<Unit> order;
  order.reserve(size_t(pl.total_work));
  for (int x = 0; x < n; ++x) {
    const FragPlan& fp = pl.frags[size_t(x)];
    int u = 0;
    for (int i = 0; i < fp.no; ++i)
      for (int j = 0; j <= i; ++j)
        for (int k = 0; k <= j; ++k, ++u)
          if (i != k) {
            const bool one = pl.pair && (i == j || j == k);
            order.push_back({x, u, one, one ? (fp.lay3 ? 2.0 / 3.0 : 0.5) * fp.unit_cost : fp.unit_cost});
          }
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const Unit& a, const Unit& b) { return a.cost > b.cost; });
  auto layouts = [&](const sie::Item& it) {   // build layouts of an item
    int i, j, k;
    const FragPlan& fp = pl.frags[size_t(it.frag)];
    const bool one = sie::unit_triple(it.unit, fp.no, pl.pair, i, j, k);
    return (fp.lay3 ? 3 : 2) - (one ? 1 : 0);
  };

  // rounds: consecutive items whose cube pairs fit in the arena.  A first
  // greedy pass counts the rounds; the cut then aims at equal rounds (bytes
  // and, for the gradient, items) so that the last round is not a small
  // remainder, keeping the greedy cut if the balanced one needs more rounds.
  std::vector<sie::Item>& items = T.items;
  std::vector<size_t>& round_begin = T.round_begin;
  items.assign(order.size(), sie::Item{});
  round_begin.clear();
  auto item_bytes = [&](size_t r) {
    const FragPlan& fp = pl.frags[size_t(order[r].frag)];
    return size_t(order[r].one ? fp.cubes_pair : fp.cubes) * fp.half_bytes;
  };
  auto count_rounds = [&](size_t cap_bytes, size_t cap_items) {
    size_t n = 0, used = 0, cnt = 0;
    for (size_t r = 0; r < order.size(); ++r) {
      const size_t b = item_bytes(r);
      if (r == 0 || used + b > cap_bytes || cnt >= cap_items) {
        ++n;
        used = 0;
        cnt = 0;
      }
      used += b;
      ++cnt;
    }
    return n;
  };
  size_t cap_bytes = arena_bytes;
  size_t cap_items = grads ? kGradRoundItems : order.size() + 1;
  {
    const size_t n_greedy = count_rounds(cap_bytes, cap_items);
    if (n_greedy > 1) {
      size_t total = 0;
      for (size_t r = 0; r < order.size(); ++r) total += item_bytes(r);
      const size_t tb = (total + n_greedy - 1) / n_greedy;
      const size_t ti = (order.size() + n_greedy - 1) / n_greedy;
      size_t bb = tb, bi = ti;
      // grow the targets until the balanced cut fits in as many rounds
      for (int tries = 0; tries < 64; ++tries) {
        const size_t cb = bb < arena_bytes ? bb : arena_bytes;
        const size_t ci = bi < cap_items ? bi : cap_items;
        if (count_rounds(cb, ci) <= n_greedy) {
          cap_bytes = cb;
          cap_items = ci;
          break;
        }
        bb += (tb + 31) / 32;
        bi += (ti + 31) / 32;
      }
    }
  }
  {
    size_t used = 0;
    int64_t blk = 0, part = 0;
    const size_t elem = pl.split ? sizeof(float) : sizeof(double);
    for (size_t r = 0; r < order.size(); ++r) {
      const FragPlan& fp = pl.frags[size_t(order[r].frag)];
      const size_t pair = item_bytes(r);
      const bool full = r > 0 && r - round_begin.back() >= cap_items;
      if (r == 0 || used + pair > cap_bytes || full) {
        round_begin.push_back(r);
        used = 0;
        blk = 0;
        part = 0;
      }
      sie::Item& it = items[r];
      it.frag = order[r].frag;
      it.unit = order[r].unit;
      it.cube_off = int64_t(used / elem);
      used += pair;
      blk += layouts(it) * desc[size_t(it.frag)].tiles;
      part += fp.n_part;
      it.blk_end = blk;
      it.part_end = part;
    }
    round_begin.push_back(order.size());
  }
  // the build launches once per tile variant of a round, so group each
  // round's items by variant (stable) and restart the block prefix sums at
  // each variant's segment; the epilogue prefix sums run over the round.
  T.segments.clear();
  for (size_t q = 0; q + 1 < round_begin.size(); ++q) {
    const size_t r0 = round_begin[q], r1 = round_begin[q + 1];
    std::stable_sort(items.begin() + r0, items.begin() + r1,
                     [&](const sie::Item& a, const sie::Item& b) {
                       return desc[size_t(a.frag)].variant < desc[size_t(b.frag)].variant;
                     });
    int64_t blk = 0, part = 0;
    size_t seg0 = r0;
    for (size_t r = r0; r < r1; ++r) {
      sie::Item& it = items[r];
      const int var = desc[size_t(it.frag)].variant;
      if (r > r0 && var != desc[size_t(items[r - 1].frag)].variant) {
        T.segments.push_back({q, seg0, r, desc[size_t(items[r - 1].frag)].variant});
        seg0 = r;
        blk = 0;
      }
      blk += layouts(it) * desc[size_t(it.frag)].tiles;
      part += pl.frags[size_t(it.frag)].n_part;
      it.blk_end = blk;
      it.part_end = part;
    }
    if (r1 > r0) T.segments.push_back({q, seg0, r1, desc[size_t(items[r1 - 1].frag)].variant});
  }
}

// float64 build launches of round q (one per tile variant present).
void build_round_f64(const Tables& T, size_t q, hipStream_t s, const sie::FragDesc* desc,
                     const sie::Item* d_items, double* arena) {
  for (const auto& sg : T.segments) {
    if (sg.round != q) continue;
    sie::launch_build_f64(sg.variant, unsigned(T.items[sg.r1 - 1].blk_end), s, desc,
                          d_items + sg.r0, int(sg.r1 - sg.r0), arena);
  }
}

void build_round_split(const Tables& T, size_t q, hipStream_t s, const sie::FragDesc* desc,
                       const sie::Item* d_items, float* arena) {
  for (const auto& sg : T.segments) {
    if (sg.round != q) continue;
    sie::launch_build_split(sg.variant, unsigned(T.items[sg.r1 - 1].blk_end), s, desc,
                            d_items + sg.r0, int(sg.r1 - sg.r0), arena);
  }
}

// bf16 hi/lo copies of every fragment's float32 inputs (see k_bf16.hpp).
// Density-fitting source of a split evaluation (sie_triples_energy_df): the
// (ia|bc) split copy is formed from the factors one occupied slice at a time
// through `slice` (n_v^3 float32) instead of from an ovvv array.
struct DfSource {
  const double* b = nullptr;
  int n_aux = 0;
  float* slice = nullptr;
};

// The factor maps of the blocks, b [n_aux][n][n] with n = n_o + n_v.
sie::DfArgs df_args(const double* b, int naux, int no, int nv) {
  sie::DfArgs a{};
  a.b = b;
  a.plane = int64_t(no + nv) * (no + nv);
  a.naux = naux;
  return a;
}

// (ia|bc) of occupied i: rows a, cols (b, c) -> out[a][b][c]
template <typename OutT>
void df_ovvv_slice(hipStream_t s, const double* b, int naux, int no, int nv, int i, OutT* out) {
  const int64_t n = no + nv;
  sie::DfArgs a = df_args(b, naux, no, nv);
  a.M = nv;
  a.N = nv * nv;
  a.x = sie::DfMap{int64_t(i) * n + no, 1 << 30, 0, 1};
  a.y = sie::DfMap{int64_t(no) * n + no, nv, n, 1};
  a.ldc = int64_t(nv) * nv;
  if (sizeof(OutT) == 8) sie::launch_df_form_f64(s, a, reinterpret_cast<double*>(out));
  else sie::launch_df_form_f32(s, a, reinterpret_cast<float*>(out));
}

// (jl|ia) -> out[j][l][i][a] and (ia|jb) -> out[i][a][j][b]
template <typename OutT>
void df_ooov_ovov(hipStream_t s, const double* b, int naux, int no, int nv, OutT* ooov,
                  OutT* ovov) {
  const int64_t n = no + nv;
  const sie::DfMap oo{0, no, n, 1}, ov{no, nv, n, 1};
  sie::DfArgs a = df_args(b, naux, no, nv);
  a.M = no * no;
  a.N = no * nv;
  a.x = oo;
  a.y = ov;
  a.ldc = int64_t(no) * nv;
  sie::DfArgs c = a;
  c.M = no * nv;
  c.x = ov;
  if (sizeof(OutT) == 8) {
    sie::launch_df_form_f64(s, a, reinterpret_cast<double*>(ooov));
    sie::launch_df_form_f64(s, c, reinterpret_cast<double*>(ovov));
  } else {
    sie::launch_df_form_f32(s, a, reinterpret_cast<float*>(ooov));
    sie::launch_df_form_f32(s, c, reinterpret_cast<float*>(ovov));
  }
}

sie_status stage_split(const std::vector<sie::FragDesc>& desc, hipStream_t s,
                       const DfSource* df = nullptr) {
  ProfScope ps(s, 3);
  auto split = [&](const void* src, int P, int X, int Y, int64_t sp, int64_t sx, int64_t sy,
                   int64_t sk, int K, int Kpad, bool kfast, const sie::u4v* dst) {
    const int64_t total = int64_t(P) * X * Y * (Kpad / 8);
    const int64_t nb = (total + 255) / 256;
    const unsigned grid = unsigned(nb < 65536 ? nb : 65536);
    sie::launch_split_bf16(grid, s, static_cast<const float*>(src), P, X, Y, sp, sx, sy, sk, K,
                           Kpad, kfast, const_cast<sie::u4v*>(dst));
  };
  for (const sie::FragDesc& d : desc) {
    const int no = d.no, nv = d.nv;
    const int64_t o = no, v = nv;
    // vS[i][a][b][d] <- ovvv, tS[i][j][a][d] <- t2 (K = d contiguous)
    if (df) {   // one formed (ia|bc) slice at a time
      for (int i = 0; i < no; ++i) {
        df_ovvv_slice(s, df->b, df->n_aux, no, nv, i, df->slice);
        split(df->slice, 1, nv, nv, v * v * v, v * v, v, 1, nv, d.Kv, true,
              d.vS + int64_t(i) * v * v * (d.Kv / 8) * 2);
      }
    } else {
      split(d.ovvv, no, nv, nv, v * v * v, v * v, v, 1, nv, d.Kv, true, d.vS);
    }
    split(d.t2, no, no, nv, o * v * v, v * v, v, 1, nv, d.Kv, true, d.tS);
    // tT[p][x][y][l] = t2[p][l][x][y], oT[x][y][v][l] = ooov[x][l][y][v] (K = l)
    split(d.t2, no, nv, nv, o * v * v, v, 1, v * v, no, d.Ko, false, d.tT);
    split(d.ooov, no, no, nv, o * o * v, v, 1, o * v, no, d.Ko, false, d.oT);
  }
  return hip_check(hipGetLastError(), "launch split staging");
}

// With the finite check on: scans every fragment's t1, t2, ovvv, ooov and
// ovov for NaN or infinity, waits for the scan, and reports the first
// offender.  This is the only path on which a call waits for the device.
sie_status scan_finite(const sie_fragment* frags, int n, bool f64, int* d_flags, hipStream_t s,
                       const std::string& w) {
  static const char* kNames[5] = {"t1", "t2", "ovvv", "ooov", "ovov"};
  sie::launch_zero_flags(s, d_flags, 5 * n);
  for (int x = 0; x < n; ++x) {
    const sie_fragment& f = frags[x];
    const int64_t o = f.n_occ, v = f.n_vir;
    const void* ptr[5] = {f.t1, f.t2, f.ovvv, f.ooov, f.ovov};
    const int64_t cnt[5] = {o * v, o * o * v * v, o * v * v * v, o * o * o * v, o * v * o * v};
    for (int a = 0; a < 5; ++a) sie::launch_nonfinite(s, ptr[a], f64, cnt[a], d_flags, 5 * x + a);
  }
  sie_status st = hip_check(hipGetLastError(), "launch finite scan");
  if (st != SIE_OK) return st;
  std::vector<int> h(size_t(5) * size_t(n), 0);
  st = hip_check(hipMemcpyAsync(h.data(), d_flags, sizeof(int) * h.size(), hipMemcpyDeviceToHost, s),
                 "read finite scan");
  if (st == SIE_OK) st = hip_check(hipStreamSynchronize(s), "finite scan");
  if (st != SIE_OK) return st;
  for (int q = 0; q < 5 * n; ++q)
    if (h[size_t(q)])
      return fail(SIE_ERR_NONFINITE, w + ": fragment " + std::to_string(q / 5) + ": " +
                                         kNames[q % 5] + " holds a non-finite value");
  return SIE_OK;
}

// One evaluation over n fragments (see work.hpp).
// With `direct` set the tables are copied straight from the host vectors
// (pageable copies, which HIP completes before returning) instead of through
// the page-locked staging ring, so the call allocates nothing anywhere.
sie_status run(const sie_fragment* frags, int n, sie_precision p, double* e_frag_out,
               double* e_total, double* e_triples, void* ws, size_t ws_bytes, void* stream,
               const char* who, bool direct = false, const DfSource* df = nullptr) {
  const std::string w(who);
  if (!frags || n < 1) return fail(SIE_ERR_INVALID_ARG, w + ": need at least one fragment");
  for (int x = 0; x < n; ++x) {
    sie_status st = check_fragment(&frags[x], p, who);
    if (st != SIE_OK) return st;
  }
  const Plan pl = make_plan(frags, n, p);
  if (!ws || !aligned(ws, 256))
    return fail(SIE_ERR_WORKSPACE, w + ": workspace is NULL or not 256-byte aligned");
  if (ws_bytes < pl.fixed_bytes + pl.min_arena)
    return fail(SIE_ERR_WORKSPACE,
                w + ": workspace smaller than required (see sie_triples_workspace_size)");
  const size_t arena_bytes = ws_bytes - pl.fixed_bytes;

  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  auto dev = [&](size_t off) { return base + off; };

  Tables T;
  make_tables(frags, n, pl, base, arena_bytes, nullptr, T);
  std::vector<sie::FragDesc>& desc = T.desc;
  std::vector<double>& eps = T.eps;
  std::vector<sie::Item>& items = T.items;
  std::vector<size_t>& round_begin = T.round_begin;

  // ---- uploads: page-locked staging, stream-ordered, no host wait ----
  sie_status st = SIE_OK;
  if (direct) {
    const std::pair<size_t, std::pair<const void*, size_t>> parts[3] = {
        {pl.off_desc, {desc.data(), sizeof(sie::FragDesc) * desc.size()}},
        {pl.off_eps, {eps.data(), sizeof(double) * eps.size()}},
        {pl.off_items, {items.data(), sizeof(sie::Item) * items.size()}}};
    for (const auto& pt : parts) {
      if (pt.second.second == 0) continue;
      st = hip_check(hipMemcpyAsync(dev(pt.first), pt.second.first, pt.second.second,
                                    hipMemcpyHostToDevice, s),
                     "upload tables");
      if (st != SIE_OK) return st;
    }
  } else {
    sie::Staging::Batch up;
    const size_t bytes = sie::Staging::padded(sizeof(sie::FragDesc) * desc.size()) +
                         sie::Staging::padded(sizeof(double) * eps.size()) +
                         sie::Staging::padded(sizeof(sie::Item) * items.size());
    st = hip_check(g_staging.begin(bytes, up), "stage tables");
    if (st != SIE_OK) return st;
    up.add(dev(pl.off_desc), desc.data(), sizeof(sie::FragDesc) * desc.size());
    up.add(dev(pl.off_eps), eps.data(), sizeof(double) * eps.size());
    up.add(dev(pl.off_items), items.data(), sizeof(sie::Item) * items.size());
    st = hip_check(up.commit(s), "upload tables");
    if (st != SIE_OK) return st;
  }
  if (check_finite_on() && !df) {   // (the density-fitting entry scans its own inputs)
    st = scan_finite(frags, n, !pl.split, reinterpret_cast<int*>(dev(pl.off_flags)), s, w);
    if (st != SIE_OK) return st;
  }

  const sie::FragDesc* d_desc = reinterpret_cast<const sie::FragDesc*>(dev(pl.off_desc));
  const sie::Item* d_items = reinterpret_cast<const sie::Item*>(dev(pl.off_items));
  double* d_units = (e_triples && n == 1) ? e_triples
                                          : reinterpret_cast<double*>(dev(pl.off_units));
  double* d_part = reinterpret_cast<double*>(dev(pl.off_part));
  double* d_efrag = e_frag_out ? e_frag_out : reinterpret_cast<double*>(dev(pl.off_efrag));

  // ---- split staging (split precision) ----
  if (pl.split) {
    st = stage_split(desc, s, df);
    if (st != SIE_OK) return st;
  }

  // ---- rounds ----
  for (size_t q = 0; q + 1 < round_begin.size(); ++q) {
    const size_t r0 = round_begin[q], r1 = round_begin[q + 1];
    if (r1 == r0) continue;
    const int cnt = int(r1 - r0);
    const unsigned n_epi = unsigned(items[r1 - 1].part_end);
    const sie::Item* ri = d_items + r0;
    if (!pl.split) {
      double* arena = reinterpret_cast<double*>(dev(pl.off_arena));
      {
        ProfScope ps(s, 0);
        build_round_f64(T, q, s, d_desc, d_items, arena);
      }
      {
        ProfScope ps(s, 1);
        sie::launch_epilogue_f64(n_epi, s, d_desc, ri, cnt, arena, d_part, pl.pstride);
      }
    } else {
      float* arena = reinterpret_cast<float*>(dev(pl.off_arena));
      {
        ProfScope ps(s, 0);
        build_round_split(T, q, s, d_desc, d_items, arena);
      }
      {
        ProfScope ps(s, 1);
        sie::launch_epilogue_f32(n_epi, s, d_desc, ri, cnt, arena, d_part, pl.pstride);
      }
    }
    st = hip_check(hipGetLastError(), "launch (T) kernels");
    if (st != SIE_OK) return st;
  }

  // ---- reductions ----
  {
    ProfScope ps(s, 2);
    int64_t max_units = 1;
    for (const auto& fp : pl.frags) max_units = fp.n_units > max_units ? fp.n_units : max_units;
    sie::launch_unit_energy(dim3(unsigned((max_units + 255) / 256), unsigned(n)), s, d_desc,
                            d_part, pl.pstride, d_units);
    sie::launch_frag_energy(unsigned(n), s, d_desc, d_units, d_efrag);
    if (e_total) sie::launch_sum_fixed(s, d_efrag, int64_t(n), e_total);
  }
  return hip_check(hipGetLastError(), "launch reductions");
}


// ---- fragment projector (k_proj.hpp) ----
// Workspace: [descriptor][e_occ|e_vir][items of every group][split copies]
// [product chunk slices][C^f][M][cube arena].  A group is the n_o ordered
// triples (i', j, k) of one occupied pair j >= k; a round holds as many
// groups as the arena fits (two row-major cubes per ordered triple).
struct ProjPlan {
  FragPlan fp;
  bool split = false;
  int64_t groups = 0, K = 0, chunk = 0;
  int chunks = 0;
  size_t off_desc = 0, off_eps = 0, off_items = 0, off_split = 0, off_part = 0, off_c = 0,
         off_m = 0, off_flags = 0, off_arena = 0, fixed = 0, group_bytes = 0;
};

ProjPlan proj_plan(const sie_fragment& f, sie_precision p) {
  ProjPlan q;
  q.split = p == SIE_SPLIT_BF16;
  q.fp = frag_plan(f.n_occ, f.n_vir, q.split);
  if (!q.split) {   // two-layout build shape (as the adjoint)
    q.fp.variant = tile_variant(q.fp.nv);
    if (sie::wshape(q.fp.variant).lay == 3) q.fp.variant = 0;
  } else {
    q.fp.variant = split_shape(q.fp.nv);
  }
  q.fp.lay3 = false;
  // 8^3-blocked cubes, as the energy's (k_proj_m runs over the padding too,
  // which k_proj_wq zeroes)
  q.fp.half_bytes = align_up((q.split ? sizeof(float) : sizeof(double)) *
                                 size_t(sie::cube_blocked_elems(q.fp.nv)), 256);
  const int64_t o = q.fp.no, v = q.fp.nv;
  q.groups = o * (o + 1) / 2;
  q.K = sie::cube_blocked_elems(q.fp.nv);
  q.chunk = 8192;   // about a thousand work-groups per product at 200 virtuals
  q.chunks = int((q.K + q.chunk - 1) / q.chunk);
  size_t off = 0;
  q.off_desc = off;
  off = align_up(off + sizeof(sie::FragDesc), 256);
  q.off_eps = off;
  off = align_up(off + sizeof(double) * size_t(o + v), 256);
  q.off_items = off;
  off = align_up(off + sizeof(sie::Item) * size_t(q.groups * o), 256);
  q.off_split = off;
  off = align_up(off + q.fp.split_bytes, 256);
  q.off_part = off;
  off = align_up(off + sizeof(double) * size_t(q.chunks) * size_t(o * o), 256);
  q.off_c = off;
  off = align_up(off + sizeof(double) * size_t(o * o), 256);
  q.off_m = off;
  off = align_up(off + sizeof(double) * size_t(o * o), 256);
  q.off_flags = off;
  off = align_up(off + sizeof(int) * 5, 256);
  q.off_arena = off;
  q.fixed = off;
  q.group_bytes = size_t(2) * size_t(o) * q.fp.half_bytes;
  return q;
}

size_t proj_workspace(const sie_fragment& f, sie_precision p, size_t max_bytes) {
  const ProjPlan q = proj_plan(f, p);
  const size_t cap = max_bytes ? max_bytes : default_cap();
  if (q.fixed + q.group_bytes > cap) {
    fail(SIE_ERR_WORKSPACE, "projector: cap below the minimum workspace (one group of cubes)");
    return 0;
  }
  size_t arena = cap - q.fixed;
  const size_t all = q.group_bytes * size_t(q.groups);
  if (arena > all) arena = all;
  arena = arena / q.group_bytes * q.group_bytes;
  return q.fixed + arena;
}

// M (device, n_o x n_o) of one fragment, and with c_host (the fragment's
// projector) also E_x = sum C M into e_out.
sie_status run_projector(const sie_fragment* f, sie_precision p, double* m_out, double* e_out,
                         void* ws, size_t ws_bytes, void* stream, const char* who) {
  const std::string w(who);
  const ProjPlan q = proj_plan(*f, p);
  if (!ws || !aligned(ws, 256))
    return fail(SIE_ERR_WORKSPACE, w + ": workspace is NULL or not 256-byte aligned");
  if (ws_bytes < q.fixed + q.group_bytes)
    return fail(SIE_ERR_WORKSPACE,
                w + ": workspace smaller than required (see sie_triples_projector_workspace_size)");
  const int64_t per_round = int64_t((ws_bytes - q.fixed) / q.group_bytes);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  auto dev = [&](size_t off) { return base + off; };
  const FragPlan& fp = q.fp;
  const int no = fp.no, nv = fp.nv;

  sie::FragDesc d{};
  d.t1 = f->t1; d.t2 = f->t2; d.ovvv = f->ovvv; d.ooov = f->ooov; d.ovov = f->ovov;
  d.eps = reinterpret_cast<const double*>(dev(q.off_eps));
  d.no = no;
  d.nv = nv;
  d.Kv = fp.Kv;
  d.Ko = fp.Ko;
  d.vec = (!q.split && nv % 2 == 0 && aligned(f->t2, 16) && aligned(f->ovvv, 16)) ? 1 : 0;
  d.epv = (nv % 2 == 0 && aligned(f->ovov, q.split ? 8 : 16)) ? 1 : 0;
  d.variant = fp.variant;
  d.pair = 0;
  d.lay3 = 0;
  d.blocked = 1;
  d.n_part = fp.n_part;
  d.unit_base = 0;
  d.half = int64_t(fp.half_bytes / (q.split ? sizeof(float) : sizeof(double)));
  d.tiles = q.split ? sie::split_tiles(nv, d.variant) : sie::wbuild_tiles(nv, d.variant);
  if (q.split) {
    const size_t o = size_t(no), v = size_t(nv);
    size_t off = q.off_split;
    d.vS = reinterpret_cast<const sie::u4v*>(dev(off));
    off += align_up(4 * o * v * v * size_t(fp.Kv), 256);
    d.tS = reinterpret_cast<const sie::u4v*>(dev(off));
    off += align_up(4 * o * o * v * size_t(fp.Kv), 256);
    d.tT = reinterpret_cast<const sie::u4v*>(dev(off));
    off += align_up(4 * o * v * v * size_t(fp.Ko), 256);
    d.oT = reinterpret_cast<const sie::u4v*>(dev(off));
  }
  std::vector<double> eps(f->eps_occ, f->eps_occ + no);
  eps.insert(eps.end(), f->eps_vir, f->eps_vir + nv);
  // items: group g = pair (j, k), j >= k in order; item i' of the group is
  // the ordered triple (i', j, k); prefix sums restart every round
  std::vector<sie::Item> items(size_t(q.groups * no));
  std::vector<std::pair<int, int>> pairs;
  for (int j = 0; j < no; ++j)
    for (int k = 0; k <= j; ++k) pairs.emplace_back(j, k);
  {
    int64_t blk = 0, part = 0;
    for (int64_t g = 0; g < q.groups; ++g) {
      if (g % per_round == 0) blk = part = 0;
      for (int i = 0; i < no; ++i) {
        sie::Item& it = items[size_t(g * no + i)];
        it.frag = 0;
        it.unit = sie::ordered_item(i, pairs[size_t(g)].first, pairs[size_t(g)].second, no);
        it.cube_off = ((g % per_round) * no + i) * 2 * d.half;
        blk += 2 * d.tiles;
        part += fp.n_part;
        it.blk_end = blk;
        it.part_end = part;
      }
    }
  }
  sie_status st = SIE_OK;
  {
    sie::Staging::Batch up;
    const size_t bytes = sie::Staging::padded(sizeof(sie::FragDesc)) +
                         sie::Staging::padded(sizeof(double) * eps.size()) +
                         sie::Staging::padded(sizeof(sie::Item) * items.size()) +
                         sie::Staging::padded(sizeof(double) * size_t(no) * no);
    st = hip_check(g_staging.begin(bytes, up), "stage tables");
    if (st != SIE_OK) return st;
    up.add(dev(q.off_desc), &d, sizeof(sie::FragDesc));
    up.add(dev(q.off_eps), eps.data(), sizeof(double) * eps.size());
    up.add(dev(q.off_items), items.data(), sizeof(sie::Item) * items.size());
    if (f->frag_proj) up.add(dev(q.off_c), f->frag_proj, sizeof(double) * size_t(no) * no);
    st = hip_check(up.commit(s), "upload tables");
    if (st != SIE_OK) return st;
  }
  if (check_finite_on()) {
    st = scan_finite(f, 1, !q.split, reinterpret_cast<int*>(dev(q.off_flags)), s, w);
    if (st != SIE_OK) return st;
  }
  const sie::FragDesc* d_desc = reinterpret_cast<const sie::FragDesc*>(dev(q.off_desc));
  const sie::Item* d_items = reinterpret_cast<const sie::Item*>(dev(q.off_items));
  double* d_m = m_out ? m_out : reinterpret_cast<double*>(dev(q.off_m));
  double* d_part = reinterpret_cast<double*>(dev(q.off_part));
  {
    const int64_t n = int64_t(no) * no;
    sie::launch_fill_zero(unsigned((n + 255) / 256), s, d_m, n);
  }
  if (q.split) {
    st = stage_split(std::vector<sie::FragDesc>{d}, s);
    if (st != SIE_OK) return st;
  }
  for (int64_t g0 = 0; g0 < q.groups; g0 += per_round) {
    const int64_t g1 = std::min(q.groups, g0 + per_round);
    const size_t r0 = size_t(g0 * no), r1 = size_t(g1 * no);
    const int cnt = int(r1 - r0);
    const sie::Item* ri = d_items + r0;
    void* arena = dev(q.off_arena);
    {
      ProfScope ps(s, 0);
      if (q.split)
        sie::launch_build_split(d.variant, unsigned(items[r1 - 1].blk_end), s, d_desc, ri, cnt,
                                static_cast<float*>(arena));
      else
        sie::launch_build_f64(d.variant, unsigned(items[r1 - 1].blk_end), s, d_desc, ri, cnt,
                              static_cast<double*>(arena));
    }
    {
      ProfScope ps(s, 1);
      if (q.split)
        sie::launch_proj_wq_f32(unsigned(items[r1 - 1].part_end), s, d_desc, ri, cnt,
                                static_cast<float*>(arena));
      else
        sie::launch_proj_wq_f64(unsigned(items[r1 - 1].part_end), s, d_desc, ri, cnt,
                                static_cast<double*>(arena));
    }
    {
      ProfScope ps(s, 2);
      for (int64_t g = g0; g < g1; ++g) {
        const int64_t off = ((g - g0) * no) * 2 * d.half;   // first item's cube pair
        const int64_t stride = 2 * d.half;
        if (q.split) {
          const float* a = static_cast<const float*>(arena) + off;
          sie::launch_proj_m_f32(s, a, a + d.half, stride, no, q.K, q.chunk, q.chunks, d_part);
        } else {
          const double* a = static_cast<const double*>(arena) + off;
          sie::launch_proj_m_f64(s, a, a + d.half, stride, no, q.K, q.chunk, q.chunks, d_part);
        }
        const bool diag = pairs[size_t(g)].first == pairs[size_t(g)].second;
        sie::launch_proj_msum(s, d_part, q.chunks, no, diag ? 1.0 / 3.0 : 2.0 / 3.0, d_m);
      }
    }
    st = hip_check(hipGetLastError(), "launch projector kernels");
    if (st != SIE_OK) return st;
  }
  if (e_out && f->frag_proj)
    sie::launch_proj_energy(s, reinterpret_cast<const double*>(dev(q.off_c)), d_m,
                            int64_t(no) * no, e_out);
  return hip_check(hipGetLastError(), "launch projector energy");
}

// Backward contraction lists of one round: for every class, the output slices
// the round's units touch (sorted), each with its records in item order.
using sie::AdjLaunch;

// Output-slice elements of a summed-block class for a fragment.
int64_t adj_slice_elems(int cls, int no, int nv) {
  return cls == sie::kAdjT2vv ? int64_t(nv) * nv : int64_t(nv) * no;
}

void adj_round_lists(const Tables& T, size_t r0, size_t r1, std::vector<sie::AdjGroup>& groups,
                     std::vector<sie::AdjRec>& recs, std::vector<sie::AdjSlice>& slices,
                     AdjLaunch (&launch)[sie::kAdjClasses]) {
  for (int cls = 0; cls < sie::kAdjClasses; ++cls) {
    struct Key {
      int frag, a0, a1;
      bool operator<(const Key& o) const {
        return frag != o.frag ? frag < o.frag : (a0 != o.a0 ? a0 < o.a0 : a1 < o.a1);
      }
    };
    std::vector<std::pair<Key, sie::AdjRec>> list;
    for (size_t r = r0; r < r1; ++r) {
      const sie::Item& it = T.items[r];
      const sie::FragDesc& d = T.desc[size_t(it.frag)];
      const bool want = cls == sie::kAdjOvvv ? d.g_ovvv != nullptr
                        : cls == sie::kAdjOoov ? d.g_ooov != nullptr
                        : cls == sie::kAdjOvov ? d.g_ovov != nullptr
                        : cls == sie::kAdjT1   ? d.g_t1 != nullptr
                                               : d.g_t2 != nullptr;
      if (!want) continue;
      // sorted triple of the unit index
      int i = 0, j = 0, k = 0;
      {
        int64_t u = it.unit;
        while (sie::tetra(i + 1) <= u) ++i;
        u -= sie::tetra(i);
        while (sie::tri(j + 1) <= u) ++j;
        k = int(u - sie::tri(j));
      }
      const int ng = sie::adj_reduce(cls) ? (d.nv + sie::kARB - 1) / sie::kARB : 1;
      for (int kind = 0; kind < sie::adj_kinds(cls); ++kind) {
        Key key{it.frag, 0, 0};
        sie::adj_slice(cls, kind, i, j, k, key.a0, key.a1);
        for (int g = 0; g < ng; ++g) {
          sie::AdjRec rec{int(r - r0), kind, g, 0};
          list.emplace_back(key, rec);
        }
      }
    }
    std::stable_sort(list.begin(), list.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    launch[cls].group_off = groups.size();
    launch[cls].n_groups = 0;
    launch[cls].rec_begin = int(recs.size());
    launch[cls].slice_off = slices.size();
    const bool red = sie::adj_reduce(cls);
    // summed-block classes: each slice's records split into contiguous
    // ranges of at most per_group[frag] records, each a group writing its
    // own partial slice.  per_group is the fragment's records over its
    // budget of kAdjParts n_o^2 partial slices less one per slice, so that
    // the ceilings stay within the budget the workspace holds and the
    // groups are of about equal length.
    std::vector<int64_t> per_group;
    if (red) {
      std::vector<int64_t> n_rec(T.desc.size(), 0), n_sl(T.desc.size(), 0);
      for (size_t q = 0; q < list.size(); ++q) {
        ++n_rec[size_t(list[q].first.frag)];
        if (q == 0 || list[q - 1].first < list[q].first) ++n_sl[size_t(list[q].first.frag)];
      }
      per_group.assign(T.desc.size(), 1);
      for (size_t f = 0; f < T.desc.size(); ++f) {
        const int64_t budget =
            int64_t(sie::kAdjParts) * T.desc[f].no * T.desc[f].no - n_sl[f];
        const int64_t b = budget > 1 ? budget : 1;
        per_group[f] = n_rec[f] > 0 ? (n_rec[f] + b - 1) / b : 1;
      }
    }
    int64_t wg = 0, part_elems = 0;
    for (size_t q = 0; q < list.size();) {
      size_t e = q;
      while (e < list.size() && !(list[q].first < list[e].first) && !(list[e].first < list[q].first))
        ++e;
      const Key& key = list[q].first;
      const sie::FragDesc& d = T.desc[size_t(key.frag)];
      const int n = int(e - q);
      const int np = red ? int((n + per_group[size_t(key.frag)] - 1) / per_group[size_t(key.frag)])
                         : 1;
      const int64_t el = red ? adj_slice_elems(cls, d.no, d.nv) : 0;
      const int64_t off0 = part_elems;
      if (red) {
        slices.push_back(sie::AdjSlice{key.frag, key.a0, key.a1, np, off0});
        part_elems += el * np;
        launch[cls].max_slice = el > launch[cls].max_slice ? el : launch[cls].max_slice;
        ++launch[cls].n_slices;
      }
      for (int pp = 0; pp < np; ++pp) {
        const size_t b0 = q + size_t(n) * pp / np, b1 = q + size_t(n) * (pp + 1) / np;
        sie::AdjGroup gr{};
        gr.frag = key.frag;
        gr.a0 = key.a0;
        gr.a1 = key.a1;
        gr.part_off = off0 + el * pp;
        gr.rec_begin = int(recs.size());
        for (size_t m = b0; m < b1; ++m) recs.push_back(list[m].second);
        gr.rec_end = int(recs.size());
        wg += sie::adj_tiles(cls, d.no, d.nv);
        gr.wg_end = wg;
        groups.push_back(gr);
        ++launch[cls].n_groups;
      }
      q = e;
    }
    if (cls <= sie::kAdjOoov) {
      // longest groups first in the grid (the dispatcher starts them in
      // order).  A summed-block group keeps its partial slice, and a
      // per-block slice has one group per launch, so no sum changes.
      const auto first = groups.begin() + std::ptrdiff_t(launch[cls].group_off);
      std::stable_sort(first, groups.end(), [](const sie::AdjGroup& a, const sie::AdjGroup& b) {
        return a.rec_end - a.rec_begin > b.rec_end - b.rec_begin;
      });
      wg = 0;
      for (auto g = first; g != groups.end(); ++g) {
        wg += sie::adj_tiles(cls, T.desc[size_t(g->frag)].no, T.desc[size_t(g->frag)].nv);
        g->wg_end = wg;
      }
    }
    launch[cls].n_wg = wg;
    launch[cls].rec_end = int(recs.size());
    launch[cls].part_elems = part_elems;
  }
}

// G / H and the gradient contractions of one backward round.
// eo_part NULL: no orbital-energy gradient is wanted.
void backward_round(bool split, const std::array<AdjLaunch, sie::kAdjClasses>& L, hipStream_t s,
                    const sie::AdjArgs& a, void* arena, double* d_part, int pstride,
                    const double* grad_e, unsigned n_epi, int n_frag, double* eo_part,
                    double* ev_part, double* ev_item, int ev_stride) {
  {
    ProfScope ps(s, 1);
    if (split)
      sie::launch_hat_f32(n_epi, s, a.desc, a.items, a.n_items, static_cast<float*>(arena),
                          d_part, pstride, grad_e, eo_part, ev_part, ev_stride);
    else
      sie::launch_hat_f64(n_epi, s, a.desc, a.items, a.n_items, static_cast<double*>(arena),
                          d_part, pstride, grad_e, eo_part, ev_part, ev_stride);
    if (eo_part)
      sie::launch_eps_vir(s, a.desc, a.items, a.n_items, n_frag, ev_part, pstride, ev_stride,
                          ev_item);
  }
  ProfScope ps(s, 4);
  if (split)
    sie::launch_adj_f32(L.data(), a, static_cast<const float*>(arena), s);
  else
    sie::launch_adj_f64(L.data(), a, static_cast<const double*>(arena), s);
}

sie_status run_backward(const sie_fragment* frags, int n, sie_precision p, const double* grad_e,
                        const sie_fragment_grad* grads, double* e_frag_out, void* ws,
                        size_t ws_bytes, void* stream) {
  const char* who = "sie_triples_backward";
  const std::string w(who);
  if (!frags || n < 1) return fail(SIE_ERR_INVALID_ARG, w + ": need at least one fragment");
  if (!grads) return fail(SIE_ERR_INVALID_ARG, w + ": gradient descriptor array is NULL");
  for (int x = 0; x < n; ++x) {
    sie_status st = check_fragment(&frags[x], p, who);
    if (st != SIE_OK) return st;
    const sie_fragment_grad& g = grads[x];
    for (const double* q : {g.t1, g.t2, g.ovvv, g.ooov, g.ovov, g.eps_occ, g.eps_vir})
      if (q && !aligned(q, sizeof(double)))
        return fail(SIE_ERR_INVALID_ARG, w + ": a gradient array is misaligned");
  }
  if (grad_e && !aligned(grad_e, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, w + ": grad_e is misaligned");
  if (e_frag_out && !aligned(e_frag_out, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, w + ": e_frag is misaligned");
  const Plan pl = make_plan(frags, n, p, true);
  if (!ws || !aligned(ws, 256))
    return fail(SIE_ERR_WORKSPACE, w + ": workspace is NULL or not 256-byte aligned");
  if (ws_bytes < pl.fixed_bytes + pl.min_arena)
    return fail(SIE_ERR_WORKSPACE,
                w + ": workspace smaller than required (see sie_triples_backward_workspace_size)");
  const size_t arena_bytes = ws_bytes - pl.fixed_bytes;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  auto dev = [&](size_t off) { return base + off; };

  Tables T;
  make_tables(frags, n, pl, base, arena_bytes, grads, T);
  const size_t n_rounds = T.round_begin.size() - 1;
  std::vector<sie::AdjGroup> groups;
  std::vector<sie::AdjRec> recs;
  std::vector<sie::AdjSlice> slices;
  std::vector<std::array<AdjLaunch, sie::kAdjClasses>> launches(n_rounds);
  for (size_t q = 0; q < n_rounds; ++q) {
    AdjLaunch l[sie::kAdjClasses];
    adj_round_lists(T, T.round_begin[q], T.round_begin[q + 1], groups, recs, slices, l);
    for (int c = 0; c < sie::kAdjClasses; ++c) {
      launches[q][size_t(c)] = l[c];
      if (size_t(l[c].part_elems) > pl.part_elems)
        return fail(SIE_ERR_HIP, w + ": internal error: partial slices exceed their bound");
    }
  }
  if (recs.size() > pl.adj_recs || groups.size() > pl.adj_recs || slices.size() > pl.adj_recs)
    return fail(SIE_ERR_HIP, w + ": internal error: contraction lists exceed their bound");
  const size_t off_recs = pl.off_adj;
  const size_t off_groups = align_up(off_recs + sizeof(sie::AdjRec) * pl.adj_recs, 256);
  const size_t off_slices = align_up(off_groups + sizeof(sie::AdjGroup) * pl.adj_recs, 256);

  sie_status st = SIE_OK;
  {
    sie::Staging::Batch up;
    const size_t bytes = sie::Staging::padded(sizeof(sie::FragDesc) * T.desc.size()) +
                         sie::Staging::padded(sizeof(double) * T.eps.size()) +
                         sie::Staging::padded(sizeof(sie::Item) * T.items.size()) +
                         sie::Staging::padded(sizeof(sie::AdjRec) * recs.size()) +
                         sie::Staging::padded(sizeof(sie::AdjGroup) * groups.size()) +
                         sie::Staging::padded(sizeof(sie::AdjSlice) * slices.size());
    st = hip_check(g_staging.begin(bytes, up), "stage tables");
    if (st != SIE_OK) return st;
    up.add(dev(pl.off_desc), T.desc.data(), sizeof(sie::FragDesc) * T.desc.size());
    up.add(dev(pl.off_eps), T.eps.data(), sizeof(double) * T.eps.size());
    up.add(dev(pl.off_items), T.items.data(), sizeof(sie::Item) * T.items.size());
    up.add(dev(off_recs), recs.data(), sizeof(sie::AdjRec) * recs.size());
    up.add(dev(off_groups), groups.data(), sizeof(sie::AdjGroup) * groups.size());
    up.add(dev(off_slices), slices.data(), sizeof(sie::AdjSlice) * slices.size());
    st = hip_check(up.commit(s), "upload tables");
    if (st != SIE_OK) return st;
  }
  if (check_finite_on()) {
    st = scan_finite(frags, n, !pl.split, reinterpret_cast<int*>(dev(pl.off_flags)), s, w);
    if (st != SIE_OK) return st;
  }

  const sie::FragDesc* d_desc = reinterpret_cast<const sie::FragDesc*>(dev(pl.off_desc));
  const sie::Item* d_items = reinterpret_cast<const sie::Item*>(dev(pl.off_items));
  const sie::AdjRec* d_recs = reinterpret_cast<const sie::AdjRec*>(dev(off_recs));
  const sie::AdjGroup* d_groups = reinterpret_cast<const sie::AdjGroup*>(dev(off_groups));
  const sie::AdjSlice* d_slices = reinterpret_cast<const sie::AdjSlice*>(dev(off_slices));
  double* d_parts = reinterpret_cast<double*>(dev(pl.off_parts));
  double* d_units = reinterpret_cast<double*>(dev(pl.off_units));
  double* d_part = reinterpret_cast<double*>(dev(pl.off_part));
  double* d_efrag = e_frag_out ? e_frag_out : reinterpret_cast<double*>(dev(pl.off_efrag));
  double* arena = reinterpret_cast<double*>(dev(pl.off_arena));
  double* t1_part = reinterpret_cast<double*>(dev(pl.off_t1));

  auto fill = [&](double* ptr, int64_t count) {
    if (!ptr || count <= 0) return;
    const int64_t nb = (count + 255) / 256;
    sie::launch_fill_zero(unsigned(nb < 65536 ? nb : 65536), s, ptr, count);
  };
  {
    ProfScope ps(s, 4);
    for (int x = 0; x < n; ++x) {
      const int64_t o = frags[x].n_occ, v = frags[x].n_vir;
      fill(grads[x].t1, o * v);
      fill(grads[x].t2, o * o * v * v);
      fill(grads[x].ovvv, o * v * v * v);
      fill(grads[x].ooov, o * o * o * v);
      fill(grads[x].ovov, o * v * o * v);
      fill(grads[x].eps_vir, v);
    }
  }
  bool want_eps = false;
  for (int x = 0; x < n; ++x) want_eps |= grads[x].eps_occ || grads[x].eps_vir;
  double* eo_part = want_eps ? reinterpret_cast<double*>(dev(pl.off_eo)) : nullptr;
  double* ev_part = reinterpret_cast<double*>(dev(pl.off_evp));
  double* ev_item = reinterpret_cast<double*>(dev(pl.off_evi));
  st = hip_check(hipGetLastError(), "launch gradient fill");
  if (st != SIE_OK) return st;

  if (pl.split) {
    st = stage_split(T.desc, s);
    if (st != SIE_OK) return st;
  }
  for (size_t q = 0; q < n_rounds; ++q) {
    const size_t r0 = T.round_begin[q], r1 = T.round_begin[q + 1];
    if (r1 == r0) continue;
    const int cnt = int(r1 - r0);
    const sie::Item* ri = d_items + r0;
    {
      ProfScope ps(s, 0);
      if (pl.split)
        build_round_split(T, q, s, d_desc, d_items, reinterpret_cast<float*>(dev(pl.off_arena)));
      else
        build_round_f64(T, q, s, d_desc, d_items, arena);
    }
    sie::AdjArgs aa{d_desc, ri, cnt, d_groups, d_recs, d_slices, d_parts, t1_part, pl.nv_max,
                    kT1Batch};
    backward_round(pl.split, launches[q], s, aa, dev(pl.off_arena), d_part, pl.pstride, grad_e,
                   unsigned(T.items[r1 - 1].part_end), n, eo_part, ev_part, ev_item, pl.nv_max);
    st = hip_check(hipGetLastError(), "launch backward kernels");
    if (st != SIE_OK) return st;
  }

  {
    ProfScope ps(s, 4);
    auto sym = [&](double* ptr, int kind, int no, int nv, int64_t count) {
      if (!ptr) return;
      const int64_t nb = (count + 255) / 256;
      sie::launch_symmetrize(unsigned(nb < 65536 ? nb : 65536), s, ptr, kind, no, nv, count);
    };
    for (int x = 0; x < n; ++x) {
      const int no = frags[x].n_occ, nv = frags[x].n_vir;
      const int64_t o = no, v = nv;
      sym(grads[x].t2, sie::kSymT2, no, nv, o * o * v * v);
      sym(grads[x].ovvv, sie::kSymOvvv, no, nv, o * v * v * v);
      sym(grads[x].ooov, sie::kSymOoov, no, nv, o * o * o * v);
      sym(grads[x].ovov, sie::kSymOvov, no, nv, o * v * o * v);
    }
  }
  {
    ProfScope ps(s, 2);
    int64_t max_units = 1;
    for (const auto& fp : pl.frags) max_units = fp.n_units > max_units ? fp.n_units : max_units;
    sie::launch_unit_energy(dim3(unsigned((max_units + 255) / 256), unsigned(n)), s, d_desc,
                            d_part, pl.pstride, d_units);
    sie::launch_frag_energy(unsigned(n), s, d_desc, d_units, d_efrag);
    if (want_eps) {
      int max_no = 1;
      for (const auto& fp : pl.frags) max_no = fp.no > max_no ? fp.no : max_no;
      sie::launch_eps_occ(s, d_desc, n, max_units, max_no, eo_part, pl.pstride,
                          reinterpret_cast<double*>(dev(pl.off_eou)));
    }
  }
  return hip_check(hipGetLastError(), "launch gradient symmetrization and reductions");
}

}  // namespace

extern "C" {

sie_status sie_triples_energy(const sie_fragment* f, sie_precision p, double* e_out,
                              double* e_triples, void* ws, size_t ws_bytes, void* stream) {
  if (!e_out || !aligned(e_out, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, "sie_triples_energy: e_out is NULL or misaligned");
  if (e_triples && !aligned(e_triples, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, "sie_triples_energy: e_triples is misaligned");
  if (f && f->frag_proj) {
    sie_status st = check_fragment(f, p, "sie_triples_energy", true);
    if (st != SIE_OK) return st;
    if (e_triples)
      return fail(SIE_ERR_UNSUPPORTED,
                  "sie_triples_energy: with a fragment projector the energy is not a sum of "
                  "per-triple terms (e_triples must be NULL)");
    return run_projector(f, p, nullptr, e_out, ws, ws_bytes, stream, "sie_triples_energy");
  }
  return run(f, 1, p, nullptr, e_out, e_triples, ws, ws_bytes, stream, "sie_triples_energy");
}

size_t sie_triples_projector_workspace_size(const sie_fragment* frag, sie_precision p,
                                            size_t max_bytes) {
  if (check_fragment(frag, p, "sie_triples_projector_workspace_size", true) != SIE_OK) return 0;
  return proj_workspace(*frag, p, max_bytes);
}

sie_status sie_triples_projector_matrix(const sie_fragment* frag, sie_precision p, double* m_out,
                                        void* ws, size_t ws_bytes, void* stream) {
  const char* who = "sie_triples_projector_matrix";
  sie_status st = check_fragment(frag, p, who, true);
  if (st != SIE_OK) return st;
  if (!m_out || !aligned(m_out, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, std::string(who) + ": m_out is NULL or misaligned");
  return run_projector(frag, p, m_out, nullptr, ws, ws_bytes, stream, who);
}

sie_status sie_triples_energy_static(const sie_fragment* f, sie_precision p, double* e_out,
                                     double* e_triples, void* stream) {
  const char* who = "sie_triples_energy_static";
  if (!e_out || !aligned(e_out, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, std::string(who) + ": e_out is NULL or misaligned");
  if (e_triples && !aligned(e_triples, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, std::string(who) + ": e_triples is misaligned");
  sie_status st = check_fragment(f, p, who);
  if (st != SIE_OK) return st;
  const Plan pl = make_plan(f, 1, p);
  if (pl.fixed_bytes + pl.min_arena > SIE_STATIC_SCRATCH_BYTES)
    return fail(SIE_ERR_WORKSPACE,
                std::string(who) + ": the fragment needs " +
                    std::to_string(pl.fixed_bytes + pl.min_arena) +
                    " bytes of workspace, more than the static scratch of " +
                    std::to_string(size_t(SIE_STATIC_SCRATCH_BYTES)) + " bytes");
  void* ws = nullptr;
  st = static_scratch(&ws, who);
  if (st != SIE_OK) return st;
  return run(f, 1, p, nullptr, e_out, e_triples, ws, SIE_STATIC_SCRATCH_BYTES, stream, who,
             /*direct=*/true);
}

sie_status sie_triples_energy_batched(const sie_fragment* frags, int32_t n, sie_precision p,
                                      double* e_frag, double* e_total, void* ws,
                                      size_t ws_bytes, void* stream) {
  if (!e_frag || !aligned(e_frag, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, "sie_triples_energy_batched: e_frag is NULL or misaligned");
  if (e_total && !aligned(e_total, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, "sie_triples_energy_batched: e_total is misaligned");
  return run(frags, n, p, e_frag, e_total, nullptr, ws, ws_bytes, stream,
             "sie_triples_energy_batched");
}

sie_status sie_triples_backward(const sie_fragment* frags, int32_t n, sie_precision p,
                                const double* grad_e, const sie_fragment_grad* grads,
                                double* e_frag, void* ws, size_t ws_bytes, void* stream) {
  return run_backward(frags, n, p, grad_e, grads, e_frag, ws, ws_bytes, stream);
}

size_t sie_triples_df_workspace_size(const sie_fragment_df* f, sie_precision p,
                                     size_t max_bytes) {
  const char* who = "sie_triples_df_workspace_size";
  if (check_df(f, p, who) != SIE_OK) return 0;
  const DfPlan q = df_plan(*f, p);
  // the formed fragment at a stand-in region address (checked, never read)
  const sie_fragment g = df_fragment(*f, p, reinterpret_cast<char*>(uintptr_t(1) << 20), q);
  const size_t cap = max_bytes ? max_bytes : default_cap();
  if (q.bytes >= cap) {
    fail(SIE_ERR_WORKSPACE, std::string(who) + ": cap below the formed integral blocks");
    return 0;
  }
  const size_t rest = workspace_size(&g, 1, p, cap - q.bytes, false, who);
  return rest ? q.bytes + rest : 0;
}

sie_status sie_triples_energy_df(const sie_fragment_df* f, sie_precision p, double* e_out,
                                 double* e_triples, void* ws, size_t ws_bytes, void* stream) {
  const char* who = "sie_triples_energy_df";
  const std::string w(who);
  sie_status st = check_df(f, p, w);
  if (st != SIE_OK) return st;
  if (!e_out || !aligned(e_out, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, w + ": e_out is NULL or misaligned");
  if (e_triples && !aligned(e_triples, sizeof(double)))
    return fail(SIE_ERR_INVALID_ARG, w + ": e_triples is misaligned");
  if (!ws || !aligned(ws, 256))
    return fail(SIE_ERR_WORKSPACE, w + ": workspace is NULL or not 256-byte aligned");
  const DfPlan q = df_plan(*f, p);
  char* region = static_cast<char*>(ws);
  const sie_fragment g = df_fragment(*f, p, region, q);
  st = check_fragment(&g, p, who);
  if (st != SIE_OK) return st;
  {
    const Plan pl = make_plan(&g, 1, p);
    if (ws_bytes < q.bytes || ws_bytes - q.bytes < pl.fixed_bytes + pl.min_arena)
      return fail(SIE_ERR_WORKSPACE,
                  w + ": workspace smaller than required (see sie_triples_df_workspace_size)");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int no = f->n_occ, nv = f->n_vir;
  if (check_finite_on()) {   // t1, t2 and the factors, before anything is formed
    int* flags = reinterpret_cast<int*>(region);
    const int64_t o = no, v = nv, n = o + v;
    sie::launch_zero_flags(s, flags, 3);
    sie::launch_nonfinite(s, f->t1, p == SIE_FP64, o * v, flags, 0);
    sie::launch_nonfinite(s, f->t2, p == SIE_FP64, o * o * v * v, flags, 1);
    sie::launch_nonfinite(s, f->b, true, int64_t(f->n_aux) * n * n, flags, 2);
    int h[3] = {0, 0, 0};
    st = hip_check(hipGetLastError(), "launch finite scan");
    if (st == SIE_OK)
      st = hip_check(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s),
                     "read finite scan");
    if (st == SIE_OK) st = hip_check(hipStreamSynchronize(s), "finite scan");
    if (st != SIE_OK) return st;
    static const char* kNames[3] = {"t1", "t2", "b"};
    for (int a = 0; a < 3; ++a)
      if (h[a]) return fail(SIE_ERR_NONFINITE, w + ": " + kNames[a] + " holds a non-finite value");
  }
  {
    ProfScope ps(s, 3);
    if (p == SIE_FP64) {
      double* ovvv = reinterpret_cast<double*>(region + q.off_ovvv);
      for (int i = 0; i < no; ++i)
        df_ovvv_slice(s, f->b, f->n_aux, no, nv, i, ovvv + int64_t(i) * nv * nv * nv);
      df_ooov_ovov(s, f->b, f->n_aux, no, nv, reinterpret_cast<double*>(region + q.off_ooov),
                   reinterpret_cast<double*>(region + q.off_ovov));
    } else {
      df_ooov_ovov(s, f->b, f->n_aux, no, nv, reinterpret_cast<float*>(region + q.off_ooov),
                   reinterpret_cast<float*>(region + q.off_ovov));
    }
  }
  st = hip_check(hipGetLastError(), "launch integral forming");
  if (st != SIE_OK) return st;
  DfSource src;
  src.b = f->b;
  src.n_aux = f->n_aux;
  src.slice = reinterpret_cast<float*>(region + q.off_slice);
  return run(&g, 1, p, nullptr, e_out, e_triples, region + q.bytes, ws_bytes - q.bytes, stream,
             who, false, &src);
}

}  // extern "C"
