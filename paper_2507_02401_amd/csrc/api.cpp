// C ABI of the wavelet E_s^* / Matern-prior library: validation, level schedules, launches.
//
// Operators (Sec. 4: W the periodic orthonormal DWT, D the level-weight diagonal with detail
// level i weighted 2^{-tau s (m-i)} and the approximation weighted 1):
//   es_adjoint = D_s W,  es_apply = W^T D_s,  matern_cov_apply = W^T D_2s W,
//   matern_sample = W^T D_s W.
//
// es_adjoint / es_apply run the full filter bank level by level (FB_DOWN / FB_UP tile
// kernels) and finish the coarse levels in one LDS-resident tail kernel per instance.
//
// matern_cov_apply / matern_sample use the projection form of W^T D W.  With P_i the
// orthogonal projection onto the level-i approximation space, P_i = (A^T)^i A^i for the
// one-level low-pass analysis A, and w_i the weight of detail level i (w_m = 1 = weight of
// the approximation):
//   W^T D W = sum_{i=1}^{m} w_i (P_{i-1} - P_i) + P_m = w_1 I + sum_{i=1}^{m-1} c_i P_i,
//   c_i = w_{i+1} - w_i,
// evaluated by the Horner recurrence
//   a_i = A a_{i-1} (a_0 = x),  z_{m-1} = c_{m-1} a_{m-1},
//   z_i = c_i a_i + A^T z_{i+1},  y = w_1 x + A^T z_1.
// Only the all-low band of every level is ever formed and level m is never visited, so the
// high-pass half of every filter pass disappears.  This is exactly the same linear operator
// as the filter-bank evaluation (a re-association of the same sum), not an approximation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/eswave.h"
#include "internal.h"
#include "tiles.h"

using namespace es;

// ------------------------------------------------------------------------------------------
// Errors.

namespace {

thread_local std::string g_last_error;

es_status fail(es_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
es_status fail(es_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

es_status dev_fail(hipError_t e, const char* where) {
  return fail(ES_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define ES_HIP(call, where)                        \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return dev_fail(e_, where); \
  } while (0)

// ------------------------------------------------------------------------------------------
// Geometry and validation.

constexpr int kMaxLevels = 30;

struct Geo {
  int D;
  int n[3];  // padded: 1-D (1,1,n), 2-D (1,n0,n1), 3-D (n0,n1,n2)
  int L;
  int m;
  double s;
  int64_t N() const { return (int64_t)n[0] * n[1] * n[2]; }
  int64_t level_size(int i) const { return (int64_t)(n[0] >> (D >= 3 ? i : 0)) * (n[1] >> (D >= 2 ? i : 0)) * (n[2] >> i); }
  void level_dims(int i, int out[3]) const {
    out[0] = D >= 3 ? n[0] >> i : 1;
    out[1] = D >= 2 ? n[1] >> i : 1;
    out[2] = n[2] >> i;
  }
};

es_status make_geo(int ndim, const int64_t* shape, int order, int levels, double s, Geo* g) {
  if (ndim < 1 || ndim > 3) return fail(ES_EINVAL, "ndim must be 1, 2 or 3 (got %d)", ndim);
  if (!shape) return fail(ES_EINVAL, "shape is NULL");
  if (order < 1 || order > 8) return fail(ES_EINVAL, "order must be in 1..8 (got %d)", order);
  if (levels < 0 || levels > kMaxLevels) return fail(ES_EINVAL, "levels must be in 0..%d (got %d)", kMaxLevels, levels);
  if (!std::isfinite(s)) return fail(ES_EINVAL, "s must be finite");
  g->D = ndim;
  g->L = 2 * order;
  g->m = levels;
  g->s = s;
  g->n[0] = g->n[1] = 1;
  int64_t prod = 1;
  for (int k = 0; k < ndim; ++k) {
    const int64_t v = shape[k];
    if (v < 1) return fail(ES_EINVAL, "shape[%d] must be positive (got %lld)", k, (long long)v);
    if (v > (1ll << 30)) return fail(ES_EINVAL, "shape[%d] too large", k);
    if (v % (1ll << levels)) return fail(ES_EINVAL, "shape[%d] = %lld is not divisible by 2^levels = %lld", k, (long long)v, 1ll << levels);
    prod *= v;
    if (prod > 0x7fffffffll) return fail(ES_EINVAL, "an instance may hold at most 2^31-1 elements");
    g->n[3 - ndim + k] = (int)v;
  }
  return ES_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return na && nb && pa < pb + nb && pb < pa + na;
}

es_status check_io(const void* in, const void* out, int64_t batch, int64_t N, const void* ws, size_t ws_bytes,
                   size_t need) {
  if (batch < 0) return fail(ES_EINVAL, "batch must be >= 0");
  if (batch > 0 && N > INT64_MAX / batch / 4) return fail(ES_EINVAL, "batch * size overflows");
  const size_t bytes = (size_t)(batch * N) * sizeof(float);
  if (batch == 0) return ES_OK;
  if (!in || !out) return fail(ES_EINVAL, "input and output pointers must be non-NULL");
  if (((uintptr_t)in & 15) || ((uintptr_t)out & 15)) return fail(ES_EINVAL, "input and output must be 16-byte aligned");
  if (overlap(in, bytes, out, bytes)) return fail(ES_EINVAL, "input and output overlap");
  if (need) {
    if (!ws) return fail(ES_EWORKSPACE, "workspace of %zu bytes required, got NULL", need);
    if (ws_bytes < need) return fail(ES_EWORKSPACE, "workspace of %zu bytes required, got %zu", need, ws_bytes);
    if ((uintptr_t)ws & 15) return fail(ES_EINVAL, "workspace must be 16-byte aligned");
    if (overlap(ws, need, in, bytes) || overlap(ws, need, out, bytes)) return fail(ES_EINVAL, "workspace overlaps input or output");
  }
  return ES_OK;
}

// gfx950 check, once per device.
es_status check_device() {
  static std::mutex mu;
  static int ok[64] = {0};  // 0 unknown, 1 ok, -1 unsupported
  int dev = 0;
  ES_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(ES_EUNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(mu);
  if (ok[dev] == 0) {
    hipDeviceProp_t prop;
    ES_HIP(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    ok[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
    if (ok[dev] < 0) return fail(ES_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  }
  if (ok[dev] < 0) return fail(ES_EUNSUPPORTED, "device %d is not gfx950", dev);
  return ES_OK;
}

bool get_filter(int L, Filter* f) {
  double h[kMaxTaps];
  if (!daubechies_filter(L / 2, h)) return false;
  for (int t = 0; t < kMaxTaps; ++t) f->h[t] = f->g[t] = 0.f;
  for (int t = 0; t < L; ++t) {
    f->h[t] = (float)h[t];
    f->g[t] = (float)((t & 1 ? -1.0 : 1.0) * h[L - 1 - t]);
  }
  return true;
}

// Detail weight of level i (1..m), FP64.
double wdet(const Geo& g, double tau, int i) { return std::exp2(-tau * g.s * (double)(g.m - i)); }

int64_t align64(int64_t v) { return (v + 63) & ~(int64_t)63; }

// Schedule mode of persistent plans (set around their schedule builds): every level launch uses
// the persistent kernel's tile variant and plain tiles, the coarse blocks fit the small LDS class
// of the coarse body, and every level array is written once (z_i gets its own array instead of
// overwriting a_i), so that no cache can hold a line of it from before it was written.
struct SchedMode {
  bool persist = false;
  int64_t coarse_limit = kCoarseMaxBlock;
};
thread_local SchedMode g_mode;

// Workspace: level arrays a_1 .. a_m of one instance, each 256-byte aligned (persistent plans:
// then z_1 .. z_m in a second region of the same size).
int64_t ws_floats_levels(const Geo& g) {
  int64_t tot = 0;
  for (int i = 1; i <= g.m; ++i) tot += align64(g.level_size(i));
  return tot;
}
int64_t ws_floats_per_instance(const Geo& g) { return (g_mode.persist ? 2 : 1) * ws_floats_levels(g); }
int64_t ws_level_offset(const Geo& g, int i) {  // offset of a_i (i >= 1)
  int64_t off = 0;
  for (int j = 1; j < i; ++j) off += align64(g.level_size(j));
  return off;
}

// ------------------------------------------------------------------------------------------
// Schedules.  A schedule is a list of launches for one geometry; each launch has one Task
// (level kernels) or one TailTask (tail kernels) whose pointers already include the
// per-instance strides of a uniform batch.

// Largest block (elements) the tail kernels keep in LDS, per dimensionality.
constexpr int64_t kTailMax[4] = {0, 4096, 8192, 8192};

// Test and tuning knobs read at every call: ESWAVE_TAIL_MAX overrides the tail threshold
// (0 disables the tail kernels), ESWAVE_FORCE_VARIANT=0/1 forces the wide/narrow tiles.
int64_t tail_max(int D) {
  const char* e = getenv("ESWAVE_TAIL_MAX");
  if (e && *e) return atoll(e);
  return kTailMax[D];
}
bool fuse_up2() {  // measured slower than two launches on 64 x 1024^2 db8: opt-in
  if (g_mode.persist) return false;
  const char* e = getenv("ESWAVE_FUSE_UP2");
  return e && *e == '1';
}
bool reverse_orders() {
  const char* e = getenv("ESWAVE_NO_REVERSE");
  return !(e && *e == '1');
}
// Kernel family of the levels that have a streamed variant (3-D full-bank levels, 2-D low-pass
// analysis): ESWAVE_STREAMED=0 plain tiles only, 2 streamed tiles at every such level,
// otherwise (default) streamed where the level fills the chip.
int streamed_mode() {
  const char* e = getenv("ESWAVE_STREAMED");
  if (e && (*e == '0' || *e == '2')) return *e - '0';
  return 1;
}
int forced_variant() {
  const char* e = getenv("ESWAVE_FORCE_VARIANT");
  if (e && *e >= '0' && *e < '0' + kNumVariants) return *e - '0';
  return -1;
}

struct Launch {
  int is_tail;
  int kind;     // KernelKind, or tail kind (0 LP, 1 FB analysis, 2 FB synthesis)
  int level;    // pyramid level passed to set_tiles (level kernels)
  int variant;
  int vec;
  int reverse;  // walk tiles in reverse order
  int D, L;
  Task task;
  TailTask tail;
  size_t lds;
};

struct Schedule {
  std::vector<Launch> launches;
  bool identity = false;  // plain copy
  Filter f;
};

void set_tiles(Task& t, int kind, const Geo& g, int level, int variant, int64_t batch) {
  int b[3];
  g.level_dims(level - 1, b);  // full-res block of the level
  const TileShape ts = tile_shape(kind, g.D, variant, g.L);
  const bool analysis = kind_is_analysis(kind);
  for (int k = 0; k < 3; ++k) {
    t.b[k] = b[k];
    const bool real = k >= 3 - g.D;
    const int extent = real ? (analysis ? b[k] / 2 : b[k]) : 1;
    t.ntile[k] = real ? (extent + ts.t[k] - 1) / ts.t[k] : 1;
  }
  t.tiles_per_inst = t.ntile[0] * t.ntile[1] * t.ntile[2];
  t.batch = (int32_t)batch;
  t.tile_begin = 0;
}

double tile_waste(int kind, const Geo& g, int level, int variant) {
  int b[3];
  g.level_dims(level - 1, b);
  const TileShape ts = tile_shape(kind, g.D, variant, g.L);
  const bool analysis = kind_is_analysis(kind);
  double covered = 1, needed = 1;
  for (int k = 3 - g.D; k < 3; ++k) {
    const int extent = analysis ? b[k] / 2 : b[k];
    covered *= (double)((extent + ts.t[k] - 1) / ts.t[k]) * ts.t[k];
    needed *= extent;
  }
  return covered / needed;
}

// Work-group count the tile heuristic assumes; ragged plans set it to their instance count so
// that a level shared by many instances is tiled for the whole launch, not for one instance.
thread_local int64_t g_variant_batch = 0;

// Largest block the low-pass coarse kernel takes: the large LDS class (an instance that fits it
// as a whole runs entirely in one work-group, in one launch).  Measured against handing over at
// the small class: equal on 64 x 1024^2 db8, 2 % faster on 256 x 512^2 db6, 14 % on 16 x 256^2
// db4.  The choice depends on the geometry only, never on the batch, so an instance gives the
// same bits in any batch.  ESWAVE_TAIL_MAX overrides (capped at the large class).
// Ragged plans whose coarse fusion depth was tuned (es_plan_autotune) set g_lp_coarse while their
// schedules are frozen.
thread_local int64_t g_lp_coarse = -1;
int64_t lp_tail_limit(const Geo&) {
  if (g_mode.persist) return std::min<int64_t>(g_mode.coarse_limit, kPCoarseMax);
  if (g_lp_coarse >= 0) return std::min<int64_t>(g_lp_coarse, kCoarseMaxBlockBig);
  const char* e = getenv("ESWAVE_TAIL_MAX");
  if (e && *e) return std::min<int64_t>(atoll(e), kCoarseMaxBlockBig);
  return kCoarseMaxBlockBig;
}

int pick_variant(int kind, const Geo& g, int level, int64_t batch) {
  if (g_mode.persist) return kPVariant;
  const int fv = forced_variant();
  if (fv >= 0) return fv;
  if (g_variant_batch > batch) batch = g_variant_batch;
  const double w0 = tile_waste(kind, g, level, 0), w1 = tile_waste(kind, g, level, 1);
  Task t{};
  set_tiles(t, kind, g, level, 0, batch);
  const int64_t wg0 = (int64_t)t.tiles_per_inst * batch;
  // large levels: wide tiles for analysis, medium tiles for the synthesis kernels (measured
  // fastest on 64 x 1024^2 db8); small levels: narrow tiles (more work-groups)
  const int big = (kind == K_LP_UP || kind == K_FB_UP || kind == K_LP_UP_S) ? 2 : 0;
  if (w0 <= 1.25 && wg0 >= 1024) return big;
  if (w0 <= w1 && wg0 >= 2048) return big;
  return 1;
}

// Row-alignment condition of the vector staging path for one launch.
bool vec_ok(const Task& t, int kind, const Geo& g) {
  auto a16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  auto m4 = [](int64_t v) { return (v & 3) == 0; };
  const bool analysis = kind_is_analysis(kind);
  const int row = analysis ? t.b[2] : (kind == K_LP_UP2 ? t.b[2] / 4 : t.b[2] / 2);  // staged input rows
  if (!m4(row)) return false;
  if (!a16(t.in0) || !m4(t.bs_in0) || !m4(t.st_in0[0]) || !m4(t.st_in0[1])) return false;
  if ((kind == K_FB_UP || kind == K_FB_UP_S) && (!a16(t.in1) || !m4(t.bs_in1) || !m4(t.st_in1[0]) || !m4(t.st_in1[1]))) return false;
  // 2-D LP_UP reads `same` and writes `out` as 16-byte vectors on the vector path
  if (kind == K_LP_UP && g.D == 2 && (!a16(t.in1) || !m4(t.bs_in1) || !a16(t.out0) || !m4(t.bs_out0))) return false;
  return true;
}

void strides_of(const int dims[3], int32_t st[2]) {
  st[0] = dims[1] * dims[2];
  st[1] = dims[2];
}

// 3-D levels (full-bank and low-pass) and 2-D low-pass analysis levels have two kernel families:
// plain tiles, and tiles streamed along the slowest axis (no halo re-reads along it, but one
// work-group walks its run in sequence).  Streaming wins when the level has enough tiles to fill
// the chip.
bool has_family(int kind, int D) {
  return (D == 3 && (kind == K_FB_DOWN || kind == K_FB_UP || kind == K_FB_DOWN_S || kind == K_FB_UP_S ||
                     kind == K_LP_DOWN || kind == K_LP_DOWN_S || kind == K_LP_UP || kind == K_LP_UP_S)) ||
         (D == 2 && (kind == K_LP_DOWN || kind == K_LP_DOWN_S));
}
bool is_family(const Launch& l) { return !l.is_tail && has_family(l.kind, l.D); }
int streamed_kind(int kind) {
  if (kind == K_LP_DOWN || kind == K_LP_DOWN_S) return K_LP_DOWN_S;
  if (kind == K_LP_UP || kind == K_LP_UP_S) return K_LP_UP_S;
  return kind_is_analysis(kind) ? K_FB_DOWN_S : K_FB_UP_S;
}
int tiled_kind(int kind) {
  if (kind == K_LP_DOWN || kind == K_LP_DOWN_S) return K_LP_DOWN;
  if (kind == K_LP_UP || kind == K_LP_UP_S) return K_LP_UP;
  return kind_is_analysis(kind) ? K_FB_DOWN : K_FB_UP;
}

Launch level_launch(int kind, const Geo& g, int level, int64_t batch) {
  const int mode = streamed_mode();
  if (has_family(kind, g.D) && mode != 0 && !g_mode.persist) {
    const int sk = streamed_kind(kind);
    Task t{};
    set_tiles(t, sk, g, level, pick_variant(sk, g, level, batch), batch);
    if (mode == 2 || (int64_t)t.tiles_per_inst * std::max<int64_t>(batch, g_variant_batch) >= 1024) kind = sk;
  }
  Launch l{};
  l.is_tail = 0;
  l.kind = kind;
  l.D = g.D;
  l.L = g.L;
  l.level = level;
  l.variant = pick_variant(kind, g, level, batch);
  set_tiles(l.task, kind, g, level, l.variant, batch);
  return l;
}

void finish_level(Launch& l, const Geo& g) { l.vec = vec_ok(l.task, l.kind, g) ? 1 : 0; }

void apply_variant(Launch& l, const Geo& g, int v, int64_t batch) {
  l.variant = v;
  set_tiles(l.task, l.kind, g, l.level, v, batch);
  finish_level(l, g);
}

// Tunable choices of a level launch: its tile variants, and for levels with two kernel families
// the tile variants of both (choice = variant + kNumVariants for the streamed family).
int num_choices(const Launch& l) { return is_family(l) ? 2 * kNumVariants : kNumVariants; }
void apply_choice(Launch& l, const Geo& g, int c, int64_t batch) {
  if (is_family(l)) l.kind = c >= kNumVariants ? streamed_kind(l.kind) : tiled_kind(l.kind);
  apply_variant(l, g, c % kNumVariants, batch);
}

// ------------------------------------------------------------------------------------------
// Autotune cache: for a geometry (op, ndim, sides, taps, levels, batch) the measured fastest
// tile variant of every launch of its schedule.  Filled by es_autotune; optionally persisted
// as text lines in the file named by ESWAVE_TUNE_CACHE.

struct TuneKey {
  int op, D, n0, n1, n2, L, m;
  int64_t batch;
  bool operator<(const TuneKey& o) const {
    return std::tie(op, D, n0, n1, n2, L, m, batch) < std::tie(o.op, o.D, o.n0, o.n1, o.n2, o.L, o.m, o.batch);
  }
};

struct TuneCache {
  std::mutex mu;
  std::map<TuneKey, std::vector<int>> map;
  bool loaded = false;
};
TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}

TuneKey tune_key(int op, const Geo& g, int64_t batch) { return TuneKey{op, g.D, g.n[0], g.n[1], g.n[2], g.L, g.m, batch}; }

void tune_load_locked(TuneCache& c) {
  if (c.loaded) return;
  c.loaded = true;
  const char* path = getenv("ESWAVE_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    TuneKey k;
    long long b;
    int used = 0;
    if (sscanf(line, "eswave-tune-v1 %d %d %d %d %d %d %d %lld :%n", &k.op, &k.D, &k.n0, &k.n1, &k.n2, &k.L, &k.m, &b,
               &used) < 8 || used == 0)
      continue;
    k.batch = b;
    std::vector<int> v;
    const char* p = line + used;
    int x, n;
    while (sscanf(p, "%d%n", &x, &n) == 1) { v.push_back(x); p += n; }
    c.map[k] = v;
  }
  fclose(f);
}

bool tune_lookup(const TuneKey& k, std::vector<int>* v) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  tune_load_locked(c);
  auto it = c.map.find(k);
  if (it == c.map.end()) return false;
  *v = it->second;
  return true;
}

void tune_store(const TuneKey& k, const std::vector<int>& v) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  tune_load_locked(c);
  c.map[k] = v;
  const char* path = getenv("ESWAVE_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "eswave-tune-v1 %d %d %d %d %d %d %d %lld :", k.op, k.D, k.n0, k.n1, k.n2, k.L, k.m, (long long)k.batch);
  for (int x : v) fprintf(f, " %d", x);
  fprintf(f, "\n");
  fclose(f);
}

// Use the tuned variants when the cache holds this geometry (and no variant is forced).
void apply_tuned(Schedule* sc, int op, const Geo& g, int64_t batch) {
  if (forced_variant() >= 0) return;
  std::vector<int> v;
  if (!tune_lookup(tune_key(op, g, batch), &v) || v.size() != sc->launches.size()) return;
  for (size_t j = 0; j < v.size(); ++j) {
    Launch& l = sc->launches[j];
    if (!l.is_tail && v[j] >= 0 && v[j] < num_choices(l)) apply_choice(l, g, v[j], batch);
  }
}

// Consecutive launches walk their tiles in opposite orders, and the last launch (the finest
// up level, which re-reads the input) runs opposite to the first (the finest down level, which
// read it first), so that data touched at the end of one launch is touched first by the next
// while it is still in the L2 / Infinity Cache.
void set_orders(Schedule* sc) {
  const int n = (int)sc->launches.size();
  for (int k = 0; k < n; ++k) sc->launches[k].reverse = reverse_orders() ? (k & 1) : 0;
  if (n >= 2 && reverse_orders()) sc->launches[n - 1].reverse = sc->launches[0].reverse ^ 1;
}

es_status build_schedule_raw(int op, const Geo& g, int64_t batch, const float* in, float* out, float* ws,
                             Schedule* sc) {
  sc->launches.clear();
  sc->identity = false;
  if (!get_filter(g.L, &sc->f)) return fail(ES_EUNSUPPORTED, "filter derivation failed for order %d", g.L / 2);
  const int64_t N = g.N();
  const int64_t wsi = ws_floats_per_instance(g);
  const int D = g.D, m = g.m;
  int full[3];
  g.level_dims(0, full);
  int32_t st_full[2];
  strides_of(full, st_full);
  auto lvl_ptr = [&](int i) -> float* { return ws + ws_level_offset(g, i); };
  // z_i: in place of a_i, or (persistent plans) in the second region
  auto zlvl_ptr = [&](int i) -> float* { return (g_mode.persist ? ws + ws_floats_levels(g) : ws) + ws_level_offset(g, i); };
  auto lvl_dims = [&](int i, int d[3]) { g.level_dims(i, d); };

  if (op == ES_OP_COV || op == ES_OP_SAMPLE) {
    if (m <= 1) {  // all weights are 1: identity
      sc->identity = true;
      return ES_OK;
    }
    const double tau = op == ES_OP_COV ? 2.0 : 1.0;
    std::vector<double> w(m + 2), c(m + 1);
    for (int i = 1; i <= m; ++i) w[i] = wdet(g, tau, i);
    for (int i = 1; i <= m - 1; ++i) c[i] = w[i + 1] - w[i];
    // Coarse levels whose block fits kCoarseMaxBlock run in one work-group per instance
    // (tail kind 3).  The first low-pass tail kernel (kind 0) stays switched off: a 1-D run of
    // it ended in a GPU memory-aperture fault whose cause has not been found.
    int T = -1;
    const int64_t limit = lp_tail_limit(g);
    for (int i = 0; i <= m - 2; ++i)
      if (g.level_size(i) <= limit) { T = i; break; }
    const bool tail = T >= 0;
    const int down_to = tail ? T : m - 1;
    for (int i = 1; i <= down_to; ++i) {
      Launch l = level_launch(K_LP_DOWN, g, i, batch);
      int d_in[3], d_out[3];
      lvl_dims(i - 1, d_in);
      lvl_dims(i, d_out);
      l.task.in0 = i == 1 ? in : lvl_ptr(i - 1);
      l.task.bs_in0 = i == 1 ? N : wsi;
      strides_of(d_in, l.task.st_in0);
      l.task.out0 = lvl_ptr(i);
      l.task.bs_out0 = wsi;
      strides_of(d_out, l.task.st_out0);
      finish_level(l, g);
      sc->launches.push_back(l);
    }
    if (tail) {
      Launch l{};
      l.is_tail = 1;
      l.kind = 3;
      l.D = D;
      l.L = g.L;
      TailTask& t = l.tail;
      const int K = m - 1 - T;
      t.in = T == 0 ? in : lvl_ptr(T);
      t.bs_in = T == 0 ? N : wsi;
      t.out = T == 0 ? out : zlvl_ptr(T);
      t.bs_out = T == 0 ? N : wsi;
      lvl_dims(T, t.b);
      t.nlev = K;
      t.batch = (int32_t)batch;
      t.coef[0] = (float)(T == 0 ? w[1] : c[T]);
      for (int j = 1; j <= K; ++j) t.coef[j] = (float)c[T + j];
      l.lds = tail_lds_bytes(3, D, t.b, K);  // selects the kernel's LDS size class
      // the kernel's LDS layout: pyramid A_0 .. A_K, then the temporaries (2-D: B/2; 3-D: B/2 + B/2)
      {
        const int64_t B = g.level_size(T);
        int64_t need = 0;
        for (int j = 0; j <= K; ++j) need += B >> (D * j);
        need += D == 2 ? B / 2 : (D == 3 ? B : 0);
        const int64_t cap = B <= kCoarseMaxBlock ? kCoarseMaxBlock / 4 * 9 : kCoarseMaxBlockBig / 4 * 9;
        if (B > kCoarseMaxBlockBig || need > cap)
          return fail(ES_EUNSUPPORTED, "coarse block of %lld floats needs %lld floats of LDS", (long long)B, (long long)need);
      }
      sc->launches.push_back(l);
    }
    const int up_from = tail ? T - 1 : m - 2;
    // 2-D: the last two up levels (z_1 and y) run fused in one kernel when both exist
    const bool fuse_last = D == 2 && up_from >= 1 && fuse_up2();
    for (int i = up_from; i >= (fuse_last ? 2 : 0); --i) {
      // produce level i (full-res block of level i = dims of a_i)
      Launch l = level_launch(K_LP_UP, g, i + 1, batch);
      int d_z[3], d_o[3];
      lvl_dims(i + 1, d_z);
      lvl_dims(i, d_o);
      // without a coarse step the first up level reads a_{m-1} itself (beta = c_{m-1})
      l.task.in0 = (!tail && i + 1 == m - 1) ? lvl_ptr(i + 1) : zlvl_ptr(i + 1);
      l.task.bs_in0 = wsi;
      strides_of(d_z, l.task.st_in0);
      l.task.in1 = i == 0 ? in : lvl_ptr(i);
      l.task.bs_in1 = i == 0 ? N : wsi;
      l.task.out0 = i == 0 ? out : zlvl_ptr(i);
      l.task.bs_out0 = i == 0 ? N : wsi;
      strides_of(d_o, l.task.st_in1);
      strides_of(d_o, l.task.st_out0);
      l.task.alpha = (float)(i == 0 ? w[1] : c[i]);
      l.task.beta = (!tail && i == m - 2) ? (float)c[m - 1] : 1.f;
      finish_level(l, g);
      sc->launches.push_back(l);
    }
    if (fuse_last) {
      Launch l = level_launch(K_LP_UP2, g, 1, batch);
      l.task.in0 = lvl_ptr(2);  // z_2
      l.task.bs_in0 = wsi;
      l.task.in1 = lvl_ptr(1);  // a_1
      l.task.bs_in1 = wsi;
      l.task.in2 = in;          // x
      l.task.bs_in2 = N;
      l.task.out0 = out;
      l.task.bs_out0 = N;
      l.task.alpha = (float)w[1];
      l.task.beta = 1.f;
      l.task.gamma = (float)c[1];
      l.task.delta = (!tail && 1 == m - 2) ? (float)c[m - 1] : 1.f;
      finish_level(l, g);
      sc->launches.push_back(l);
    }
    set_orders(sc);
    return ES_OK;
  }

  // full filter bank
  if (m == 0) {
    sc->identity = true;
    return ES_OK;
  }
  std::vector<double> w(m + 1);
  for (int i = 1; i <= m; ++i) w[i] = wdet(g, 1.0, i);
  int T = m;  // tail handles levels T+1..m from a_T
  for (int i = 0; i <= m - 1; ++i)
    if (g.level_size(i) <= std::min<int64_t>(tail_max(D), kFbCoarseMaxBlock)) { T = i; break; }
  const bool tail = T < m;
  auto approx_region = [&](int32_t st[2]) { st[0] = st_full[0]; st[1] = st_full[1]; };

  if (op == ES_OP_ADJOINT) {
    for (int i = 1; i <= T; ++i) {
      Launch l = level_launch(K_FB_DOWN, g, i, batch);
      int d_in[3], d_ll[3];
      lvl_dims(i - 1, d_in);
      lvl_dims(i, d_ll);
      l.task.in0 = i == 1 ? in : lvl_ptr(i - 1);
      l.task.bs_in0 = i == 1 ? N : wsi;
      strides_of(d_in, l.task.st_in0);
      l.task.out0 = out;
      l.task.bs_out0 = N;
      l.task.st_out0[0] = st_full[0];
      l.task.st_out0[1] = st_full[1];
      if (i == m) {  // last level without tail: approximation into the coefficient array
        l.task.out1 = out;
        l.task.bs_out1 = N;
        approx_region(l.task.st_out1);
      } else {
        l.task.out1 = lvl_ptr(i);
        l.task.bs_out1 = wsi;
        strides_of(d_ll, l.task.st_out1);
      }
      l.task.alpha = (float)w[i];
      l.task.beta = 1.f;
      finish_level(l, g);
      sc->launches.push_back(l);
    }
    if (tail) {
      Launch l{};
      l.is_tail = 1;
      l.kind = 1;
      l.D = D;
      l.L = g.L;
      TailTask& t = l.tail;
      t.in = T == 0 ? in : lvl_ptr(T);
      t.bs_in = T == 0 ? N : wsi;
      t.out = out;
      t.bs_out = N;
      t.st_out[0] = st_full[0];
      t.st_out[1] = st_full[1];
      lvl_dims(T, t.b);
      int db[3];
      lvl_dims(T, db);
      strides_of(db, t.st_in);
      t.nlev = m - T;
      t.batch = (int32_t)batch;
      for (int j = 0; j < m - T; ++j) t.coef[j] = (float)w[T + 1 + j];
      t.coef[m - T] = 1.f;
      l.lds = tail_lds_bytes(1, D, t.b, t.nlev);
      sc->launches.push_back(l);
    }
    set_orders(sc);
    return ES_OK;
  }

  // ES_OP_APPLY
  if (tail) {
    Launch l{};
    l.is_tail = 1;
    l.kind = 2;
    l.D = D;
    l.L = g.L;
    TailTask& t = l.tail;
    t.in = in;
    t.bs_in = N;
    t.st_in[0] = st_full[0];
    t.st_in[1] = st_full[1];
    t.out = T == 0 ? out : lvl_ptr(T);
    t.bs_out = T == 0 ? N : wsi;
    lvl_dims(T, t.b);
    int db[3];
    lvl_dims(T, db);
    if (T == 0) {
      t.st_out[0] = st_full[0];
      t.st_out[1] = st_full[1];
    } else {
      strides_of(db, t.st_out);
    }
    t.nlev = m - T;
    t.batch = (int32_t)batch;
    for (int j = 0; j < m - T; ++j) t.coef[j] = (float)w[T + 1 + j];
    t.coef[m - T] = 1.f;
    l.lds = tail_lds_bytes(2, D, t.b, t.nlev);
    sc->launches.push_back(l);
  }
  for (int i = T; i >= 1; --i) {
    Launch l = level_launch(K_FB_UP, g, i, batch);
    int d_ll[3], d_out[3];
    lvl_dims(i, d_ll);
    lvl_dims(i - 1, d_out);
    if (i == m) {  // no tail: approximation read from the coefficient array
      l.task.in0 = in;
      l.task.bs_in0 = N;
      approx_region(l.task.st_in0);
    } else {
      l.task.in0 = lvl_ptr(i);
      l.task.bs_in0 = wsi;
      strides_of(d_ll, l.task.st_in0);
    }
    l.task.in1 = in;
    l.task.bs_in1 = N;
    l.task.st_in1[0] = st_full[0];
    l.task.st_in1[1] = st_full[1];
    l.task.out0 = i == 1 ? out : lvl_ptr(i - 1);
    l.task.bs_out0 = i == 1 ? N : wsi;
    strides_of(d_out, l.task.st_out0);
    l.task.alpha = (float)w[i];
    l.task.beta = 1.f;
    finish_level(l, g);
    sc->launches.push_back(l);
  }
  set_orders(sc);
  return ES_OK;
}

es_status build_schedule(int op, const Geo& g, int64_t batch, const float* in, float* out, float* ws,
                         Schedule* sc) {
  es_status st = build_schedule_raw(op, g, batch, in, out, ws, sc);
  if (st == ES_OK && !sc->identity && !g_mode.persist) apply_tuned(sc, op, g, batch);
  return st;
}

// ------------------------------------------------------------------------------------------
// Footprint check.  Every level kernel reduces its tile indices modulo the level block or
// guards them against it, and every coarse kernel walks exactly its block, so the memory one
// launch may touch is, per array, the block that array is addressed with (its own dims and
// strides) for each instance of the task.  Before anything is enqueued the host checks these
// ranges against the caller's buffers: a launch that would read outside every buffer, or write
// outside the writable ones, is rejected with ES_EINVAL instead of reaching the device.

struct Region {
  uintptr_t lo, hi;  // [lo, hi) bytes
  bool writable;
};

struct Access {
  const void* base;
  int64_t per_inst;  // bytes between instances
  int64_t span;      // bytes one instance may touch from base
  bool write;
};

// Largest element offset + 1 of a (d0, d1, d2) block addressed with strides (s0, s1, 1).
int64_t block_span(const int d[3], int64_t s0, int64_t s1) {
  if (d[0] <= 0 || d[1] <= 0 || d[2] <= 0) return 0;
  return (int64_t)(d[0] - 1) * s0 + (int64_t)(d[1] - 1) * s1 + d[2];
}
int64_t dense_span(const int d[3]) { return (int64_t)d[0] * d[1] * d[2]; }
void half_of(const int b[3], int D, int h[3]) {
  for (int k = 0; k < 3; ++k) h[k] = k >= 3 - D ? b[k] / 2 : 1;
}

void launch_accesses(const Launch& l, std::vector<Access>* acc) {
  acc->clear();
  auto add = [&](const void* p, int64_t bs, int64_t span_floats, bool w) {
    acc->push_back(Access{p, bs * (int64_t)sizeof(float), span_floats * (int64_t)sizeof(float), w});
  };
  if (l.is_tail) {
    const TailTask& t = l.tail;
    const int64_t B = dense_span(t.b);
    if (l.kind == 3) {  // low-pass coarse: contiguous block in, contiguous block out
      add(t.in, t.bs_in, B, false);
      add(t.out, t.bs_out, B, true);
    } else if (l.kind == 1) {  // full-bank analysis: contiguous in, strided packed block out
      add(t.in, t.bs_in, B, false);
      if (t.flags & kNormSq) acc->push_back(Access{t.out, 0, (int64_t)t.batch * 8, true});
      else add(t.out, t.bs_out, block_span(t.b, t.st_out[0], t.st_out[1]), true);
    } else {  // full-bank synthesis: strided packed block in, strided block out
      add(t.in, t.bs_in, block_span(t.b, t.st_in[0], t.st_in[1]), false);
      add(t.out, t.bs_out, block_span(t.b, t.st_out[0], t.st_out[1]), true);
    }
    return;
  }
  const Task& t = l.task;
  int h[3];
  half_of(t.b, l.D, h);
  switch (l.kind) {
    case K_LP_DOWN:
    case K_LP_DOWN_S:
      add(t.in0, t.bs_in0, block_span(t.b, t.st_in0[0], t.st_in0[1]), false);
      add(t.out0, t.bs_out0, dense_span(h), true);
      break;
    case K_LP_UP:
    case K_LP_UP_S:
      add(t.in0, t.bs_in0, dense_span(h), false);
      add(t.in1, t.bs_in1, dense_span(t.b), false);
      add(t.out0, t.bs_out0, dense_span(t.b), true);
      break;
    case K_LP_UP2: {
      int q[3];
      half_of(h, l.D, q);
      add(t.in0, t.bs_in0, dense_span(q), false);
      add(t.in1, t.bs_in1, dense_span(h), false);
      add(t.in2, t.bs_in2, dense_span(t.b), false);
      add(t.out0, t.bs_out0, dense_span(t.b), true);
      break;
    }
    case K_FB_DOWN:
    case K_FB_DOWN_S:
      add(t.in0, t.bs_in0, block_span(t.b, t.st_in0[0], t.st_in0[1]), false);
      if (t.flags & kNormSq) {  // per-work-group partial sums (8-byte pairs) in place of the bands
        acc->push_back(Access{t.out0, 0, (int64_t)t.tiles_per_inst * t.batch * 8, true});
        if (!(t.flags & kNormLL)) add(t.out1, t.bs_out1, block_span(h, t.st_out1[0], t.st_out1[1]), true);
      } else {
        add(t.out0, t.bs_out0, block_span(t.b, t.st_out0[0], t.st_out0[1]), true);
        add(t.out1, t.bs_out1, block_span(h, t.st_out1[0], t.st_out1[1]), true);
      }
      break;
    default:  // K_FB_UP, K_FB_UP_S
      add(t.in0, t.bs_in0, block_span(h, t.st_in0[0], t.st_in0[1]), false);
      add(t.in1, t.bs_in1, block_span(t.b, t.st_in1[0], t.st_in1[1]), false);
      add(t.out0, t.bs_out0, block_span(t.b, t.st_out0[0], t.st_out0[1]), true);
      break;
  }
}

// Tile bookkeeping of a level launch: the counts the kernel decodes work-group indices with.
bool tiles_consistent(const Launch& l) {
  if (l.is_tail) return l.tail.batch >= 1 && l.tail.nlev >= 1;
  const Task& t = l.task;
  for (int k = 0; k < 3; ++k)
    if (t.ntile[k] < 1 || t.b[k] < 1) return false;
  return t.batch >= 1 && (int64_t)t.tiles_per_inst == (int64_t)t.ntile[0] * t.ntile[1] * t.ntile[2];
}

// Checks every access of every instance of one launch against the regions.
es_status check_launch(const Launch& l, const Region* regions, int nreg, const char* what) {
  if (!tiles_consistent(l)) return fail(ES_EINVAL, "%s: inconsistent tile counts", what);
  std::vector<Access> acc;
  launch_accesses(l, &acc);
  const int64_t batch = l.is_tail ? l.tail.batch : l.task.batch;
  for (const Access& a : acc) {
    if (a.span <= 0) continue;
    const uintptr_t lo = (uintptr_t)a.base;
    const uintptr_t hi = lo + (uintptr_t)((batch - 1) * a.per_inst + a.span);
    bool ok = false;
    for (int r = 0; r < nreg && !ok; ++r)
      ok = lo >= regions[r].lo && hi <= regions[r].hi && (!a.write || regions[r].writable);
    if (!ok)
      return fail(ES_EINVAL, "%s: a %s of %lld bytes at %p lies outside the caller's %sbuffers", what,
                  a.write ? "write" : "read", (long long)(hi - lo), a.base, a.write ? "writable " : "");
  }
  return ES_OK;
}

es_status check_schedule(const Schedule& sc, const Region* regions, int nreg) {
  if (sc.identity) return ES_OK;
  char what[64];
  for (size_t j = 0; j < sc.launches.size(); ++j) {
    snprintf(what, sizeof what, "launch %zu of the schedule", j);
    es_status st = check_launch(sc.launches[j], regions, nreg, what);
    if (st != ES_OK) return st;
  }
  return ES_OK;
}

// The regions of a uniform-batch call: input (read), output and workspace (read and write).
int call_regions(const void* in, const void* out, int64_t bytes, const void* ws, size_t ws_bytes, Region r[3]) {
  int n = 0;
  r[n++] = Region{(uintptr_t)in, (uintptr_t)in + (uintptr_t)bytes, false};
  r[n++] = Region{(uintptr_t)out, (uintptr_t)out + (uintptr_t)bytes, true};
  if (ws && ws_bytes) r[n++] = Region{(uintptr_t)ws, (uintptr_t)ws + ws_bytes, true};
  return n;
}

int64_t round8(int64_t v) { return (v + 7) & ~(int64_t)7; }

es_status run_launch(const Launch& l, const Filter& f, hipStream_t stream, const Task* table, int count,
                     int total_wg, const TailTask* ttable) {
  if (total_wg <= 0) return ES_OK;
  const int grid = (int)round8(total_wg);
  if (!l.is_tail) {
    TaskArgs a{};
    a.table = table;
    a.count = count;
    a.total_wg = total_wg;
    a.vec = l.vec;
    a.reverse = l.reverse;
    a.t0 = l.task;
    ES_HIP(launch_level(l.kind, l.D, l.L, l.variant, a, grid, f, stream), "level kernel launch");
  } else {
    TailArgs a{};
    a.table = ttable;
    a.count = count;
    a.total_wg = total_wg;
    a.t0 = l.tail;
    ES_HIP(launch_tail(l.kind, l.D, l.L, a, grid, l.lds, f, stream), "tail kernel launch");
  }
  return ES_OK;
}

es_status run_schedule(const Schedule& sc, const Geo& g, int64_t batch, const float* in, float* out,
                       hipStream_t stream) {
  if (batch == 0) return ES_OK;
  if (sc.identity) {
    const int64_t n = batch * g.N();
    if (n % 4 == 0) {
      ES_HIP(launch_copy(in, out, n, stream), "copy kernel launch");
    } else {
      ES_HIP(hipMemcpyAsync(out, in, n * sizeof(float), hipMemcpyDeviceToDevice, stream), "hipMemcpyAsync");
    }
    return ES_OK;
  }
  for (const Launch& l : sc.launches) {
    const int64_t per = l.is_tail ? 1 : l.task.tiles_per_inst;
    const int64_t total = per * batch;
    if (total > 0x7fffffffll) return fail(ES_EINVAL, "too many work-groups in one launch");
    es_status st = run_launch(l, sc.f, stream, nullptr, 1, (int)total, nullptr);
    if (st != ES_OK) return st;
  }
  return ES_OK;
}

// ------------------------------------------------------------------------------------------
// Sub-batch streams (opt-in, ESWAVE_STREAMS=S).  A large uniform batch is split into S
// sub-batches whose launch chains run
// on S streams (the caller's and S-1 library streams, all at default priority), forked from and
// joined back to the caller's stream with events.  The coarse levels of one sub-batch
// (latency-bound, few work-groups) then overlap the bandwidth-bound fine levels of another,
// and each sub-batch re-reads its input sooner after the first read (cache reuse).

constexpr int kMaxStreams = 4;

struct SideStreams {
  std::mutex mu;
  bool init = false;
  hipStream_t s[kMaxStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxStreams] = {};
};

SideStreams& side_streams(int dev) {
  static SideStreams pool[64];
  return pool[dev & 63];
}

int stream_count(const Geo& g, int64_t batch) {
  int S = 1;  // measured: two or more streams were slower on 64 x 1024^2 db8 (opt-in)
  const char* e = getenv("ESWAVE_STREAMS");
  if (e && *e) S = atoi(e);
  if (S < 1) S = 1;
  if (S > kMaxStreams) S = kMaxStreams;
  // only worth it for batches of large instances (ESWAVE_SPLIT_MIN: minimum voxels per
  // sub-batch, default 2^22)
  int64_t min_vox = (int64_t)1 << 22;
  const char* m = getenv("ESWAVE_SPLIT_MIN");
  if (m && *m) min_vox = atoll(m);
  while (S > 1 && (batch < 2 * S || g.N() * (batch / S) < min_vox)) --S;
  return S;
}

int64_t sub_batch(int64_t batch, int S) { return (batch + S - 1) / S; }

es_status run_split(int op, const Geo& g, int64_t batch, int S, const float* in, float* out, float* ws,
                    hipStream_t user) {
  int dev = 0;
  ES_HIP(hipGetDevice(&dev), "hipGetDevice");
  SideStreams& ss = side_streams(dev);
  std::lock_guard<std::mutex> lk(ss.mu);
  if (!ss.init) {
    for (int k = 1; k < kMaxStreams; ++k) {
      ES_HIP(hipStreamCreateWithFlags(&ss.s[k], hipStreamNonBlocking), "hipStreamCreateWithFlags");
      ES_HIP(hipEventCreateWithFlags(&ss.join[k], hipEventDisableTiming), "hipEventCreate");
    }
    ES_HIP(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming), "hipEventCreate");
    ss.init = true;
  }
  const int64_t N = g.N(), wsi = ws_floats_per_instance(g), bk = sub_batch(batch, S);
  ES_HIP(hipEventRecord(ss.fork, user), "hipEventRecord");
  for (int k = 1; k < S; ++k) ES_HIP(hipStreamWaitEvent(ss.s[k], ss.fork, 0), "hipStreamWaitEvent");
  for (int k = 0; k < S; ++k) {
    const int64_t b0 = k * bk, nb = std::min(bk, batch - b0);
    if (nb <= 0) break;
    hipStream_t st = k == 0 ? user : ss.s[k];
    Schedule sc;
    es_status r = build_schedule(op, g, nb, in + b0 * N, out + b0 * N, ws ? ws + b0 * wsi : nullptr, &sc);
    Region reg[3];
    const int nreg = call_regions(in + b0 * N, out + b0 * N, nb * N * (int64_t)sizeof(float), ws ? ws + b0 * wsi : nullptr,
                                  (size_t)(nb * wsi) * sizeof(float), reg);
    if (r == ES_OK) r = check_schedule(sc, reg, nreg);
    if (r == ES_OK) r = run_schedule(sc, g, nb, in + b0 * N, out + b0 * N, st);
    if (r != ES_OK) return r;
  }
  for (int k = 1; k < S; ++k) {
    ES_HIP(hipEventRecord(ss.join[k], ss.s[k]), "hipEventRecord");
    ES_HIP(hipStreamWaitEvent(user, ss.join[k], 0), "hipStreamWaitEvent");
  }
  return ES_OK;
}

es_status run_op(int op, int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                 const float* in, float* out, void* ws, size_t ws_bytes, void* stream) {
  Geo g;
  es_status st = make_geo(ndim, shape, order, levels, s, &g);
  if (st != ES_OK) return st;
  const size_t need = (size_t)(batch > 0 ? batch : 0) * (size_t)ws_floats_per_instance(g) * sizeof(float);
  const bool identity = (op >= ES_OP_COV) ? levels <= 1 : levels == 0;
  st = check_io(in, out, batch, g.N(), ws, ws_bytes, identity ? 0 : need);
  if (st != ES_OK) return st;
  if (batch == 0) return ES_OK;
  if (batch > 0x7fffffffll) return fail(ES_EINVAL, "batch too large");
  st = check_device();
  if (st != ES_OK) return st;
  const int S = identity ? 1 : stream_count(g, batch);
  if (S > 1) return run_split(op, g, batch, S, in, out, (float*)ws, (hipStream_t)stream);
  Schedule sc;
  st = build_schedule(op, g, batch, in, out, (float*)ws, &sc);
  if (st != ES_OK) return st;
  Region reg[3];
  const int nreg = call_regions(in, out, batch * g.N() * (int64_t)sizeof(float), ws, need, reg);
  st = check_schedule(sc, reg, nreg);
  if (st != ES_OK) return st;
  return run_schedule(sc, g, batch, in, out, (hipStream_t)stream);
}

// ------------------------------------------------------------------------------------------
// Plain reference path: per instance, per level, per axis, one launch each.

int64_t plain_ws_floats(const Geo& g, int op) {
  const int64_t N = align64(g.N());
  if (op == ES_OP_COV || op == ES_OP_SAMPLE) return 3 * N;  // coefficients + two temporaries
  return 2 * N;
}

es_status plain_instance(int op, const Geo& g, const Filter& f, const float* in, float* out, float* ws,
                         hipStream_t s) {
  const int64_t N = align64(g.N());
  float* T1 = ws;
  float* T2 = ws + N;
  float* C = ws + 2 * N;  // coefficient buffer (cov / sample)
  int full[3];
  g.level_dims(0, full);
  int32_t stf[2];
  strides_of(full, stf);
  const int D = g.D, m = g.m;
  auto pass = [&](const float* src, float* dst, int i, int ax, int synth, int scale, float w) -> es_status {
    PlainPass p{};
    p.src = src;
    p.dst = dst;
    g.level_dims(i - 1, p.b);
    p.st_src[0] = p.st_dst[0] = stf[0];
    p.st_src[1] = p.st_dst[1] = stf[1];
    p.axis = ax;
    p.synth = synth;
    p.scale_mode = scale;
    p.ndim = D;
    p.w = w;
    ES_HIP(launch_plain_pass(p, g.L, f, s), "plain pass launch");
    return ES_OK;
  };
  auto blk_copy = [&](const float* src, float* dst, int i) -> es_status {
    int b[3];
    g.level_dims(i - 1, b);
    int st[2] = {stf[0], stf[1]};
    ES_HIP(launch_block_copy(src, dst, b, st, st, s), "block copy launch");
    return ES_OK;
  };
  // analysis of `src` into packed coefficients `dst` (dst may equal the level-2+ source)
  auto analysis = [&](const float* src, float* dst, double tau) -> es_status {
    for (int i = 1; i <= m; ++i) {
      const float w = (float)wdet(g, tau, i);
      const float* a = i == 1 ? src : dst;
      // axes last to first, ping-pong T1/T2, the level's last pass scales and writes dst
      int axes[3], na = 0;
      for (int ax = 2; ax >= 3 - D; --ax) axes[na++] = ax;
      const float* cur = a;
      for (int k = 0; k < na; ++k) {
        const bool last = k == na - 1;
        float* nxt = last ? dst : (k % 2 == 0 ? T1 : T2);
        if (last && cur == dst) nxt = (k % 2 == 0 ? T1 : T2);  // avoid in-place pass
        es_status st = pass(cur, nxt, i, axes[k], 0, last ? 1 : 0, w);
        if (st != ES_OK) return st;
        if (last && nxt != dst) {
          st = blk_copy(nxt, dst, i);
          if (st != ES_OK) return st;
        }
        cur = nxt;
      }
    }
    return ES_OK;
  };
  // synthesis of packed coefficients `src` into `dst` (src is copied to dst first)
  auto synthesis = [&](const float* src, float* dst, double tau) -> es_status {
    ES_HIP(launch_copy_any(src, dst, g.N(), s), "copy kernel launch");
    for (int i = m; i >= 1; --i) {
      const float w = (float)wdet(g, tau, i);
      int axes[3], na = 0;
      for (int ax = 3 - D; ax <= 2; ++ax) axes[na++] = ax;
      const float* cur = dst;
      for (int k = 0; k < na; ++k) {
        const bool last = k == na - 1;
        float* nxt = last ? dst : (k % 2 == 0 ? T1 : T2);
        if (last && cur == dst) nxt = (k % 2 == 0 ? T1 : T2);
        es_status st = pass(cur, nxt, i, axes[k], 1, k == 0 ? 2 : 0, w);
        if (st != ES_OK) return st;
        if (last && nxt != dst) {
          st = blk_copy(nxt, dst, i);
          if (st != ES_OK) return st;
        }
        cur = nxt;
      }
    }
    return ES_OK;
  };
  switch (op) {
    case ES_OP_ADJOINT: return analysis(in, out, 1.0);
    case ES_OP_APPLY: return synthesis(in, out, 1.0);
    default: {
      // D_tau = D_{tau/2} D_{tau/2}: half of the weight on each side
      const double half_tau = op == ES_OP_COV ? 1.0 : 0.5;
      es_status st = analysis(in, C, half_tau);
      if (st != ES_OK) return st;
      return synthesis(C, out, half_tau);
    }
  }
}



// ------------------------------------------------------------------------------------------
// Ragged plans.  Every instance gets the schedule a single call would run; launches of the
// same phase (down level i, tail, up level i) and the same kernel instantiation are merged
// into one launch whose work-groups look their instance up in a device task table.  Phases
// run in dependency order: down levels ascending, tails, up levels descending, so each
// instance's steps keep their order.  The whole sequence is captured once into a hipGraph.

struct PlanGroup {
  int phase;
  Launch proto;           // kernel instantiation (kind, D, L, variant, vec, lds)
  std::vector<int> inst;  // instances, in table order
  std::vector<int> step;  // index of the step in the instance's schedule
  int64_t table_off;      // first entry in the task (or tail) table
  int total_wg;
};

}  // namespace

struct es_plan {
  int op = 0;
  int device = 0;
  std::vector<Geo> geos;
  std::vector<int64_t> ws_off;
  std::vector<int64_t> ws_len;  // floats of each instance's workspace slice
  int64_t ws_total = 0;
  std::vector<std::vector<int>> phase_of;  // per instance: phase of each schedule step
  std::vector<PlanGroup> groups;
  std::vector<Task> h_tasks;
  std::vector<TailTask> h_tails;
  Task* d_tasks = nullptr;
  TailTask* d_tails = nullptr;
  Filter filt[17];
  std::vector<const float*> last_in;
  std::vector<float*> last_out;
  void* last_ws = nullptr;
  bool tables_valid = false;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  // the streams and events used to capture the graph, kept until the graph is destroyed
  std::vector<hipStream_t> cap_streams;
  std::vector<hipEvent_t> cap_events;
  std::vector<int> identity_inst;  // instances whose op is the identity (plain copy)
  int64_t lp_coarse = -1;          // phase-merged cov / sample: largest coarse block (-1: the default)
  std::vector<std::vector<Launch>> frozen;  // per instance: its schedule at creation (sentinel pointers)
  bool host_only = false;                   // es_plan_create_host: tables only, no device resources
  // persistent execution (cov / sample): one launch per dimensionality over a work-item queue
  bool persistent = false;
  double lag = 1.0;                 // pipeline lag scale of the item order
  int64_t coarse_limit = kPCoarseMax;
  int spin_limit = 1 << 16;  // polls of one dependency wait (of the order of 0.1 s)
  int nq = kPMaxQueues;      // queues of a persistent launch: the device's XCDs
  int chunk = 4;             // tiles per work item of large steps
  struct PGroup {  // one persistent launch: the instances of one (dimensionality, taps)
    int D = 0;
    int L = 0;
    std::vector<PStep> h_steps;     // frozen steps (sentinel pointers)
    std::vector<PStep> cur_steps;   // steps with the caller's pointers
    std::vector<PItem> h_items;     // execution order, queue after queue
    std::vector<int32_t> qbegin;    // queue q: items [qbegin[q], qbegin[q + 1])
    PStep* d_steps = nullptr;
    PItem* d_items = nullptr;
    int32_t* d_ctr = nullptr;
    int grid = 0;
  };
  std::vector<PGroup> pgroups;
};

namespace {

// Plans freeze every instance schedule when they are created: kernel, tile variant, tile
// counts, vector path and coarse-kernel LDS class are decided once, from the knobs and the
// tune cache as they are at es_plan_create.  The schedules are built against sentinel base
// addresses (one range each for the input, the output and the workspace, far apart and never
// dereferenced); when the caller's pointers change, each table entry is the frozen launch with
// its pointers moved from the sentinel ranges to the caller's buffers, nothing else.
constexpr uintptr_t kSentinelIn = (uintptr_t)1 << 44;
constexpr uintptr_t kSentinelOut = (uintptr_t)2 << 44;
constexpr uintptr_t kSentinelWs = (uintptr_t)3 << 44;
constexpr uintptr_t kSentinelSpan = (uintptr_t)1 << 44;

es_status instance_schedule_frozen(const es_plan* p, int k, Schedule* sc) {
  const Geo& g = p->geos[k];
  g_variant_batch = (int64_t)p->geos.size();
  const es_status st = build_schedule(p->op, g, 1, (const float*)kSentinelIn, (float*)kSentinelOut,
                                      (float*)kSentinelWs + p->ws_off[k], sc);
  g_variant_batch = 0;
  return st;
}

// Moves one pointer from its sentinel range to the caller's buffer; false if it lies in none.
template <class T>
bool rebase(T*& ptr, const float* in, float* out, void* ws) {
  if (!ptr) return true;
  const uintptr_t v = (uintptr_t)ptr;
  const uintptr_t bases[3] = {kSentinelIn, kSentinelOut, kSentinelWs};
  const uintptr_t real[3] = {(uintptr_t)in, (uintptr_t)out, (uintptr_t)ws};
  for (int i = 0; i < 3; ++i)
    if (v >= bases[i] && v < bases[i] + kSentinelSpan) {
      ptr = (T*)(real[i] + (v - bases[i]));
      return true;
    }
  return false;
}

// Phase of step j of an instance schedule: down steps get their level index, the tail 1000,
// up steps 2000 - (level they produce).
void step_phases(int op, const Geo& g, const Schedule& sc, std::vector<int>* ph) {
  ph->clear();
  int down = 0;
  for (const Launch& l : sc.launches) {
    if (l.is_tail) {
      ph->push_back(op == ES_OP_APPLY ? 0 : 1000);
    } else if (kind_is_analysis(l.kind)) {
      ph->push_back(++down);
    } else {
      // LP_UP / FB_UP: task.b is the full-res output block; its level index follows from size
      int lev = 0;
      while (lev < 31 && (g.n[2] >> lev) != l.task.b[2]) ++lev;
      ph->push_back(2000 - lev);
    }
  }
}

// A member launch may share a group's kernel only if it is the same instantiation.
bool same_kernel(const Launch& a, const Launch& proto) {
  return a.is_tail == proto.is_tail && a.kind == proto.kind && a.D == proto.D && a.L == proto.L &&
         a.variant == proto.variant && a.vec == proto.vec && (!a.is_tail || a.lds <= proto.lds);
}

es_status plan_fill_tables(es_plan* p, const float* const* in, float* const* out, void* ws) {
  const int n = (int)p->geos.size();
  Region reg[3];
  for (PlanGroup& gr : p->groups) {
    int64_t wg = 0;
    for (size_t q = 0; q < gr.inst.size(); ++q) {
      const int k = gr.inst[q];
      if (k < 0 || k >= n || gr.step[q] < 0 || gr.step[q] >= (int)p->frozen[k].size())
        return fail(ES_EINVAL, "plan table: instance %d step %d is not in its frozen schedule", k, gr.step[q]);
      Launch l = p->frozen[k][gr.step[q]];
      if (!same_kernel(l, gr.proto))
        return fail(ES_EINVAL, "plan table: instance %d step %d does not match its launch group's kernel", k, gr.step[q]);
      const float* ik = in ? in[k] : nullptr;
      float* ok = out ? out[k] : nullptr;
      bool moved = true;
      if (l.is_tail) {
        moved = rebase(l.tail.in, ik, ok, ws) && rebase(l.tail.out, ik, ok, ws);
      } else {
        moved = rebase(l.task.in0, ik, ok, ws) && rebase(l.task.in1, ik, ok, ws) && rebase(l.task.in2, ik, ok, ws) &&
                rebase(l.task.out0, ik, ok, ws) && rebase(l.task.out1, ik, ok, ws);
      }
      if (!moved) return fail(ES_EINVAL, "plan table: instance %d step %d has a pointer outside its buffers", k, gr.step[q]);
      if (!l.is_tail) {
        // the launch's vector path was chosen when the plan was built; every instance must allow it
        if (l.vec && !vec_ok(l.task, l.kind, p->geos[k]))
          return fail(ES_EINVAL, "instance %d: pointers not aligned as the plan's vector path requires", k);
      }
      // instance k may touch its input, its output and its own slice of the workspace only
      const int64_t nbytes = p->geos[k].N() * (int64_t)sizeof(float);
      const int nreg = call_regions(ik, ok, nbytes, ws ? (float*)ws + p->ws_off[k] : nullptr,
                                    (size_t)p->ws_len[k] * sizeof(float), reg);
      char what[64];
      snprintf(what, sizeof what, "plan instance %d step %d", k, gr.step[q]);
      es_status st = check_launch(l, reg, nreg, what);
      if (st != ES_OK) return st;
      if (l.is_tail) {
        TailTask t = l.tail;
        t.tile_begin = (int32_t)wg;
        t.batch = 1;
        p->h_tails[gr.table_off + q] = t;
        wg += 1;
      } else {
        Task t = l.task;
        t.tile_begin = (int32_t)wg;
        t.batch = 1;
        p->h_tasks[gr.table_off + q] = t;
        wg += t.tiles_per_inst;
      }
      if (wg > 0x7fffffffll) return fail(ES_EINVAL, "plan launch group has too many work-groups");
    }
    gr.total_wg = (int)wg;
  }
  return ES_OK;
}

es_status plan_launch_group(es_plan* p, const PlanGroup& gr, hipStream_t s) {
  const Filter& f = p->filt[gr.proto.L];
  return run_launch(gr.proto, f, s, gr.proto.is_tail ? nullptr : p->d_tasks + gr.table_off, (int)gr.inst.size(),
                    gr.total_wg, gr.proto.is_tail ? p->d_tails + gr.table_off : nullptr);
}

// All groups in order on one stream.
es_status plan_launch_all(es_plan* p, hipStream_t s) {
  for (const PlanGroup& gr : p->groups) {
    es_status st = plan_launch_group(p, gr, s);
    if (st != ES_OK) return st;
  }
  return ES_OK;
}

// Graph capture with concurrent groups: the groups of one phase touch disjoint instances, so they
// are forked onto `nside` side streams (joined back before the next phase); the captured graph
// then holds them as parallel branches and the device overlaps their launches.  Events are
// created here and destroyed by the caller after the capture ends.
es_status plan_launch_all_forked(es_plan* p, hipStream_t s, hipStream_t* side, int nside,
                                 std::vector<hipEvent_t>* events) {
  auto new_event = [&](hipEvent_t* e) -> es_status {
    ES_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming), "hipEventCreate");
    events->push_back(*e);
    return ES_OK;
  };
  const size_t n = p->groups.size();
  for (size_t g = 0; g < n;) {
    size_t e = g;
    while (e < n && p->groups[e].phase == p->groups[g].phase) ++e;
    const int width = (int)std::min<size_t>(e - g, (size_t)nside + 1);
    if (width == 1) {
      for (size_t q = g; q < e; ++q) {
        es_status st = plan_launch_group(p, p->groups[q], s);
        if (st != ES_OK) return st;
      }
      g = e;
      continue;
    }
    hipEvent_t fork;
    es_status st = new_event(&fork);
    if (st != ES_OK) return st;
    ES_HIP(hipEventRecord(fork, s), "hipEventRecord");
    for (int k = 1; k < width; ++k) ES_HIP(hipStreamWaitEvent(side[k - 1], fork, 0), "hipStreamWaitEvent");
    for (size_t q = g; q < e; ++q) {
      const int k = (int)((q - g) % width);
      st = plan_launch_group(p, p->groups[q], k == 0 ? s : side[k - 1]);
      if (st != ES_OK) return st;
    }
    for (int k = 1; k < width; ++k) {
      hipEvent_t join;
      st = new_event(&join);
      if (st != ES_OK) return st;
      ES_HIP(hipEventRecord(join, side[k - 1]), "hipEventRecord");
      ES_HIP(hipStreamWaitEvent(s, join, 0), "hipStreamWaitEvent");
    }
    g = e;
  }
  return ES_OK;
}

es_status plan_identity_copies(es_plan* p, const float* const* in, float* const* out, hipStream_t s) {
  for (int k : p->identity_inst) {
    const int64_t N = p->geos[k].N();
    if (N % 4 == 0) {
      ES_HIP(launch_copy(in[k], out[k], N, s), "copy kernel launch");
    } else {
      ES_HIP(hipMemcpyAsync(out[k], in[k], N * sizeof(float), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
    }
  }
  return ES_OK;
}

// ---- persistent plans -------------------------------------------------------------------

// Persistent execution (ESWAVE_PLAN_PERSISTENT=1 at plan creation) is available for plans of the
// projection-form operators whose level launches all take the vector staging path.  It is not
// the default: measured on 64 x 1024^2 db8 (0.54 ms against 0.35 ms phase-merged and 0.27 ms
// for one uniform call) and on 200 ragged instances (1.51 against 0.98 ms), its work-groups run
// at 4 per CU (the union of tile bodies holds 128 registers) where the level kernels run 6 to 8,
// and every work item pays a queue pop and a dependency poll.
bool persistent_wanted(int op) {
  if (op != ES_OP_COV && op != ES_OP_SAMPLE) return false;
  const char* e = getenv("ESWAVE_PLAN_PERSISTENT");
  return e && *e == '1';
}

// Cost model of the item order: the bytes a step moves (its footprint) and the latency between
// its last item being taken and its completion (a tile's duration; a coarse block's serial work).
double step_bytes(const Launch& l) {
  std::vector<Access> acc;
  launch_accesses(l, &acc);
  double b = 0;
  for (const Access& a : acc) b += (double)a.span;
  return b;
}
double step_latency_us(const Launch& l) {
  if (!l.is_tail) return 6.0;
  const double B = (double)dense_span(l.tail.b);
  return 4.0 + B * l.L / 8000.0;
}

// Builds the persistent step tables of a plan from its frozen schedules, and the item order:
// a list-scheduling simulation of the device (throughput kRate bytes/us) in which an instance's
// next step becomes ready `lag` x its predecessor's latency after that predecessor was issued;
// at each point the oldest started instance with a ready step is issued, else a new instance is
// started.  lag -> 0 gives instance after instance, a large lag gives level after level.
// Every instance's steps appear in order, so each step's dependency precedes it in the list.
void persistent_tables(es_plan* p) {
  constexpr double kRate = 5000.0;  // bytes per microsecond
  p->pgroups.clear();
  const int n = (int)p->geos.size();
  for (int D = 1; D <= 3; ++D)
  for (int L = 2; L <= kMaxTaps; L += 2) {
    es_plan::PGroup G;
    G.D = D;
    G.L = L;
    std::vector<int> inst;
    for (int k = 0; k < n; ++k)
      if (p->geos[k].D == D && p->geos[k].L == L) inst.push_back(k);
    if (inst.empty()) continue;
    // steps, instance by instance
    std::vector<int> first(inst.size()), count(inst.size());
    std::vector<double> bytes, lat;
    for (size_t q = 0; q < inst.size(); ++q) {
      const int k = inst[q];
      first[q] = (int)G.h_steps.size();
      const Geo& g = p->geos[k];
      if (p->frozen[k].empty()) {  // identity: a copy of the input
        PStep st{};
        st.kind = P_COPY;
        st.L = g.L;
        st.wait = -1;
        st.inst = k;
        st.task.in0 = (const float*)kSentinelIn;
        st.task.out0 = (float*)kSentinelOut;
        st.task.bs_in0 = g.N();
        st.ntiles = (int)((g.N() + kPCopyChunk - 1) / kPCopyChunk);
        G.h_steps.push_back(st);
        bytes.push_back(8.0 * (double)g.N());
        lat.push_back(2.0);
      } else {
        for (const Launch& l : p->frozen[k]) {
          PStep st{};
          st.inst = k;
          st.L = l.L;
          if (l.is_tail) {
            st.kind = P_COARSE;
            st.tail = l.tail;
            st.tail.batch = 1;
            st.tail.tile_begin = 0;
            st.ntiles = 1;
          } else {
            st.kind = kind_is_analysis(l.kind) ? P_LP_DOWN : P_LP_UP;
            st.task = l.task;
            st.task.batch = 1;
            st.task.tile_begin = 0;
            st.ntiles = l.task.tiles_per_inst;
          }
          const int idx = (int)G.h_steps.size();
          st.wait = idx > first[q] ? idx - 1 : -1;
          st.wait_count = st.wait >= 0 ? G.h_steps[st.wait].ntiles : 0;
          G.h_steps.push_back(st);
          bytes.push_back(step_bytes(l));
          lat.push_back(step_latency_us(l));
        }
      }
      count[q] = (int)G.h_steps.size() - first[q];
    }
    // instances to queues (one per XCD): longest first onto the least loaded queue
    const int ni = (int)inst.size();
    const int nq = std::max(1, std::min(p->nq, kPMaxQueues));
    std::vector<double> work(ni, 0.0), load(nq, 0.0);
    for (int q = 0; q < ni; ++q)
      for (int j = first[q]; j < first[q] + count[q]; ++j) work[q] += bytes[j];
    std::vector<int> by_work(ni), queue_of(ni);
    for (int q = 0; q < ni; ++q) by_work[q] = q;
    std::stable_sort(by_work.begin(), by_work.end(), [&](int a, int b) { return work[a] > work[b]; });
    for (int q : by_work) {
      const int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      queue_of[q] = best;
      load[best] += work[q];
    }
    // item order of each queue: the queue's XCD (throughput kRate / nq) simulated as above
    G.qbegin.assign(nq + 1, 0);
    for (int Q = 0; Q < nq; ++Q) {
      G.qbegin[Q] = (int32_t)G.h_items.size();
      std::vector<int> mine;
      for (int q = 0; q < ni; ++q)
        if (queue_of[q] == Q) mine.push_back(q);
      const int nm = (int)mine.size();
      std::vector<int> next(nm, 0);
      std::vector<double> ready(nm, 0.0);
      int started = 0, finished = 0;
      double t = 0;
      while (finished < nm) {
        int pick = -1;
        for (int r = 0; r < started; ++r)
          if (next[r] < count[mine[r]] && ready[r] <= t) { pick = r; break; }
        if (pick < 0) {
          if (started < nm) {
            pick = started++;
          } else {
            double tmin = 1e300;
            for (int r = 0; r < started; ++r)
              if (next[r] < count[mine[r]]) tmin = std::min(tmin, ready[r]);
            t = tmin;
            continue;
          }
        }
        const int q = mine[pick];
        const int j = first[q] + next[pick];
        // consecutive tiles share filter halos: larger steps hand out a few per item
        const int nt = G.h_steps[j].ntiles;
        const int chunk = G.h_steps[j].kind == P_COPY ? 1 : (nt >= 64 ? p->chunk : (nt >= 16 ? std::min(2, p->chunk) : 1));
        for (int tile = 0; tile < nt; tile += chunk) G.h_items.push_back(PItem{j, tile, std::min(chunk, nt - tile), 0});
        t += bytes[j] / (kRate / nq);
        ready[pick] = t + p->lag * lat[j];
        if (++next[pick] == count[q]) ++finished;
      }
    }
    G.qbegin[nq] = (int32_t)G.h_items.size();
    G.cur_steps = G.h_steps;
    p->pgroups.push_back(std::move(G));
  }
}

// Fills the persistent step tables for the caller's pointers, checking every step's footprint
// against the instance's buffers.
es_status persistent_fill(es_plan* p, const float* const* in, float* const* out, void* ws) {
  Region reg[3];
  for (es_plan::PGroup& G : p->pgroups) {
    for (size_t j = 0; j < G.h_steps.size(); ++j) {
      PStep st = G.h_steps[j];
      const int k = st.inst;
      const float* ik = in ? in[k] : nullptr;
      float* ok = out ? out[k] : nullptr;
      bool moved = true;
      if (st.kind == P_COARSE) {
        moved = rebase(st.tail.in, ik, ok, ws) && rebase(st.tail.out, ik, ok, ws);
      } else {
        moved = rebase(st.task.in0, ik, ok, ws) && rebase(st.task.in1, ik, ok, ws) &&
                rebase(st.task.in2, ik, ok, ws) && rebase(st.task.out0, ik, ok, ws) &&
                rebase(st.task.out1, ik, ok, ws);
      }
      if (!moved) return fail(ES_EINVAL, "plan instance %d: a step has a pointer outside its buffers", k);
      const int64_t nbytes = p->geos[k].N() * (int64_t)sizeof(float);
      const int nreg = call_regions(ik, ok, nbytes, ws ? (float*)ws + p->ws_off[k] : nullptr,
                                    (size_t)p->ws_len[k] * sizeof(float), reg);
      char what[64];
      snprintf(what, sizeof what, "plan instance %d step %zu", k, j);
      if (st.kind == P_COPY) {
        const Access a{st.task.in0, 0, st.task.bs_in0 * 4, false}, b{st.task.out0, 0, st.task.bs_in0 * 4, true};
        for (const Access& x : {a, b}) {
          bool fits = false;
          for (int r = 0; r < nreg && !fits; ++r)
            fits = (uintptr_t)x.base >= reg[r].lo && (uintptr_t)x.base + x.span <= reg[r].hi && (!x.write || reg[r].writable);
          if (!fits) return fail(ES_EINVAL, "%s: copy outside the caller's buffers", what);
        }
      } else {
        Launch l{};
        l.is_tail = st.kind == P_COARSE;
        l.kind = l.is_tail ? 3 : (st.kind == P_LP_DOWN ? K_LP_DOWN : K_LP_UP);
        l.D = G.D;
        l.L = st.L;
        l.task = st.task;
        l.tail = st.tail;
        if (!l.is_tail && !vec_ok(l.task, l.kind, p->geos[k]))
          return fail(ES_EINVAL, "instance %d: pointers not aligned as the plan's vector path requires", k);
        es_status e = check_launch(l, reg, nreg, what);
        if (e != ES_OK) return e;
      }
      G.cur_steps[j] = st;
    }
  }
  return ES_OK;
}

// Workspace slice of every instance (persistent plans: write-once level arrays, twice the size).
void plan_layout(es_plan* p, bool persist) {
  const int n = (int)p->geos.size();
  p->ws_off.assign(n, 0);
  p->ws_len.assign(n, 0);
  p->ws_total = 0;
  const SchedMode keep = g_mode;
  g_mode.persist = persist;
  for (int k = 0; k < n; ++k) {
    p->ws_off[k] = p->ws_total;
    p->ws_len[k] = ws_floats_per_instance(p->geos[k]);
    p->ws_total += p->ws_len[k];
  }
  g_mode = keep;
}

// Host part of plan creation: geometries, workspace offsets, frozen schedules, launch groups and
// host tables (no device call).
es_status plan_build(const es_desc* descs, int32_t count, int op, es_plan** out, int64_t lp_coarse = -1) {
  *out = nullptr;
  if (count < 0 || (count > 0 && !descs)) return fail(ES_EINVAL, "descs must hold count >= 0 entries");
  if (op < 0 || op > 3) return fail(ES_EINVAL, "unknown op %d", op);
  es_plan* p = new (std::nothrow) es_plan();
  if (!p) return fail(ES_ENOMEM, "plan allocation failed");
  p->op = op;
  for (int o = 1; o <= 8; ++o)
    if (!get_filter(2 * o, &p->filt[2 * o])) { delete p; return fail(ES_EUNSUPPORTED, "filter derivation failed"); }
  p->geos.resize(count);
  es_status st = ES_OK;
  for (int k = 0; k < count; ++k) {
    const es_desc& d = descs[k];
    st = make_geo(d.ndim, d.shape, d.order, d.levels, d.s, &p->geos[k]);
    if (st != ES_OK) { delete p; return fail(st, "desc %d: %s", k, g_last_error.c_str()); }
  }
  plan_layout(p, persistent_wanted(op));
  // freeze every instance schedule: for persistent execution when every level launch can take
  // the persistent kernel's (vector) path, else for phase-merged launches
  std::vector<Schedule> scs(count);
  p->frozen.resize(count);
  p->persistent = persistent_wanted(op);
  if (p->persistent) {
    const char* e = getenv("ESWAVE_PLAN_COARSE_MAX");
    if (e && *e) p->coarse_limit = std::max<int64_t>(0, std::min<int64_t>(atoll(e), kPCoarseMax));
    const char* lg = getenv("ESWAVE_PLAN_LAG");
    if (lg && *lg) p->lag = std::max(0.0, atof(lg));
    const char* sp = getenv("ESWAVE_PERSIST_SPIN");
    if (sp && *sp) p->spin_limit = atoi(sp);
    const char* ch = getenv("ESWAVE_PLAN_CHUNK");
    if (ch && *ch) p->chunk = std::max(1, std::min(64, atoi(ch)));
    g_mode.persist = true;
    g_mode.coarse_limit = p->coarse_limit;
    for (int k = 0; k < count && p->persistent; ++k) {
      st = instance_schedule_frozen(p, k, &scs[k]);
      if (st != ES_OK) break;
      for (const Launch& l : scs[k].launches)
        if (!l.is_tail && !l.vec) p->persistent = false;
    }
    g_mode = SchedMode{};
    if (st != ES_OK) { delete p; return st; }
    if (p->persistent) {
      for (int k = 0; k < count; ++k)
        if (!scs[k].identity) p->frozen[k] = scs[k].launches;
      persistent_tables(p);
      *out = p;
      return ES_OK;
    }
    plan_layout(p, false);  // phase-merged after all: in-place level arrays
  }
  p->lp_coarse = lp_coarse;
  for (int k = 0; k < count; ++k) {
    g_lp_coarse = lp_coarse;
    st = instance_schedule_frozen(p, k, &scs[k]);
    g_lp_coarse = -1;
    if (st != ES_OK) { delete p; return st; }
    if (scs[k].identity) { p->identity_inst.push_back(k); continue; }
    p->frozen[k] = scs[k].launches;
    std::vector<int> ph;
    step_phases(op, p->geos[k], scs[k], &ph);
    for (size_t j = 0; j < scs[k].launches.size(); ++j) {
      const Launch& l = scs[k].launches[j];
      PlanGroup* gr = nullptr;
      for (PlanGroup& c : p->groups)
        if (c.phase == ph[j] && c.proto.is_tail == l.is_tail && c.proto.kind == l.kind && c.proto.D == l.D &&
            c.proto.L == l.L && c.proto.variant == l.variant && c.proto.vec == l.vec) { gr = &c; break; }
      if (!gr) {
        p->groups.push_back(PlanGroup{});
        gr = &p->groups.back();
        gr->phase = ph[j];
        gr->proto = l;
        gr->proto.lds = 0;
      }
      gr->inst.push_back(k);
      gr->step.push_back((int)j);
      if (l.is_tail) gr->proto.lds = std::max(gr->proto.lds, l.lds);
    }
  }
  std::stable_sort(p->groups.begin(), p->groups.end(), [](const PlanGroup& a, const PlanGroup& b) { return a.phase < b.phase; });
  int64_t nt = 0, ntail = 0;
  for (PlanGroup& gr : p->groups) {
    if (gr.proto.is_tail) { gr.table_off = ntail; ntail += gr.inst.size(); }
    else { gr.table_off = nt; nt += gr.inst.size(); }
  }
  p->h_tasks.resize(nt);
  p->h_tails.resize(ntail);
  *out = p;
  return ES_OK;
}

// Host checks of the caller's pointers for one execution (no device call).
es_status plan_check_io(const es_plan* p, const float* const* in, float* const* out, void* ws, size_t ws_bytes) {
  if (!in || !out) return fail(ES_EINVAL, "in and out must be non-NULL host arrays");
  const int n = (int)p->geos.size();
  if (p->ws_total > 0) {
    if (!ws) return fail(ES_EWORKSPACE, "workspace of %zu bytes required", (size_t)p->ws_total * sizeof(float));
    if (ws_bytes < (size_t)p->ws_total * sizeof(float)) return fail(ES_EWORKSPACE, "workspace too small");
    if ((uintptr_t)ws & 15) return fail(ES_EINVAL, "workspace must be 16-byte aligned");
  }
  for (int k = 0; k < n; ++k) {
    const size_t bytes = (size_t)p->geos[k].N() * sizeof(float);
    es_status st = check_io(in[k], out[k], 1, p->geos[k].N(), nullptr, 0, 0);
    if (st != ES_OK) return fail(st, "instance %d: %s", k, g_last_error.c_str());
    if (ws && p->ws_total && (overlap(ws, p->ws_total * sizeof(float), in[k], bytes) ||
                              overlap(ws, p->ws_total * sizeof(float), out[k], bytes)))
      return fail(ES_EINVAL, "instance %d overlaps the workspace", k);
  }
  return ES_OK;
}

es_status plan_prepare(es_plan* p, const float* const* in, float* const* out, void* ws, size_t ws_bytes,
                       hipStream_t s, bool* changed) {
  if (p->host_only) return fail(ES_EINVAL, "plan was created by es_plan_create_host (no device resources)");
  es_status st0 = plan_check_io(p, in, out, ws, ws_bytes);
  if (st0 != ES_OK) return st0;
  const int n = (int)p->geos.size();
  int dev = 0;
  ES_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev != p->device) return fail(ES_EINVAL, "plan was created on device %d, current device is %d", p->device, dev);
  bool same = p->tables_valid && ws == p->last_ws;
  for (int k = 0; same && k < n; ++k) same = in[k] == p->last_in[k] && out[k] == p->last_out[k];
  *changed = !same;
  if (!same && p->persistent) {
    es_status st = persistent_fill(p, in, out, ws);
    if (st != ES_OK) return st;
    for (es_plan::PGroup& G : p->pgroups)
      ES_HIP(hipMemcpyAsync(G.d_steps, G.cur_steps.data(), G.cur_steps.size() * sizeof(PStep), hipMemcpyHostToDevice, s),
             "step table upload");
    p->last_in.assign(in, in + n);
    p->last_out.assign(out, out + n);
    p->last_ws = ws;
    p->tables_valid = true;
    return ES_OK;
  }
  if (!same) {
    es_status st = plan_fill_tables(p, in, out, ws);
    if (st != ES_OK) return st;
    if (!p->h_tasks.empty())
      ES_HIP(hipMemcpyAsync(p->d_tasks, p->h_tasks.data(), p->h_tasks.size() * sizeof(Task), hipMemcpyHostToDevice, s),
             "task table upload");
    if (!p->h_tails.empty())
      ES_HIP(hipMemcpyAsync(p->d_tails, p->h_tails.data(), p->h_tails.size() * sizeof(TailTask),
                            hipMemcpyHostToDevice, s),
             "tail table upload");
    p->last_in.assign(in, in + n);
    p->last_out.assign(out, out + n);
    p->last_ws = ws;
    p->tables_valid = true;
  }
  return ES_OK;
}

// Device tables of a persistent plan (items are fixed at creation; steps are uploaded at fill).
void persistent_free(es_plan* p) {
  for (es_plan::PGroup& G : p->pgroups) {
    if (G.d_steps) (void)hipFree(G.d_steps);
    if (G.d_items) (void)hipFree(G.d_items);
    if (G.d_ctr) (void)hipFree(G.d_ctr);
    G.d_steps = nullptr;
    G.d_items = nullptr;
    G.d_ctr = nullptr;
  }
}

es_status persistent_alloc(es_plan* p) {
  for (es_plan::PGroup& G : p->pgroups) {
    if (hipMalloc(&G.d_steps, G.h_steps.size() * sizeof(PStep)) != hipSuccess ||
        hipMalloc(&G.d_items, std::max<size_t>(1, G.h_items.size()) * sizeof(PItem)) != hipSuccess ||
        hipMalloc(&G.d_ctr, (kPDone + G.h_steps.size()) * sizeof(int32_t)) != hipSuccess)
      return fail(ES_ENOMEM, "persistent plan table allocation failed");
    if (!G.h_items.empty())
      ES_HIP(hipMemcpy(G.d_items, G.h_items.data(), G.h_items.size() * sizeof(PItem), hipMemcpyHostToDevice),
             "item table upload");
    ES_HIP(hipMemset(G.d_ctr, 0, (kPDone + G.h_steps.size()) * sizeof(int32_t)), "counter clear");
    const int resident = persist_resident_groups(G.D, G.L);
    if (resident <= 0) return fail(ES_EDEVICE, "occupancy query of the persistent kernel failed");
    // every XCD must receive work-groups (they are handed out round-robin): at least one per
    // queue, in multiples of the queue count
    const int nq = (int)G.qbegin.size() - 1;
    int64_t grid = std::min<int64_t>((int64_t)G.h_items.size(), resident);
    grid = (grid + nq - 1) / nq * nq;
    G.grid = (int)std::max<int64_t>(grid, nq);
  }
  return ES_OK;
}

// One persistent group: clear its counters (a fill kernel, also inside captured graphs), run it.
es_status persistent_launch_group(es_plan* p, const es_plan::PGroup& G, hipStream_t s) {
  ES_HIP(launch_zero_ints(G.d_ctr, kPDone + (int64_t)G.h_steps.size(), s), "counter reset launch");
  PArgs a{};
  a.items = G.d_items;
  a.steps = G.d_steps;
  a.counters = G.d_ctr;
  a.nq = (int32_t)G.qbegin.size() - 1;
  for (int q = 0; q <= a.nq; ++q) a.qbegin[q] = G.qbegin[q];
  a.spin_limit = p->spin_limit;
  a.f = p->filt[G.L];
  ES_HIP(launch_persist(G.D, G.L, a, G.grid, s), "persistent kernel launch");
  return ES_OK;
}

// Every group; groups after the first run on side streams forked from and joined back to `s`
// (their instances are disjoint), when side streams are given.
es_status persistent_launch_all(es_plan* p, hipStream_t s, hipStream_t* side, int nside,
                                std::vector<hipEvent_t>* events) {
  const int ng = (int)p->pgroups.size();
  if (ng <= 1 || nside <= 0 || !events) {
    for (const es_plan::PGroup& G : p->pgroups) {
      es_status st = persistent_launch_group(p, G, s);
      if (st != ES_OK) return st;
    }
    return ES_OK;
  }
  hipEvent_t fork;
  ES_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming), "hipEventCreate");
  events->push_back(fork);
  ES_HIP(hipEventRecord(fork, s), "hipEventRecord");
  const int width = std::min(ng, nside + 1);
  for (int k = 1; k < width; ++k) ES_HIP(hipStreamWaitEvent(side[k - 1], fork, 0), "hipStreamWaitEvent");
  for (int g = 0; g < ng; ++g) {
    const int k = g % width;
    es_status st = persistent_launch_group(p, p->pgroups[g], k == 0 ? s : side[k - 1]);
    if (st != ES_OK) return st;
  }
  for (int k = 1; k < width; ++k) {
    hipEvent_t join;
    ES_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming), "hipEventCreate");
    events->push_back(join);
    ES_HIP(hipEventRecord(join, side[k - 1]), "hipEventRecord");
    ES_HIP(hipStreamWaitEvent(s, join, 0), "hipStreamWaitEvent");
  }
  return ES_OK;
}

void plan_drop_graph(es_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  for (hipEvent_t ev : p->cap_events) (void)hipEventDestroy(ev);
  for (hipStream_t st : p->cap_streams) (void)hipStreamDestroy(st);
  p->cap_events.clear();
  p->cap_streams.clear();
}

// Rebuilds a persistent plan's frozen schedules, step tables and item order for its current
// lag and coarse limit (used by the plan autotuner), with fresh device tables.
es_status persistent_rebuild(es_plan* p) {
  plan_drop_graph(p);
  persistent_free(p);
  const int n = (int)p->geos.size();
  std::vector<Schedule> scs(n);
  g_mode.persist = true;
  g_mode.coarse_limit = p->coarse_limit;
  es_status st = ES_OK;
  for (int k = 0; k < n && st == ES_OK; ++k) {
    st = instance_schedule_frozen(p, k, &scs[k]);
    for (const Launch& l : scs[k].launches)
      if (st == ES_OK && !l.is_tail && !l.vec) st = fail(ES_EUNSUPPORTED, "instance %d needs the scalar staging path", k);
  }
  g_mode = SchedMode{};
  if (st != ES_OK) return st;
  for (int k = 0; k < n; ++k) p->frozen[k] = scs[k].identity ? std::vector<Launch>() : scs[k].launches;
  persistent_tables(p);
  p->tables_valid = false;
  return persistent_alloc(p);
}

// Device task tables of a phase-merged plan.
es_status plan_alloc_tables(es_plan* p) {
  const size_t nt = p->h_tasks.size(), ntail = p->h_tails.size();
  if (nt && hipMalloc(&p->d_tasks, nt * sizeof(Task)) != hipSuccess) return fail(ES_ENOMEM, "task table allocation failed");
  if (ntail && hipMalloc(&p->d_tails, ntail * sizeof(TailTask)) != hipSuccess)
    return fail(ES_ENOMEM, "tail table allocation failed");
  return ES_OK;
}

// Best of three rounds of `reps` eager executions (after one warm execution), in ms.
es_status plan_time_eager(es_plan* p, const float* const* in, float* const* out, void* ws, size_t ws_bytes, int reps,
                          hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* best) {
  es_status st = es_plan_execute_eager(p, in, out, ws, ws_bytes, s);
  *best = 1e30f;
  for (int round = 0; round < 3 && st == ES_OK; ++round) {
    if (hipEventRecord(e0, s) != hipSuccess) return fail(ES_EDEVICE, "hipEventRecord");
    for (int r = 0; r < reps && st == ES_OK; ++r) st = es_plan_execute_eager(p, in, out, ws, ws_bytes, s);
    float ms = 0.f;
    if (st == ES_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = fail(ES_EDEVICE, "event timing failed");
    if (st == ES_OK) *best = std::min(*best, ms);
  }
  return st;
}

// Tuning of a phase-merged plan.
//  1. Coarse fusion depth (cov / sample): the largest block the coarse-level kernel takes, among
//     16384, 4096 and 1024 floats; each candidate is a plan rebuilt with that limit and timed as a
//     whole (it changes the launch count and the summation order: results agree to rounding).
//  2. Tile choice of every launch group (tile variant, and kernel family where a level has two),
//     greedily in decreasing order of work-groups, each candidate timed inside the whole plan
//     (bit-identical results).  A candidate whose tiles fail the host footprint checks is skipped.
es_status plan_autotune_merged(es_plan* p, const float* const* in, float* const* out, void* ws, size_t ws_bytes,
                               int reps, hipStream_t s) {
  ES_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  plan_drop_graph(p);  // re-captured by the next es_plan_execute
  p->tables_valid = false;
  hipEvent_t e0, e1;
  ES_HIP(hipEventCreate(&e0), "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(ES_EDEVICE, "hipEventCreate"); }
  es_status st = ES_OK;
  bool has_tail = false;
  for (const PlanGroup& gr : p->groups) has_tail = has_tail || gr.proto.is_tail;
  if ((p->op == ES_OP_COV || p->op == ES_OP_SAMPLE) && has_tail) {
    const int n = (int)p->geos.size();
    std::vector<es_desc> descs(n);
    for (int k = 0; k < n; ++k) {
      const Geo& g = p->geos[k];
      es_desc d{};
      d.ndim = g.D;
      d.order = g.L / 2;
      for (int a = 0; a < g.D; ++a) d.shape[a] = g.n[3 - g.D + a];
      d.levels = g.m;
      d.s = g.s;
      descs[k] = d;
    }
    float t_cur = 0.f;
    st = plan_time_eager(p, in, out, ws, ws_bytes, reps, s, e0, e1, &t_cur);
    const int64_t cands[] = {kCoarseMaxBlockBig, kCoarseMaxBlock, kCoarseMaxBlock / 4};
    for (int64_t c : cands) {
      if (st != ES_OK) break;
      if (c == (p->lp_coarse < 0 ? kCoarseMaxBlockBig : p->lp_coarse)) continue;
      es_plan* q = nullptr;
      st = plan_build(descs.data(), n, p->op, &q, c);
      if (st != ES_OK) break;
      q->device = p->device;
      st = plan_alloc_tables(q);
      float t = 0.f;
      if (st == ES_OK) st = plan_time_eager(q, in, out, ws, ws_bytes, reps, s, e0, e1, &t);
      if (st == ES_OK && t < t_cur) {
        t_cur = t;
        std::swap(*p, *q);  // p takes the faster plan; q now holds the previous one
      }
      if (hipDeviceSynchronize() != hipSuccess && st == ES_OK) st = fail(ES_EDEVICE, "hipDeviceSynchronize");
      es_plan_destroy(q);
    }
  }
  // 2. tile choices, groups with the most work-groups first (tables filled by the last execution)
  if (st == ES_OK) st = es_plan_execute_eager(p, in, out, ws, ws_bytes, s);
  std::vector<int> order;
  for (int gi = 0; gi < (int)p->groups.size(); ++gi)
    if (!p->groups[gi].proto.is_tail) order.push_back(gi);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return p->groups[a].total_wg > p->groups[b].total_wg; });
  for (int gi : order) {
    if (st != ES_OK) break;
    PlanGroup& gr = p->groups[gi];
    const Launch proto0 = gr.proto;
    std::vector<Launch> keep(gr.inst.size());
    for (size_t q = 0; q < gr.inst.size(); ++q) keep[q] = p->frozen[gr.inst[q]][gr.step[q]];
    auto apply = [&](int c) {
      for (size_t q = 0; q < gr.inst.size(); ++q) {
        Launch l = keep[q];
        apply_choice(l, p->geos[gr.inst[q]], c, 1);
        p->frozen[gr.inst[q]][gr.step[q]] = l;
        if (q == 0) gr.proto = l;
      }
      gr.proto.lds = proto0.lds;
      p->tables_valid = false;
    };
    const int nc = num_choices(proto0);
    int best = -1;
    float t_best = 1e30f;
    for (int c = 0; c < nc && st == ES_OK; ++c) {
      apply(c);
      bool same = true;  // every member must take the same kernel instantiation
      for (size_t q = 0; q < gr.inst.size(); ++q) same = same && same_kernel(p->frozen[gr.inst[q]][gr.step[q]], gr.proto);
      if (!same) continue;
      float t = 0.f;
      st = plan_time_eager(p, in, out, ws, ws_bytes, reps, s, e0, e1, &t);
      if (st == ES_EINVAL) { st = ES_OK; continue; }  // tiles refused by the footprint checks
      if (st == ES_OK && t < t_best) { t_best = t; best = c; }
    }
    if (st != ES_OK) break;
    if (best < 0) {  // no candidate ran: keep the frozen launches
      for (size_t q = 0; q < gr.inst.size(); ++q) p->frozen[gr.inst[q]][gr.step[q]] = keep[q];
      gr.proto = proto0;
      p->tables_valid = false;
    } else {
      apply(best);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ES_OK) return st;
  // the timing runs repeated in-place launches: recompute the result with the tuned plan
  st = es_plan_execute_eager(p, in, out, ws, ws_bytes, s);
  if (st == ES_OK) ES_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  plan_drop_graph(p);
  p->tables_valid = false;
  return st;
}

}  // namespace

namespace es {

int64_t cov_dot_partials_max(int ndim, const int64_t* shape) {
  if (ndim != 2 || !shape || shape[0] < 1 || shape[1] < 1) return 0;
  int64_t best = 0;
  for (int v = 0; v < kNumVariants; ++v) {
    const TileShape ts = tile_shape(K_LP_UP, 2, v, kMaxTaps);  // 2-D synthesis tiles do not depend on the taps
    best = std::max<int64_t>(best, ((shape[0] + ts.t[1] - 1) / ts.t[1]) * ((shape[1] + ts.t[2] - 1) / ts.t[2]));
  }
  return best;
}

es_status cov_apply_masked_dot(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                               const float* x, float* y, void* ws, size_t ws_bytes, const float* mask, float gamma,
                               float scale, float* partials, int64_t partials_cap, int64_t* per, hipStream_t stream) {
  Geo g;
  es_status st = make_geo(ndim, shape, order, levels, s, &g);
  if (st != ES_OK) return st;
  if (ndim != 2 || levels <= 1 || batch < 1 || batch > 0x7fffffffll)
    return fail(ES_EUNSUPPORTED, "the fused solver step needs a 2-D geometry, at least 2 levels and 1 <= batch < 2^31");
  const size_t need = (size_t)batch * (size_t)ws_floats_per_instance(g) * sizeof(float);
  st = check_io(x, y, batch, g.N(), ws, ws_bytes, need);
  if (st != ES_OK) return st;
  if (stream_count(g, batch) > 1) return fail(ES_EUNSUPPORTED, "sub-batch streams split this schedule");
  Schedule sc;
  st = build_schedule(ES_OP_COV, g, batch, x, y, (float*)ws, &sc);
  if (st != ES_OK) return st;
  if (sc.identity || sc.launches.empty()) return fail(ES_EUNSUPPORTED, "identity schedule");
  const Launch& last = sc.launches.back();
  if (last.is_tail || last.kind != K_LP_UP || !last.vec || last.task.out0 != y || last.task.in1 != x)
    return fail(ES_EUNSUPPORTED, "the schedule does not end in a 2-D vector-path synthesis of x");
  const int64_t tpi = last.task.tiles_per_inst;
  if (!partials || tpi * batch > partials_cap) return fail(ES_EINVAL, "partial-sum buffer too small");
  Region reg[3];
  const int nreg = call_regions(x, y, batch * g.N() * (int64_t)sizeof(float), ws, need, reg);
  st = check_schedule(sc, reg, nreg);
  if (st != ES_OK) return st;
  st = check_device();
  if (st != ES_OK) return st;
  for (size_t j = 0; j + 1 < sc.launches.size(); ++j) {
    const Launch& l = sc.launches[j];
    const int64_t total = (l.is_tail ? 1 : l.task.tiles_per_inst) * batch;
    if (total > 0x7fffffffll) return fail(ES_EINVAL, "too many work-groups in one launch");
    st = run_launch(l, sc.f, stream, nullptr, 1, (int)total, nullptr);
    if (st != ES_OK) return st;
  }
  Task t = last.task;
  t.in2 = mask;
  t.bs_in2 = g.N();
  t.gamma = mask ? gamma : 0.f;
  t.alpha *= scale;
  t.beta *= scale;
  t.out1 = partials;
  const int64_t total = tpi * batch;
  if (total > 0x7fffffffll) return fail(ES_EINVAL, "too many work-groups in one launch");
  TaskArgs a{};
  a.table = nullptr;
  a.count = 1;
  a.total_wg = (int)total;
  a.vec = 1;
  a.reverse = last.reverse;
  a.t0 = t;
  ES_HIP(launch_lp_up_cge(last.L, last.variant, a, (int)round8(total), sc.f, stream), "fused solver step launch");
  *per = tpi;
  return ES_OK;
}

es_status report_error(es_status st, const char* msg) {
  g_last_error = msg;
  return st;
}
es_status device_check() { return check_device(); }
}  // namespace es

// ------------------------------------------------------------------------------------------
// Exports.

extern "C" {

es_status es_adjoint(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s, const float* x,
                     float* coeff, void* ws, size_t ws_bytes, void* stream) {
  return run_op(ES_OP_ADJOINT, ndim, shape, batch, order, levels, s, x, coeff, ws, ws_bytes, stream);
}

es_status es_apply(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s, const float* coeff,
                   float* x, void* ws, size_t ws_bytes, void* stream) {
  return run_op(ES_OP_APPLY, ndim, shape, batch, order, levels, s, coeff, x, ws, ws_bytes, stream);
}

es_status matern_cov_apply(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                           const float* x, float* y, void* ws, size_t ws_bytes, void* stream) {
  return run_op(ES_OP_COV, ndim, shape, batch, order, levels, s, x, y, ws, ws_bytes, stream);
}

es_status matern_sample(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                        const float* xi, float* x, void* ws, size_t ws_bytes, void* stream) {
  return run_op(ES_OP_SAMPLE, ndim, shape, batch, order, levels, s, xi, x, ws, ws_bytes, stream);
}

size_t es_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels, int op) {
  Geo g;
  if (make_geo(ndim, shape, order, levels, 0.0, &g) != ES_OK || batch < 0 || op < 0 || op > 3) return 0;
  const bool identity = (op >= ES_OP_COV) ? levels <= 1 : levels == 0;
  if (identity) return 0;
  return (size_t)batch * (size_t)ws_floats_per_instance(g) * sizeof(float);
}

// ------------------------------------------------------------------------------------------
// Squared H^s norm: ||x||^2_{H^s} = ||D_{-s} W x||^2 = sum of 2^{2 s j} c^2 over the orthonormal
// coefficients c = W x (detail level i: j = m - i; approximation: 1).  The analysis launch
// sequence of es_adjoint with smoothness -s runs in squared-norm mode: coefficients are squared
// and summed per work-group instead of stored, and one finalising launch adds the partials of
// each instance in a fixed order.

// Partial sums (compensated FP32 pairs, 8 bytes each) the squared-norm mode needs per instance: for every level launch the
// most tiles any of its candidates uses, plus one for the coarse-level kernel.
int64_t norm_partials_per_instance(const Geo& g) {
  Schedule sc;
  if (build_schedule_raw(ES_OP_ADJOINT, g, 1, (const float*)(uintptr_t)256, (float*)(uintptr_t)512,
                         (float*)(uintptr_t)1024, &sc) != ES_OK)
    return -1;
  int64_t n = 0;
  for (const Launch& l : sc.launches) {
    if (l.is_tail) { n += 1; continue; }
    int64_t mx = 0;
    for (int c = 0; c < num_choices(l); ++c) {
      Launch k = l;
      apply_choice(k, g, c, 1);
      mx = std::max<int64_t>(mx, k.task.tiles_per_inst);
    }
    n += mx;
  }
  return n;
}

size_t norm_ws_bytes(const Geo& g, int64_t batch) {
  if (g.m == 0 || batch <= 0) return 0;
  const int64_t per = norm_partials_per_instance(g);
  if (per < 0) return 0;
  const size_t lv = ((size_t)batch * (size_t)ws_floats_per_instance(g) * sizeof(float) + 255) & ~(size_t)255;
  return lv + (size_t)batch * (size_t)per * sizeof(float2);
}

size_t es_hs_norm_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels) {
  Geo g;
  if (make_geo(ndim, shape, order, levels, 0.0, &g) != ES_OK || batch < 0) return 0;
  return norm_ws_bytes(g, batch);
}

es_status es_hs_norm_sq(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                        const float* x, float* norms, void* ws, size_t ws_bytes, void* stream) {
  Geo g;
  es_status st = make_geo(ndim, shape, order, levels, -s, &g);  // weights 2^{+s j}
  if (st != ES_OK) return st;
  if (batch < 0) return fail(ES_EINVAL, "batch must be >= 0");
  if (batch == 0) return ES_OK;
  if (batch > 0x7fffffffll) return fail(ES_EINVAL, "batch too large");
  if (!x || !norms) return fail(ES_EINVAL, "input and output pointers must be non-NULL");
  if (((uintptr_t)x & 15) || ((uintptr_t)norms & 3))
    return fail(ES_EINVAL, "input must be 16-byte and output 4-byte aligned");
  const size_t xbytes = (size_t)(batch * g.N()) * sizeof(float);
  if (overlap(x, xbytes, norms, (size_t)batch * sizeof(float))) return fail(ES_EINVAL, "input and output overlap");
  const size_t need = norm_ws_bytes(g, batch);
  if (need) {
    if (!ws) return fail(ES_EWORKSPACE, "workspace of %zu bytes required, got NULL", need);
    if (ws_bytes < need) return fail(ES_EWORKSPACE, "workspace of %zu bytes required, got %zu", need, ws_bytes);
    if ((uintptr_t)ws & 255) return fail(ES_EINVAL, "workspace must be 256-byte aligned");
    if (overlap(ws, need, x, xbytes) || overlap(ws, need, norms, (size_t)batch * sizeof(float)))
      return fail(ES_EINVAL, "workspace overlaps input or output");
  }
  st = check_device();
  if (st != ES_OK) return st;
  const hipStream_t hs = (hipStream_t)stream;
  if (g.m == 0) {  // W = I
    ES_HIP(launch_sumsq(x, g.N(), batch, norms, hs), "sum-of-squares launch");
    return ES_OK;
  }
  float* lv = (float*)ws;
  float2* partials = (float2*)((char*)ws + (((size_t)batch * (size_t)ws_floats_per_instance(g) * sizeof(float) + 255) &
                                            ~(size_t)255));
  Schedule sc;
  // the coefficient array is never written in squared-norm mode: pass the partials as its address
  st = build_schedule(ES_OP_ADJOINT, g, batch, x, (float*)partials, lv, &sc);
  if (st != ES_OK) return st;
  bool has_tail = false;
  for (const Launch& l : sc.launches) has_tail |= l.is_tail != 0;
  NormSegs segs{};
  int64_t off = 0;
  for (size_t j = 0; j < sc.launches.size(); ++j) {
    Launch& l = sc.launches[j];
    if (segs.count >= kMaxNormSegs) return fail(ES_EUNSUPPORTED, "too many levels for the squared-norm mode");
    segs.off[segs.count] = off;
    if (l.is_tail) {
      l.tail.flags = kNormSq;
      l.tail.out = (float*)(partials + off);
      segs.per[segs.count++] = 1;
      off += batch;
    } else {
      l.task.flags = kNormSq | ((!has_tail && j + 1 == sc.launches.size()) ? kNormLL : 0);
      l.task.out0 = (float*)(partials + off);
      l.task.bs_out0 = 0;
      segs.per[segs.count++] = l.task.tiles_per_inst;
      off += (int64_t)l.task.tiles_per_inst * batch;
    }
  }
  {
    const Region reg[2] = {{(uintptr_t)x, (uintptr_t)x + xbytes, false}, {(uintptr_t)ws, (uintptr_t)ws + need, true}};
    st = check_schedule(sc, reg, 2);
    if (st != ES_OK) return st;
  }
  st = run_schedule(sc, g, batch, x, (float*)partials, hs);
  if (st != ES_OK) return st;
  ES_HIP(launch_norm_finalize(partials, segs, norms, batch, hs), "norm finalize launch");
  return ES_OK;
}

size_t es_workspace_bytes_plain(int ndim, const int64_t* shape, int64_t batch, int order, int levels, int op) {
  Geo g;
  (void)batch;
  if (make_geo(ndim, shape, order, levels, 0.0, &g) != ES_OK || op < 0 || op > 3) return 0;
  return (size_t)plain_ws_floats(g, op) * sizeof(float);
}

es_status es_plain_apply_op(int op, int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                            const float* in, float* out, void* ws, size_t ws_bytes, void* stream) {
  if (op < 0 || op > 3) return fail(ES_EINVAL, "unknown op %d", op);
  Geo g;
  es_status st = make_geo(ndim, shape, order, levels, s, &g);
  if (st != ES_OK) return st;
  if (g.N() % 4) return fail(ES_EUNSUPPORTED, "the plain path needs instance sizes divisible by 4");
  const size_t need = (size_t)plain_ws_floats(g, op) * sizeof(float);
  st = check_io(in, out, batch, g.N(), ws, ws_bytes, need);
  if (st != ES_OK) return st;
  if (batch == 0) return ES_OK;
  st = check_device();
  if (st != ES_OK) return st;
  Filter f;
  if (!get_filter(g.L, &f)) return fail(ES_EUNSUPPORTED, "filter derivation failed");
  const hipStream_t hs = (hipStream_t)stream;
  for (int64_t b = 0; b < batch; ++b) {
    const float* ib = in + b * g.N();
    float* ob = out + b * g.N();
    if (g.m == 0) {
      ES_HIP(launch_copy_any(ib, ob, g.N(), hs), "copy kernel launch");
      continue;
    }
    st = plain_instance(op, g, f, ib, ob, (float*)ws, hs);
    if (st != ES_OK) return st;
  }
  return ES_OK;
}

es_status es_plan_create(const es_desc* descs, int32_t count, int op, void* stream, es_plan** out) {
  if (!out) return fail(ES_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 0 || (count > 0 && !descs)) return fail(ES_EINVAL, "descs must hold count >= 0 entries");
  if (op < 0 || op > 3) return fail(ES_EINVAL, "unknown op %d", op);
  es_status st = check_device();
  if (st != ES_OK) return st;
  (void)stream;
  es_plan* p = nullptr;
  st = plan_build(descs, count, op, &p);
  if (st != ES_OK) return st;
  if (hipGetDevice(&p->device) != hipSuccess) { es_plan_destroy(p); return fail(ES_EDEVICE, "hipGetDevice failed"); }
  if (p->persistent) {
    int nxcc = 0;
    if (hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, p->device) != hipSuccess || nxcc < 1) nxcc = 1;
    if (nxcc != p->nq) {  // the item lists were built for kPMaxQueues XCDs
      p->nq = std::min(nxcc, kPMaxQueues);
      persistent_tables(p);
    }
    st = persistent_alloc(p);
    if (st != ES_OK) { es_plan_destroy(p); return st; }
    *out = p;
    return ES_OK;
  }
  st = plan_alloc_tables(p);
  if (st != ES_OK) { es_plan_destroy(p); return st; }
  *out = p;
  return ES_OK;
}

es_status es_plan_create_host(const es_desc* descs, int32_t count, int op, es_plan** out) {
  if (!out) return fail(ES_EINVAL, "out is NULL");
  *out = nullptr;
  es_plan* p = nullptr;
  es_status st = plan_build(descs, count, op, &p);
  if (st != ES_OK) return st;
  p->host_only = true;
  *out = p;
  return ES_OK;
}

es_status es_plan_fill_host(es_plan* p, const uint64_t* in, const uint64_t* out, uint64_t ws, size_t ws_bytes) {
  if (!p) return fail(ES_EINVAL, "plan is NULL");
  if (p->geos.empty()) return ES_OK;
  if (!in || !out) return fail(ES_EINVAL, "in and out must be non-NULL host arrays");
  const int n = (int)p->geos.size();
  std::vector<const float*> ip(n);
  std::vector<float*> op(n);
  for (int k = 0; k < n; ++k) {
    ip[k] = (const float*)(uintptr_t)in[k];
    op[k] = (float*)(uintptr_t)out[k];
  }
  es_status st = plan_check_io(p, ip.data(), op.data(), (void*)(uintptr_t)ws, ws_bytes);
  if (st != ES_OK) return st;
  if (p->persistent) return persistent_fill(p, ip.data(), op.data(), (void*)(uintptr_t)ws);
  return plan_fill_tables(p, ip.data(), op.data(), (void*)(uintptr_t)ws);
}

int64_t es_plan_work_groups(const es_plan* p) {
  if (!p) return -1;
  int64_t n = 0;
  if (p->persistent) {
    for (const es_plan::PGroup& G : p->pgroups)
      for (const PItem& it : G.h_items) n += it.ntile;
    return n;
  }
  for (const PlanGroup& gr : p->groups) n += gr.total_wg;
  return n;
}

es_status es_plan_execute_eager(es_plan* p, const float* const* in, float* const* out, void* ws, size_t ws_bytes,
                                void* stream) {
  if (!p) return fail(ES_EINVAL, "plan is NULL");
  if (p->geos.empty()) return ES_OK;
  const hipStream_t s = (hipStream_t)stream;
  bool changed = false;
  es_status st = plan_prepare(p, in, out, ws, ws_bytes, s, &changed);
  if (st != ES_OK) return st;
  if (p->persistent) return persistent_launch_all(p, s, nullptr, 0, nullptr);
  st = plan_identity_copies(p, in, out, s);
  if (st != ES_OK) return st;
  return plan_launch_all(p, s);
}

es_status es_plan_execute(es_plan* p, const float* const* in, float* const* out, void* ws, size_t ws_bytes,
                          void* stream) {
  if (!p) return fail(ES_EINVAL, "plan is NULL");
  if (p->geos.empty()) return ES_OK;
  const hipStream_t s = (hipStream_t)stream;
  bool changed = false;
  es_status st = plan_prepare(p, in, out, ws, ws_bytes, s, &changed);
  if (st != ES_OK) return st;
  // identity instances are plain copies of caller pointers: launched eagerly (persistent plans
  // copy them in their own launches)
  st = plan_identity_copies(p, in, out, s);
  if (st != ES_OK) return st;
  if (p->groups.empty() && p->pgroups.empty()) return ES_OK;
  if (!p->exec) {
    // kernels read everything through the device tables, so the captured graph stays valid
    // when the caller's pointers change (only the tables are refreshed, above)
    // groups of a phase run as parallel branches, ESWAVE_PLAN_BRANCHES of them at most
    // (default: 4, or 1 -- one chain -- for plans under 2^22 voxels, where the cross-queue
    // synchronisation of the branches costs more than their overlap gains)
    constexpr int kSide = 15;
    constexpr int64_t kBranchMinVoxels = 1 << 22;
    hipStream_t cap = nullptr, side[kSide] = {};
    ES_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate");
    const char* br = getenv("ESWAVE_PLAN_BRANCHES");
    int64_t voxels = 0;
    for (const Geo& g : p->geos) voxels += g.N();
    const int def_br = voxels < kBranchMinVoxels ? 1 : 4;
    int nside = std::max(0, std::min(kSide, (br && *br ? atoi(br) : def_br) - 1));
    if (p->persistent) nside = std::min(kSide, (int)p->pgroups.size() - 1);  // one branch per launch
    hipError_t e = hipSuccess;
    for (int k = 0; k < nside && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking);
    std::vector<hipEvent_t> events;
    auto cleanup = [&]() {
      for (hipEvent_t ev : events) (void)hipEventDestroy(ev);
      for (int k = 0; k < kSide; ++k)
        if (side[k]) (void)hipStreamDestroy(side[k]);
      (void)hipStreamDestroy(cap);
    };
    if (e != hipSuccess) { cleanup(); return dev_fail(e, "hipStreamCreate"); }
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { cleanup(); return dev_fail(e, "hipStreamBeginCapture"); }
    if (p->persistent) st = persistent_launch_all(p, cap, side, nside, &events);
    else st = nside ? plan_launch_all_forked(p, cap, side, nside, &events) : plan_launch_all(p, cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap, &graph);
    if (st != ES_OK) { cleanup(); if (graph) (void)hipGraphDestroy(graph); return st; }
    if (e != hipSuccess) { cleanup(); return dev_fail(e, "hipStreamEndCapture"); }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { cleanup(); (void)hipGraphDestroy(graph); return dev_fail(e, "hipGraphInstantiate"); }
    p->graph = graph;
    p->exec = exec;
    // the capture streams and events are released with the graph (es_plan_destroy), not before
    p->cap_events = events;
    p->cap_streams.push_back(cap);
    for (int k = 0; k < kSide; ++k)
      if (side[k]) p->cap_streams.push_back(side[k]);
  }
  ES_HIP(hipGraphLaunch(p->exec, s), "hipGraphLaunch");
  return ES_OK;
}

size_t es_plan_workspace_bytes(const es_plan* p) { return p ? (size_t)p->ws_total * sizeof(float) : 0; }

int32_t es_plan_num_launches(const es_plan* p) {
  if (p && p->persistent) return (int32_t)p->pgroups.size();
  return p ? (int32_t)(p->groups.size() + p->identity_inst.size()) : 0;
}

int32_t es_plan_is_persistent(const es_plan* p) { return p && p->persistent ? 1 : 0; }

es_status es_plan_errors(es_plan* p, void* stream) {
  if (!p) return fail(ES_EINVAL, "plan is NULL");
  if (!p->persistent || p->host_only) return ES_OK;
  ES_HIP(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
  for (const es_plan::PGroup& G : p->pgroups) {
    int32_t words[kPDone] = {};
    ES_HIP(hipMemcpy(words, G.d_ctr, sizeof words, hipMemcpyDeviceToHost), "error word read");
    if (words[kPMaxQueues] != 0)
      return fail(ES_EDEVICE, "persistent plan (%d-D, %d-tap launch): a dependency wait gave up after its poll "
                              "limit; the results of the last execution are invalid", G.D, G.L);
    const int nq = (int)G.qbegin.size() - 1;
    for (int q = 0; q < nq; ++q)
      if (words[q] < G.qbegin[q + 1] - G.qbegin[q])
        return fail(ES_EDEVICE, "persistent plan (%d-D, %d-tap launch): queue %d was not drained (no work-group ran "
                                "on its XCD); the results of the last execution are invalid", G.D, G.L, q);
  }
  return ES_OK;
}

es_status es_plan_autotune(es_plan* p, const float* const* in, float* const* out, void* ws, size_t ws_bytes,
                           int32_t reps, void* stream) {
  if (!p) return fail(ES_EINVAL, "plan is NULL");
  if (p->geos.empty()) return ES_OK;
  if (p->host_only) return fail(ES_EINVAL, "plan was created by es_plan_create_host (no device resources)");
  if (reps < 1) reps = 3;
  const hipStream_t s = (hipStream_t)stream;
  if (!p->persistent) {
    const es_status st0 = plan_check_io(p, in, out, ws, ws_bytes);
    if (st0 != ES_OK) return st0;
    return plan_autotune_merged(p, in, out, ws, ws_bytes, reps, s);
  }
  // candidates: coarse fusion depth (largest block the coarse step takes) x pipeline lag
  const int64_t coarse[] = {kPCoarseMax, kPCoarseMax / 4};
  const double lags[] = {0.25, 1.0, 4.0, 64.0};
  hipEvent_t e0, e1;
  ES_HIP(hipEventCreate(&e0), "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(ES_EDEVICE, "hipEventCreate"); }
  es_status st = ES_OK;
  float best = 1e30f;
  int64_t best_c = p->coarse_limit;
  double best_l = p->lag;
  for (int64_t c : coarse) {
    for (double l : lags) {
      p->coarse_limit = c;
      p->lag = l;
      st = persistent_rebuild(p);
      if (st == ES_OK) st = es_plan_execute_eager(p, in, out, ws, ws_bytes, stream);  // warm + table fill
      if (st != ES_OK) break;
      float tmin = 1e30f;
      for (int round = 0; round < 3 && st == ES_OK; ++round) {
        if (hipEventRecord(e0, s) != hipSuccess) { st = fail(ES_EDEVICE, "hipEventRecord"); break; }
        for (int r = 0; r < reps && st == ES_OK; ++r) st = es_plan_execute_eager(p, in, out, ws, ws_bytes, stream);
        float ms = 0.f;
        if (st == ES_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          st = fail(ES_EDEVICE, "event timing failed");
        tmin = std::min(tmin, ms);
      }
      if (st == ES_OK) st = es_plan_errors(p, stream);
      if (st != ES_OK) break;
      if (tmin < best) { best = tmin; best_c = c; best_l = l; }
    }
    if (st != ES_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->coarse_limit = best_c;
  p->lag = best_l;
  es_status st2 = persistent_rebuild(p);
  if (st != ES_OK) return st;
  return st2;
}

es_status es_plan_config(const es_plan* p, int64_t* coarse_limit, double* lag, int64_t* items) {
  if (!p) return fail(ES_EINVAL, "plan is NULL");
  if (coarse_limit)
    *coarse_limit = p->persistent ? p->coarse_limit : (p->lp_coarse >= 0 ? p->lp_coarse : -1);
  if (lag) *lag = p->persistent ? p->lag : -1.0;
  if (items) {
    int64_t n = 0;
    for (const es_plan::PGroup& G : p->pgroups) n += (int64_t)G.h_items.size();
    *items = n;
  }
  return ES_OK;
}

void es_plan_destroy(es_plan* p) {
  if (!p) return;
  persistent_free(p);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  for (hipEvent_t ev : p->cap_events) (void)hipEventDestroy(ev);
  for (hipStream_t s : p->cap_streams) (void)hipStreamDestroy(s);
  if (p->d_tasks) (void)hipFree(p->d_tasks);
  if (p->d_tails) (void)hipFree(p->d_tails);
  delete p;
}

int32_t es_schedule_length(int op, int ndim, const int64_t* shape, int64_t batch, int order, int levels) {
  Geo g;
  if (op < 0 || op > 3 || batch < 1 || make_geo(ndim, shape, order, levels, 0.0, &g) != ES_OK) return -1;
  Schedule sc;
  if (build_schedule(op, g, batch, (const float*)(uintptr_t)256, (float*)(uintptr_t)512, (float*)(uintptr_t)1024, &sc) !=
      ES_OK)
    return -1;
  return sc.identity ? 0 : (int32_t)sc.launches.size();
}

es_status es_schedule_describe(int op, int ndim, const int64_t* shape, int64_t batch, int order, int levels,
                               int32_t index, char* name, size_t name_len, int64_t* work_groups, int32_t* level) {
  Geo g;
  if (op < 0 || op > 3) return fail(ES_EINVAL, "unknown op %d", op);
  if (batch < 1) return fail(ES_EINVAL, "batch must be >= 1");
  es_status st = make_geo(ndim, shape, order, levels, 0.0, &g);
  if (st != ES_OK) return st;
  Schedule sc;
  st = build_schedule(op, g, batch, (const float*)(uintptr_t)256, (float*)(uintptr_t)512, (float*)(uintptr_t)1024, &sc);
  if (st != ES_OK) return st;
  if (index < 0 || index >= (int32_t)sc.launches.size()) return fail(ES_EINVAL, "step index out of range");
  const Launch& l = sc.launches[index];
  static const char* kinds[9] = {"lp_down", "lp_up", "fb_down", "fb_up", "lp_up2", "fb_down_s", "fb_up_s", "lp_down_s",
                                 "lp_up_s"};
  static const char* tails[4] = {"tail_lp_off", "tail_fb_analysis", "tail_fb_synthesis", "lp_coarse"};
  char buf[128];
  int lev = 0;
  while (lev < 31 && (g.n[2] >> lev) != (l.is_tail ? l.tail.b[2] : l.task.b[2])) ++lev;
  if (l.is_tail) {
    snprintf(buf, sizeof buf, "%s_%dd_L%d", tails[l.kind], l.D, l.L);
  } else {
    const TileShape ts = tile_shape(l.kind, l.D, l.variant, l.L);
    snprintf(buf, sizeof buf, "%s_%dd_L%d_v%d_t%dx%dx%d%s", kinds[l.kind], l.D, l.L, l.variant, ts.t[0], ts.t[1],
             ts.t[2], l.vec ? "" : "_scalar");
  }
  if (name && name_len) {
    strncpy(name, buf, name_len - 1);
    name[name_len - 1] = 0;
  }
  if (work_groups) *work_groups = (l.is_tail ? 1 : (int64_t)l.task.tiles_per_inst) * batch;
  if (level) *level = lev;
  return ES_OK;
}

es_status es_schedule_run_step(int op, int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                               const float* in, float* out, void* ws, size_t ws_bytes, int32_t index, void* stream) {
  if (op < 0 || op > 3) return fail(ES_EINVAL, "unknown op %d", op);
  Geo g;
  es_status st = make_geo(ndim, shape, order, levels, s, &g);
  if (st != ES_OK) return st;
  const size_t need = (size_t)(batch > 0 ? batch : 0) * (size_t)ws_floats_per_instance(g) * sizeof(float);
  st = check_io(in, out, batch, g.N(), ws, ws_bytes, need);
  if (st != ES_OK) return st;
  if (batch < 1) return fail(ES_EINVAL, "batch must be >= 1");
  st = check_device();
  if (st != ES_OK) return st;
  Schedule sc;
  st = build_schedule(op, g, batch, in, out, (float*)ws, &sc);
  if (st != ES_OK) return st;
  if (sc.identity || index < 0 || index >= (int32_t)sc.launches.size()) return fail(ES_EINVAL, "step index out of range");
  Region reg[3];
  const int nreg = call_regions(in, out, batch * g.N() * (int64_t)sizeof(float), ws, need, reg);
  st = check_launch(sc.launches[index], reg, nreg, "launch");
  if (st != ES_OK) return st;
  const Launch& l = sc.launches[index];
  const int64_t total = (l.is_tail ? 1 : l.task.tiles_per_inst) * batch;
  return run_launch(l, sc.f, (hipStream_t)stream, nullptr, 1, (int)total, nullptr);
}

es_status es_autotune(int op, int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                      const float* in, float* out, void* ws, size_t ws_bytes, int32_t reps, void* stream) {
  if (op < 0 || op > 3) return fail(ES_EINVAL, "unknown op %d", op);
  Geo g;
  es_status st = make_geo(ndim, shape, order, levels, s, &g);
  if (st != ES_OK) return st;
  const size_t need = (size_t)(batch > 0 ? batch : 0) * (size_t)ws_floats_per_instance(g) * sizeof(float);
  const bool identity = (op >= ES_OP_COV) ? levels <= 1 : levels == 0;
  st = check_io(in, out, batch, g.N(), ws, ws_bytes, identity ? 0 : need);
  if (st != ES_OK) return st;
  if (batch < 1 || identity) return ES_OK;
  if (reps < 1) reps = 3;
  st = check_device();
  if (st != ES_OK) return st;
  // tune the schedule the operator runs: the first sub-batch when the batch is split
  const int64_t full_batch = batch;
  batch = sub_batch(batch, stream_count(g, batch));
  Schedule sc;
  st = build_schedule_raw(op, g, batch, in, out, (float*)ws, &sc);
  if (st != ES_OK) return st;
  {
    // candidates change tiles only, never the blocks a launch addresses
    Region reg[3];
    const int nreg = call_regions(in, out, batch * g.N() * (int64_t)sizeof(float), ws, need, reg);
    st = check_schedule(sc, reg, nreg);
    if (st != ES_OK) return st;
  }
  const hipStream_t hs = (hipStream_t)stream;
  // one full pass so that every launch finds valid inputs in the workspace
  st = run_schedule(sc, g, batch, in, out, hs);
  if (st != ES_OK) return st;
  hipEvent_t e0, e1;
  ES_HIP(hipEventCreate(&e0), "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(ES_EDEVICE, "hipEventCreate"); }
  // Each launch's candidates are timed inside the whole launch sequence (the other launches
  // keep their current choice), because a launch's speed depends on what the launches before
  // it left in the caches.  Launches are settled in order (greedy descent); candidates are
  // timed round-robin over kTuneRounds rounds of `reps` sequences and keep their fastest round.
  constexpr int kTuneRounds = 3;
  std::vector<int> best(sc.launches.size(), -1);
  auto time_sequence = [&](float* ms) -> es_status {
    es_status r = run_schedule(sc, g, batch, in, out, hs);  // warm
    if (r != ES_OK) return r;
    if (hipEventRecord(e0, hs) != hipSuccess) return fail(ES_EDEVICE, "hipEventRecord");
    for (int k = 0; k < reps && r == ES_OK; ++k) r = run_schedule(sc, g, batch, in, out, hs);
    if (r != ES_OK) return r;
    if (hipEventRecord(e1, hs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
      return fail(ES_EDEVICE, "event timing failed");
    return ES_OK;
  };
  for (size_t j = 0; j < sc.launches.size() && st == ES_OK; ++j) {
    if (sc.launches[j].is_tail) continue;
    const Launch keep = sc.launches[j];
    const int nc = num_choices(keep);
    std::vector<float> t_min(nc, 1e30f);
    for (int round = 0; round < kTuneRounds && st == ES_OK; ++round) {
      for (int v = 0; v < nc && st == ES_OK; ++v) {
        sc.launches[j] = keep;
        apply_choice(sc.launches[j], g, v, batch);
        float ms = 0.f;
        st = time_sequence(&ms);
        if (st == ES_OK) t_min[v] = std::min(t_min[v], ms);
      }
    }
    for (int v = 0; v < nc; ++v)
      if (best[j] < 0 || t_min[v] < t_min[best[j]]) best[j] = v;
    sc.launches[j] = keep;
    apply_choice(sc.launches[j], g, best[j], batch);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ES_OK) return st;
  tune_store(tune_key(op, g, batch), best);
  // the timing runs repeated in-place launches: recompute the result with the tuned schedule
  return run_op(op, ndim, shape, full_batch, order, levels, s, in, out, ws, ws_bytes, stream);
}

es_status es_filter(int order, double* h_out) {
  if (!h_out) return fail(ES_EINVAL, "h_out is NULL");
  if (order < 1 || order > 8) return fail(ES_EINVAL, "order must be in 1..8 (got %d)", order);
  if (!daubechies_filter(order, h_out)) return fail(ES_EUNSUPPORTED, "filter derivation failed for order %d", order);
  return ES_OK;
}

es_status es_level_weights(int levels, double s, double tau, float* w_out) {
  if (!w_out) return fail(ES_EINVAL, "w_out is NULL");
  if (levels < 0 || levels > kMaxLevels) return fail(ES_EINVAL, "levels out of range");
  if (!std::isfinite(s) || !std::isfinite(tau)) return fail(ES_EINVAL, "s and tau must be finite");
  for (int i = 1; i <= levels; ++i) w_out[i - 1] = (float)std::exp2(-tau * s * (double)(levels - i));
  w_out[levels] = 1.f;
  return ES_OK;
}

const char* es_status_string(es_status st) {
  switch (st) {
    case ES_OK: return "ES_OK";
    case ES_EINVAL: return "ES_EINVAL: invalid argument";
    case ES_EWORKSPACE: return "ES_EWORKSPACE: workspace missing or too small";
    case ES_EUNSUPPORTED: return "ES_EUNSUPPORTED: unsupported request";
    case ES_EDEVICE: return "ES_EDEVICE: HIP runtime error";
    case ES_ENOMEM: return "ES_ENOMEM: allocation failed";
  }
  return "unknown es_status";
}

const char* es_last_error(void) { return g_last_error.c_str(); }

const char* es_version(void) { return "eswave 0.1 (gfx950)"; }

}  // extern "C"

