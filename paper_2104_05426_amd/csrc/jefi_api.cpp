// libjefi C ABI: argument validation, the FP64 time prelude, launch
// planning, per-stream scratch, batched evaluation with a graph-replayed
// persistent launch, and the launch-shape autotuner.  Device work is in
// jefi_kernels.hip.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/libjefi.h"
#include "jefi_internal.h"

using namespace jefi;

namespace {

thread_local std::string g_err;
std::atomic<int> g_device_failed{0};

jefi_status fail(jefi_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

jefi_status hip_fail(hipError_t e, const char* what) {
  g_device_failed.store(1);
  return fail(JEFI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool grid_ok(const jefi_grid* g, const char* name, long long* cells) {
  if (!g) {
    fail(JEFI_EINVAL, "%s grid is NULL", name);
    return false;
  }
  const bool empty = g->n[0] == 0 && g->n[1] == 0 && g->n[2] == 0;
  long long c = 1;
  for (int a = 0; a < 3; ++a) {
    if (!empty && (g->n[a] < 1 || g->n[a] > (1 << 20))) {
      fail(JEFI_EINVAL, "%s grid: n[%d] = %d out of range", name, a, g->n[a]);
      return false;
    }
    if (!std::isfinite(g->origin[a]) || !std::isfinite(g->spacing[a]) || !(g->spacing[a] > 0.0)) {
      fail(JEFI_EINVAL, "%s grid: origin/spacing[%d] must be finite with spacing > 0", name, a);
      return false;
    }
    c *= empty ? 0 : g->n[a];
  }
  if (c > 0x7fffffffLL) {
    fail(JEFI_EINVAL, "%s grid has %lld cells (limit 2^31-1)", name, c);
    return false;
  }
  *cells = c;
  return true;
}

GridD to_gd(const jefi_grid* g) {
  GridD d;
  for (int a = 0; a < 3; ++a) {
    d.n[a] = g->n[a];
    d.o[a] = g->origin[a];
    d.h[a] = g->spacing[a];
  }
  return d;
}

long long brick_count(const jefi_grid* g, int* nbx, int* nby, int* nbz) {
  *nbx = (g->n[0] + 1) / 2;
  *nby = (g->n[1] + 1) / 2;
  *nbz = (g->n[2] + 1) / 2;
  return (long long)*nbx * *nby * *nbz;
}

size_t dtype_size(int dt) { return dt == JEFI_F64 ? 8 : 4; }

// The evaluation time on the logical slice axis (the FP64 sequence the
// header documents): a = (t - t0)/dt - s_old split into a_i + a_f.
struct TimeSplit {
  long long a_i;
  double a_f;
  double inv_cdt;
};

jefi_status time_split(double t, double t0, double dt, long long newest, int nt, double c,
                       TimeSplit* ts) {
  const long long s_old = newest - (long long)nt + 1;
  double a = (t - t0) / dt - (double)s_old;
  const double top = (double)(nt - 1);
  if (!(a <= top)) {
    const double slack = 1e-9 * (1.0 + std::fabs(a) + std::fabs((double)s_old));
    if (a - top <= slack)
      a = top;
    else
      return fail(JEFI_EINVAL, "t = %.17g lies after the newest slice (%.17g slices past it)", t,
                  a - top);
  }
  const double fl = std::floor(a);
  ts->a_i = (long long)fl;
  ts->a_f = a - fl;
  ts->inv_cdt = 1.0 / (c * dt);
  return JEFI_OK;
}

struct Resolved {
  double c;
  double screen[3];
  int precision;
  int tile_config;
  unsigned flags;
  int reserve_cus;
};

jefi_status resolve_options(const jefi_options* opt, const jefi_grid* src, Resolved* r) {
  jefi_options d;
  jefi_options_default(&d);
  if (!opt) opt = &d;
  if (!std::isfinite(opt->c) || !(opt->c > 0.0)) return fail(JEFI_EINVAL, "c must be finite and > 0");
  if (opt->precision != JEFI_PREC_F64 && opt->precision != JEFI_PREC_F32_COMP)
    return fail(JEFI_EINVAL, "unknown precision %d", opt->precision);
  if (opt->tile_config < 0 || opt->tile_config > 3)
    return fail(JEFI_EINVAL, "tile_config %d (0 = auto, 1 = 8x8x8, 2 = 8x8x4, 3 = size rule per problem)",
                opt->tile_config);
  if (opt->reserve_cus < 0 || opt->reserve_cus > 1024)
    return fail(JEFI_EINVAL, "reserve_cus %d (0 .. 1024)", opt->reserve_cus);
  const unsigned known = JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE | JEFI_FLAG_DERIV_SLOPE |
                         JEFI_FLAG_PAST_HOLD | JEFI_FLAG_TIME_CUBIC | JEFI_FLAG_PAST_CUT;
  const unsigned idx = opt->flags & (JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE);
  const unsigned slope_cubic = JEFI_FLAG_DERIV_SLOPE | JEFI_FLAG_TIME_CUBIC;
  const unsigned pasts = JEFI_FLAG_PAST_HOLD | JEFI_FLAG_PAST_CUT;
  if ((opt->flags & ~known) != 0 || idx == (JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE) ||
      (opt->flags & slope_cubic) == slope_cubic || (opt->flags & pasts) == pasts)
    return fail(JEFI_EINVAL,
                "flags 0x%x (at most one JEFI_FLAG_INDEX_* value, at most one of JEFI_FLAG_DERIV_SLOPE "
                "and JEFI_FLAG_TIME_CUBIC, at most one of JEFI_FLAG_PAST_HOLD and JEFI_FLAG_PAST_CUT)",
                opt->flags);
  r->flags = opt->flags;
  r->c = opt->c;
  r->precision = opt->precision;
  r->tile_config = opt->tile_config;
  r->reserve_cus = opt->reserve_cus;
  for (int a = 0; a < 3; ++a) {
    if (opt->screen_set) {
      if (!std::isfinite(opt->screen[a]) || opt->screen[a] < 0.0)
        return fail(JEFI_EINVAL, "screen[%d] must be finite and >= 0", a);
      r->screen[a] = opt->screen[a];
    } else {
      r->screen[a] = 0.5 * src->spacing[a];
    }
  }
  return JEFI_OK;
}

// ---- launch configurations (table filled by the autotuner) -----------------
// A launch configuration: observation tile (1 = 8x8x8, 2 = 8x8x4, 0 = the
// size rule), FP32 index mode (0 = from the guard-pair estimate, 1 = guard
// band, 2 = threshold table for every pair of a full brick) and work
// granularity (0 = default, 1 = coarser, 2 = finer: half or twice the
// workgroup target of a single launch, or 6 or 24 instead of 12 work items
// per workgroup slot of a batch).
struct LaunchCfg {
  int tile = 0, idx = 0, gran = 0;
};
int cfg_pack(const LaunchCfg& c) { return c.tile | (c.idx << 2) | (c.gran << 4); }
LaunchCfg cfg_unpack(int v) {
  LaunchCfg c;
  c.tile = v & 3;
  c.idx = (v >> 2) & 3;
  c.gran = (v >> 4) & 3;
  return c;
}
bool cfg_valid(int v) {
  const LaunchCfg c = cfg_unpack(v);
  return v >= 0 && v < 64 && c.tile <= 2 && c.idx <= 2 && c.gran <= 2;
}

// Table keys (a kind tag in bits 40..): one problem launched alone, one
// instance inside a batch, a whole batch.  The size class of a problem is
// its precision, staging window class (32, 64 or 128 slots per cell, or
// chunked), log2 of its observation points and log2 of its pairs; that of
// a batch is its precision, log2 of its instance count and log2 of its
// pairs.
enum { kKeySingle = 1, kKeyMember = 2, kKeyBatch = 3 };
std::mutex g_tune_mu;
std::map<long long, int> g_tune;
bool g_tune_loaded = false;

int log2_bucket(double v) { return v < 1.0 ? 0 : (int)std::floor(std::log2(v)); }

long long size_key(int kind, int precision, int wcls, double a, double b) {
  return ((long long)kind << 40) | ((long long)precision << 32) | ((long long)wcls << 24) |
         ((long long)log2_bucket(a) << 12) | (long long)log2_bucket(b);
}

const char* tune_path() {
  const char* p = std::getenv("JEFI_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = tune_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  long long k;
  int v;
  while (std::fscanf(f, "%lld %d", &k, &v) == 2)
    if ((k >> 40) >= kKeySingle && (k >> 40) <= kKeyBatch && cfg_valid(v)) g_tune[k] = v;
  std::fclose(f);
}

void tune_store_locked() {
  const char* path = tune_path();
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  for (auto& kv : g_tune) std::fprintf(f, "%lld %d\n", kv.first, kv.second);
  std::fclose(f);
}

LaunchCfg lookup_cfg(long long key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(key);
  return it == g_tune.end() ? LaunchCfg{} : cfg_unpack(it->second);
}

void store_cfgs(const std::vector<std::pair<long long, LaunchCfg>>& entries) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  for (const auto& e : entries) g_tune[e.first] = cfg_pack(e.second);
  tune_store_locked();
}

// Observation tile edge in z: the caller's tile_config, else the tuned
// tile, else the size rule (small observation grids take the 256-thread
// 8x8x4 tile); tile_config 3 asks for the size rule.
int choose_tile_z(int tile_config, int tuned_tile, double obs_per_inst) {
  int cfg = tile_config == 3 ? 0 : tile_config ? tile_config : tuned_tile;
  if (cfg == 0) cfg = obs_per_inst >= 32768.0 ? 1 : 2;
  return cfg == 1 ? 8 : 4;
}

// Box of cell centres of a grid (canonical FP64 corners).
void grid_box(const jefi_grid* g, double lo[3], double hi[3]) {
  for (int a = 0; a < 3; ++a) {
    lo[a] = g->origin[a] + 0.0 * g->spacing[a];
    hi[a] = g->origin[a] + (double)(g->n[a] - 1) * g->spacing[a];
  }
}

struct Plan {
  PairParams p;
  int multi;  // window longer than any staging shape: the chunked kernel
  int wsel;   // slots staged per cell otherwise (32, 64, 128)
  bool all_dead;
  bool empty;
};

void set_tiles(PairParams& p, const jefi_grid* obs, int tile_z) {
  p.tile_z = tile_z;
  p.ntx = (obs->n[0] + kTileEdge - 1) / kTileEdge;
  p.nty = (obs->n[1] + kTileEdge - 1) / kTileEdge;
  p.ntz = (obs->n[2] + tile_z - 1) / tile_z;
  p.n_tiles = p.ntx * p.nty * p.ntz;
}

// Whether so many pairs fall in the FP32 guard band that nearly every
// (wavefront, brick) step would take the FP64 fix-up anyway; then the pair
// kernels decide every pair by the threshold table instead.  Aligned grids
// whose spacing is a multiple of c*dt put a few percent of all pairs at
// exact integer positions; generic grids put about 2g of them in the band.
// Estimated on 2048 pairs drawn by a fixed LCG: the cost of both schemes
// breaks even when a 512-pair step holds a guard pair with probability 1/2,
// i.e. at about 1.4e-3 of the pairs.
bool guard_pairs_common(const jefi_grid* src, const jefi_grid* obs, const TimeSplit& ts, double g) {
  const long long ns = (long long)src->n[0] * src->n[1] * src->n[2];
  const long long no = (long long)obs->n[0] * obs->n[1] * obs->n[2];
  if (ns <= 0 || no <= 0) return false;
  unsigned long long st = 0x9e3779b97f4a7c15ull;
  auto next = [&st](long long n) {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return (long long)((st >> 17) % (unsigned long long)n);
  };
  const int kSamples = 2048;
  int hits = 0;
  for (int q = 0; q < kSamples; ++q) {
    const long long o = next(no), s = next(ns);
    const long long oi[3] = {o % obs->n[0], (o / obs->n[0]) % obs->n[1], o / ((long long)obs->n[0] * obs->n[1])};
    const long long si[3] = {s % src->n[0], (s / src->n[0]) % src->n[1], s / ((long long)src->n[0] * src->n[1])};
    double d[3];
    for (int a = 0; a < 3; ++a)
      d[a] = (obs->origin[a] + (double)oi[a] * obs->spacing[a]) - (src->origin[a] + (double)si[a] * src->spacing[a]);
    const double u = ts.a_f - std::sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) * ts.inv_cdt;
    const double fr = u - std::floor(u);
    if (std::fabs(fr - 0.5) > 0.5 - g) ++hits;
  }
  return hits * 700 >= kSamples;  // about 1.4e-3
}

constexpr long long kMinRounds = 32;

// Source splits of a single launch for a target workgroup count.
void apply_splits(Plan* plan, int precision, long long splits_target_wg) {
  PairParams& p = plan->p;
  long long splits = (splits_target_wg + p.n_tiles - 1) / p.n_tiles;
  // at least kMinRounds staging rounds per workgroup, so that its set-up
  // (tile geometry, threshold table, first window) stays small
  const int w = plan->multi ? 32 : plan->wsel;
  long long g = (long long)(precision == JEFI_PREC_F64 ? 1 : 2) * (p.tile_z == 8 ? 2 : 1) * 32 / w;
  if (g < 1) g = 1;
  long long max_splits = p.n_bricks / (kMinRounds * g);
  if (max_splits < 1) max_splits = 1;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  // a multiple of 8 splits lets the launch deal them round-robin over the
  // 8 XCDs (balanced shares of the source); the last ones may be empty
  if (splits >= 8) splits &= ~7LL;
  long long bps = (p.n_bricks + splits - 1) / splits;
  if (splits < 8) splits = (p.n_bricks + bps - 1) / bps;
  p.n_splits = (int)splits;
  p.bricks_per_split = (int)bps;
  p.n_wg = (int)((long long)p.n_tiles * splits);
}

// Everything about a launch except the history pointer and outputs.
// `splits_target_wg`: workgroups to aim for (single launches) or 0 to
// leave n_splits = 1 for the caller to set.
jefi_status make_plan(const jefi_grid* src, const jefi_grid* obs, int nt, double dt, long long newest,
                      double t0, double t, const Resolved& r, int tile_z, long long splits_target_wg,
                      Plan* plan) {
  TimeSplit ts;
  jefi_status st = time_split(t, t0, dt, newest, nt, r.c, &ts);
  if (st != JEFI_OK) return st;
  PairParams& p = plan->p;
  std::memset(&p, 0, sizeof p);
  plan->multi = 0;
  plan->wsel = 32;
  // every pair's stencil lies before the oldest slice: zero fields, unless
  // the past is held (then every pair reads slice 0 through slot -2, and
  // a_i = -2 places them all there)
  const bool hold = (r.flags & JEFI_FLAG_PAST_HOLD) != 0;
  plan->all_dead = !hold && ts.a_i <= -2;
  p.src = to_gd(src);
  p.obs = to_gd(obs);
  p.n_bricks = (int)brick_count(src, &p.nbx, &p.nby, &p.nbz);
  set_tiles(p, obs, tile_z);
  plan->empty = p.n_tiles == 0 || p.n_bricks == 0;
  p.a_i = ts.a_i <= -2 ? -2 : (int)ts.a_i;
  p.stencil = ((r.flags & JEFI_FLAG_DERIV_SLOPE) ? kStencilSlope : 0) | (hold ? kStencilHold : 0) |
              ((r.flags & JEFI_FLAG_TIME_CUBIC) ? kStencilCubic : 0) |
              ((r.flags & JEFI_FLAG_PAST_CUT) ? kStencilCut : 0);
  p.a_f = ts.a_f;
  p.inv_cdt = ts.inv_cdt;
  p.inv_dt = 1.0 / dt;
  p.nt = nt;
  for (int a = 0; a < 3; ++a) p.screen[a] = r.screen[a];
  p.margin = 1e-7;
  p.near_slack = 1e-12;
  p.pref = (src->spacing[0] * src->spacing[1] * src->spacing[2]) / (4.0 * M_PI);
  // the FP32 kernels sum in units of c dt: every term carries (1/(c dt))^2
  if (r.precision == JEFI_PREC_F32_COMP) p.pref *= ts.inv_cdt * ts.inv_cdt;
  p.n_splits = 1;
  p.bricks_per_split = p.n_bricks;
  p.n_wg = p.n_tiles;
  if (plan->empty) return JEFI_OK;

  // Largest separation of any pair, and the tile/brick diagonals.
  double slo[3], shi[3], olo[3], ohi[3];
  grid_box(src, slo, shi);
  grid_box(obs, olo, ohi);
  double rmax2 = 0.0, dt2 = 0.0, db2 = 0.0, hsd2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double far = std::fmax(std::fabs(shi[a] - olo[a]), std::fabs(ohi[a] - slo[a]));
    rmax2 += far * far;
    // the 8x8x8 tile is the widest either shape uses
    const double te = (double)std::min(obs->n[a] - 1, kTileEdge - 1) * obs->spacing[a];
    const double be = (double)std::min(src->n[a] - 1, 1) * src->spacing[a];
    dt2 += te * te;
    db2 += be * be;
    hsd2 += src->spacing[a] * src->spacing[a];
  }
  const double rmax = std::sqrt(rmax2), diam_t = std::sqrt(dt2), diam_b = std::sqrt(db2);
  // FP32 index guard: a bound on |u32 - u64| for the FP32 sequence of the
  // pair kernels, which works in units of c dt, with u = 2^-24 the FP32
  // unit roundoff (lengths below in the caller's units):
  //  - coordinates relative to the tile's first point, brick corner, cell
  //    offset, each scaled by 1/(c dt) in FP64 and rounded once (three
  //    roundings deep): |d32 - d| <= u (3R + 2 D_tile + 3 h);
  //  - r2 = x^2 + (y^2 + z^2): 3u relative, i.e. 1.5u on R; v_rsq_f32 taken
  //    as 2 ulp (4u): 5.5u relative on R = r2 * ri, which the FMA below
  //    does not round; 1u more covers the FP64 scaling products;
  //  - u = fma(-r2, ri, a_f) with a_f rounded to FP32: u on a_f, u on the
  //    result.
  // The band used is 1.25x that bound; a fractional part inside it sends
  // the pair through the canonical FP64 decision.
  const double eps = std::ldexp(1.0, -24);
  const double e_coord = eps * (3.0 * rmax + 2.0 * diam_t + 3.0 * std::sqrt(hsd2));
  const double e_R = e_coord + 6.5 * eps * rmax;
  const double umax = ts.inv_cdt * rmax + 2.0;
  const double e_u = ts.inv_cdt * e_R + eps * (umax + 1.0);
  double g = 1.25 * e_u + 1e-7;
  const bool f64 = r.precision == JEFI_PREC_F64;
  p.use_thr = 0;
  if (!(g < 0.5)) g = 0.5;  // every FP32 pair then takes the FP64 path
  if (f64 || g < 0.5) {
    // Pairs whose position u lies near an integer N have floor(u64) in
    // {N-1, N}; u is monotone in r2, so floor(u64) >= N iff r2 <= T(N), with
    // T(N) the largest FP64 r2 whose canonical u reaches N.  A threshold
    // kernel builds the table for every N the launch can meet.  The FP32
    // kernels decide guard-band pairs (or every pair) by it; the FP64
    // kernels decide every pair of a full brick by it, with no correctly
    // rounded square root.
    const double ulow = std::floor(ts.a_f - rmax * ts.inv_cdt) - 2.0;
    if (ulow > -1e9) {
      const long long lo = (long long)ulow;
      const long long n = 1 - lo + 1;
      if (n <= (f64 ? kThrMax64 : kThrMax)) {
        p.use_thr = 1;
        p.thr_lo = (int)lo;
        p.thr_n = (int)n;
      }
    }
  }
  p.guard = (float)g;
  // A brick counts as far (fast path, no per-pair screening test) only when
  // its box is farther than the screening width plus more than the FP32
  // coordinate error on some axis: every FP32 separation there is nonzero.
  p.near_slack = std::max(1e-12, 4.0 * e_coord);
  p.exact_idx = 0;
  const unsigned idx_mode = r.flags & (JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE);
  if (!f64 && p.use_thr && idx_mode != JEFI_FLAG_INDEX_GUARD)
    p.exact_idx = idx_mode == JEFI_FLAG_INDEX_TABLE || guard_pairs_common(src, obs, ts, g) ? 1 : 0;
  // Longest slice window any brick can need (the 8x8x8 tile bounds both shapes).
  const double wb = std::floor((diam_t + diam_b) * ts.inv_cdt * (1.0 + 1e-12) + 2.0 * p.margin + 1e-6) + 3.0;
  // Staging shape: 32 slots per cell, else 64 or 128 with fewer bricks per
  // round (8x8x8 tiles; FP64 stops at 64), else the chunked kernel.
  const int wcap = r.precision == JEFI_PREC_F64 ? 64 : 128;
  plan->wsel = 0;
  for (int w = 32; w <= wcap && plan->wsel == 0; w *= 2)
    if (wb <= (double)w) plan->wsel = w;
  plan->multi = plan->wsel == 0;
  if (plan->multi || plan->wsel > 32) set_tiles(p, obs, 8);  // those kernels run 8x8x8 tiles only

  if (splits_target_wg > 0) apply_splits(plan, r.precision, splits_target_wg);
  return JEFI_OK;
}

// ---- per-(device, stream) scratch for the single-problem path ----------------
struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
  // threshold table last built into the head of the scratch
  bool thr_valid = false;
  double thr_af = 0.0, thr_icdt = 0.0;
  int thr_lo = 0, thr_n = 0;
};
std::mutex g_scratch_mu;
std::map<std::pair<int, void*>, Scratch> g_scratch;
constexpr size_t kThrBytes = kThrMax * sizeof(double);

jefi_status scratch_get(void* stream, size_t bytes, Scratch** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  Scratch& s = g_scratch[{dev, stream}];
  if (s.bytes < bytes) {
    if (s.ptr) {
      e = hipStreamSynchronize((hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      (void)hipFree(s.ptr);
      s.ptr = nullptr;
      s.bytes = 0;
    }
    const size_t want = bytes + bytes / 4;
    e = hipMalloc(&s.ptr, want);
    if (e != hipSuccess) {
      s.ptr = nullptr;
      (void)hipGetLastError();
      return fail(JEFI_ENOMEM, "scratch allocation of %zu bytes failed", want);
    }
    s.bytes = want;
    s.thr_valid = false;
  }
  *out = &s;
  return JEFI_OK;
}

// Point p.thr at the scratch head and (re)build the table when the time
// split changed since the last build on this stream.
jefi_status prepare_thresholds(PairParams& p, Scratch* s, hipStream_t stream) {
  if (!p.use_thr) return JEFI_OK;
  p.thr = (double*)s->ptr;
  if (s->thr_valid && s->thr_af == p.a_f && s->thr_icdt == p.inv_cdt && s->thr_lo == p.thr_lo &&
      s->thr_n == p.thr_n)
    return JEFI_OK;
  hipError_t e = launch_thresholds(p.thr, p.thr_lo, p.thr_n, p.a_f, p.inv_cdt, stream);
  if (e != hipSuccess) return hip_fail(e, "threshold kernel launch");
  s->thr_valid = true;
  s->thr_af = p.a_f;
  s->thr_icdt = p.inv_cdt;
  s->thr_lo = p.thr_lo;
  s->thr_n = p.thr_n;
  return JEFI_OK;
}

jefi_status check_history(const jefi_history* h, int nt) {
  if (!h) return fail(JEFI_EINVAL, "history is NULL");
  if (!h->data) return fail(JEFI_EINVAL, "history data is NULL");
  if (h->dtype != JEFI_F32 && h->dtype != JEFI_F64) return fail(JEFI_EINVAL, "history dtype %d", h->dtype);
  if (h->capacity < 1) return fail(JEFI_EINVAL, "history capacity %d < 1", h->capacity);
  if (!std::isfinite(h->t0)) return fail(JEFI_EINVAL, "history t0 must be finite");
  if (nt < 1 || nt > h->capacity)
    return fail(JEFI_EINVAL, "nt = %d must be in [1, capacity = %d]", nt, h->capacity);
  if ((long long)nt > h->newest + 1)
    return fail(JEFI_EINVAL, "nt = %d exceeds the %lld slices pushed", nt, (long long)h->newest + 1);
  return JEFI_OK;
}

// Validated single problem: everything eval needs.
struct Checked {
  long long ns, no;
  Resolved r;
  Plan plan;
  LaunchCfg cfg;  // the configuration the plan follows (single launches)
};

// Validation and a plan with the given observation tile edge in z.
jefi_status check_problem(const jefi_grid* src, const jefi_history* hist, double dt, int nt,
                          const jefi_grid* obs, double t, const jefi_fields* out, const jefi_options* opt,
                          long long splits_target_wg, int tile_z, Checked* c) {
  if (!grid_ok(src, "source", &c->ns) || !grid_ok(obs, "observation", &c->no)) return JEFI_EINVAL;
  jefi_status st = check_history(hist, nt);
  if (st != JEFI_OK) return st;
  if (out) {
    if (!out->E || !out->B) return fail(JEFI_EINVAL, "output fields are NULL");
    if (out->dtype != JEFI_F32 && out->dtype != JEFI_F64) return fail(JEFI_EINVAL, "output dtype %d", out->dtype);
  }
  if (!std::isfinite(dt) || !(dt > 0.0)) return fail(JEFI_EINVAL, "dt must be finite and > 0");
  if (!std::isfinite(t)) return fail(JEFI_EINVAL, "t must be finite");
  if ((st = resolve_options(opt, src, &c->r)) != JEFI_OK) return st;
  const int want = c->r.precision == JEFI_PREC_F64 ? JEFI_F64 : JEFI_F32;
  if (hist->dtype != want)
    return fail(JEFI_EINVAL, "precision %s needs a %s history",
                c->r.precision == JEFI_PREC_F64 ? "F64" : "F32_COMP", want == JEFI_F64 ? "F64" : "F32");
  c->cfg = LaunchCfg{};
  return make_plan(src, obs, nt, dt, hist->newest, hist->t0, t, c->r, tile_z, splits_target_wg, &c->plan);
}

// Window class of a plan: 0, 1, 2 = 32, 64, 128 staged slots per cell, 3 = chunked.
int window_class(const Plan& pl) { return pl.multi ? 3 : pl.wsel == 32 ? 0 : pl.wsel == 64 ? 1 : 2; }

// The FP32 index mode of a configuration, unless the caller's flags fix one
// (both modes give identical slice indices; they differ in speed only).
void apply_idx(const LaunchCfg& cfg, const Resolved& r, PairParams& p) {
  if (cfg.idx == 0 || r.precision != JEFI_PREC_F32_COMP || !p.use_thr) return;
  if (r.flags & (JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE)) return;
  p.exact_idx = cfg.idx == 2 ? 1 : 0;
}

// Workgroups a single launch aims for: many waves of them over the 256 CUs,
// so that the cheap tiles (mostly culled) and the expensive ones even out
// at the end; split partials grow with it (6 doubles per point and split),
// which stays far below the time it saves on the 64^3 workload.  A
// configuration's granularity halves or doubles it.
long long single_target_wg(int tile_z, int gran) {
  const long long base = tile_z == 8 ? 32768 : 65536;
  return gran == 1 ? base / 2 : gran == 2 ? base * 2 : base;
}

// One problem for a single launch.  The 8x8x8 plan gives its window class
// and so its size class; the configuration (forced, else tuned, else the
// defaults; the caller's tile_config wins) then fixes the tile, the split
// target and the FP32 index mode.  max_splits > 0 caps the split count.
jefi_status plan_single(const jefi_grid* src, const jefi_history* hist, double dt, int nt, const jefi_grid* obs,
                        double t, const jefi_fields* out, const jefi_options* opt, const LaunchCfg* force,
                        long long max_splits, Checked* c) {
  jefi_status st = check_problem(src, hist, dt, nt, obs, t, out, opt, 0, 8, c);
  if (st != JEFI_OK) return st;
  Plan& pl = c->plan;
  const LaunchCfg cfg =
      force ? *force
            : lookup_cfg(size_key(kKeySingle, c->r.precision, window_class(pl), (double)c->no,
                                  (double)c->no * (double)c->ns));
  c->cfg = cfg;
  int tz = choose_tile_z(c->r.tile_config, cfg.tile, (double)c->no);
  if (pl.multi || pl.wsel > 32) tz = 8;  // those kernels run 8x8x8 tiles only
  if (pl.empty) return JEFI_OK;
  if (tz != pl.p.tile_z) set_tiles(pl.p, obs, tz);
  long long target = single_target_wg(tz, cfg.gran);
  if (max_splits > 0) target = std::min(target, max_splits * (long long)pl.p.n_tiles);
  apply_splits(&pl, c->r.precision, target);
  apply_idx(cfg, c->r, pl.p);
  return JEFI_OK;
}

void attach_history(PairParams& p, const jefi_history* hist, int nt) {
  p.capacity = hist->capacity;
  p.slot_base = (int)((hist->newest - nt + 1) % hist->capacity);
  p.ring = hist->data;
  p.slot_elems = (long long)p.n_bricks * kBrickCells * 4;
  const unsigned long long rb =
      (unsigned long long)hist->capacity * (unsigned long long)p.slot_elems * (hist->dtype == JEFI_F64 ? 8ull : 4ull);
  p.ring_bytes_rs = rb < 0x7ffffff0ull ? (unsigned)rb : 0u;
}


// ---- batched evaluation ----------------------------------------------------------
struct BatchWorkspace {
  void* dev = nullptr;
  size_t dev_bytes = 0;
  void* host[2] = {nullptr, nullptr};
  size_t host_bytes = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_used[2] = {false, false};
  int turn = 0;
  // graph per (launch width, cubic stencil, is_f64, index mode, groups),
  // valid for the current `dev` buffer
  std::map<long long, hipGraphExec_t> graphs;
  BatchDevice bd{};
  BatchDevice bdg[2]{};  // the kernel arguments of the two group launches
};
std::mutex g_batch_mu;
std::map<std::pair<int, void*>, BatchWorkspace> g_batch;

constexpr int kBatchMaxInst = 1 << 16;

void drop_graphs(BatchWorkspace& w) {
  for (auto& kv : w.graphs) (void)hipGraphExecDestroy(kv.second);
  w.graphs.clear();
}

int slots_per_cu(int wz) { return wz == 2 ? 2 : 4; }
// Work items per workgroup slot of a batched launch, by granularity.
int items_per_slot(int gran) { return gran == 1 ? 6 : gran == 2 ? 24 : 12; }
// Launch groups of a batch: 8x8x8 tiles (wz 2), then 8x8x4 tiles (wz 1).
constexpr int kGroupWz[2] = {2, 1};

// Compute units whose workgroup slots a persistent launch fills: all of
// them less the caller's reserve, which is capped at half the device.
int launch_cus(int reserve) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus - std::min(reserve, cus / 2);
}

// Graph of one batched evaluation: queue reset -> threshold tables -> one
// persistent pair launch per non-empty group -> split reduction.  Its
// arguments are workspace pointers only (counts live in device memory), so
// it replays any batch that fits the workspace.
jefi_status build_graph(BatchWorkspace& w, int is_f64, const bool has[2], int idx, int stg, int cus,
                        hipGraphExec_t* out) {
  hipGraph_t g;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphCreate");
  for (int q = 0; q < 2; ++q) {
    w.bdg[q] = w.bd;
    w.bdg[q].group = q;
  }
  void* args0[] = {&w.bdg[0]};
  void* args1[] = {&w.bdg[1]};
  hipKernelNodeParams kp{};
  kp.kernelParams = args0;
  kp.extra = nullptr;
  kp.sharedMemBytes = 0;
  hipGraphNode_t n0, n1, prev;
  kp.func = batch_reset_kernel();
  kp.gridDim = dim3(1);
  kp.blockDim = dim3(64);
  e = hipGraphAddKernelNode(&n0, g, nullptr, 0, &kp);
  if (e == hipSuccess) {
    kp.func = batch_threshold_kernel();
    kp.gridDim = dim3(4, 256);
    kp.blockDim = dim3(128);
    e = hipGraphAddKernelNode(&n1, g, &n0, 1, &kp);
  }
  prev = n1;
  for (int q = 0; q < 2 && e == hipSuccess; ++q) {
    if (!has[q]) continue;
    hipGraphNode_t np;
    kp.kernelParams = q == 0 ? args0 : args1;
    kp.func = batch_pair_kernel(is_f64, kGroupWz[q], idx, stg);
    kp.gridDim = dim3(cus * slots_per_cu(kGroupWz[q]));
    kp.blockDim = dim3(batch_pair_threads(kGroupWz[q]));
    e = hipGraphAddKernelNode(&np, g, &prev, 1, &kp);
    prev = np;
  }
  if (e == hipSuccess) {
    hipGraphNode_t n3;
    kp.kernelParams = args0;
    kp.func = batch_epilogue_kernel();
    kp.gridDim = dim3(2048);
    kp.blockDim = dim3(256);
    e = hipGraphAddKernelNode(&n3, g, &prev, 1, &kp);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "batch graph build");
  return JEFI_OK;
}

struct BatchItem {
  int inst, wg;
  double cost;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

extern "C" {

const char* jefi_version(void) { return "libjefi 0.2 (gfx950)"; }

const char* jefi_last_error(void) { return g_err.c_str(); }

void jefi_options_default(jefi_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof *opt);
  opt->c = 1.0;
  opt->screen_set = 0;
  opt->precision = JEFI_PREC_F32_COMP;
  opt->flags = 0;
  opt->tile_config = 0;
  opt->reserve_cus = 0;
}

uint64_t jefi_history_bytes(const jefi_grid* src, int32_t capacity, int32_t dtype) {
  long long cells = 0;
  if (!grid_ok(src, "source", &cells) || capacity < 1 || (dtype != JEFI_F32 && dtype != JEFI_F64)) return 0;
  int nbx, nby, nbz;
  const long long nb = brick_count(src, &nbx, &nby, &nbz);
  return (uint64_t)capacity * (uint64_t)nb * kBrickCells * 4 * dtype_size(dtype);
}

jefi_status jefi_history_init(jefi_history* h, void* data, uint64_t bytes, const jefi_grid* src,
                              int32_t capacity, int32_t dtype, double t0, void* stream) {
  if (g_device_failed.load()) return fail(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  if (!h || !data) return fail(JEFI_EINVAL, "history or data is NULL");
  if (!std::isfinite(t0)) return fail(JEFI_EINVAL, "t0 must be finite");
  long long cells;
  if (!grid_ok(src, "source", &cells)) return JEFI_EINVAL;
  if (capacity < 1 || (dtype != JEFI_F32 && dtype != JEFI_F64))
    return fail(JEFI_EINVAL, "bad capacity %d or dtype %d", capacity, dtype);
  const uint64_t need = jefi_history_bytes(src, capacity, dtype);
  if (bytes < need)
    return fail(JEFI_EINVAL, "history buffer has %llu bytes, needs %llu", (unsigned long long)bytes,
                (unsigned long long)need);
  if (need > 0) {
    hipError_t e = launch_zero(data, need, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "history zero-fill launch");
  }
  h->data = data;
  h->dtype = dtype;
  h->capacity = capacity;
  h->newest = -1;
  h->t0 = t0;
  return JEFI_OK;
}

jefi_status jefi_history_push(jefi_history* h, const jefi_grid* src, const void* slice, void* stream) {
  if (g_device_failed.load()) return fail(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  long long cells = 0;
  if (!grid_ok(src, "source", &cells)) return JEFI_EINVAL;
  if (!h || !h->data) return fail(JEFI_EINVAL, "history is NULL or has no data");
  if (h->dtype != JEFI_F32 && h->dtype != JEFI_F64) return fail(JEFI_EINVAL, "history dtype %d", h->dtype);
  if (h->capacity < 1) return fail(JEFI_EINVAL, "history capacity %d", h->capacity);
  if (cells > 0 && !slice) return fail(JEFI_EINVAL, "slice is NULL");
  const long long step = h->newest + 1;
  const int slot = (int)(step % h->capacity);
  int nbx, nby, nbz;
  const long long nb = brick_count(src, &nbx, &nby, &nbz);
  const size_t slot_bytes = (size_t)nb * kBrickCells * 4 * dtype_size(h->dtype);
  if (cells > 0) {
    hipError_t e = launch_ingest(slice, (char*)h->data + (size_t)slot * slot_bytes, to_gd(src), nbx, nby,
                                 h->dtype == JEFI_F64, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "history ingest launch");
  }
  h->newest = step;
  return JEFI_OK;
}

}  // extern "C"

namespace {

// One field evaluation; force (or NULL) replaces the tuned configuration.
jefi_status eval_single(const jefi_grid* src, const jefi_history* hist, double dt, int32_t nt, const jefi_grid* obs,
                        double t, const jefi_fields* out, const jefi_options* opt, const LaunchCfg* force,
                        void* stream) {
  if (g_device_failed.load()) return fail(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  if (!out) return fail(JEFI_EINVAL, "output fields are NULL");
  Checked c;
  {
    jefi_status st = plan_single(src, hist, dt, nt, obs, t, out, opt, force, 0, &c);
    if (st != JEFI_OK) return st;
  }
  if (c.no == 0) return JEFI_OK;
  hipStream_t s = (hipStream_t)stream;
  const int out_f64 = out->dtype == JEFI_F64;
  if (c.ns == 0 || c.plan.all_dead) {
    hipError_t e = launch_fill_zero_fields(out->E, out->B, c.no, out_f64, s);
    return e == hipSuccess ? JEFI_OK : hip_fail(e, "zero-fill launch");
  }
  PairParams& p = c.plan.p;
  attach_history(p, hist, nt);
  p.E = out->E;
  p.B = out->B;
  p.out_f64 = out_f64;
  p.direct = p.n_splits == 1;
  Scratch* scr = nullptr;
  const size_t part_bytes = p.direct ? 0 : (size_t)p.n_splits * 6 * (size_t)c.no * sizeof(double);
  jefi_status st = scratch_get(stream, kThrBytes + part_bytes, &scr);
  if (st != JEFI_OK) return st;
  if (!p.direct) p.partial = (double*)((char*)scr->ptr + kThrBytes);
  if (!c.plan.multi) {
    if ((st = prepare_thresholds(p, scr, s)) != JEFI_OK) return st;
  } else {
    p.use_thr = 0;
  }
  hipError_t e = launch_pairs(p, c.r.precision == JEFI_PREC_F64, 0, c.plan.multi, c.plan.wsel, s);
  if (e != hipSuccess) return hip_fail(e, "pair kernel launch");
  if (!p.direct) {
    EpilogueParams ep{p.partial, p.n_splits, c.no, p.pref, out->E, out->B, out_f64};
    e = launch_epilogue(ep, s);
    if (e != hipSuccess) return hip_fail(e, "epilogue launch");
  }
  return JEFI_OK;
}

}  // namespace

extern "C" {

jefi_status jefi_eval_fields(const jefi_grid* src, const jefi_history* hist, double dt, int32_t nt,
                             const jefi_grid* obs, double t, const jefi_fields* out,
                             const jefi_options* opt, void* stream) {
  return eval_single(src, hist, dt, nt, obs, t, out, opt, nullptr, stream);
}

jefi_status jefi_eval_fields_noalloc(const jefi_grid* src, const jefi_history* hist, double dt, int32_t nt,
                                     const jefi_grid* obs, double t, const jefi_fields* out,
                                     const jefi_options* opt, void* stream) {
  if (g_device_failed.load()) return fail(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  if (!out) return fail(JEFI_EINVAL, "output fields are NULL");
  Checked c;
  {
    // the split count of jefi_eval_fields, capped so that the FP64 split
    // partials fit the fixed scratch behind the threshold table (one split
    // needs none: the pair kernel then writes E and B itself)
    long long obs_pts = 0;
    if (!grid_ok(obs, "observation", &obs_pts)) return JEFI_EINVAL;
    long long max_splits = 0;
    if (obs_pts > 0) {
      const unsigned long long room = kNoAllocScratchBytes - kThrBytes;
      max_splits = std::max(1LL, (long long)(room / (6ull * sizeof(double) * (unsigned long long)obs_pts)));
    }
    jefi_status st = plan_single(src, hist, dt, nt, obs, t, out, opt, nullptr, max_splits, &c);
    if (st != JEFI_OK) return st;
  }
  if (c.no == 0) return JEFI_OK;
  hipStream_t s = (hipStream_t)stream;
  const int out_f64 = out->dtype == JEFI_F64;
  if (c.ns == 0 || c.plan.all_dead) {
    hipError_t e = launch_fill_zero_fields(out->E, out->B, c.no, out_f64, s);
    return e == hipSuccess ? JEFI_OK : hip_fail(e, "zero-fill launch");
  }
  PairParams& p = c.plan.p;
  attach_history(p, hist, nt);
  p.E = out->E;
  p.B = out->B;
  p.out_f64 = out_f64;
  p.direct = p.n_splits == 1;
  const unsigned long long part_bytes = p.direct ? 0ull : (unsigned long long)p.n_splits * 6ull * (unsigned long long)c.no * sizeof(double);
  if (kThrBytes + part_bytes > kNoAllocScratchBytes)
    return fail(JEFI_ETOOLARGE, "%d splits x %lld points need %llu scratch bytes; the fixed scratch has %llu",
                p.n_splits, c.no, (unsigned long long)(kThrBytes + part_bytes), kNoAllocScratchBytes);
  void* base = nullptr;
  hipError_t e = noalloc_scratch(&base);
  if (e != hipSuccess) return hip_fail(e, "scratch symbol address");
  if (!p.direct) p.partial = (double*)((char*)base + kThrBytes);
  if (!c.plan.multi && p.use_thr) {
    // rebuilt on every call: another call may have left its own table here
    p.thr = (double*)base;
    e = launch_thresholds(p.thr, p.thr_lo, p.thr_n, p.a_f, p.inv_cdt, s);
    if (e != hipSuccess) return hip_fail(e, "threshold kernel launch");
  } else {
    p.use_thr = 0;
  }
  e = launch_pairs(p, c.r.precision == JEFI_PREC_F64, 0, c.plan.multi, c.plan.wsel, s);
  if (e != hipSuccess) return hip_fail(e, "pair kernel launch");
  if (!p.direct) {
    EpilogueParams ep{p.partial, p.n_splits, c.no, p.pref, out->E, out->B, out_f64};
    e = launch_epilogue(ep, s);
    if (e != hipSuccess) return hip_fail(e, "epilogue launch");
  }
  return JEFI_OK;
}

jefi_status jefi_slice_index_dump(const jefi_grid* src, int32_t nt, double dt, int64_t newest, double t0,
                                  const jefi_grid* obs, double t, const jefi_options* opt, int32_t* out,
                                  void* stream) {
  if (g_device_failed.load()) return fail(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  long long ns = 0, no = 0;
  if (!grid_ok(src, "source", &ns) || !grid_ok(obs, "observation", &no)) return JEFI_EINVAL;
  if (!out && ns * no > 0) return fail(JEFI_EINVAL, "out is NULL");
  if (ns * no > 0x7fffffffLL) return fail(JEFI_EINVAL, "dump limited to 2^31-1 pairs");
  if (nt < 1 || (long long)nt > newest + 1) return fail(JEFI_EINVAL, "nt = %d with newest = %lld", nt, (long long)newest);
  if (!std::isfinite(dt) || !(dt > 0.0) || !std::isfinite(t) || !std::isfinite(t0))
    return fail(JEFI_EINVAL, "dt, t and t0 must be finite with dt > 0");
  Resolved r;
  jefi_status st = resolve_options(opt, src, &r);
  if (st != JEFI_OK) return st;
  Plan plan;
  if ((st = make_plan(src, obs, nt, dt, newest, t0, t, r, 8, 0, &plan)) != JEFI_OK) return st;
  DumpParams d;
  std::memset(&d, 0, sizeof d);
  d.src = to_gd(src);
  d.obs = to_gd(obs);
  d.a_i = plan.p.a_i;
  d.a_f = plan.p.a_f;
  d.inv_cdt = plan.p.inv_cdt;
  for (int a = 0; a < 3; ++a) d.screen[a] = r.screen[a];
  d.guard = plan.p.guard;
  d.use_f64 = r.precision == JEFI_PREC_F64;
  d.out = out;
  hipError_t e = launch_dump(d, (hipStream_t)stream);
  return e == hipSuccess ? JEFI_OK : hip_fail(e, "dump launch");
}

jefi_status jefi_slice_fingerprint(const jefi_grid* src, const jefi_history* hist, double dt, int32_t nt,
                                   const jefi_grid* obs, double t, const jefi_options* opt, int64_t* fp,
                                   void* stream) {
  if (g_device_failed.load()) return fail(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  Checked c;
  jefi_status st = plan_single(src, hist, dt, nt, obs, t, nullptr, opt, nullptr, 0, &c);
  if (st != JEFI_OK) return st;
  if (!fp && c.no > 0) return fail(JEFI_EINVAL, "fp is NULL");
  if (c.no == 0) return JEFI_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_zero(fp, (unsigned long long)c.no * 4 * sizeof(int64_t), s);
  if (e != hipSuccess) return hip_fail(e, "fingerprint zero-fill");
  // every pair wholly in the past still runs: screened pairs are counted
  if (c.ns == 0) return JEFI_OK;
  PairParams& p = c.plan.p;
  attach_history(p, hist, nt);
  p.fp = (unsigned long long*)fp;
  Scratch* scr = nullptr;
  if ((st = scratch_get(stream, kThrBytes, &scr)) != JEFI_OK) return st;
  if (!c.plan.multi) {
    if ((st = prepare_thresholds(p, scr, s)) != JEFI_OK) return st;
  } else {
    p.use_thr = 0;
  }
  e = launch_pairs(p, c.r.precision == JEFI_PREC_F64, 1, c.plan.multi, c.plan.wsel, s);
  return e == hipSuccess ? JEFI_OK : hip_fail(e, "fingerprint kernel launch");
}

}  // extern "C"

namespace {

// A batched evaluation.  force_tiles (per problem: 1 = 8x8x8, 2 = 8x8x4)
// and force_batch (index mode and items per slot) replace the tuned table,
// for the autotuner's trials; grid_cus > 0 sizes the persistent launches
// for that many compute units.
jefi_status eval_batch_impl(const jefi_problem* probs, int32_t n, const jefi_options* opt, void* stream,
                            const std::vector<int>* force_tiles, const LaunchCfg* force_batch, int grid_cus = 0) {
  if (g_device_failed.load()) return fail(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  if (n < 0 || n > kBatchMaxInst) return fail(JEFI_EINVAL, "batch of %d problems (limit %d)", n, kBatchMaxInst);
  if (n == 0) return JEFI_OK;
  if (!probs) return fail(JEFI_EINVAL, "problems are NULL");
  hipStream_t s = (hipStream_t)stream;
  // Validate everything before any device work.
  std::vector<Checked> cs((size_t)n);
  double obs_sum = 0.0, pair_sum = 0.0;
  for (int i = 0; i < n; ++i) {
    const jefi_problem& q = probs[i];
    jefi_status st = check_problem(&q.src, &q.hist, q.dt, q.nt, &q.obs, q.t, &q.out, opt, 0, 8, &cs[i]);
    if (st != JEFI_OK) {
      std::string m = g_err;
      return fail(st, "problem %d: %s", i, m.c_str());
    }
    obs_sum += (double)cs[i].no;
    pair_sum += (double)cs[i].no * (double)cs[i].ns;
  }
  const Resolved& r0 = cs[0].r;
  const int is_f64 = r0.precision == JEFI_PREC_F64;
  for (int i = 1; i < n; ++i)
    if (cs[i].r.precision != r0.precision) return fail(JEFI_EINVAL, "mixed precisions in one batch");
  // Tile per problem: forced, else the caller's tile_config, else the tuned
  // entry of its size class within batches, else one size rule for the
  // whole batch (on the mean observation grid).
  const int rule_tile = choose_tile_z(0, 0, obs_sum / n) == 8 ? 1 : 2;
  const LaunchCfg bcfg = force_batch ? *force_batch : lookup_cfg(size_key(kKeyBatch, r0.precision, 0, n, pair_sum));

  // Instances the persistent kernel does not take: empty, all-dead, or
  // windows longer than one staging chunk.  They run on their own launches.
  std::vector<int> batch_idx, group_of;
  for (int i = 0; i < n; ++i) {
    const jefi_problem& q = probs[i];
    Checked& c = cs[i];
    if (c.no == 0) continue;
    if (c.ns == 0 || c.plan.all_dead) {
      hipError_t e = launch_fill_zero_fields(q.out.E, q.out.B, c.no, q.out.dtype == JEFI_F64, s);
      if (e != hipSuccess) return hip_fail(e, "zero-fill launch");
      continue;
    }
    if (c.plan.multi || c.plan.wsel > 32) {
      // windows longer than the persistent kernel's 32 slots: their own launch
      jefi_status st = jefi_eval_fields(&q.src, &q.hist, q.dt, q.nt, &q.obs, q.t, &q.out, opt, stream);
      if (st != JEFI_OK) return st;
      continue;
    }
    int tile = force_tiles ? (*force_tiles)[i] : c.r.tile_config;
    if (tile == 3) tile = choose_tile_z(3, 0, (double)c.no) == 8 ? 1 : 2;  // each problem by its own size
    if (tile == 0)
      tile = lookup_cfg(size_key(kKeyMember, c.r.precision, window_class(c.plan), (double)c.no,
                                 (double)c.no * (double)c.ns)).tile;
    if (tile == 0) tile = rule_tile;
    const int tile_z = tile == 1 ? 8 : 4;
    jefi_status st = make_plan(&q.src, &q.obs, q.nt, q.dt, q.hist.newest, q.hist.t0, q.t, c.r, tile_z, 0, &c.plan);
    if (st != JEFI_OK) return st;
    batch_idx.push_back(i);
    group_of.push_back(tile_z == 8 ? 0 : 1);
  }
  const int nb = (int)batch_idx.size();
  if (nb == 0) return JEFI_OK;

  // Splits: equal-cost items, about items_per_slot(gran) per workgroup slot
  // of each group's launch, so that the last items to finish leave little
  // of the device idle.
  int dev = 0;
  (void)hipGetDevice(&dev);
  // items are sized for the whole device, so that a reserve changes only how
  // many workgroups run at once, not the decomposition (nor the results)
  const int cus = launch_cus(0);
  // the options are shared; a caller's explicit grid wins over its reserve
  const int run_cus = grid_cus > 0 ? std::min(grid_cus, cus) : launch_cus(cs[0].r.reserve_cus);
  const int ips = items_per_slot(bcfg.gran);
  double group_cost[2] = {0.0, 0.0};
  for (int k = 0; k < nb; ++k) {
    const PairParams& p = cs[batch_idx[k]].plan.p;
    const int tile_pts = 64 * p.tile_z;
    group_cost[group_of[k]] += (double)p.n_tiles * tile_pts * (double)p.n_bricks * kBrickCells;
  }
  double group_target[2];
  for (int q = 0; q < 2; ++q)
    group_target[q] = std::max(group_cost[q] / ((double)ips * cus * slots_per_cu(kGroupWz[q])), 1.0);
  std::vector<BatchItem> gitems[2];
  std::vector<PairParams> params((size_t)nb);
  std::vector<EpilogueParams> epi((size_t)nb);
  std::vector<long long> prefix((size_t)nb + 1, 0);
  size_t part_doubles = 0;
  for (int k = 0; k < nb; ++k) {
    const int i = batch_idx[k];
    const int q = group_of[k];
    PairParams p = cs[i].plan.p;
    const int tile_pts = 64 * p.tile_z;
    const int G = (is_f64 ? 1 : 2) * kGroupWz[q];
    const double per_tile = (double)tile_pts * (double)p.n_bricks * kBrickCells;
    long long splits = (long long)std::ceil(per_tile / group_target[q]);
    long long max_splits = std::max(1, p.n_bricks / (4 * G));
    splits = std::max(1LL, std::min(splits, max_splits));
    long long bps = (p.n_bricks + splits - 1) / splits;
    splits = (p.n_bricks + bps - 1) / bps;
    p.n_splits = (int)splits;
    p.bricks_per_split = (int)bps;
    p.n_wg = p.n_tiles * p.n_splits;
    attach_history(p, &probs[i].hist, probs[i].nt);
    p.E = probs[i].out.E;
    p.B = probs[i].out.B;
    p.out_f64 = probs[i].out.dtype == JEFI_F64;
    p.direct = p.n_splits == 1;
    if (!p.direct) part_doubles += (size_t)p.n_splits * 6 * (size_t)cs[i].no;
    params[k] = p;
    const double item_cost = (double)tile_pts * (double)bps * kBrickCells;
    for (int wg = 0; wg < p.n_wg; ++wg) gitems[q].push_back({k, wg, item_cost});
  }
  for (int q = 0; q < 2; ++q)
    std::stable_sort(gitems[q].begin(), gitems[q].end(),
                     [](const BatchItem& a, const BatchItem& b) { return a.cost > b.cost; });
  // One FP32 index mode for the whole launch (both give the same indices):
  // the tuned one, else the threshold table when every instance has one
  // and instances that prefer it carry at least half of the work.
  int idx = 0;
  if (!is_f64) {
    bool all_thr = true;
    double want = 0.0, total = 0.0;
    for (int k = 0; k < nb; ++k) {
      const PairParams& p = params[k];
      const double cost = (double)p.n_tiles * 64 * p.tile_z * (double)p.n_bricks;
      all_thr = all_thr && p.use_thr;
      total += cost;
      if (p.exact_idx) want += cost;
    }
    const bool forced = (r0.flags & (JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE)) != 0;
    if (!forced && bcfg.idx != 0)
      idx = bcfg.idx == 2 && all_thr ? 1 : 0;
    else
      idx = all_thr && 2.0 * want >= total ? 1 : 0;
  }
  const int n_items0 = (int)gitems[0].size();
  const int n_items = n_items0 + (int)gitems[1].size();
  const bool has[2] = {!gitems[0].empty(), !gitems[1].empty()};
  // Workspace layout (device): params | items | counts | counter | epi | prefix | thresholds | partials
  const size_t o_params = 0;
  const size_t o_items = align_up(o_params + sizeof(PairParams) * nb, 256);
  const size_t o_counts = align_up(o_items + sizeof(int2) * n_items, 256);
  const size_t o_counter = o_counts + 64;
  const size_t o_epi = align_up(o_counter + 64, 256);
  const size_t o_prefix = align_up(o_epi + sizeof(EpilogueParams) * nb, 256);
  const size_t o_thr = align_up(o_prefix + sizeof(long long) * (nb + 1), 256);
  const size_t o_part = align_up(o_thr + kThrBytes * nb, 256);
  const size_t dev_bytes = o_part + part_doubles * sizeof(double);
  const size_t host_bytes = o_thr;  // the uploaded head

  std::lock_guard<std::mutex> lk(g_batch_mu);
  BatchWorkspace& w = g_batch[{dev, stream}];
  hipError_t e;
  if (w.dev_bytes < dev_bytes) {
    if (w.dev) {
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      (void)hipFree(w.dev);
      w.dev = nullptr;
    }
    drop_graphs(w);
    const size_t want = dev_bytes + dev_bytes / 4;
    if ((e = hipMalloc(&w.dev, want)) != hipSuccess) {
      (void)hipGetLastError();
      w.dev = nullptr;
      w.dev_bytes = 0;
      return fail(JEFI_ENOMEM, "batch workspace of %zu bytes", want);
    }
    w.dev_bytes = want;
  }
  if (w.host_bytes < host_bytes) {
    for (int b = 0; b < 2; ++b) {
      if (w.ev_used[b]) (void)hipEventSynchronize(w.ev[b]);
      if (w.host[b]) (void)hipHostFree(w.host[b]);
      w.host[b] = nullptr;
    }
    const size_t want = host_bytes + host_bytes / 4;
    for (int b = 0; b < 2; ++b) {
      if ((e = hipHostMalloc(&w.host[b], want, hipHostMallocDefault)) != hipSuccess) {
        (void)hipGetLastError();
        w.host_bytes = 0;
        return fail(JEFI_ENOMEM, "pinned staging of %zu bytes", want);
      }
    }
    w.host_bytes = want;
  }
  for (int b = 0; b < 2; ++b)
    if (!w.ev[b] && (e = hipEventCreateWithFlags(&w.ev[b], hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreate");
  char* dbase = (char*)w.dev;
  for (int k = 0; k < nb; ++k) {
    PairParams& p = params[k];
    if (p.use_thr) p.thr = (double*)(dbase + o_thr + kThrBytes * k);
  }
  size_t part_at = 0;
  for (int k = 0; k < nb; ++k) {
    PairParams& p = params[k];
    const long long no = (long long)p.obs.n[0] * p.obs.n[1] * p.obs.n[2];
    if (!p.direct) {
      p.partial = (double*)(dbase + o_part) + part_at;
      epi[k] = EpilogueParams{p.partial, p.n_splits, no, p.pref, p.E, p.B, p.out_f64};
      part_at += (size_t)p.n_splits * 6 * (size_t)no;
      prefix[k + 1] = prefix[k] + 6 * no;
    } else {
      epi[k] = EpilogueParams{nullptr, 0, no > 0 ? no : 1, p.pref, p.E, p.B, p.out_f64};
      prefix[k + 1] = prefix[k];
    }
  }
  // Stage the head in pinned memory (wait until its previous upload finished).
  const int b = w.turn;
  w.turn ^= 1;
  if (w.ev_used[b] && (e = hipEventSynchronize(w.ev[b])) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  char* hb = (char*)w.host[b];
  std::memcpy(hb + o_params, params.data(), sizeof(PairParams) * nb);
  int2* hi = (int2*)(hb + o_items);
  for (int q = 0; q < 2; ++q)
    for (size_t a = 0; a < gitems[q].size(); ++a)
      hi[(q ? n_items0 : 0) + a] = make_int2(gitems[q][a].inst, gitems[q][a].wg);
  int* hc = (int*)(hb + o_counts);
  hc[0] = nb;
  hc[1] = n_items0;
  hc[2] = 0;
  hc[3] = n_items - n_items0;
  hc[4] = n_items0;
  std::memcpy(hb + o_epi, epi.data(), sizeof(EpilogueParams) * nb);
  std::memcpy(hb + o_prefix, prefix.data(), sizeof(long long) * (nb + 1));
  if ((e = hipMemcpyAsync(w.dev, hb, host_bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "batch descriptor upload");
  if ((e = hipEventRecord(w.ev[b], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  w.ev_used[b] = true;
  // Graph of reset -> thresholds -> persistent pairs -> epilogue, pointer
  // arguments only: rebuilt only when the workspace moves.
  BatchDevice bd;
  std::memset(&bd, 0, sizeof bd);  // compared bytewise below, padding included
  bd.params = (const PairParams*)(dbase + o_params);
  bd.items = (const int2*)(dbase + o_items);
  bd.counts = (const int*)(dbase + o_counts);
  bd.counter = (int*)(dbase + o_counter);
  bd.epi = (const EpilogueParams*)(dbase + o_epi);
  bd.epi_prefix = (const long long*)(dbase + o_prefix);
  if (std::memcmp(&bd, &w.bd, sizeof bd) != 0) {
    drop_graphs(w);
    w.bd = bd;
  }
  // one stencil for the whole batch (the options are shared)
  // staging mode of the persistent kernels: bit 0 cubic, bit 1 history start (one per batch)
  const int stg = nb > 0 ? ((params[0].stencil & kStencilCubic) ? 1 : 0) | ((params[0].stencil & kStencilCut) ? 2 : 0) : 0;
  const long long gkey = (long long)run_cus * 64 + stg * 16 + is_f64 * 8 + idx * 4 + (has[0] ? 2 : 0) + (has[1] ? 1 : 0);
  auto it = w.graphs.find(gkey);
  if (it == w.graphs.end()) {
    hipGraphExec_t ge;
    jefi_status st = build_graph(w, is_f64, has, idx, stg, run_cus, &ge);
    if (st != JEFI_OK) return st;
    it = w.graphs.emplace(gkey, ge).first;
  }
  if ((e = hipGraphLaunch(it->second, s)) != hipSuccess) return hip_fail(e, "batch graph launch");
  return JEFI_OK;
}

}  // namespace

namespace jefi {

jefi_status report_error(jefi_status st, const char* msg) { return fail(st, "%s", msg); }

jefi_status report_hip(hipError_t e, const char* what) { return hip_fail(e, what); }

bool device_failed() { return g_device_failed.load() != 0; }

int device_cus() { return launch_cus(0); }

bool create_stream_on_cus(hipStream_t* s, int first_cu, int n_cus) {
  const int cus = launch_cus(0);
  if (first_cu < 0 || n_cus < 1 || first_cu + n_cus > cus) return false;
  std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0u);
  for (int c = first_cu; c < first_cu + n_cus; ++c) mask[(size_t)c / 32] |= 1u << (c % 32);
  const hipError_t e = hipExtStreamCreateWithCUMask(s, (uint32_t)mask.size(), mask.data());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

jefi_status eval_batch_on_cus(const jefi_problem* probs, int32_t n, const jefi_options* opt, void* stream,
                              int grid_cus) {
  return eval_batch_impl(probs, n, opt, stream, nullptr, nullptr, grid_cus);
}

}  // namespace jefi

extern "C" {

jefi_status jefi_eval_batch(const jefi_problem* probs, int32_t n, const jefi_options* opt, void* stream) {
  return eval_batch_impl(probs, n, opt, stream, nullptr, nullptr);
}

}  // extern "C"

namespace {

// Mean milliseconds per run of `run` over `reps` runs after one warm-up
// (which also builds graphs), timed with events on the stream.
template <class F>
jefi_status time_runs(F run, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, double* ms) {
  jefi_status st = run();
  if (st != JEFI_OK) return st;
  hipError_t e = hipEventRecord(e0, s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  for (int q = 0; q < reps; ++q)
    if ((st = run()) != JEFI_OK) return st;
  if ((e = hipEventRecord(e1, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  float f = 0.f;
  (void)hipEventElapsedTime(&f, e0, e1);
  *ms = (double)f / reps;
  return JEFI_OK;
}

// A change of configuration is kept only when it is faster by this factor
// (run-to-run noise of a few tenths of a percent must not flip choices).
constexpr double kTuneGain = 0.99;

jefi_status tune_single(const jefi_problem& q, const jefi_options& o, int reps, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1, int* best_config, double* best_ms) {
  Checked c;
  jefi_status st = plan_single(&q.src, &q.hist, q.dt, q.nt, &q.obs, q.t, &q.out, &o, nullptr, 0, &c);
  if (st != JEFI_OK) return st;
  // 8x8x4 tiles only with 32-slot windows; both index modes only where the
  // FP32 path has a threshold table and the caller's flags leave it open
  Checked c8;
  if ((st = check_problem(&q.src, &q.hist, q.dt, q.nt, &q.obs, q.t, &q.out, &o, 0, 8, &c8)) != JEFI_OK) return st;
  const int wcls = window_class(c8.plan);
  const int n_tiles = wcls == 0 ? 2 : 1;
  const bool idx_free = c.r.precision == JEFI_PREC_F32_COMP && c8.plan.p.use_thr &&
                        !(c.r.flags & (JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE));
  LaunchCfg best{};
  double best_t = -1.0;
  for (int tile = 1; tile <= n_tiles; ++tile)
    for (int idx = idx_free ? 1 : 0; idx <= (idx_free ? 2 : 0); ++idx)
      for (int gran = 0; gran <= 2; ++gran) {
        const LaunchCfg cfg{tile, idx, gran};
        double ms = 0.0;
        st = time_runs([&]() { return eval_single(&q.src, &q.hist, q.dt, q.nt, &q.obs, q.t, &q.out, &o, &cfg, s); },
                       reps, s, e0, e1, &ms);
        if (st != JEFI_OK) return st;
        if (best_t < 0.0 || ms < best_t) {
          best = cfg;
          best_t = ms;
        }
      }
  store_cfgs({{size_key(kKeySingle, c.r.precision, wcls, (double)c.no, (double)c.no * (double)c.ns), best}});
  *best_config = cfg_pack(best);
  *best_ms = best_t;
  return JEFI_OK;
}

// A batch: greedy coordinate search from the untuned launch.  Each size
// class of instances (precision, window class, observation points, pairs)
// tries the other tile; then the batch tries both index modes and the
// other work granularities.  Kept changes go to the table: member entries
// per size class, one entry for the batch's class.
jefi_status tune_batch(const jefi_problem* probs, int n, const jefi_options& o, int reps, hipStream_t s,
                       hipEvent_t e0, hipEvent_t e1, int* best_config, double* best_ms) {
  std::vector<Checked> cs((size_t)n);
  double obs_sum = 0.0, pair_sum = 0.0;
  for (int i = 0; i < n; ++i) {
    const jefi_problem& q = probs[i];
    jefi_status st = check_problem(&q.src, &q.hist, q.dt, q.nt, &q.obs, q.t, &q.out, &o, 0, 8, &cs[i]);
    if (st != JEFI_OK) return st;
    obs_sum += (double)cs[i].no;
    pair_sum += (double)cs[i].no * (double)cs[i].ns;
  }
  const Resolved& r0 = cs[0].r;
  const int rule_tile = choose_tile_z(0, 0, obs_sum / n) == 8 ? 1 : 2;
  std::vector<int> tiles((size_t)n, rule_tile);
  // size classes of the instances the persistent launch takes, heaviest first
  std::map<long long, double> weight;
  std::vector<long long> key((size_t)n, -1);
  for (int i = 0; i < n; ++i) {
    const Checked& c = cs[i];
    if (c.no == 0 || c.ns == 0 || c.plan.all_dead || c.plan.multi || c.plan.wsel > 32) continue;
    key[i] = size_key(kKeyMember, c.r.precision, window_class(c.plan), (double)c.no, (double)c.no * (double)c.ns);
    weight[key[i]] += (double)c.no * (double)c.ns;
  }
  std::vector<std::pair<double, long long>> order;
  for (const auto& kv : weight) order.push_back({kv.second, kv.first});
  std::sort(order.rbegin(), order.rend());
  LaunchCfg bc{};
  auto trial = [&](const std::vector<int>& t, const LaunchCfg& b, double* ms) {
    return time_runs([&]() { return eval_batch_impl(probs, n, &o, s, &t, &b); }, reps, s, e0, e1, ms);
  };
  double best_t = 0.0;
  jefi_status st = trial(tiles, bc, &best_t);
  if (st != JEFI_OK) return st;
  for (const auto& cls : order) {
    std::vector<int> t2 = tiles;
    for (int i = 0; i < n; ++i)
      if (key[i] == cls.second) t2[i] = 3 - t2[i];
    double ms = 0.0;
    if ((st = trial(t2, bc, &ms)) != JEFI_OK) return st;
    if (ms < kTuneGain * best_t) {
      tiles = t2;
      best_t = ms;
    }
  }
  const bool idx_free = r0.precision == JEFI_PREC_F32_COMP && !(r0.flags & (JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE));
  if (idx_free) {
    LaunchCfg keep = bc;
    for (int idx = 1; idx <= 2; ++idx) {
      LaunchCfg b2 = bc;
      b2.idx = idx;
      double ms = 0.0;
      if ((st = trial(tiles, b2, &ms)) != JEFI_OK) return st;
      if (ms < kTuneGain * best_t) {
        keep = b2;
        best_t = ms;
      }
    }
    bc = keep;
  }
  {
    LaunchCfg keep = bc;
    for (int gran = 1; gran <= 2; ++gran) {
      LaunchCfg b2 = bc;
      b2.gran = gran;
      double ms = 0.0;
      if ((st = trial(tiles, b2, &ms)) != JEFI_OK) return st;
      if (ms < kTuneGain * best_t) {
        keep = b2;
        best_t = ms;
      }
    }
    bc = keep;
  }
  std::vector<std::pair<long long, LaunchCfg>> entries;
  for (const auto& cls : order) {
    for (int i = 0; i < n; ++i)
      if (key[i] == cls.second) {
        entries.push_back({cls.second, LaunchCfg{tiles[i], 0, 0}});
        break;
      }
  }
  entries.push_back({size_key(kKeyBatch, r0.precision, 0, n, pair_sum), bc});
  store_cfgs(entries);
  *best_config = cfg_pack(bc);
  *best_ms = best_t;
  return JEFI_OK;
}

}  // namespace

extern "C" {

jefi_status jefi_autotune(const jefi_problem* probs, int32_t n, const jefi_options* opt, int32_t reps,
                          void* stream, int32_t* best_config, double* best_ms) {
  if (g_device_failed.load()) return fail(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  if (!probs || n < 1) return fail(JEFI_EINVAL, "autotune needs at least one problem");
  if (n > kBatchMaxInst) return fail(JEFI_EINVAL, "batch of %d problems (limit %d)", n, kBatchMaxInst);
  if (reps < 1) reps = 3;
  jefi_options o;
  if (opt)
    o = *opt;
  else
    jefi_options_default(&o);
  o.tile_config = 0;  // the trials set the tile
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  int best = 0;
  double ms = 0.0;
  const jefi_status st = n == 1 ? tune_single(probs[0], o, reps, s, e0, e1, &best, &ms)
                                : tune_batch(probs, n, o, reps, s, e0, e1, &best, &ms);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != JEFI_OK) return st;
  if (best_config) *best_config = best;
  if (best_ms) *best_ms = ms;
  return JEFI_OK;
}

}  // extern "C"
