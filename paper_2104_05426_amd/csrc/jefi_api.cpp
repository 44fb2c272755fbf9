// libjefi C ABI: argument validation, the FP64 time prelude, launch
// configuration and per-stream scratch.  Device work is in jefi_kernels.hip.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

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

// The evaluation time on the logical slice axis (the same FP64 sequence the
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

// Per-(device, stream) scratch for FP64 split partials.
struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_scratch_mu;
std::map<std::pair<int, void*>, Scratch> g_scratch;

jefi_status scratch_get(void* stream, size_t bytes, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  Scratch& s = g_scratch[{dev, stream}];
  if (s.bytes < bytes) {
    if (s.ptr) {
      e = hipStreamSynchronize((hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      hipFree(s.ptr);
      s.ptr = nullptr;
      s.bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    e = hipMalloc(&s.ptr, want);
    if (e != hipSuccess) {
      s.ptr = nullptr;
      (void)hipGetLastError();
      return fail(JEFI_ENOMEM, "scratch allocation of %zu bytes failed", want);
    }
    s.bytes = want;
  }
  *out = s.ptr;
  return JEFI_OK;
}

struct Resolved {
  double c;
  double screen[3];
  int precision;
};

jefi_status resolve_options(const jefi_options* opt, const jefi_grid* src, Resolved* r) {
  jefi_options d;
  jefi_options_default(&d);
  if (!opt) opt = &d;
  if (!std::isfinite(opt->c) || !(opt->c > 0.0)) return fail(JEFI_EINVAL, "c must be finite and > 0");
  if (opt->precision != JEFI_PREC_F64 && opt->precision != JEFI_PREC_F32_COMP)
    return fail(JEFI_EINVAL, "unknown precision %d", opt->precision);
  r->c = opt->c;
  r->precision = opt->precision;
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

// Box of cell centres of a grid (canonical FP64 corners).
void grid_box(const jefi_grid* g, double lo[3], double hi[3]) {
  for (int a = 0; a < 3; ++a) {
    lo[a] = g->origin[a] + 0.0 * g->spacing[a];
    hi[a] = g->origin[a] + (double)(g->n[a] - 1) * g->spacing[a];
  }
}

// Launch description shared by the field evaluation and the fingerprint.
struct Plan {
  PairParams p;
  int multi;
  bool all_dead;
};

jefi_status make_plan(const jefi_grid* src, const jefi_grid* obs, int nt, double dt, long long newest,
                      double t0, double t, const Resolved& r, Plan* plan) {
  TimeSplit ts;
  jefi_status st = time_split(t, t0, dt, newest, nt, r.c, &ts);
  if (st != JEFI_OK) return st;
  PairParams& p = plan->p;
  std::memset(&p, 0, sizeof p);
  plan->all_dead = ts.a_i <= -2;  // every pair's stencil lies before the oldest slice
  p.src = to_gd(src);
  p.obs = to_gd(obs);
  p.n_bricks = (int)brick_count(src, &p.nbx, &p.nby, &p.nbz);
  p.ntx = (obs->n[0] + kTileEdge - 1) / kTileEdge;
  p.nty = (obs->n[1] + kTileEdge - 1) / kTileEdge;
  p.ntz = (obs->n[2] + kTileEdge - 1) / kTileEdge;
  p.n_tiles = p.ntx * p.nty * p.ntz;
  // Enough workgroups to fill 256 CUs several times over; splits of the
  // source bricks make up what the observation tiles alone do not give.
  const long long target_wg = 8192;
  if (p.n_tiles == 0 || p.n_bricks == 0) {
    plan->multi = 0;
    return JEFI_OK;  // nothing to launch
  }
  long long splits = (target_wg + p.n_tiles - 1) / p.n_tiles;
  long long max_splits = p.n_bricks / 8 > 0 ? p.n_bricks / 8 : 1;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  long long bps = (p.n_bricks + splits - 1) / splits;
  splits = (p.n_bricks + bps - 1) / bps;
  p.n_splits = (int)splits;
  p.bricks_per_split = (int)bps;
  p.n_wg = (int)((long long)p.n_tiles * splits);
  p.a_i = plan->all_dead ? -2 : (int)ts.a_i;
  p.a_f = ts.a_f;
  p.inv_cdt = ts.inv_cdt;
  p.inv_dt = 1.0 / dt;
  p.nt = nt;
  for (int a = 0; a < 3; ++a) p.screen[a] = r.screen[a];
  p.margin = 1e-7;
  p.near_slack = 1e-12;
  p.pref = (src->spacing[0] * src->spacing[1] * src->spacing[2]) / (4.0 * M_PI);

  // Largest separation of any pair, and the tile/brick diagonals.
  double slo[3], shi[3], olo[3], ohi[3];
  grid_box(src, slo, shi);
  grid_box(obs, olo, ohi);
  double rmax2 = 0.0, dt2 = 0.0, db2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double far = std::fmax(std::fabs(shi[a] - olo[a]), std::fabs(ohi[a] - slo[a]));
    rmax2 += far * far;
    const double te = (double)std::min(obs->n[a] - 1, kTileEdge - 1) * obs->spacing[a];
    const double be = (double)std::min(src->n[a] - 1, 1) * src->spacing[a];
    dt2 += te * te;
    db2 += be * be;
  }
  const double rmax = std::sqrt(rmax2), diam_t = std::sqrt(dt2), diam_b = std::sqrt(db2);
  // FP32 index guard: a bound on |u32 - u64| for the FP32 sequence of the
  // pair kernels, with u = 2^-24 the FP32 unit roundoff:
  //  - coordinates relative to the tile's first point, brick corner, cell
  //    offset (three roundings deep): |d32 - d| <= u (3R + 2 D_tile + 3 h);
  //  - r2 = x^2 + (y^2 + z^2): 3u relative, i.e. 1.5u on R; v_rsq_f32 taken
  //    as 2 ulp (4u); R = r2 * ri one more rounding: 6.5u relative on R;
  //  - u = fma(-R, 1/(c dt), a_f) with both constants rounded to FP32: u on
  //    1/(c dt), u on a_f, u on the result.
  // The band used is 1.25x that bound; a fractional part inside it sends
  // the pair through the canonical FP64 sequence.
  const double eps = std::ldexp(1.0, -24);
  double hsd2 = 0.0;
  for (int a = 0; a < 3; ++a) hsd2 += src->spacing[a] * src->spacing[a];
  const double e_coord = eps * (3.0 * rmax + 2.0 * diam_t + 3.0 * std::sqrt(hsd2));
  const double e_R = e_coord + 7.5 * eps * rmax;
  const double umax = ts.inv_cdt * rmax + 2.0;
  const double e_u = ts.inv_cdt * e_R + eps * (umax + 1.0);
  double g = 1.25 * e_u + 1e-7;
  p.use_thr = 0;
  if (!(g < 0.5)) {
    g = 0.5;  // every pair then takes the FP64 path
  } else {
    // Guard-band pairs have floor(u64) in {N-1, N}, N the integer nearest
    // u32; u is monotone in r2, so floor(u64) >= N iff r2 <= T(N), with T(N)
    // the largest FP64 r2 whose canonical u reaches N.  Kernels build the
    // table for every N the launch can meet.
    const double ulow = std::floor(ts.a_f - rmax * ts.inv_cdt) - 2.0;
    if (ulow > -1e9) {
      const long long lo = (long long)ulow;
      const long long n = 1 - lo + 1;
      if (n <= kThrMax) {
        p.use_thr = 1;
        p.thr_lo = (int)lo;
        p.thr_n = (int)n;
      }
    }
  }
  p.guard = (float)g;
  // Longest slice window any brick can need.
  const double wb = std::floor((diam_t + diam_b) * ts.inv_cdt * (1.0 + 1e-12) + 2.0 * p.margin + 1e-6) + 3.0;
  plan->multi = !(wb <= (double)kWmax);
  return JEFI_OK;
}

jefi_status check_history(const jefi_history* h, const jefi_grid* src, int nt) {
  if (!h) return fail(JEFI_EINVAL, "history is NULL");
  if (!h->data) return fail(JEFI_EINVAL, "history data is NULL");
  if (h->dtype != JEFI_F32 && h->dtype != JEFI_F64) return fail(JEFI_EINVAL, "history dtype %d", h->dtype);
  if (h->capacity < 1) return fail(JEFI_EINVAL, "history capacity %d < 1", h->capacity);
  if (!std::isfinite(h->t0)) return fail(JEFI_EINVAL, "history t0 must be finite");
  if (nt < 1 || nt > h->capacity)
    return fail(JEFI_EINVAL, "nt = %d must be in [1, capacity = %d]", nt, h->capacity);
  if ((long long)nt > h->newest + 1)
    return fail(JEFI_EINVAL, "nt = %d exceeds the %lld slices pushed", nt, (long long)h->newest + 1);
  (void)src;
  return JEFI_OK;
}

}  // namespace

extern "C" {

const char* jefi_version(void) { return "libjefi 0.1 (gfx950)"; }

const char* jefi_last_error(void) { return g_err.c_str(); }

void jefi_options_default(jefi_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof *opt);
  opt->c = 1.0;
  opt->screen_set = 0;
  opt->precision = JEFI_PREC_F32_COMP;
  opt->flags = 0;
  opt->tile_config = 0;
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
  const uint64_t need = jefi_history_bytes(src, capacity, dtype);
  if (need == 0 && capacity >= 1) {
    long long cells;
    if (!grid_ok(src, "source", &cells)) return JEFI_EINVAL;
  }
  if (capacity < 1 || (dtype != JEFI_F32 && dtype != JEFI_F64))
    return fail(JEFI_EINVAL, "bad capacity %d or dtype %d", capacity, dtype);
  if (bytes < need) return fail(JEFI_EINVAL, "history buffer has %llu bytes, needs %llu",
                                (unsigned long long)bytes, (unsigned long long)need);
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

jefi_status jefi_eval_fields(const jefi_grid* src, const jefi_history* hist, double dt, int32_t nt,
                             const jefi_grid* obs, double t, const jefi_fields* out,
                             const jefi_options* opt, void* stream) {
  if (g_device_failed.load()) return fail(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  long long ns = 0, no = 0;
  if (!grid_ok(src, "source", &ns) || !grid_ok(obs, "observation", &no)) return JEFI_EINVAL;
  jefi_status st = check_history(hist, src, nt);
  if (st != JEFI_OK) return st;
  if (!out || !out->E || !out->B) return fail(JEFI_EINVAL, "output fields are NULL");
  if (out->dtype != JEFI_F32 && out->dtype != JEFI_F64) return fail(JEFI_EINVAL, "output dtype %d", out->dtype);
  if (!std::isfinite(dt) || !(dt > 0.0)) return fail(JEFI_EINVAL, "dt must be finite and > 0");
  if (!std::isfinite(t)) return fail(JEFI_EINVAL, "t must be finite");
  Resolved r;
  if ((st = resolve_options(opt, src, &r)) != JEFI_OK) return st;
  const int want = r.precision == JEFI_PREC_F64 ? JEFI_F64 : JEFI_F32;
  if (hist->dtype != want)
    return fail(JEFI_EINVAL, "precision %s needs a %s history", r.precision == JEFI_PREC_F64 ? "F64" : "F32_COMP",
                want == JEFI_F64 ? "F64" : "F32");
  Plan plan;
  if ((st = make_plan(src, obs, nt, dt, hist->newest, hist->t0, t, r, &plan)) != JEFI_OK) return st;
  if (no == 0) return JEFI_OK;
  hipStream_t s = (hipStream_t)stream;
  const int out_f64 = out->dtype == JEFI_F64;
  if (ns == 0 || plan.all_dead) {
    hipError_t e = launch_fill_zero_fields(out->E, out->B, no, out_f64, s);
    return e == hipSuccess ? JEFI_OK : hip_fail(e, "zero-fill launch");
  }
  PairParams& p = plan.p;
  p.capacity = hist->capacity;
  p.slot_base = (int)((hist->newest - nt + 1) % hist->capacity);
  p.ring = hist->data;
  p.slot_elems = (long long)p.n_bricks * kBrickCells * 4;
  p.E = out->E;
  p.B = out->B;
  p.out_f64 = out_f64;
  p.direct = p.n_splits == 1;
  if (!p.direct) {
    void* scr = nullptr;
    if ((st = scratch_get(stream, (size_t)p.n_splits * 6 * (size_t)no * sizeof(double), &scr)) != JEFI_OK)
      return st;
    p.partial = (double*)scr;
  }
  hipError_t e = launch_pairs(p, r.precision == JEFI_PREC_F64, 0, plan.multi, s);
  if (e != hipSuccess) return hip_fail(e, "pair kernel launch");
  if (!p.direct) {
    EpilogueParams ep{p.partial, p.n_splits, no, p.pref, out->E, out->B, out_f64};
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
  if ((st = make_plan(src, obs, nt, dt, newest, t0, t, r, &plan)) != JEFI_OK) return st;
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
  long long ns = 0, no = 0;
  if (!grid_ok(src, "source", &ns) || !grid_ok(obs, "observation", &no)) return JEFI_EINVAL;
  jefi_status st = check_history(hist, src, nt);
  if (st != JEFI_OK) return st;
  if (!fp && no > 0) return fail(JEFI_EINVAL, "fp is NULL");
  if (!std::isfinite(dt) || !(dt > 0.0) || !std::isfinite(t)) return fail(JEFI_EINVAL, "dt and t must be finite, dt > 0");
  Resolved r;
  if ((st = resolve_options(opt, src, &r)) != JEFI_OK) return st;
  const int want = r.precision == JEFI_PREC_F64 ? JEFI_F64 : JEFI_F32;
  if (hist->dtype != want) return fail(JEFI_EINVAL, "history dtype does not match the precision");
  Plan plan;
  if ((st = make_plan(src, obs, nt, dt, hist->newest, hist->t0, t, r, &plan)) != JEFI_OK) return st;
  if (no == 0) return JEFI_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_zero(fp, (unsigned long long)no * 4 * sizeof(int64_t), s);
  if (e != hipSuccess) return hip_fail(e, "fingerprint zero-fill");
  if (ns == 0 || plan.all_dead) return JEFI_OK;
  PairParams& p = plan.p;
  p.capacity = hist->capacity;
  p.slot_base = (int)((hist->newest - nt + 1) % hist->capacity);
  p.ring = hist->data;
  p.slot_elems = (long long)p.n_bricks * kBrickCells * 4;
  p.fp = (unsigned long long*)fp;
  e = launch_pairs(p, r.precision == JEFI_PREC_F64, 1, plan.multi, s);
  return e == hipSuccess ? JEFI_OK : hip_fail(e, "fingerprint kernel launch");
}

}  // extern "C"
