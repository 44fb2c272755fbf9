// libjefi serving loop: sessions with resident source histories in a
// caller-provided device arena, admission by arena bytes with LRU eviction
// of idle sessions (a host shadow of each ring re-materialises them), and
// continuous batching: a scheduler thread turns admitted requests into
// batched evaluations on several streams, so requests arriving while others
// run are launched as soon as a stream slot and memory are free.  Small
// requests may take an express lane: one more stream whose batches run on a
// few compute units that the other batches leave free, so that they never
// wait behind a persistent launch holding the whole device.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/libjefi.h"
#include "jefi_arena.h"
#include "jefi_internal.h"

using jefi::Arena;

namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

long long cells_of(const jefi_grid& g) { return (long long)g.n[0] * g.n[1] * g.n[2]; }

bool grid_valid(const jefi_grid& g) {
  const bool empty = g.n[0] == 0 && g.n[1] == 0 && g.n[2] == 0;
  for (int a = 0; a < 3; ++a) {
    if (!empty && (g.n[a] < 1 || g.n[a] > (1 << 20))) return false;
    if (!std::isfinite(g.origin[a]) || !std::isfinite(g.spacing[a]) || !(g.spacing[a] > 0.0)) return false;
  }
  return cells_of(g) <= 0x7fffffffLL;
}

struct Session {
  uint64_t id = 0;
  jefi_grid src{};
  int32_t capacity = 0, window = 0;
  double t0 = 0.0, dt = 0.0;
  size_t elem = 4;
  long long n_src = 0;
  int64_t newest = -1;
  std::vector<unsigned char> shadow;  // host copy [capacity][4][n_src], slot = step % capacity
  bool resident = false;
  bool evicted = false;  // left the arena at least once since it was opened
  uint64_t ring_off = 0, ring_bytes = 0;
  int busy = 0;      // requests admitted and not finished
  hipEvent_t last_done = nullptr;  // completion event of the batch holding its latest admitted request
  int queued = 0;    // requests submitted and not admitted
  uint64_t last_use = 0;
};

enum { kQueued = 0, kRunning = 1, kDone = 2 };

struct Req {
  uint64_t ticket = 0, session = 0;
  std::vector<unsigned char> slice;
  jefi_grid obs{};
  double t = 0.0;
  void* E = nullptr;
  void* B = nullptr;
  int32_t out_dtype = 0, out_on_host = 0;
  long long n_obs = 0;
  int state = kQueued;
  jefi_status status = JEFI_PENDING;
  uint64_t t_submit = 0, t_admit = 0, t_start = 0, t_done = 0, pairs = 0;
  int batch_size = 0;
  // arena resources (device) and pinned staging, released at completion
  uint64_t slice_off = 0, slice_bytes = 0, out_off = 0, out_bytes = 0;
  uint64_t pin_off = 0, pin_bytes = 0;
};

struct Region {
  bool device;
  uint64_t off, bytes;
};

struct Batch {
  int stream = 0;
  hipEvent_t done = nullptr;
  std::vector<uint64_t> tickets;
  std::vector<Region> extra;  // re-materialisation staging, freed with the batch
};

}  // namespace

struct jefi_server {
  jefi_server_config cfg{};
  int device = 0;
  char* dbase = nullptr;
  Arena darena;
  char* pbase = nullptr;
  Arena parena;
  // streams: regular lane [0, n_regular); express lane streams[express];
  // with CU masks, [express + 1, express + 1 + n_regular): regular streams
  // on every compute unit, used while a backlog has switched the lane off
  std::vector<hipStream_t> streams;
  int n_regular = 0;
  int express = -1;      // stream index of the express lane, -1 without one
  int express_cus = 0;   // compute units its batches run on
  bool cu_masked = false;  // lane streams restricted to their compute units
  std::vector<hipEvent_t> events;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  std::unordered_map<uint64_t, Session> sessions;
  std::deque<Batch> inflight;
  hipStream_t setup = nullptr;  // eager ring uploads at open_session
  std::thread th;
  bool stop = false;
  uint64_t next_ticket = 1, use_clock = 0;
  jefi_status sticky = JEFI_OK;
  char sticky_msg[256] = {0};
  jefi_server_stats stats{};
};

namespace {

void set_sticky(jefi_server* s, hipError_t e, const char* what) {
  if (s->sticky == JEFI_OK) {
    s->sticky = JEFI_EDEVICE;
    snprintf(s->sticky_msg, sizeof s->sticky_msg, "%s: %s", what, hipGetErrorString(e));
  }
}

size_t elem_size(int precision) { return precision == JEFI_PREC_F64 ? 8 : 4; }

uint64_t ring_bytes_of(const jefi_grid& src, int capacity, int precision) {
  return jefi_history_bytes(&src, capacity, precision == JEFI_PREC_F64 ? JEFI_F64 : JEFI_F32);
}

// Make room for `bytes` in the device arena by evicting idle resident
// sessions, least recently used first (never those in `keep`).
bool make_room(jefi_server* sv, uint64_t bytes, const std::unordered_set<uint64_t>& keep) {
  while (!sv->darena.fits(bytes)) {
    Session* victim = nullptr;
    for (auto& kv : sv->sessions) {
      Session& s = kv.second;
      if (!s.resident || s.busy > 0 || keep.count(s.id)) continue;
      if (!victim || s.last_use < victim->last_use) victim = &s;
    }
    if (!victim) return false;
    sv->darena.release(victim->ring_off, victim->ring_bytes);
    victim->resident = false;
    victim->evicted = true;
    sv->stats.evictions++;
  }
  return true;
}

// Bring a session's ring onto the device: the whole host shadow (every
// slot, zeros where nothing was pushed) goes to a device staging region and
// one kernel lays every slot out into the ring.  The copy reads pageable host
// memory, so the shadow may change as soon as this returns; the staging
// region (returned in *staging) must outlive the kernel, i.e. be released
// only after `st` has passed this point.
jefi_status materialise(jefi_server* sv, Session& s, hipStream_t st, const std::unordered_set<uint64_t>& keep,
                        Region* staging) {
  staging->device = true;
  staging->off = staging->bytes = 0;
  if (!make_room(sv, s.ring_bytes, keep)) return JEFI_ENOMEM;
  uint64_t off;
  if (!sv->darena.alloc(s.ring_bytes, &off)) return JEFI_ENOMEM;
  const uint64_t sh_bytes = s.shadow.size();
  uint64_t so = 0;
  if (s.newest >= 0 && (!make_room(sv, sh_bytes, keep) || !sv->darena.alloc(sh_bytes, &so))) {
    sv->darena.release(off, s.ring_bytes);
    return JEFI_ENOMEM;
  }
  s.ring_off = off;
  s.resident = true;
  jefi_history h{};
  const int dt = sv->cfg.precision == JEFI_PREC_F64 ? JEFI_F64 : JEFI_F32;
  jefi_status rc = jefi_history_init(&h, sv->dbase + off, s.ring_bytes, &s.src, s.capacity, dt, s.t0, st);
  if (rc == JEFI_OK && s.newest >= 0) {
    staging->off = so;
    staging->bytes = sh_bytes;
    hipError_t e = hipMemcpyAsync(sv->dbase + so, s.shadow.data(), sh_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      jefi::GridD g;
      for (int a = 0; a < 3; ++a) {
        g.n[a] = s.src.n[a];
        g.o[a] = s.src.origin[a];
        g.h[a] = s.src.spacing[a];
      }
      e = jefi::launch_ingest_slots(sv->dbase + so, sv->dbase + off, g, (g.n[0] + 1) / 2, (g.n[1] + 1) / 2, s.capacity,
                              dt == JEFI_F64, st);
    }
    if (e != hipSuccess) {
      set_sticky(sv, e, "session upload");
      rc = JEFI_EDEVICE;
    }
    if (s.evicted) sv->stats.rematerialisations++;
  }
  return rc;
}

void release_req(jefi_server* sv, Req& r) {
  if (r.slice_bytes) sv->darena.release(r.slice_off, r.slice_bytes);
  if (r.out_bytes) sv->darena.release(r.out_off, r.out_bytes);
  if (r.pin_bytes) sv->parena.release(r.pin_off, r.pin_bytes);
  r.slice_bytes = r.out_bytes = r.pin_bytes = 0;
}

void finish(jefi_server* sv, Req& r, jefi_status st) {
  r.status = st;
  r.state = kDone;
  r.t_done = now_ns();
  if (st == JEFI_OK) {
    sv->stats.completed++;
    sv->stats.pairs += r.pairs;
  } else {
    sv->stats.failed++;
  }
}

void complete_batch(jefi_server* sv, Batch& b, jefi_status st) {
  for (uint64_t tk : b.tickets) {
    Req& r = sv->reqs[tk];
    Session& s = sv->sessions[r.session];
    if (st == JEFI_OK && r.out_on_host) {
      const size_t each = (size_t)3 * r.n_obs * (r.out_dtype == JEFI_F64 ? 8 : 4);
      const uint64_t at = r.pin_off + Arena::round_up(r.slice.size());
      std::memcpy(r.E, sv->pbase + at, each);
      std::memcpy(r.B, sv->pbase + at + each, each);
    }
    release_req(sv, r);
    std::vector<unsigned char>().swap(r.slice);
    s.busy--;
    s.last_use = ++sv->use_clock;
    finish(sv, r, st);
  }
  for (Region& g : b.extra) {
    if (g.device)
      sv->darena.release(g.off, g.bytes);
    else
      sv->parena.release(g.off, g.bytes);
  }
  sv->events.push_back(b.done);
}

bool small_request(const jefi_server* sv, const Req& r) {
  return sv->express >= 0 && r.pairs <= sv->cfg.express_pairs;
}

// Choose the next batch of one lane: FIFO over the queue, one request per
// session, every resource reserved up front; a request that does not fit yet
// stops the scan (admission in arrival order).  With an express lane, it
// takes only requests of at most express_pairs pairs and the regular lane
// the others.  A session whose earlier request is left for the other lane
// is passed over, so each session's requests still run in order.  While
// more requests wait than one batch holds (a backlog, where latency is the
// queue's anyway), the express lane admits nothing and the regular lane
// takes every request, on streams that use every compute unit.
void admit_and_launch(jefi_server* sv, bool express_lane) {
  if (sv->queue.empty()) return;
  const bool backlog = sv->queue.size() > (size_t)sv->cfg.max_batch;
  const bool lanes = sv->express >= 0 && !backlog;
  if (express_lane && !lanes) return;
  // a stream of this lane with no batch in flight, so that this batch
  // overlaps the others; at most n_regular regular batches at once
  int si = -1;
  if (express_lane) {
    bool used = false;
    for (const Batch& f : sv->inflight) used = used || f.stream == sv->express;
    if (!used) si = sv->express;
  } else {
    int regular_inflight = 0;
    for (const Batch& f : sv->inflight) regular_inflight += f.stream != sv->express;
    if (regular_inflight >= sv->n_regular) return;
    const bool full = backlog && sv->cu_masked;
    const int first = full ? sv->express + 1 : 0;
    for (int i = first; i < first + sv->n_regular && si < 0; ++i) {
      bool used = false;
      for (const Batch& f : sv->inflight) used = used || f.stream == i;
      if (!used) si = i;
    }
  }
  if (si < 0) return;
  hipStream_t st = sv->streams[si];
  Batch b;
  b.stream = si;
  std::unordered_set<uint64_t> in_batch, passed;
  std::vector<uint64_t> chosen;
  std::vector<hipEvent_t> deps;
  const size_t el = elem_size(sv->cfg.precision);
  // An express batch stays short (at most four express-sized requests of
  // work): a later request of one of its sessions in the regular lane waits
  // for it, and so would that request's whole batch.
  const uint64_t express_budget = 4 * sv->cfg.express_pairs;
  uint64_t batch_pairs = 0;
  for (auto it = sv->queue.begin(); it != sv->queue.end() && (int)chosen.size() < sv->cfg.max_batch;) {
    Req& r = sv->reqs[*it];
    Session& s = sv->sessions[r.session];
    if (express_lane && !chosen.empty() && batch_pairs + r.pairs > express_budget) break;
    if (passed.count(s.id)) {  // an earlier request of the session is the other lane's
      ++it;
      continue;
    }
    const bool small = small_request(sv, r);
    if (lanes && small != express_lane) {
      passed.insert(s.id);
      ++it;
      continue;
    }
    if (in_batch.count(s.id)) {  // one request per session and batch
      ++it;
      continue;
    }
    // the evaluation time must not lie after the newest slice (after this push)
    const int64_t newest = s.newest + (r.slice.empty() ? 0 : 1);
    const double t_new = s.t0 + (double)newest * s.dt;
    const double t = std::isnan(r.t) ? t_new : r.t;
    if (newest < 0 || !(t <= t_new + 1e-9 * (1.0 + std::fabs(t_new)))) {
      r.t_admit = r.t_start = now_ns();
      s.queued--;
      finish(sv, r, JEFI_EINVAL);
      it = sv->queue.erase(it);
      continue;
    }
    in_batch.insert(s.id);
    bool fresh = false;  // ring uploaded on `st` in this pass
    Region stg{true, 0, 0};
    if (!s.resident) {
      jefi_status rc = materialise(sv, s, st, in_batch, &stg);
      if (stg.bytes) b.extra.push_back(stg);
      if (rc != JEFI_OK) {
        in_batch.erase(s.id);
        if (rc == JEFI_EDEVICE) return;
        break;  // no room yet: wait for completions
      }
      fresh = true;
    }
    const uint64_t slice_bytes = r.slice.size();
    const uint64_t out_bytes = r.out_on_host ? (uint64_t)6 * r.n_obs * (r.out_dtype == JEFI_F64 ? 8 : 4) : 0;
    const uint64_t pin_bytes = Arena::round_up(slice_bytes) + out_bytes;
    bool ok = true;
    if (slice_bytes) ok = make_room(sv, slice_bytes, in_batch) && sv->darena.alloc(slice_bytes, &r.slice_off);
    if (ok) r.slice_bytes = slice_bytes;
    if (ok && out_bytes) ok = make_room(sv, out_bytes, in_batch) && sv->darena.alloc(out_bytes, &r.out_off);
    if (ok) r.out_bytes = out_bytes;
    if (ok && pin_bytes) ok = sv->parena.alloc(pin_bytes, &r.pin_off);
    if (ok) r.pin_bytes = pin_bytes;
    if (!ok) {
      release_req(sv, r);
      in_batch.erase(s.id);
      if (fresh) {
        // The ring upload is queued on `st` but the session joins no batch
        // here: its next request may run on another stream, with nothing
        // ordering it after the upload (nor its eviction after it).  Let the
        // upload finish before the session is used again.
        const hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
          set_sticky(sv, e, "session upload");
          return;
        }
        if (stg.bytes) {
          sv->darena.release(stg.off, stg.bytes);
          b.extra.pop_back();
        }
      }
      break;
    }
    (void)el;
    if (slice_bytes) std::memcpy(sv->pbase + r.pin_off, r.slice.data(), slice_bytes);
    // A session with a request still on the device: this batch's stream
    // waits for that batch before its push and evaluation (the push may
    // overwrite a slot the earlier evaluation reads).
    if (s.busy > 0 && s.last_done && std::find(deps.begin(), deps.end(), s.last_done) == deps.end())
      deps.push_back(s.last_done);
    r.t_admit = now_ns();
    r.state = kRunning;
    s.queued--;
    s.busy++;
    batch_pairs += r.pairs;
    chosen.push_back(*it);
    it = sv->queue.erase(it);
  }
  if (chosen.empty()) {
    if (!b.extra.empty()) {
      // a session was materialised but no request fits yet: let its
      // staging drain, then give the staging back
      (void)hipStreamSynchronize(st);
      for (Region& g : b.extra) {
        if (g.device)
          sv->darena.release(g.off, g.bytes);
        else
          sv->parena.release(g.off, g.bytes);
      }
    }
    return;
  }
  // Launch: slice uploads and pushes, one batched evaluation, output copies.
  for (hipEvent_t ev : deps) {
    const hipError_t e = hipStreamWaitEvent(st, ev, 0);
    if (e != hipSuccess) set_sticky(sv, e, "hipStreamWaitEvent");
  }
  std::vector<jefi_problem> probs;
  probs.reserve(chosen.size());
  const uint64_t t_start = now_ns();
  for (uint64_t tk : chosen) {
    Req& r = sv->reqs[tk];
    Session& s = sv->sessions[r.session];
    r.t_start = t_start;
    r.batch_size = (int)chosen.size();
    jefi_history h{sv->dbase + s.ring_off, sv->cfg.precision == JEFI_PREC_F64 ? JEFI_F64 : JEFI_F32, s.capacity,
                   s.newest, s.t0};
    if (!r.slice.empty()) {
      hipError_t e = hipMemcpyAsync(sv->dbase + r.slice_off, sv->pbase + r.pin_off, r.slice.size(),
                                    hipMemcpyHostToDevice, st);
      if (e != hipSuccess) {
        set_sticky(sv, e, "slice upload");
        break;
      }
      if (jefi_history_push(&h, &s.src, sv->dbase + r.slice_off, st) != JEFI_OK) {
        set_sticky(sv, hipErrorUnknown, "slice ingest");
        break;
      }
      const size_t slot = (size_t)(h.newest % s.capacity);
      std::memcpy(s.shadow.data() + slot * r.slice.size(), r.slice.data(), r.slice.size());
      s.newest = h.newest;
    }
    const int nt = (int)std::min<int64_t>(s.window, s.newest + 1);
    jefi_problem q{};
    q.src = s.src;
    q.hist = h;
    q.dt = s.dt;
    q.nt = nt;
    q.obs = r.obs;
    q.t = std::isnan(r.t) ? s.t0 + (double)s.newest * s.dt : r.t;
    if (r.out_on_host) {
      const size_t each = (size_t)3 * r.n_obs * (r.out_dtype == JEFI_F64 ? 8 : 4);
      q.out = jefi_fields{sv->dbase + r.out_off, sv->dbase + r.out_off + each, r.out_dtype};
    } else {
      q.out = jefi_fields{r.E, r.B, r.out_dtype};
    }
    r.pairs = (uint64_t)cells_of(s.src) * (uint64_t)r.n_obs;
    probs.push_back(q);
  }
  jefi_status rc = JEFI_OK;
  if (sv->sticky != JEFI_OK) {
    rc = sv->sticky;
  } else {
    jefi_options opt;
    jefi_options_default(&opt);
    opt.precision = sv->cfg.precision;
    opt.flags = sv->cfg.flags;
    if (express_lane) {
      rc = jefi::eval_batch_on_cus(probs.data(), (int32_t)probs.size(), &opt, st, sv->express_cus);
    } else {
      // regular batches on the lane's masked streams leave the express
      // lane's compute units free
      const bool beside_express = sv->express >= 0 && si < sv->express;
      opt.reserve_cus = std::max(sv->cfg.reserve_cus, beside_express ? sv->express_cus : 0);
      rc = jefi_eval_batch(probs.data(), (int32_t)probs.size(), &opt, st);
    }
    if (rc == JEFI_EDEVICE) set_sticky(sv, hipErrorUnknown, jefi_last_error());
  }
  if (rc == JEFI_OK) {
    for (uint64_t tk : chosen) {
      Req& r = sv->reqs[tk];
      if (!r.out_on_host) continue;
      hipError_t e = hipMemcpyAsync(sv->pbase + r.pin_off + Arena::round_up(r.slice.size()), sv->dbase + r.out_off,
                                    r.out_bytes, hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) {
        set_sticky(sv, e, "output copy");
        rc = JEFI_EDEVICE;
        break;
      }
    }
  }
  b.tickets = chosen;
  if (sv->events.empty()) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) sv->events.push_back(ev);
  }
  if (rc != JEFI_OK || sv->events.empty()) {
    // the batch never reached the device in full: wait for the stream, fail it
    (void)hipStreamSynchronize(st);
    if (!sv->events.empty()) {
      b.done = sv->events.back();
      sv->events.pop_back();
    }
    complete_batch(sv, b, rc != JEFI_OK ? rc : JEFI_EDEVICE);
    return;
  }
  b.done = sv->events.back();
  sv->events.pop_back();
  hipError_t e = hipEventRecord(b.done, st);
  if (e != hipSuccess) set_sticky(sv, e, "hipEventRecord");
  for (uint64_t tk : chosen) sv->sessions[sv->reqs[tk].session].last_done = b.done;
  sv->stats.batches++;
  if (express_lane) sv->stats.express_batches++;
  if ((uint64_t)chosen.size() > sv->stats.max_batch) sv->stats.max_batch = chosen.size();
  sv->inflight.push_back(std::move(b));
}

void scheduler(jefi_server* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    bool progress = false;
    for (auto it = sv->inflight.begin(); it != sv->inflight.end();) {
      hipError_t q = hipEventQuery(it->done);
      if (q == hipErrorNotReady) {
        ++it;
        continue;
      }
      if (q != hipSuccess) set_sticky(sv, q, "batch completion");
      complete_batch(sv, *it, q == hipSuccess ? JEFI_OK : JEFI_EDEVICE);
      it = sv->inflight.erase(it);
      progress = true;
    }
    if (progress) sv->done_cv.notify_all();
    if (!sv->queue.empty()) {
      const size_t before = sv->queue.size();
      admit_and_launch(sv, true);
      admit_and_launch(sv, false);
      if (sv->queue.size() != before) progress = true;
      sv->done_cv.notify_all();
    }
    if (sv->stop && sv->queue.empty() && sv->inflight.empty()) break;
    if (!progress) sv->cv.wait_for(lk, std::chrono::microseconds(sv->inflight.empty() ? 2000 : 50));
  }
}

}  // namespace

extern "C" {

jefi_status jefi_server_create(const jefi_server_config* cfg, jefi_server** out) {
  if (!cfg || !out) return JEFI_EINVAL;
  if (!cfg->arena || cfg->arena_bytes < Arena::kGranule) return JEFI_EINVAL;
  if (cfg->precision != JEFI_PREC_F64 && cfg->precision != JEFI_PREC_F32_COMP) return JEFI_EINVAL;
  const uint32_t known = JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE | JEFI_FLAG_DERIV_SLOPE | JEFI_FLAG_PAST_HOLD |
                         JEFI_FLAG_TIME_CUBIC | JEFI_FLAG_PAST_CUT;
  const uint32_t both = JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE;
  const uint32_t slope_cubic = JEFI_FLAG_DERIV_SLOPE | JEFI_FLAG_TIME_CUBIC;
  const uint32_t pasts = JEFI_FLAG_PAST_HOLD | JEFI_FLAG_PAST_CUT;
  if ((cfg->flags & ~known) != 0 || (cfg->flags & both) == both || (cfg->flags & slope_cubic) == slope_cubic ||
      (cfg->flags & pasts) == pasts)
    return JEFI_EINVAL;
  if (cfg->reserve_cus < 0 || cfg->reserve_cus > 1024) return JEFI_EINVAL;
  if (cfg->express_cus < 0 || cfg->express_cus > 1024) return JEFI_EINVAL;
  jefi_server* sv = new jefi_server();
  sv->cfg = *cfg;
  if (sv->cfg.max_inflight < 1) sv->cfg.max_inflight = 2;
  if (sv->cfg.max_inflight > 8) sv->cfg.max_inflight = 8;
  if (sv->cfg.max_batch < 1) sv->cfg.max_batch = 256;
  if (sv->cfg.max_queue < 1) sv->cfg.max_queue = 65536;
  if (sv->cfg.pinned_bytes == 0) sv->cfg.pinned_bytes = 256ull << 20;
  (void)hipGetDevice(&sv->device);
  sv->dbase = (char*)cfg->arena;
  sv->darena.reset(cfg->arena_bytes);
  if (hipHostMalloc((void**)&sv->pbase, sv->cfg.pinned_bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete sv;
    return JEFI_ENOMEM;
  }
  sv->parena.reset(sv->cfg.pinned_bytes);
  sv->n_regular = sv->cfg.max_inflight;
  int n_streams = sv->n_regular + (sv->cfg.express_pairs > 0 ? 1 : 0);
  if (sv->cfg.express_pairs > 0) {
    // the express lane: the last express_cus compute units (16 by default,
    // at most half the device); the regular streams take the others
    const int cus = jefi::device_cus();
    sv->express_cus = std::max(1, std::min(sv->cfg.express_cus > 0 ? sv->cfg.express_cus : 16, cus / 2));
    sv->express = sv->n_regular;
    sv->cu_masked = true;
    for (int i = 0; i < n_streams && sv->cu_masked; ++i) {
      hipStream_t s;
      const bool ok = i == sv->express ? jefi::create_stream_on_cus(&s, cus - sv->express_cus, sv->express_cus)
                                       : jefi::create_stream_on_cus(&s, 0, cus - sv->express_cus);
      if (ok)
        sv->streams.push_back(s);
      else
        sv->cu_masked = false;
    }
    if (!sv->cu_masked) {
      // the runtime refused the masks: plain streams, and the lanes kept apart
      // by launch sizes alone (regular launches leave the units free)
      for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
      sv->streams.clear();
    } else {
      n_streams += sv->n_regular;  // unmasked regular streams for backlogs
    }
  }
  for (int i = (int)sv->streams.size(); i < n_streams; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
      (void)hipHostFree(sv->pbase);
      delete sv;
      return JEFI_EDEVICE;
    }
    sv->streams.push_back(s);
  }
  sv->stats.express_cus = (uint64_t)sv->express_cus;
  sv->stats.cu_masked = sv->cu_masked ? 1u : 0u;
  if (hipStreamCreateWithFlags(&sv->setup, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
    (void)hipHostFree(sv->pbase);
    delete sv;
    return JEFI_EDEVICE;
  }
  sv->stats.arena_bytes = cfg->arena_bytes;
  sv->th = std::thread(scheduler, sv);
  *out = sv;
  return JEFI_OK;
}

jefi_status jefi_server_open_session(jefi_server* sv, uint64_t session, const jefi_grid* src, int32_t capacity,
                                     int32_t window, double t0, double dt, const void* init_history,
                                     int32_t init_nt) {
  if (!sv || !src) return JEFI_EINVAL;
  if (!grid_valid(*src) || cells_of(*src) == 0) return JEFI_EINVAL;
  if (capacity < 1 || window < 1 || window > capacity) return JEFI_EINVAL;
  if (!std::isfinite(t0) || !std::isfinite(dt) || !(dt > 0.0)) return JEFI_EINVAL;
  if (init_nt < 0 || init_nt > capacity || (init_nt > 0 && !init_history)) return JEFI_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->sticky != JEFI_OK) return sv->sticky;
  if (sv->sessions.count(session)) return JEFI_EINVAL;
  Session s;
  s.id = session;
  s.src = *src;
  s.capacity = capacity;
  s.window = window;
  s.t0 = t0;
  s.dt = dt;
  s.elem = elem_size(sv->cfg.precision);
  s.n_src = cells_of(*src);
  s.ring_bytes = ring_bytes_of(*src, capacity, sv->cfg.precision);
  const size_t slice_bytes = (size_t)4 * s.n_src * s.elem;
  if (Arena::round_up(s.ring_bytes) + Arena::round_up((uint64_t)capacity * slice_bytes) > sv->cfg.arena_bytes)
    return JEFI_ETOOLARGE;
  s.shadow.assign((size_t)capacity * slice_bytes, 0);
  for (int j = 0; j < init_nt; ++j)
    std::memcpy(s.shadow.data() + (size_t)j * slice_bytes, (const char*)init_history + (size_t)j * slice_bytes,
                slice_bytes);
  s.newest = init_nt - 1;
  s.last_use = ++sv->use_clock;
  Session& ss = sv->sessions.emplace(session, std::move(s)).first->second;
  // Upload the ring now when the arena has room (idle sessions may be
  // evicted for it), so that the first request does not pay for it;
  // otherwise the first admitted request brings it in.
  Region stg;
  const jefi_status rc = materialise(sv, ss, sv->setup, {}, &stg);
  if (rc == JEFI_EDEVICE) return JEFI_EDEVICE;
  if (rc == JEFI_OK || stg.bytes) {
    const hipError_t e = hipStreamSynchronize(sv->setup);
    if (e != hipSuccess) {
      set_sticky(sv, e, "session upload");
      return JEFI_EDEVICE;
    }
  }
  if (stg.bytes) sv->darena.release(stg.off, stg.bytes);
  return JEFI_OK;
}

jefi_status jefi_server_submit(jefi_server* sv, const jefi_request* rq, uint64_t* ticket) {
  if (!sv || !rq || !ticket) return JEFI_EINVAL;
  if (!grid_valid(rq->obs)) return JEFI_EINVAL;
  if (rq->out_dtype != JEFI_F32 && rq->out_dtype != JEFI_F64) return JEFI_EINVAL;
  const long long n_obs = cells_of(rq->obs);
  if (n_obs > 0 && (!rq->E || !rq->B)) return JEFI_EINVAL;
  if (!std::isnan(rq->t) && !std::isfinite(rq->t)) return JEFI_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->sticky != JEFI_OK) return sv->sticky;
  auto sit = sv->sessions.find(rq->session);
  if (sit == sv->sessions.end()) return JEFI_ENOENT;
  Session& s = sit->second;
  const size_t slice_bytes = (size_t)4 * s.n_src * s.elem;
  const uint64_t out_bytes = rq->out_on_host ? (uint64_t)6 * n_obs * (rq->out_dtype == JEFI_F64 ? 8 : 4) : 0;
  // Worst case for one request on an otherwise empty arena: the ring, the
  // staging of its host shadow (when it has to be brought back), the slice
  // and the outputs, all held until its batch completes.
  const uint64_t shadow_bytes = Arena::round_up(s.shadow.size());
  uint64_t need = Arena::round_up(s.ring_bytes) + shadow_bytes + Arena::round_up(out_bytes);
  if (rq->new_slice) need += Arena::round_up(slice_bytes);
  const uint64_t pin_need = Arena::round_up(rq->new_slice ? slice_bytes : 0) + out_bytes;
  if (need > sv->cfg.arena_bytes || pin_need > sv->cfg.pinned_bytes) return JEFI_ETOOLARGE;
  // only requests that could ever run are told to retry
  if ((int)sv->queue.size() >= sv->cfg.max_queue) return JEFI_EBUSY;
  Req r;
  r.ticket = sv->next_ticket++;
  r.session = rq->session;
  if (rq->new_slice) r.slice.assign((const unsigned char*)rq->new_slice, (const unsigned char*)rq->new_slice + slice_bytes);
  r.obs = rq->obs;
  r.t = rq->t;
  r.E = rq->E;
  r.B = rq->B;
  r.out_dtype = rq->out_dtype;
  r.out_on_host = rq->out_on_host;
  r.n_obs = n_obs;
  r.pairs = (uint64_t)s.n_src * (uint64_t)n_obs;
  r.t_submit = now_ns();
  s.queued++;
  sv->stats.submitted++;
  *ticket = r.ticket;
  if (n_obs == 0 && !rq->new_slice) {
    // nothing to compute or store
    r.t_admit = r.t_start = r.t_submit;
    s.queued--;
    finish(sv, r, JEFI_OK);
    sv->reqs.emplace(r.ticket, std::move(r));
    return JEFI_OK;
  }
  sv->queue.push_back(r.ticket);
  sv->reqs.emplace(r.ticket, std::move(r));
  lk.unlock();
  sv->cv.notify_all();
  return JEFI_OK;
}

static void fill_result(const Req& r, jefi_result* res) {
  res->status = r.state == kDone ? r.status : JEFI_PENDING;
  res->batch_size = r.batch_size;
  res->t_submit_ns = r.t_submit;
  res->t_admit_ns = r.t_admit;
  res->t_start_ns = r.t_start;
  res->t_done_ns = r.t_done;
  res->pairs = r.pairs;
}

jefi_status jefi_server_poll(jefi_server* sv, uint64_t ticket, jefi_result* res) {
  if (!sv || !res) return JEFI_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return JEFI_ENOENT;
  fill_result(it->second, res);
  if (it->second.state != kDone) return JEFI_PENDING;
  sv->reqs.erase(it);
  sv->done_cv.notify_all();  // a waiter on the same ticket now sees it gone
  return JEFI_OK;
}

jefi_status jefi_server_wait(jefi_server* sv, uint64_t ticket, jefi_result* res) {
  if (!sv || !res) return JEFI_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return JEFI_ENOENT;
  // another thread may poll or wait the same ticket and release it first
  sv->done_cv.wait(lk, [&]() {
    const auto f = sv->reqs.find(ticket);
    return f == sv->reqs.end() || f->second.state == kDone;
  });
  it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return JEFI_ENOENT;
  fill_result(it->second, res);
  sv->reqs.erase(it);
  return JEFI_OK;
}

jefi_status jefi_server_close_session(jefi_server* sv, uint64_t session) {
  if (!sv) return JEFI_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->sessions.find(session);
  if (it == sv->sessions.end()) return JEFI_ENOENT;
  if (it->second.busy > 0 || it->second.queued > 0) return JEFI_EBUSY;
  if (it->second.resident) sv->darena.release(it->second.ring_off, it->second.ring_bytes);
  sv->sessions.erase(it);
  return JEFI_OK;
}

jefi_status jefi_server_get_stats(jefi_server* sv, jefi_server_stats* out) {
  if (!sv || !out) return JEFI_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->stats;
  out->arena_high_water = sv->darena.high_water();
  out->arena_used = sv->darena.used();
  return JEFI_OK;
}

jefi_status jefi_server_destroy(jefi_server* sv) {
  if (!sv) return JEFI_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  sv->th.join();
  const jefi_status st = sv->sticky;
  for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
  (void)hipStreamDestroy(sv->setup);
  for (hipEvent_t e : sv->events) (void)hipEventDestroy(e);
  (void)hipHostFree(sv->pbase);
  delete sv;
  return st;
}

}  // extern "C"
