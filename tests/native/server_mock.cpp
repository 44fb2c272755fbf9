// Host implementations of the mock HIP runtime (tests/native/mock_hip) and
// of the library calls the serving loop makes, with a simple ring layout
// [capacity][4][n_src] and a stand-in "evaluation" whose outputs record
// exactly which slices the ring held when it ran: a weighted sum over the
// window, so that any reordering of a push and an evaluation shows up.
// Test infrastructure only: nothing here computes fields.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/libjefi.h"
#include "../../paper_2104_05426_amd/csrc/jefi_internal.h"

struct MockStream {
  std::mutex mu;
  std::condition_variable cv, idle_cv;
  std::deque<std::function<void()>> ops;
  bool busy = false, stop = false;
  std::thread th;
  MockStream() {
    th = std::thread([this]() {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        cv.wait(lk, [&]() { return stop || !ops.empty(); });
        if (ops.empty() && stop) break;
        std::function<void()> op = std::move(ops.front());
        ops.pop_front();
        busy = true;
        lk.unlock();
        op();
        lk.lock();
        busy = false;
        idle_cv.notify_all();
      }
    });
  }
  void push(std::function<void()> op) {
    std::lock_guard<std::mutex> lk(mu);
    ops.push_back(std::move(op));
    cv.notify_all();
  }
  void sync() {
    std::unique_lock<std::mutex> lk(mu);
    idle_cv.wait(lk, [&]() { return ops.empty() && !busy; });
  }
  ~MockStream() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
      cv.notify_all();
    }
    th.join();
  }
};

struct MockEvent {
  std::mutex mu;
  std::condition_variable cv;
  uint64_t recorded = 0, done = 0;
};

int g_eval_sleep_us = 0;    // set by the test to keep batches on the "device" longer
int g_ingest_sleep_us = 0;  // likewise for ring uploads (re-materialisation)

// Batches launched so far, and a gate that keeps the next n batches on their
// streams until the test releases them, in launch order (scenarios that need
// a fixed order of completions whatever the threads' timing).
static std::mutex g_gate_mu;
static std::condition_variable g_gate_cv;
static int g_launched = 0, g_gate_base = 0, g_gate_n = 0, g_gate_released = 0;

hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "mock error"; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new MockStream();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  s->sync();
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  s->sync();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new MockEvent();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    gen = ++e->recorded;
  }
  s->push([e, gen]() {
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->done < gen) e->done = gen;
    e->cv.notify_all();
  });
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(e->mu);
  return e->done >= e->recorded ? hipSuccess : hipErrorNotReady;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    gen = e->recorded;
  }
  s->push([e, gen]() {
    std::unique_lock<std::mutex> lk(e->mu);
    e->cv.wait(lk, [&]() { return e->done >= gen; });
  });
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s) {
  if (kind == hipMemcpyHostToDevice) {
    // pageable semantics: the source is consumed before the call returns
    auto tmp = std::make_shared<std::vector<unsigned char>>((const unsigned char*)src,
                                                            (const unsigned char*)src + bytes);
    s->push([dst, tmp]() { std::memcpy(dst, tmp->data(), tmp->size()); });
  } else {
    s->push([dst, src, bytes]() { std::memcpy(dst, src, bytes); });
  }
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  *p = std::malloc(bytes);
  return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}

// ---- library calls (mock layout) ----------------------------------------------
static long long cells(const jefi_grid* g) { return (long long)g->n[0] * g->n[1] * g->n[2]; }

extern "C" {

const char* jefi_last_error(void) { return "mock"; }

void jefi_options_default(jefi_options* o) {
  std::memset(o, 0, sizeof *o);
  o->c = 1.0;
  o->precision = JEFI_PREC_F32_COMP;
}

uint64_t jefi_history_bytes(const jefi_grid* src, int32_t capacity, int32_t dtype) {
  return (uint64_t)capacity * 4 * (uint64_t)cells(src) * (dtype == JEFI_F64 ? 8 : 4);
}

jefi_status jefi_history_init(jefi_history* h, void* data, uint64_t bytes, const jefi_grid* src, int32_t capacity,
                              int32_t dtype, double t0, void* stream) {
  if (bytes < jefi_history_bytes(src, capacity, dtype)) return JEFI_EINVAL;
  h->data = data;
  h->dtype = dtype;
  h->capacity = capacity;
  h->newest = -1;
  h->t0 = t0;
  ((hipStream_t)stream)->push([data, bytes]() { std::memset(data, 0, bytes); });
  return JEFI_OK;
}

jefi_status jefi_history_push(jefi_history* h, const jefi_grid* src, const void* slice, void* stream) {
  const size_t sb = (size_t)4 * cells(src) * (h->dtype == JEFI_F64 ? 8 : 4);
  h->newest += 1;
  void* dst = (char*)h->data + (size_t)(h->newest % h->capacity) * sb;
  ((hipStream_t)stream)->push([dst, slice, sb]() { std::memcpy(dst, slice, sb); });
  return JEFI_OK;
}

// E[0][o] = sum over the window (oldest first, j = 0..nt-1) of (j + 1) * rho
// of cell 0 in that slot; E[1][o] = newest step; E[2][o] = t; B[c][o] = o.
std::atomic<unsigned> g_last_batch_flags{0};

jefi_status jefi_eval_batch(const jefi_problem* probs, int32_t n, const jefi_options* opt, void* stream) {
  g_last_batch_flags.store(opt->flags);
  int held = -1;
  {
    std::lock_guard<std::mutex> lk(g_gate_mu);
    const int idx = g_launched++;
    if (idx >= g_gate_base && idx < g_gate_base + g_gate_n) held = idx - g_gate_base;
  }
  if (held >= 0)
    ((hipStream_t)stream)->push([held]() {
      std::unique_lock<std::mutex> lk(g_gate_mu);
      g_gate_cv.wait(lk, [held]() { return g_gate_released > held; });
    });
  // the whole batch "runs" for a while before it reads any ring, which
  // leaves room for a later batch to overtake it if nothing orders them
  const int sleep_us = g_eval_sleep_us;
  if (sleep_us) ((hipStream_t)stream)->push([sleep_us]() { std::this_thread::sleep_for(std::chrono::microseconds(sleep_us)); });
  for (int i = 0; i < n; ++i) {
    const jefi_problem q = probs[i];
    const bool f64 = opt->precision == JEFI_PREC_F64;
    ((hipStream_t)stream)->push([q, f64]() {
      const long long ns = cells(&q.src), no = cells(&q.obs);
      const size_t sb = (size_t)4 * ns;
      double acc = 0.0;
      for (int j = 0; j < q.nt; ++j) {
        const long long step = q.hist.newest - q.nt + 1 + j;
        const size_t slot = (size_t)(step % q.hist.capacity);
        const double v = f64 ? ((const double*)q.hist.data)[slot * sb] : ((const float*)q.hist.data)[slot * sb];
        acc += (double)(j + 1) * v;
      }
      for (long long o = 0; o < no; ++o) {
        const double e[3] = {acc, (double)q.hist.newest, q.t};
        for (int c = 0; c < 3; ++c) {
          if (q.out.dtype == JEFI_F64) {
            ((double*)q.out.E)[c * no + o] = e[c];
            ((double*)q.out.B)[c * no + o] = (double)o;
          } else {
            ((float*)q.out.E)[c * no + o] = (float)e[c];
            ((float*)q.out.B)[c * no + o] = (float)o;
          }
        }
      }
    });
  }
  return JEFI_OK;
}

}  // extern "C"

namespace jefi {
int device_cus() { return 256; }
bool create_stream_on_cus(hipStream_t* s, int first_cu, int n_cus) {
  if (first_cu < 0 || n_cus < 1 || first_cu + n_cus > 256) return false;
  *s = new MockStream();
  return true;
}
std::atomic<int> g_express_grid_cus{0};  // grid of the last express-lane batch
jefi_status eval_batch_on_cus(const jefi_problem* probs, int32_t n, const jefi_options* opt, void* stream,
                              int grid_cus) {
  g_express_grid_cus.store(grid_cus);
  return jefi_eval_batch(probs, n, opt, stream);
}
hipError_t launch_ingest_slots(const void* hist, void* ring, const GridD& src, int, int, int n_slots, int is_f64,
                               hipStream_t s) {
  const size_t bytes = (size_t)n_slots * 4 * (size_t)src.n[0] * src.n[1] * src.n[2] * (is_f64 ? 8 : 4);
  const int sleep_us = g_ingest_sleep_us;
  s->push([hist, ring, bytes, sleep_us]() {
    if (sleep_us) std::this_thread::sleep_for(std::chrono::microseconds(sleep_us));
    std::memcpy(ring, hist, bytes);
  });
  return hipSuccess;
}
}  // namespace jefi

int jefi_mock_express_grid() { return jefi::g_express_grid_cus.load(); }

int jefi_mock_batches_launched() {
  std::lock_guard<std::mutex> lk(g_gate_mu);
  return g_launched;
}

void jefi_mock_hold_next_batches(int n) {
  std::lock_guard<std::mutex> lk(g_gate_mu);
  g_gate_base = g_launched;
  g_gate_n = n;
  g_gate_released = 0;
}

void jefi_mock_release_batch() {
  std::lock_guard<std::mutex> lk(g_gate_mu);
  ++g_gate_released;
  g_gate_cv.notify_all();
}
