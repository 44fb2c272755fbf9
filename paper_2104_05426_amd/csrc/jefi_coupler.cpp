// Per-step coupling with a time-stepping producer: each step hands one new
// source slice and takes E and B of that step back, and the copies of one
// step overlap the evaluation of its neighbours.  Three streams:
//   copy-in:  slice s (pinned host, or the caller's device buffer) -> device;
//   compute:  push slice s into the ring, evaluate E and B at its time;
//   copy-out: E and B of step s -> pinned host.
// Two slots of staging buffers take alternate steps, so step s + 1's slice
// travels while step s evaluates and step s's fields travel while step s + 1
// evaluates.  Events order every reuse of a slot's buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "../../include/libjefi.h"
#include "jefi_internal.h"

namespace {

struct Slot {
  void* pin_in = nullptr;    // pinned staging of a host slice
  void* dev_in = nullptr;    // device copy of the slice
  void* pin_out = nullptr;   // pinned E then B
  void* dev_out = nullptr;   // device E then B
  hipEvent_t in_ready = nullptr;   // slice on the device (copy-in or producer stream)
  hipEvent_t pushed = nullptr;     // push done: dev_in (or the caller's buffer) free again
  hipEvent_t evaluated = nullptr;  // E and B on the device (compute stream)
  hipEvent_t out_ready = nullptr;  // E and B in pin_out; dev_out free again
  long long step = -1;             // step the slot holds, -1 = none
  bool collected = true;
  bool used = false;               // its events have been recorded at least once
};

}  // namespace

struct jefi_coupler {
  jefi_grid src{}, obs{};
  jefi_history* hist = nullptr;
  double dt = 0.0;
  int32_t nt = 0;
  jefi_options opt{};
  int32_t out_dtype = JEFI_F32;
  size_t slice_bytes = 0, out_bytes = 0;
  long long n_obs = 0;
  hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
  Slot slot[2];
};

namespace {

void release(jefi_coupler* c) {
  for (hipStream_t s : {c->s_in, c->s_comp, c->s_out})
    if (s) (void)hipStreamSynchronize(s);
  for (Slot& sl : c->slot) {
    if (sl.pin_in) (void)hipHostFree(sl.pin_in);
    if (sl.pin_out) (void)hipHostFree(sl.pin_out);
    if (sl.dev_in) (void)hipFree(sl.dev_in);
    if (sl.dev_out) (void)hipFree(sl.dev_out);
    for (hipEvent_t e : {sl.in_ready, sl.pushed, sl.evaluated, sl.out_ready})
      if (e) (void)hipEventDestroy(e);
  }
  for (hipStream_t s : {c->s_in, c->s_comp, c->s_out})
    if (s) (void)hipStreamDestroy(s);
  delete c;
}

long long cells(const jefi_grid& g) { return (long long)g.n[0] * g.n[1] * g.n[2]; }

}  // namespace

extern "C" {

jefi_status jefi_coupler_create(const jefi_grid* src, jefi_history* hist, double dt, int32_t nt,
                                const jefi_grid* obs, const jefi_options* opt, int32_t out_dtype,
                                jefi_coupler** out) {
  if (jefi::device_failed()) return jefi::report_error(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  if (!src || !hist || !obs || !out) return jefi::report_error(JEFI_EINVAL, "coupler: NULL argument");
  if (!hist->data || (hist->dtype != JEFI_F32 && hist->dtype != JEFI_F64))
    return jefi::report_error(JEFI_EINVAL, "coupler: history has no data or a bad dtype");
  if (nt < 1 || nt > hist->capacity) return jefi::report_error(JEFI_EINVAL, "coupler: nt must be in [1, capacity]");
  if (!(dt > 0.0)) return jefi::report_error(JEFI_EINVAL, "coupler: dt must be > 0");
  if (out_dtype != JEFI_F32 && out_dtype != JEFI_F64) return jefi::report_error(JEFI_EINVAL, "coupler: out_dtype");
  for (int a = 0; a < 3; ++a)
    if (src->n[a] < 1 || obs->n[a] < 1) return jefi::report_error(JEFI_EINVAL, "coupler: empty grid");
  jefi_coupler* c = new jefi_coupler();
  c->src = *src;
  c->obs = *obs;
  c->hist = hist;
  c->dt = dt;
  c->nt = nt;
  if (opt)
    c->opt = *opt;
  else
    jefi_options_default(&c->opt);
  c->out_dtype = out_dtype;
  c->slice_bytes = (size_t)4 * (size_t)cells(*src) * (hist->dtype == JEFI_F64 ? 8 : 4);
  c->n_obs = cells(*obs);
  c->out_bytes = (size_t)6 * (size_t)c->n_obs * (out_dtype == JEFI_F64 ? 8 : 4);
  hipError_t e = hipSuccess;
  for (hipStream_t* s : {&c->s_in, &c->s_comp, &c->s_out})
    if (e == hipSuccess) e = hipStreamCreateWithFlags(s, hipStreamNonBlocking);
  for (Slot& sl : c->slot) {
    if (e == hipSuccess) e = hipHostMalloc(&sl.pin_in, c->slice_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&sl.pin_out, c->out_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&sl.dev_in, c->slice_bytes);
    if (e == hipSuccess) e = hipMalloc(&sl.dev_out, c->out_bytes);
    for (hipEvent_t* ev : {&sl.in_ready, &sl.pushed, &sl.evaluated, &sl.out_ready})
      if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release(c);
    return jefi::report_error(JEFI_ENOMEM, "coupler: staging buffers, streams or events could not be created");
  }
  *out = c;
  return JEFI_OK;
}

jefi_status jefi_coupler_step(jefi_coupler* c, const void* slice, int32_t slice_on_host, void* stream,
                              int64_t* step) {
  if (jefi::device_failed()) return jefi::report_error(JEFI_EDEVICE, "an earlier HIP failure is sticky");
  if (!c || !slice) return jefi::report_error(JEFI_EINVAL, "coupler step: NULL argument");
  const long long s = c->hist->newest + 1;
  Slot& sl = c->slot[s & 1];
  if (!sl.collected)
    return jefi::report_error(JEFI_EBUSY, "coupler step: collect the step two back first (its slot is in use)");
  hipError_t e = hipSuccess;
  const void* dev_slice = slice;
  if (slice_on_host) {
    // the slot's previous copy-in must have left its pinned buffer
    if (sl.used && (e = hipEventSynchronize(sl.in_ready)) != hipSuccess) return jefi::report_hip(e, "coupler step");
    std::memcpy(sl.pin_in, slice, c->slice_bytes);
    // the device buffer is free once the push two steps back has read it
    if (sl.used && (e = hipStreamWaitEvent(c->s_in, sl.pushed, 0)) != hipSuccess)
      return jefi::report_hip(e, "coupler step");
    if ((e = hipMemcpyAsync(sl.dev_in, sl.pin_in, c->slice_bytes, hipMemcpyHostToDevice, c->s_in)) != hipSuccess)
      return jefi::report_hip(e, "coupler slice upload");
    if ((e = hipEventRecord(sl.in_ready, c->s_in)) != hipSuccess) return jefi::report_hip(e, "coupler step");
    if ((e = hipStreamWaitEvent(c->s_comp, sl.in_ready, 0)) != hipSuccess) return jefi::report_hip(e, "coupler step");
    dev_slice = sl.dev_in;
  } else {
    // a device slice of the caller's: the push waits for the work enqueued
    // on the producer's stream so far; the slot's staging stays unused
    if ((e = hipEventRecord(sl.in_ready, (hipStream_t)stream)) != hipSuccess)
      return jefi::report_hip(e, "coupler step");
    if ((e = hipStreamWaitEvent(c->s_comp, sl.in_ready, 0)) != hipSuccess) return jefi::report_hip(e, "coupler step");
  }
  // E and B of the step two back must have left the device buffer
  if (sl.used && (e = hipStreamWaitEvent(c->s_comp, sl.out_ready, 0)) != hipSuccess)
    return jefi::report_hip(e, "coupler step");
  jefi_status st = jefi_history_push(c->hist, &c->src, dev_slice, c->s_comp);
  if (st != JEFI_OK) return st;
  if ((e = hipEventRecord(sl.pushed, c->s_comp)) != hipSuccess) return jefi::report_hip(e, "coupler step");
  const size_t each = c->out_bytes / 2;
  const jefi_fields f{sl.dev_out, (char*)sl.dev_out + each, c->out_dtype};
  const int32_t nt = (int32_t)std::min<long long>(c->nt, c->hist->newest + 1);
  st = jefi_eval_fields(&c->src, c->hist, c->dt, nt, &c->obs, c->hist->t0 + (double)c->hist->newest * c->dt, &f,
                        &c->opt, c->s_comp);
  if (st != JEFI_OK) return st;
  if ((e = hipEventRecord(sl.evaluated, c->s_comp)) != hipSuccess) return jefi::report_hip(e, "coupler step");
  if ((e = hipStreamWaitEvent(c->s_out, sl.evaluated, 0)) != hipSuccess) return jefi::report_hip(e, "coupler step");
  if ((e = hipMemcpyAsync(sl.pin_out, sl.dev_out, c->out_bytes, hipMemcpyDeviceToHost, c->s_out)) != hipSuccess)
    return jefi::report_hip(e, "coupler field download");
  if ((e = hipEventRecord(sl.out_ready, c->s_out)) != hipSuccess) return jefi::report_hip(e, "coupler step");
  sl.step = s;
  sl.collected = false;
  sl.used = true;
  if (step) *step = s;
  return JEFI_OK;
}

jefi_status jefi_coupler_collect(jefi_coupler* c, int64_t step, void* E, void* B) {
  if (!c || !E || !B) return jefi::report_error(JEFI_EINVAL, "coupler collect: NULL argument");
  Slot& sl = c->slot[step & 1];
  if (sl.step != step || sl.collected)
    return jefi::report_error(JEFI_ENOENT, "coupler collect: that step is not waiting to be collected");
  const hipError_t e = hipEventSynchronize(sl.out_ready);
  if (e != hipSuccess) return jefi::report_hip(e, "coupler collect");
  const size_t each = c->out_bytes / 2;
  std::memcpy(E, sl.pin_out, each);
  std::memcpy(B, (const char*)sl.pin_out + each, each);
  sl.collected = true;
  return JEFI_OK;
}

jefi_status jefi_coupler_destroy(jefi_coupler* c) {
  if (!c) return JEFI_EINVAL;
  release(c);
  return jefi::device_failed() ? JEFI_EDEVICE : JEFI_OK;
}

}  // extern "C"
