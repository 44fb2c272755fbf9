/*
 * libjefi -- evaluation of the discretised Jefimenko equations on gfx950.
 *
 * For every observation point r of a uniform grid at time t the library sums,
 * over every cell r' of a uniform source grid, the charge density rho and the
 * current density J and their backward-difference time derivatives, read at
 * the retarded time t_r = t - |r - r'|/c from a stored history of source
 * slices, weighted by the 1/R^3, 1/R^2 and 1/R kernels, and returns E and B
 * (paper: section "GPU implementation of Jefimenko's equations", the
 * discretised equations for E, B and t_r; units: rationalised
 * Lorentz-Heaviside, section "Jefimenko's equations").
 *
 *   E(r,t) =  1/(4 pi) sum [ d rho/R^3 + d rho_dot/R^2 - J_dot/R ] dOmega
 *   B(r,t) = -1/(4 pi) sum [ d x J/R^3 + d x J_dot/R^2 ] dOmega
 *
 * Conventions shared by every entry point:
 *   - A grid's cell (i,j,k) has its centre at origin + (i,j,k)*spacing
 *     (evaluated in FP64 as a multiply then an add); linear cell index
 *     i + n0*(j + n1*k) (x fastest).  dOmega is the source cell volume.
 *   - History step s sits at time t0 + s*dt.  An evaluation with nt slices
 *     uses steps newest-nt+1 .. newest.  Between slices values are linear in
 *     time; the derivative is the same linear interpolation of the
 *     slice-wise backward differences (h_k - h_(k-1))/dt.  Slices before the
 *     oldest used step count as zero.
 *   - Slice index: with a = (t - t0)/dt - (newest - nt + 1) split as
 *     a = a_i + a_f (a_i = floor(a)) on the host in FP64, each pair uses
 *     k = a_i + floor(u), f = u - floor(u), u = a_f - R/(c dt), where
 *     R = sqrt((dx*dx + dy*dy) + dz*dz) of d = r - r' -- all FP64 without
 *     contraction.  This decision is bit-exact in both precisions.
 *   - Coarse screening: a pair with |dx| <= s_x, |dy| <= s_y, |dz| <= s_z
 *     (and any pair with R == 0) contributes nothing.
 *   - Device pointers are HIP device memory on the current device; the
 *     library never frees caller memory.  `stream` is a hipStream_t passed as
 *     void* (NULL = the null stream).  Calls are stream-ordered and
 *     asynchronous: outputs are valid once the stream reaches the call.
 *   - Every function returns jefi_status; on an error nothing is written to
 *     the outputs and jefi_last_error() explains (thread-local text).
 *     JEFI_EDEVICE after a HIP failure is sticky for the process.
 *   - Threads: any number of host threads may call the library on different
 *     streams at once.  The library keeps scratch memory per (device,
 *     stream), so calls on one stream must come from one host thread at a
 *     time (as stream order already implies).  The serving loop (below) is
 *     safe to use from any thread.
 */
#ifndef LIBJEFI_H
#define LIBJEFI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  JEFI_OK = 0,
  JEFI_PENDING = 1,      /* server request not finished yet */
  JEFI_EINVAL = -1,      /* bad argument or descriptor */
  JEFI_ENOMEM = -2,      /* device allocation failed */
  JEFI_EDEVICE = -3,     /* a HIP call failed (sticky) */
  JEFI_EBUSY = -4,       /* server queue full: retry */
  JEFI_ENOENT = -5,      /* unknown ticket or session */
  JEFI_ETOOLARGE = -6    /* can never fit the memory budget */
} jefi_status;

typedef enum { JEFI_F32 = 0, JEFI_F64 = 1 } jefi_dtype;

/* JEFI_PREC_F64: all pair arithmetic in FP64 (needs an F64 history).
 * JEFI_PREC_F32_COMP: FP32 pair arithmetic (rsqrt, FMA) with compensated
 * accumulation, FP64 for the slice index near slice boundaries and for the
 * final per-point reduction (needs an F32 history).  The FP32 arithmetic
 * measures lengths in units of c*dt, so separations must stay well inside
 * the FP32 range in those units (roughly 1e-18 to 1e18 c*dt; squares are
 * formed). */
typedef enum { JEFI_PREC_F64 = 0, JEFI_PREC_F32_COMP = 1 } jefi_precision;

/* Uniform grid: n cells per axis (n >= 1 each, or all three 0 for an empty
 * grid), centre of cell 0 and spacing (spacing > 0, finite). */
typedef struct {
  int32_t n[3];
  double origin[3];
  double spacing[3];
} jefi_grid;

/* Resident source history: a ring of `capacity` slices in DEVICE memory.
 * Slot layout (the library's, written by jefi_history_push): per slot,
 * bricks of 2x2x2 source cells in brick order bx + nbx*(by + nby*bz)
 * (nbx = ceil(n0/2) ...), inside a brick cell cx + 2*cy + 4*cz, and per cell
 * the 4 channels rho, Jx, Jy, Jz contiguous in `dtype`; cells beyond the grid
 * edge are zero.  Step s lives in slot s % capacity.  `newest` is the
 * absolute step of the newest pushed slice (-1 = none), `t0` the time of
 * step 0.  The caller owns `data` (jefi_history_bytes() bytes). */
typedef struct {
  void* data;
  int32_t dtype;       /* jefi_dtype */
  int32_t capacity;
  int64_t newest;
  double t0;
} jefi_history;

/* Output fields in DEVICE memory: E and B each [3][n_obs] of `dtype`,
 * component-major (x, y, z), points in linear order. */
typedef struct {
  void* E;
  void* B;
  int32_t dtype;       /* jefi_dtype */
} jefi_fields;

typedef struct {
  double c;              /* speed of light, > 0 (default 1) */
  double screen[3];      /* screening half-widths, used when screen_set != 0 */
  int32_t screen_set;    /* 0: half the source spacing per axis (default) */
  int32_t precision;     /* jefi_precision (default JEFI_PREC_F32_COMP) */
  uint32_t flags;        /* at most one JEFI_FLAG_INDEX_* value, at most one of
                            JEFI_FLAG_DERIV_SLOPE and JEFI_FLAG_TIME_CUBIC, and at
                            most one of JEFI_FLAG_PAST_HOLD and JEFI_FLAG_PAST_CUT;
                            other bits and combinations are rejected (EINVAL) */
  int32_t tile_config;   /* launch shape: 0 = automatic (autotuned table, else a size
                            rule: 8x8x8 tiles from 32768 observation points on, taken
                            over the mean problem of a batch), 1 = 8x8x8 observation
                            tiles (512 threads), 2 = 8x8x4 tiles (256 threads), 3 = the
                            size rule per problem (a batch of large and small problems
                            then runs one persistent launch per tile) */
  int32_t reserve_cus;   /* jefi_eval_batch only: the persistent launch leaves this many
                            compute units' worth of workgroup slots free (at most half the
                            device), so that launches on other streams can start while it
                            runs; 0 (default) = every slot; 0 .. 1024, else EINVAL */
} jefi_options;

/* How the FP32 path reaches the canonical FP64 slice index of each pair
 * (both give the same indices and results; only speed differs).  Default:
 * chosen per call from the expected share of pairs within the FP32 rounding
 * band of an integer retarded position (large on aligned grids whose
 * spacing is a multiple of c*dt). */
enum {
  JEFI_FLAG_INDEX_GUARD = 1, /* decide in FP32, redo in FP64 only inside the guard band */
  JEFI_FLAG_INDEX_TABLE = 2  /* decide every pair by its FP64 r2 against a threshold table */
};

/* Readings of the time stencil.  The paper takes time derivatives as the
 * backward difference over one step and its sources vanish before they are
 * switched on (section "GPU implementation of Jefimenko's equations" and the
 * source definitions of the constant and sinusoidal tests); between slices
 * the library interpolates linearly.  By default the derivative at t_r is
 * therefore the linear interpolation of the slice-wise backward differences
 * (h_k - h_(k-1))/dt, and the history is zero before the oldest slice of the
 * window (pairs whose stencil lies wholly before it contribute nothing).
 * These flags select the alternatives, in any combination with each other
 * (except JEFI_FLAG_DERIV_SLOPE with JEFI_FLAG_TIME_CUBIC, and
 * JEFI_FLAG_PAST_HOLD with JEFI_FLAG_PAST_CUT) and with an index flag:
 *   JEFI_FLAG_DERIV_SLOPE: the derivative is the slope of the linear
 *     interpolant on the interval that holds t_r, (h_(k+1) - h_k)/dt.
 *   JEFI_FLAG_PAST_HOLD: before the oldest slice of the window the history
 *     holds that slice's values (sources constant before the window); no
 *     pair is then culled as lying in the past, so every unscreened pair is
 *     computed.
 *   JEFI_FLAG_TIME_CUBIC: value and time derivative at t_r come from the
 *     cubic through slices k-2, k-1, k, k+1 (exact for sources cubic in
 *     time).  Its nodes end at k+1, like the linear stencil's, so the same
 *     pairs are live and no slice after the newest is read.
 *   JEFI_FLAG_PAST_CUT: the history starts at the oldest slice of the
 *     window: a pair whose retarded time precedes it (k < 0) contributes
 *     nothing, and stencils that reach before it read its values, so no time
 *     derivative is taken across the start.  For sources switched on at the
 *     oldest slice this drops the shell that the step's derivative puts on
 *     the light cone; it is the reading under which the constant-source
 *     comparison (section "Constant sources") shows the paper's field scale.
 * None of them changes the slice index k, the screening decision or the
 * fingerprint (jefi_slice_fingerprint, jefi_slice_index_dump). */
enum {
  JEFI_FLAG_DERIV_SLOPE = 4,
  JEFI_FLAG_PAST_HOLD = 8,
  JEFI_FLAG_TIME_CUBIC = 16,
  JEFI_FLAG_PAST_CUT = 32
};

const char* jefi_version(void);
const char* jefi_last_error(void);
void jefi_options_default(jefi_options* opt);

/* ---- source history ------------------------------------------------------
 * The stored history of rho and J slices the sums read at retarded times
 * (paper, section "Parameter dependence": rho and J are kept in GPU memory
 * for all relevant times and are not released between calls). */

/* Bytes of a ring of `capacity` slices for `src` in `dtype`; 0 on bad input. */
uint64_t jefi_history_bytes(const jefi_grid* src, int32_t capacity, int32_t dtype);

/* Fill in `h` for a caller-owned device buffer of `bytes` bytes and zero it
 * (stream-ordered).  newest = -1.  EINVAL on a short buffer or bad sizes. */
jefi_status jefi_history_init(jefi_history* h, void* data, uint64_t bytes, const jefi_grid* src,
                              int32_t capacity, int32_t dtype, double t0, void* stream);

/* Append one slice: `slice` is DEVICE memory [4][n_src] of h->dtype in linear
 * cell order (channel 0 = rho, 1..3 = Jx, Jy, Jz).  It becomes step
 * h->newest + 1 (written to its slot in the library layout, overwriting the
 * oldest step once the ring is full); h->newest is incremented on return. */
jefi_status jefi_history_push(jefi_history* h, const jefi_grid* src, const void* slice,
                              void* stream);

/* ---- field evaluation (section "GPU implementation": the discretised E, B
 * and retarded-time equations, one result per observation point) ----------
 * E and B at time t on the observation grid from the last `nt` steps of the
 * history (1 <= nt <= min(capacity, newest + 1)); t must not lie after the
 * newest step (beyond FP64 rounding of t): EINVAL otherwise.  `opt` NULL =
 * defaults.  The history dtype must match the precision (F32 for
 * F32_COMP, F64 for F64); `out->dtype` may be either.  An empty observation
 * grid is a no-op; an empty source grid gives zero fields. */
jefi_status jefi_eval_fields(const jefi_grid* src, const jefi_history* hist, double dt, int32_t nt,
                             const jefi_grid* obs, double t, const jefi_fields* out,
                             const jefi_options* opt, void* stream);

/* jefi_eval_fields for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid it).
 * Same arguments, same validation and errors; it calls no hipMalloc or
 * hipFree.  Its scratch (threshold table and FP64 split partials) is one
 * fixed array of 128 MiB per GPU inside the library, held until the
 * process ends.  The split count is that of jefi_eval_fields, capped so the
 * partials fit (one split needs none), so the fields agree with
 * jefi_eval_fields within the stated tolerances (not bit for bit when the
 * cap applies); ETOOLARGE if a plan would still not fit.  Every call on a
 * GPU shares that array, and nothing in it needs to start at zero: calls
 * that overlap on one GPU (several streams or threads) race and must be
 * serialised by the caller. */
jefi_status jefi_eval_fields_noalloc(const jefi_grid* src, const jefi_history* hist, double dt, int32_t nt,
                                     const jefi_grid* obs, double t, const jefi_fields* out,
                                     const jefi_options* opt, void* stream);

/* ---- batched evaluation ---------------------------------------------------
 * Many independent problems of uneven sizes in one persistent launch:
 * workgroups pull (problem, observation tile, source split) items, heaviest
 * first, from a device queue; the launch sequence (queue reset, threshold
 * tables, persistent pair kernel, split reduction) is a hipGraph built once
 * per stream workspace and replayed.  Each problem means what
 * jefi_eval_fields means for the same arguments (results agree within the
 * precision's tolerance; FP64 split sums may associate differently). */
typedef struct {
  jefi_grid src;
  jefi_history hist;     /* each problem's own resident history */
  double dt;
  int32_t nt;
  jefi_grid obs;
  double t;
  jefi_fields out;       /* each problem's own DEVICE outputs (must not overlap) */
} jefi_problem;

/* All problems share `opt` (precision, c, screening rule, launch shape);
 * 0 <= n <= 65536.  Stream-ordered like jefi_eval_fields.  Validation of
 * every problem precedes any device work: on EINVAL nothing is launched.
 * The library keeps a per-(device, stream) workspace (descriptor tables,
 * split partials, two pinned staging buffers and the graph): a call may wait
 * for the upload of the call before last on the same stream. */
jefi_status jefi_eval_batch(const jefi_problem* probs, int32_t n, const jefi_options* opt, void* stream);

/* Autotuner.  A launch configuration is an observation tile (8x8x8 or
 * 8x8x4), an FP32 slice-index mode (guard band or threshold table: the
 * same indices, different speed) and a work granularity (half, default or
 * twice the workgroup target of a single launch; 6, 12 or 24 work items per
 * workgroup slot of a batch).  Every trial is `reps` timed runs after a
 * warm-up on `stream`; the problems' outputs are written.
 *   n == 1: times every configuration the problem admits (the 8x8x4 tile
 *     only with 32-slot windows) and records the fastest for its size
 *     class: precision, staging window class (32, 64 or 128 slots per cell,
 *     or chunked), log2 observation points, log2 pairs.
 *   n > 1: a greedy search from the untuned batch: each size class of
 *     instances, heaviest first, tries the other tile (instances of one
 *     batch may then run in two persistent launches, one per tile); then
 *     the batch tries both index modes and the other granularities.  A
 *     change is kept when it is at least 1 % faster.  Records the tile per
 *     instance size class (within batches) and the batch's index mode and
 *     granularity for its class (precision, log2 instances, log2 pairs).
 * tile_config = 0 then uses the table (JEFI_FLAG_INDEX_* flags still fix
 * the index mode); the table persists in the file named by
 * $JEFI_TUNE_CACHE when that is set.  best_config = the chosen
 * configuration (the batch-level one for n > 1) packed as
 * tile | index mode << 2 | granularity << 4 (tile 1 = 8x8x8, 2 = 8x8x4,
 * 0 = size rule; index 1 = guard, 2 = table, 0 = estimated; granularity
 * 0 = default, 1 = coarser, 2 = finer); best_ms = its time per run.
 * Either may be NULL. */
jefi_status jefi_autotune(const jefi_problem* probs, int32_t n, const jefi_options* opt, int32_t reps,
                          void* stream, int32_t* best_config, double* best_ms);

/* ---- per-step coupling with a producer ------------------------------------
 * The paper's per-step use (section "Parameter dependence", Table 4 upper
 * panel; the transport-code coupling of the introduction): every time step
 * a producer hands the new rho/J slice over and takes E and B of that step
 * back.  A coupler runs each step as: slice to the device (copy-in stream),
 * push and evaluation at the new step's time (compute stream), E and B back
 * to pinned host memory (copy-out stream).  Two staging slots take
 * alternate steps, so the next step's slice travels while a step evaluates
 * and a step's fields travel while the next one evaluates.  The coupler
 * owns its streams and staging (pinned host and device memory for two
 * slices and two sets of fields); the caller owns the history, which the
 * coupler pushes into (hist->newest advances at each step call).  Use it
 * from one thread. */
typedef struct jefi_coupler jefi_coupler;

/* Evaluations on `obs` from the last min(nt, pushed) steps of `hist`, with
 * `opt` (NULL = defaults; its precision must match the history dtype) and
 * fields of out_dtype.  EINVAL on bad arguments, ENOMEM when the staging
 * cannot be allocated. */
jefi_status jefi_coupler_create(const jefi_grid* src, jefi_history* hist, double dt, int32_t nt,
                                const jefi_grid* obs, const jefi_options* opt, int32_t out_dtype,
                                jefi_coupler** out);

/* Enqueue the next step (absolute step hist->newest + 1, returned in *step):
 * slice = [4][n_src] of the history dtype, in HOST memory (slice_on_host = 1:
 * copied into pinned staging before return; `stream` unused) or DEVICE
 * memory (0: the push waits for the work enqueued on the producer's
 * `stream` (a hipStream_t, NULL = the null stream) so far, and reads the
 * slice then, so it must stay unchanged until the step is collected).
 * Asynchronous.  EBUSY while the step two back (same slot) has not been
 * collected; EINVAL/EDEVICE as jefi_history_push and jefi_eval_fields. */
jefi_status jefi_coupler_step(jefi_coupler* c, const void* slice, int32_t slice_on_host, void* stream,
                              int64_t* step);

/* Wait for `step` and copy its E and B (HOST [3][n_obs] of out_dtype each).
 * ENOENT if that step is not waiting to be collected. */
jefi_status jefi_coupler_collect(jefi_coupler* c, int64_t step, void* E, void* B);

/* Waits for all enqueued work, frees the coupler. */
jefi_status jefi_coupler_destroy(jefi_coupler* c);

/* ---- serving loop ----------------------------------------------------------
 * Field evaluations of many sessions (a time-stepping source each) arrive at
 * any time.  Each session keeps its history resident in a caller-provided
 * device arena (the HBM budget); each request pushes the session's next
 * slice and evaluates on its own observation grid: the paper's per-step use
 * (section "Parameter dependence", Table 4 upper panel: one slice to the
 * device, one evaluation, E and B back, per time step).  What a session
 * occupies follows the paper's memory count (same section, the equation for
 * N: (lts + 1) slices of 4 values per source cell plus 6 per observation
 * point); admission charges the ring, the slice staging and the outputs
 * against the arena in the same way.  A scheduler thread
 * admits requests in arrival order as arena bytes and batch slots free up
 * (evicting idle sessions least-recently-used first and re-uploading their
 * history from a host copy when they return) and launches them as batched
 * evaluations on several streams, so new arrivals start while earlier
 * batches still run (continuous batching).  One request per session is on
 * the device at a time; a session's requests run in submission order.
 * Per-request timestamps give latency percentiles.  The per-stream batch
 * workspace (descriptor tables, split partials) lies outside the arena. */
typedef struct jefi_server jefi_server;

typedef struct {
  void* arena;              /* DEVICE memory the server may use (histories, slices, outputs) */
  uint64_t arena_bytes;
  uint64_t pinned_bytes;    /* host staging pool (0 = 256 MiB) */
  int32_t precision;        /* jefi_precision of every evaluation */
  int32_t max_inflight;     /* batches on the device at once, 1..8 (0 = 2) */
  int32_t max_batch;        /* requests per batch (0 = 256) */
  int32_t max_queue;        /* waiting requests before submit returns EBUSY (0 = 65536) */
  uint32_t flags;           /* jefi_options.flags of every evaluation (index mode, time-stencil
                               readings); 0 = defaults; invalid combinations: EINVAL at create */
  int32_t reserve_cus;      /* jefi_options.reserve_cus of every batch: with max_inflight >= 3,
                               small requests then start beside large ones instead of waiting
                               for them (lower tail latency, some throughput); 0 = none */
  int32_t express_cus;      /* compute units of the express lane (0 = 16; at most half the
                               device; 0 .. 1024, else EINVAL) */
  uint64_t express_pairs;   /* 0 = no express lane.  Else requests of at most this many pairs
                               (n_src * n_obs) run in an express lane: one more stream whose
                               batches use express_cus compute units that the other batches
                               (max_inflight streams) leave free, through CU-masked streams
                               where the runtime allows, else through launch sizes; a small
                               request then never waits behind a persistent launch that holds
                               the device.  Each session's requests still run in order. */
} jefi_server_config;

typedef struct {
  uint64_t session;
  const void* new_slice;    /* HOST [4][n_src] (float for F32_COMP, double for F64), or NULL;
                               copied before submit returns; pushed as the next step */
  jefi_grid obs;
  double t;                 /* NaN = the time of the newest step after the push */
  void* E;                  /* outputs [3][n_obs] of out_dtype: HOST memory when */
  void* B;                  /*   out_on_host, else DEVICE memory; valid once done */
  int32_t out_dtype;
  int32_t out_on_host;
} jefi_request;

typedef struct {
  int32_t status;           /* JEFI_PENDING, JEFI_OK or the request's error */
  int32_t batch_size;       /* requests in the batch it ran in */
  uint64_t t_submit_ns, t_admit_ns, t_start_ns, t_done_ns;  /* CLOCK_MONOTONIC */
  uint64_t pairs;           /* n_src * n_obs */
} jefi_result;

typedef struct {
  uint64_t submitted, completed, failed, batches, max_batch;
  uint64_t evictions;          /* idle rings dropped from the arena to make room */
  uint64_t rematerialisations; /* rings brought back from their host shadow after an eviction */
  uint64_t arena_bytes, arena_used, arena_high_water;
  uint64_t pairs;
  uint64_t express_batches;  /* batches run in the express lane */
  uint64_t express_cus;      /* its compute units (0 without one) */
  uint64_t cu_masked;        /* 1 when the lanes run on CU-masked streams */
} jefi_server_stats;

/* Start a server on the current device.  EINVAL on a bad config, ENOMEM
 * when the pinned pool cannot be allocated. */
jefi_status jefi_server_create(const jefi_server_config* cfg, jefi_server** out);

/* A session: source grid, ring capacity, evaluation window (slices used,
 * 1 <= window <= capacity), time axis (step s at t0 + s*dt), and optionally
 * its first init_nt steps (HOST [init_nt][4][n_src], oldest first; copied
 * before return).  The ring is uploaded into the arena before return when
 * there is room (idle sessions may be evicted for it), else when its first
 * request is admitted.  EINVAL for a used id or bad sizes; ETOOLARGE when
 * the ring can never fit the arena; EDEVICE on a HIP failure. */
jefi_status jefi_server_open_session(jefi_server* sv, uint64_t session, const jefi_grid* src, int32_t capacity,
                                     int32_t window, double t0, double dt, const void* init_history,
                                     int32_t init_nt);

/* Non-blocking.  ENOENT: unknown session; EBUSY: queue full (retry);
 * ETOOLARGE: the request can never fit the arena or the pinned pool (its
 * worst case holds the ring, the staged host shadow, the slice and the
 * outputs at once);
 * EINVAL: bad grid or outputs.  A request whose time lies after its
 * session's newest step fails with EINVAL when it is admitted. */
jefi_status jefi_server_submit(jefi_server* sv, const jefi_request* rq, uint64_t* ticket);

/* JEFI_PENDING while running; once done returns the request's status (the
 * ticket is then released), res filled either way.  ENOENT: unknown ticket. */
jefi_status jefi_server_poll(jefi_server* sv, uint64_t ticket, jefi_result* res);

/* Blocks until the ticket is done, then as poll.  If another thread polls
 * or waits the same ticket and releases it first, returns ENOENT. */
jefi_status jefi_server_wait(jefi_server* sv, uint64_t ticket, jefi_result* res);

/* Frees an idle session's ring.  EBUSY while it has queued or running requests. */
jefi_status jefi_server_close_session(jefi_server* sv, uint64_t session);

jefi_status jefi_server_get_stats(jefi_server* sv, jefi_server_stats* out);

/* Runs every queued request to completion, then stops and frees the
 * server; returns JEFI_EDEVICE if a device failure occurred. */
jefi_status jefi_server_destroy(jefi_server* sv);

/* ---- slice-decision diagnostics ------------------------------------------
 * The integer decisions the field kernels take, exposed for bit-exact
 * checks against an independent implementation. */

/* Per-pair decision of the device index code, DEVICE int32 out[n_obs][n_src]:
 * INT32_MIN = screened (or R == 0), -2 = stencil wholly before the oldest
 * slice (k < -1), else k in [-1, nt-1].  `precision` picks the FP32 guarded
 * or the FP64 device sequence.  For small problems (n_obs*n_src <= 2^31). */
jefi_status jefi_slice_index_dump(const jefi_grid* src, int32_t nt, double dt, int64_t newest,
                                  double t0, const jefi_grid* obs, double t,
                                  const jefi_options* opt, int32_t* out, void* stream);

/* Per-observation-point fingerprint computed by the field kernel's own path
 * (same tiling, staging windows, culling and index code), DEVICE int64
 * fp[n_obs][4]: number of pairs that are neither screened nor wholly before
 * the oldest slice, the sum of their k, the sum of k*(s+1) (wrapping, s =
 * linear source index), and the number of screened pairs (all of them, also
 * those wholly before the oldest slice). */
jefi_status jefi_slice_fingerprint(const jefi_grid* src, const jefi_history* hist, double dt,
                                   int32_t nt, const jefi_grid* obs, double t,
                                   const jefi_options* opt, int64_t* fp, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LIBJEFI_H */
