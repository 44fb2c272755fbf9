// CPU test of the serving loop (jefi_server.cpp) against the host mock of
// the HIP runtime and of the library calls (server_mock.cpp): concurrent
// submitters, overlapping batches and per-session ordering of pushes and
// evaluations, eviction and re-materialisation, a full queue, requests that
// can never fit, session closing, timestamps.  Built with ThreadSanitizer.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "../../include/libjefi.h"

extern int g_eval_sleep_us;
extern int g_ingest_sleep_us;
extern std::atomic<unsigned> g_last_batch_flags;
int jefi_mock_express_grid();  // grid (compute units) of the last express-lane batch
int jefi_mock_batches_launched();
void jefi_mock_hold_next_batches(int n);  // the next n batches wait on their streams ...
void jefi_mock_release_batch();           // ... until released, one per call, in launch order

static std::atomic<int> g_fail{0};
#define CHECK(c)                                                \
  do {                                                          \
    if (!(c)) {                                                 \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);  \
      g_fail.fetch_add(1);                                      \
    }                                                           \
  } while (0)

namespace {

constexpr int kCap = 6;  // ring capacity = evaluation window: a push reuses the slot the previous window began with

jefi_grid grid(int n) {
  jefi_grid g;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = n;
    g.origin[a] = -0.5;
    g.spacing[a] = 1.0 / n;
  }
  return g;
}

float value(int sid, long long step) { return step < 0 ? 0.0f : (float)(1000 * sid + step); }

// What the mock evaluation reports for a session whose newest step is `newest`.
double expected(int sid, long long newest) {
  const long long nt = std::min<long long>(kCap, newest + 1);
  double acc = 0.0;
  for (long long j = 0; j < nt; ++j) acc += (double)(j + 1) * value(sid, newest - nt + 1 + j);
  return acc;
}

struct Session {
  int sid;
  int edge;
  long long next_step;
};

struct Pending {
  int sid;
  long long step;
  uint64_t ticket;
  std::vector<float> E, B;
  std::vector<float> slice;
};

jefi_server* make_server(size_t arena_bytes, int max_inflight, int max_queue, std::vector<char>& arena,
                         uint32_t flags = 0, uint64_t express_pairs = 0) {
  arena.assign(arena_bytes, 0);
  jefi_server_config cfg;
  std::memset(&cfg, 0, sizeof cfg);
  cfg.arena = arena.data();
  cfg.arena_bytes = arena_bytes;
  cfg.precision = JEFI_PREC_F32_COMP;
  cfg.max_inflight = max_inflight;
  cfg.max_batch = 64;
  cfg.max_queue = max_queue;
  cfg.flags = flags;
  cfg.express_pairs = express_pairs;
  jefi_server* sv = nullptr;
  CHECK(jefi_server_create(&cfg, &sv) == JEFI_OK);
  return sv;
}

void open_sessions(jefi_server* sv, std::vector<Session>& ss, int init_nt) {
  for (Session& s : ss) {
    const jefi_grid g = grid(s.edge);
    const long long n = (long long)s.edge * s.edge * s.edge;
    std::vector<float> h((size_t)init_nt * 4 * n);
    for (int k = 0; k < init_nt; ++k)
      for (long long i = 0; i < 4 * n; ++i) h[(size_t)k * 4 * n + i] = value(s.sid, k);
    CHECK(jefi_server_open_session(sv, (uint64_t)s.sid, &g, kCap, kCap, 0.0, 0.1, h.data(), init_nt) == JEFI_OK);
    s.next_step = init_nt;
  }
}

// Submit one request (retrying while the queue is full); returns 0 or the
// number of EBUSY answers seen.
int submit(jefi_server* sv, Session& s, Pending& p, int n_obs_edge) {
  const jefi_grid g = grid(s.edge);
  const long long n = (long long)s.edge * s.edge * s.edge;
  p.sid = s.sid;
  p.step = s.next_step++;
  p.slice.assign((size_t)4 * n, value(s.sid, p.step));
  const jefi_grid obs = grid(n_obs_edge);
  const long long no = (long long)n_obs_edge * n_obs_edge * n_obs_edge;
  p.E.assign((size_t)3 * no, NAN);
  p.B.assign((size_t)3 * no, NAN);
  jefi_request rq;
  std::memset(&rq, 0, sizeof rq);
  rq.session = (uint64_t)s.sid;
  rq.new_slice = p.slice.data();
  rq.obs = obs;
  rq.t = NAN;
  rq.E = p.E.data();
  rq.B = p.B.data();
  rq.out_dtype = JEFI_F32;
  rq.out_on_host = 1;
  int busy = 0;
  for (;;) {
    const jefi_status st = jefi_server_submit(sv, &rq, &p.ticket);
    if (st == JEFI_OK) break;
    CHECK(st == JEFI_EBUSY);
    if (st != JEFI_EBUSY) break;
    ++busy;
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
  (void)g;
  return busy;
}

void check_result(jefi_server* sv, Pending& p) {
  jefi_result res;
  CHECK(jefi_server_wait(sv, p.ticket, &res) == JEFI_OK);
  CHECK(res.status == JEFI_OK);
  CHECK(res.t_submit_ns <= res.t_admit_ns && res.t_admit_ns <= res.t_start_ns && res.t_start_ns <= res.t_done_ns);
  CHECK(res.batch_size >= 1);
  const size_t no = p.E.size() / 3;
  const double want = expected(p.sid, p.step);
  for (size_t o = 0; o < no; ++o) {
    // the weighted sums are integers below 2^24: exact in FP32
    if (p.E[o] != (float)want || p.E[no + o] != (float)p.step ||
        p.B[o] != (float)o) {
      std::printf("FAIL session %d step %lld point %zu: E0 %g want %g, E1 %g\n", p.sid, p.step, o, p.E[o], want,
                  p.E[no + o]);
      g_fail.fetch_add(1);
      return;
    }
  }
}

void concurrent_submitters() {
  std::vector<char> arena;
  jefi_server* sv = make_server(64 << 20, 3, 65536, arena);
  g_eval_sleep_us = 150;
  std::vector<Session> a = {{1, 3, 0}, {2, 4, 0}, {3, 5, 0}}, b = {{4, 6, 0}, {5, 2, 0}};
  open_sessions(sv, a, 3);
  open_sessions(sv, b, 2);
  auto worker = [&](std::vector<Session>& ss, unsigned seed, int count) {
    std::mt19937 rng(seed);
    std::vector<Pending> ps((size_t)count);
    for (int i = 0; i < count; ++i) submit(sv, ss[rng() % ss.size()], ps[(size_t)i], 1 + (int)(rng() % 3));
    for (Pending& p : ps) check_result(sv, p);
  };
  std::thread t1(worker, std::ref(a), 1u, 150);
  std::thread t2(worker, std::ref(b), 2u, 120);
  t1.join();
  t2.join();
  jefi_server_stats st;
  CHECK(jefi_server_get_stats(sv, &st) == JEFI_OK);
  CHECK(st.completed == 270 && st.failed == 0 && st.submitted == 270);
  CHECK(st.batches >= 1 && st.max_batch >= 2);
  std::printf("concurrent: %llu batches, largest %llu\n", (unsigned long long)st.batches,
              (unsigned long long)st.max_batch);
  CHECK(jefi_server_destroy(sv) == JEFI_OK);
}

// An express lane for requests of at most 64 pairs: on sessions of 2^3
// cells, 1^3 and 2^3 observation points go express, 3^3 and 4^3 regular;
// every session mixes both kinds, so each session's pushes and evaluations
// must keep their order across the lanes.
void express_lane() {
  std::vector<char> arena;
  jefi_server* sv = make_server(64 << 20, 2, 65536, arena, 0, 64);
  g_eval_sleep_us = 100;
  std::vector<Session> ss = {{21, 2, 0}, {22, 2, 0}, {23, 2, 0}};
  open_sessions(sv, ss, 3);
  std::mt19937 rng(7);
  std::vector<Pending> ps(120);
  int small = 0;
  for (int i = 0; i < 120; ++i) {
    const int edge = 1 + (int)(rng() % 4);  // 8 * edge^3 pairs: 8, 64 express; 216, 512 regular
    small += edge <= 2;
    submit(sv, ss[rng() % ss.size()], ps[(size_t)i], edge);
    // paced, so that the queue stays shorter than a batch (a backlog
    // switches the express lane off)
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
  for (Pending& p : ps) check_result(sv, p);
  jefi_server_stats st;
  CHECK(jefi_server_get_stats(sv, &st) == JEFI_OK);
  CHECK(st.completed == 120 && st.failed == 0);
  CHECK(st.express_batches >= 1 && st.express_batches < st.batches);
  CHECK(st.express_cus == 16 && st.cu_masked == 1);
  CHECK(jefi_mock_express_grid() == 16);
  std::printf("express lane: %d small of 120 requests, %llu of %llu batches express\n", small,
              (unsigned long long)st.express_batches, (unsigned long long)st.batches);
  CHECK(jefi_server_destroy(sv) == JEFI_OK);
}

void eviction() {
  // rings of 10^3 cells: 6 slots x 4 channels x 1000 x 4 B = 96 000 B, the
  // shadow staging as much again; room for about two sessions at once
  std::vector<char> arena;
  jefi_server* sv = make_server(330 * 1024, 2, 65536, arena);
  g_eval_sleep_us = 50;
  std::vector<Session> ss = {{11, 10, 0}, {12, 10, 0}, {13, 10, 0}, {14, 10, 0}, {15, 10, 0}};
  open_sessions(sv, ss, 4);
  std::vector<Pending> ps(60);
  for (int i = 0; i < 60; ++i) submit(sv, ss[(size_t)(i * 7 % 5)], ps[(size_t)i], 2);
  for (Pending& p : ps) check_result(sv, p);
  jefi_server_stats st;
  CHECK(jefi_server_get_stats(sv, &st) == JEFI_OK);
  CHECK(st.evictions > 0 && st.rematerialisations > 0);
  CHECK(st.arena_high_water <= 330 * 1024);
  std::printf("eviction: %llu evictions, %llu rematerialisations\n", (unsigned long long)st.evictions,
              (unsigned long long)st.rematerialisations);
  CHECK(jefi_server_destroy(sv) == JEFI_OK);
}

void full_queue_and_rejections() {
  std::vector<char> arena;
  jefi_server* sv = make_server(8 << 20, 1, 3, arena);
  g_eval_sleep_us = 3000;
  std::vector<Session> ss = {{21, 3, 0}, {22, 3, 0}, {23, 3, 0}, {24, 3, 0}};
  open_sessions(sv, ss, 1);
  std::vector<Pending> ps(24);
  int busy = 0;
  for (int i = 0; i < 24; ++i) busy += submit(sv, ss[(size_t)(i % 4)], ps[(size_t)i], 1);
  CHECK(busy > 0);  // the queue of 3 filled up at least once
  // unknown session, request that can never fit the arena
  jefi_request rq;
  std::memset(&rq, 0, sizeof rq);
  std::vector<float> E(3), B(3);
  rq.session = 99;
  rq.obs = grid(1);
  rq.t = NAN;
  rq.E = E.data();
  rq.B = B.data();
  rq.out_on_host = 1;
  uint64_t tk;
  CHECK(jefi_server_submit(sv, &rq, &tk) == JEFI_ENOENT);
  rq.session = 21;
  rq.obs = grid(400);  // 6.4e7 points: outputs far beyond the arena
  CHECK(jefi_server_submit(sv, &rq, &tk) == JEFI_ETOOLARGE);
  // closing a session with requests outstanding is refused
  CHECK(jefi_server_close_session(sv, 24) == JEFI_EBUSY);
  for (Pending& p : ps) check_result(sv, p);
  CHECK(jefi_server_close_session(sv, 24) == JEFI_OK);
  CHECK(jefi_server_close_session(sv, 24) == JEFI_ENOENT);
  rq.session = 24;
  rq.obs = grid(1);
  CHECK(jefi_server_submit(sv, &rq, &tk) == JEFI_ENOENT);
  jefi_server_stats st;
  CHECK(jefi_server_get_stats(sv, &st) == JEFI_OK);
  CHECK(st.completed == 24 && st.failed == 0);
  CHECK(jefi_server_destroy(sv) == JEFI_OK);
}

void time_after_newest_fails_at_admission() {
  std::vector<char> arena;
  jefi_server* sv = make_server(8 << 20, 2, 64, arena);
  g_eval_sleep_us = 0;
  std::vector<Session> ss = {{31, 3, 0}};
  open_sessions(sv, ss, 2);
  jefi_request rq;
  std::memset(&rq, 0, sizeof rq);
  std::vector<float> E(3), B(3);
  rq.session = 31;
  rq.obs = grid(1);
  rq.t = 100.0;  // step 1000 of a session whose newest step is 1
  rq.E = E.data();
  rq.B = B.data();
  rq.out_on_host = 1;
  uint64_t tk;
  CHECK(jefi_server_submit(sv, &rq, &tk) == JEFI_OK);
  jefi_result res;
  CHECK(jefi_server_wait(sv, tk, &res) == JEFI_OK);
  CHECK(res.status == JEFI_EINVAL);
  // the session still serves later requests
  Pending p;
  submit(sv, ss[0], p, 2);
  check_result(sv, p);
  CHECK(jefi_server_destroy(sv) == JEFI_OK);
}

void option_flags() {
  // invalid combinations are refused at create; valid ones reach every evaluation
  std::vector<char> arena(1 << 20);
  jefi_server_config cfg;
  std::memset(&cfg, 0, sizeof cfg);
  cfg.arena = arena.data();
  cfg.arena_bytes = arena.size();
  cfg.precision = JEFI_PREC_F32_COMP;
  jefi_server* bad = nullptr;
  cfg.flags = JEFI_FLAG_INDEX_GUARD | JEFI_FLAG_INDEX_TABLE;
  CHECK(jefi_server_create(&cfg, &bad) == JEFI_EINVAL);
  cfg.flags = 64;
  CHECK(jefi_server_create(&cfg, &bad) == JEFI_EINVAL);
  cfg.flags = JEFI_FLAG_DERIV_SLOPE | JEFI_FLAG_TIME_CUBIC;
  CHECK(jefi_server_create(&cfg, &bad) == JEFI_EINVAL);
  cfg.flags = JEFI_FLAG_PAST_HOLD | JEFI_FLAG_PAST_CUT;
  CHECK(jefi_server_create(&cfg, &bad) == JEFI_EINVAL);
  cfg.flags = 0;
  cfg.reserve_cus = -1;
  CHECK(jefi_server_create(&cfg, &bad) == JEFI_EINVAL);
  cfg.reserve_cus = 0;
  std::vector<char> ar;
  const uint32_t flags = JEFI_FLAG_PAST_HOLD | JEFI_FLAG_DERIV_SLOPE | JEFI_FLAG_INDEX_TABLE;
  jefi_server* sv = make_server(8 << 20, 2, 64, ar, flags);
  g_eval_sleep_us = 0;
  std::vector<Session> ss = {{41, 3, 0}};
  open_sessions(sv, ss, 2);
  Pending p;
  submit(sv, ss[0], p, 2);
  check_result(sv, p);
  CHECK(g_last_batch_flags.load() == flags);
  CHECK(jefi_server_destroy(sv) == JEFI_OK);
  // the cubic reading reaches the evaluations the same way
  const uint32_t cflags = JEFI_FLAG_PAST_HOLD | JEFI_FLAG_TIME_CUBIC;
  std::vector<char> ar2;
  jefi_server* sv2 = make_server(8 << 20, 2, 64, ar2, cflags);
  std::vector<Session> ss2 = {{43, 3, 0}};
  open_sessions(sv2, ss2, 2);
  Pending p2;
  submit(sv2, ss2[0], p2, 2);
  check_result(sv2, p2);
  CHECK(g_last_batch_flags.load() == cflags);
  CHECK(jefi_server_destroy(sv2) == JEFI_OK);
}

// A session brought back into the arena in a pass whose request then does
// not fit (its slice finds no room) must not be used on another stream
// before its ring upload has finished.  Two streams; the first-fit arena of
// 312000 B is laid out as follows (rings of 4^3-cell sessions: 6144 B, of
// the 10^3-cell session B: 96000 B, as much again to stage its shadow):
//   - sessions B, A, C, G open in that order: rings at 0, 96000, 102144,
//     108288;
//   - G's request takes its slice and 192000 B of outputs at 114432;
//   - C's request (outputs 81152 B) finds no room at the end and evicts B,
//     the least recently used idle session: its outputs go to 0;
//   - A and B queue while G and C run.  When G completes, one pass admits A
//     and brings B back into G's old region (ring and shadow staging), but
//     B's slice (16128 B) fits nowhere, also after evicting the idle G: the
//     batch holds A only, and B's (slow) ring upload is queued on its stream;
//   - when C completes, B's request runs on C's stream.
// B's result is right only if its push and evaluation follow the upload.
// G and C are held on their streams until released, so that A and B queue
// behind them and G completes first whatever the threads' timing.
void wait_launched(int n) {
  for (int i = 0; i < 100000 && jefi_mock_batches_launched() < n; ++i)
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  CHECK(jefi_mock_batches_launched() >= n);
}

void materialised_but_not_admitted() {
  std::vector<char> arena;
  jefi_server* sv = make_server(312000, 2, 64, arena);
  g_eval_sleep_us = 0;
  g_ingest_sleep_us = 0;
  std::vector<Session> ss = {{51, 10, 0}, {52, 4, 0}, {53, 4, 0}, {54, 4, 0}};  // B A C G
  open_sessions(sv, ss, 3);
  Session &B = ss[0], &A = ss[1], &C = ss[2], &G = ss[3];
  Pending pg, pc, pa, pb;
  const int base = jefi_mock_batches_launched();
  jefi_mock_hold_next_batches(2);
  submit(sv, G, pg, 20);  // 8000 points: 192000 B of outputs
  wait_launched(base + 1);
  submit(sv, C, pc, 15);  // 3375 points: 81152 B
  wait_launched(base + 2);
  g_ingest_sleep_us = 40000;
  submit(sv, A, pa, 1);
  submit(sv, B, pb, 1);
  jefi_mock_release_batch();  // G completes: A is admitted, B brought back but not admitted
  wait_launched(base + 3);
  jefi_mock_release_batch();  // C completes: B runs on its stream
  check_result(sv, pg);
  check_result(sv, pc);
  check_result(sv, pa);
  check_result(sv, pb);
  g_ingest_sleep_us = 0;
  jefi_server_stats st;
  CHECK(jefi_server_get_stats(sv, &st) == JEFI_OK);
  CHECK(st.evictions >= 2 && st.rematerialisations >= 1 && st.batches == 4);
  std::printf("materialised but not admitted: %llu evictions, %llu rematerialisations, %llu batches\n",
              (unsigned long long)st.evictions, (unsigned long long)st.rematerialisations,
              (unsigned long long)st.batches);
  CHECK(jefi_server_destroy(sv) == JEFI_OK);
}

// One ticket polled and waited from two threads: exactly one of them takes
// the result, the other sees the ticket gone; neither blocks forever.
void poll_and_wait_one_ticket() {
  std::vector<char> arena;
  jefi_server* sv = make_server(8 << 20, 2, 64, arena);
  g_eval_sleep_us = 5000;
  std::vector<Session> ss = {{61, 3, 0}};
  open_sessions(sv, ss, 2);
  for (int round = 0; round < 20; ++round) {
    Pending p;
    submit(sv, ss[0], p, 1);
    std::atomic<int> ok{0}, gone{0};
    std::thread waiter([&]() {
      jefi_result res;
      const jefi_status st = jefi_server_wait(sv, p.ticket, &res);
      if (st == JEFI_OK) ok++;
      else if (st == JEFI_ENOENT) gone++;
    });
    std::thread poller([&]() {
      jefi_result res;
      for (;;) {
        const jefi_status st = jefi_server_poll(sv, p.ticket, &res);
        if (st == JEFI_PENDING) {
          std::this_thread::sleep_for(std::chrono::microseconds(100));
          continue;
        }
        if (st == JEFI_OK) ok++;
        else if (st == JEFI_ENOENT) gone++;
        break;
      }
    });
    waiter.join();
    poller.join();
    CHECK(ok.load() == 1 && gone.load() == 1);
  }
  CHECK(jefi_server_destroy(sv) == JEFI_OK);
}

}  // namespace

int main() {
  std::setvbuf(stdout, nullptr, _IONBF, 0);
  concurrent_submitters();
  express_lane();
  eviction();
  full_queue_and_rejections();
  time_after_newest_fails_at_admission();
  option_flags();
  materialised_but_not_admitted();
  poll_and_wait_one_ticket();
  if (g_fail.load() == 0) std::printf("server ok\n");
  return g_fail.load() == 0 ? 0 : 1;
}
