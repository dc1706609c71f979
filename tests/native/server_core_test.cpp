// CPU tests of the server's scheduling core (paper_1812_07122_amd/csrc/server_core.h)
// driven by a fake executor instead of HIP kernels and events: FIFO admission by
// arena bytes and slots, DONE and FAILED retirement (a failed launch, an error
// reported while the step runs), drain on stop, a full queue (BLFLS_E_AGAIN), a
// workspace larger than the arena (BLFLS_E_NOMEM), submissions after stop,
// unknown tickets, and the bounded latency window.  Prints one line per check and
// exits non-zero on the first failure.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "server_core.h"

using namespace blfls;

struct TJob : CoreJob {
  int tag = 0;
};

struct FakeExec {
  std::mutex m;
  std::set<int> fail_launch, fail_query;  // tags whose step fails at launch / while running
  std::atomic<bool> hold{false};          // steps do not complete while set
  std::vector<int> slot_tags[2];
  size_t bytes_now = 0, bytes_peak = 0;
  int running_now = 0, running_peak = 0;
  std::vector<size_t> slot_bytes = std::vector<size_t>(2, 0);
  std::vector<int> slot_count = std::vector<int>(2, 0);

  int launch(std::vector<TJob*>& jobs, int slot) {
    std::lock_guard<std::mutex> lk(m);
    slot_tags[slot].clear();
    size_t b = 0;
    bool fail = false;
    for (TJob* j : jobs) {
      slot_tags[slot].push_back(j->tag);
      b += j->ws_bytes;
      fail = fail || fail_launch.count(j->tag);
    }
    slot_bytes[slot] = b;
    slot_count[slot] = static_cast<int>(jobs.size());
    bytes_now += b;
    running_now += slot_count[slot];
    bytes_peak = std::max(bytes_peak, bytes_now);
    running_peak = std::max(running_peak, running_now);
    return fail ? -7 : 0;
  }
  int query(int slot) {
    if (hold.load()) return 1;
    std::lock_guard<std::mutex> lk(m);
    for (int t : slot_tags[slot])
      if (fail_query.count(t)) return -9;
    return 0;
  }
  void drain(int slot, int) {
    while (hold.load()) std::this_thread::sleep_for(std::chrono::microseconds(200));
    std::lock_guard<std::mutex> lk(m);
    bytes_now -= slot_bytes[slot];
    running_now -= slot_count[slot];
    slot_bytes[slot] = 0;
    slot_count[slot] = 0;
  }
};

static int g_fail = 0;
#define CHECK(cond, what)                                                   \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::printf("FAIL %s (%s:%d)\n", what, __FILE__, __LINE__);           \
      std::fflush(stdout);                                                  \
      std::exit(1);                                                         \
    }                                                                       \
  } while (0)

static CoreConfig cfg(size_t arena, int slots, int cap, size_t window = 1 << 16) {
  CoreConfig c;
  c.arena_base = 4096;
  c.arena_bytes = arena;
  c.max_slots = slots;
  c.queue_cap = cap;
  c.step_budget = 1 << 20;
  c.step_overhead = 1024;
  c.latency_window = window;
  return c;
}

static TJob* job(int tag, size_t ws, size_t desc = 64) {
  auto* j = new TJob();
  j->tag = tag;
  j->ws_bytes = ws;
  j->desc_bytes = desc;
  return j;
}

static void wait_state(SchedulerCore<TJob>& core, uint64_t t, int32_t* state, blfls_status* res) {
  for (int i = 0; i < 200000; ++i) {
    const blfls_status st = core.poll(t, state, res);
    CHECK(st == BLFLS_OK, "poll of a live ticket");
    if (*state == BLFLS_DONE || *state == BLFLS_FAILED) return;
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
  CHECK(false, "ticket never finished");
}

static void fifo_admission_by_bytes() {
  FakeExec ex;
  auto core_holder = std::make_unique<SchedulerCore<TJob>>();
  SchedulerCore<TJob>& core = *core_holder;
  core.configure(cfg(1024, 8, 64));
  core.start(&ex);
  std::vector<uint64_t> t(40);
  for (int i = 0; i < 40; ++i) CHECK(core.submit(job(i, i % 3 == 0 ? 600 : 200), &t[i]) == BLFLS_OK, "submit");
  for (int i = 0; i < 40; ++i) {
    int32_t s;
    blfls_status r;
    wait_state(core, t[i], &s, &r);
    CHECK(s == BLFLS_DONE && r == BLFLS_OK, "every request DONE");
  }
  blfls_stats st{};
  core.fill_stats(&st);
  CHECK(st.completed == 40 && st.failed == 0 && st.admitted == 40, "counters");
  CHECK(st.arena_in_use == 0 && st.arena_peak <= 1024, "arena released, never over-committed");
  CHECK(ex.bytes_peak <= 1024, "admitted bytes in flight within the arena");
  CHECK(st.running_now == 0 && st.queued_now == 0, "idle at the end");
  core.stop();
  std::printf("ok fifo_admission_by_bytes (peak %zu of 1024 bytes, %d requests in flight at most)\n", ex.bytes_peak,
              ex.running_peak);
}

static void slots_bound_requests_in_flight() {
  FakeExec ex;
  auto core_holder = std::make_unique<SchedulerCore<TJob>>();
  SchedulerCore<TJob>& core = *core_holder;
  core.configure(cfg(1 << 20, 3, 64));
  core.start(&ex);
  std::vector<uint64_t> t(30);
  for (int i = 0; i < 30; ++i) CHECK(core.submit(job(i, 256), &t[i]) == BLFLS_OK, "submit");
  for (int i = 0; i < 30; ++i) {
    int32_t s;
    blfls_status r;
    wait_state(core, t[i], &s, &r);
    CHECK(s == BLFLS_DONE, "DONE");
  }
  CHECK(ex.running_peak <= 3, "at most max_slots requests in flight");
  core.stop();
  std::printf("ok slots_bound_requests_in_flight (%d at most)\n", ex.running_peak);
}

static void failed_steps() {
  for (int mode = 0; mode < 2; ++mode) {
    FakeExec ex;
    (mode == 0 ? ex.fail_launch : ex.fail_query).insert(3);
    auto core_holder = std::make_unique<SchedulerCore<TJob>>();
  SchedulerCore<TJob>& core = *core_holder;
    core.configure(cfg(1 << 20, 1, 64));   // one request per step
    core.start(&ex);
    std::vector<uint64_t> t(8);
    for (int i = 0; i < 8; ++i) CHECK(core.submit(job(i, 256), &t[i]) == BLFLS_OK, "submit");
    for (int i = 0; i < 8; ++i) {
      int32_t s;
      blfls_status r;
      wait_state(core, t[i], &s, &r);
      if (i == 3) CHECK(s == BLFLS_FAILED && r == BLFLS_E_HIP, "the failing request is FAILED with E_HIP");
      else CHECK(s == BLFLS_DONE && r == BLFLS_OK, "the others complete");
    }
    blfls_stats st{};
    core.fill_stats(&st);
    CHECK(st.failed == 1 && st.completed == 7 && st.arena_in_use == 0, "counters and arena after a failure");
    core.stop();
    std::printf("ok failed_steps (%s)\n", mode == 0 ? "launch error" : "error while running");
  }
}

static void drain_on_stop() {
  FakeExec ex;
  ex.hold = true;
  auto core_holder = std::make_unique<SchedulerCore<TJob>>();
  SchedulerCore<TJob>& core = *core_holder;
  core.configure(cfg(1 << 20, 2, 64));
  core.start(&ex);
  std::vector<uint64_t> t(10);
  for (int i = 0; i < 10; ++i) CHECK(core.submit(job(i, 256), &t[i]) == BLFLS_OK, "submit");
  std::thread release([&] {
    std::this_thread::sleep_for(std::chrono::milliseconds(50));
    ex.hold = false;
  });
  core.stop();   // returns only after every queued and running request finished
  release.join();
  for (int i = 0; i < 10; ++i) {
    int32_t s;
    blfls_status r;
    CHECK(core.poll(t[i], &s, &r) == BLFLS_OK && s == BLFLS_DONE, "drained to DONE by stop");
  }
  uint64_t t2;
  TJob* late = job(99, 256);
  CHECK(core.submit(late, &t2) == BLFLS_E_INVALID, "no submissions after stop");
  delete late;   // refused: still the caller's
  std::printf("ok drain_on_stop\n");
}

static void queue_full_and_nomem() {
  FakeExec ex;
  ex.hold = true;
  auto core_holder = std::make_unique<SchedulerCore<TJob>>();
  SchedulerCore<TJob>& core = *core_holder;
  core.configure(cfg(1024, 1, 2));
  core.start(&ex);
  uint64_t a, b, c, d;
  TJob* big = job(50, 2048);
  CHECK(core.submit(big, &d) == BLFLS_E_NOMEM, "a workspace beyond the arena is refused");
  delete big;
  CHECK(core.submit(job(0, 256), &a) == BLFLS_OK, "first");
  blfls_stats st{};
  for (int i = 0; i < 20000; ++i) {
    core.fill_stats(&st);
    if (st.running_now == 1) break;
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
  CHECK(st.running_now == 1, "first request admitted");
  CHECK(core.submit(job(1, 256), &b) == BLFLS_OK && core.submit(job(2, 256), &c) == BLFLS_OK, "queue fills");
  TJob* extra = job(3, 256);
  CHECK(core.submit(extra, &d) == BLFLS_E_AGAIN, "a full queue answers E_AGAIN");
  delete extra;
  ex.hold = false;
  int32_t s;
  blfls_status r;
  for (uint64_t t : {a, b, c}) {
    wait_state(core, t, &s, &r);
    CHECK(s == BLFLS_DONE, "queued requests complete");
  }
  CHECK(core.submit(job(4, 256), &d) == BLFLS_OK, "accepts again once drained");
  wait_state(core, d, &s, &r);
  CHECK(core.poll(d, &s, &r) == BLFLS_E_UNKNOWN_TICKET, "a retired ticket is unknown");
  CHECK(core.poll(123456, &s, &r) == BLFLS_E_UNKNOWN_TICKET, "a ticket never issued is unknown");
  core.stop();
  std::printf("ok queue_full_and_nomem\n");
}

static void bounded_latency_window() {
  FakeExec ex;
  auto core_holder = std::make_unique<SchedulerCore<TJob>>();
  SchedulerCore<TJob>& core = *core_holder;
  core.configure(cfg(1 << 20, 4, 256, 16));
  core.start(&ex);
  std::vector<uint64_t> t(40);
  for (int i = 0; i < 40; ++i) CHECK(core.submit(job(i, 256), &t[i]) == BLFLS_OK, "submit");
  int32_t s;
  blfls_status r;
  for (uint64_t x : t) wait_state(core, x, &s, &r);
  blfls_stats st{};
  core.fill_stats(&st);
  CHECK(st.completed == 40 && st.latency_samples == 16, "latency window keeps the last 16 samples");
  CHECK(st.latency_p50_ms <= st.latency_p99_ms && st.latency_p99_ms <= st.latency_max_ms, "percentiles ordered");
  core.stop();
  std::printf("ok bounded_latency_window\n");
}

int main() {
  fifo_admission_by_bytes();
  slots_bound_requests_in_flight();
  failed_steps();
  drain_on_stop();
  queue_full_and_nomem();
  bounded_latency_window();
  std::printf("all server core checks passed\n");
  return g_fail;
}
