// Scheduling core of the continuous-batching server, independent of the GPU.
//
// It owns the request queue, the tickets, admission (FIFO, while a slot is free
// and the request's workspace fits in the arena: admission by HBM bytes), the
// steps in flight, their retirement (DONE, or FAILED with BLFLS_E_HIP when the
// executor reports an error), the bounded window of submit-to-done latencies
// and the counters.  A scheduler thread runs steps through an executor:
//
//   int  launch(std::vector<JobT*>& jobs, int slot)  queue a step's work (0 = ok)
//   int  query(int slot)       1 while the slot's step runs, 0 when done, < 0 error
//   void drain(int slot, int err)  block until the slot's queued work has finished
//                              (err: the step's error so far, 0 if none)
//
// kDepth steps are in flight: while step k runs, step k+1 is prepared and
// queued; steps retire in launch order.  Destroying the core (stop) drains
// every queued and running request first.  The server drives it with HIP
// kernels and events; the CPU tests drive it with a fake executor.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/blfls.h"

namespace blfls {

inline size_t core_align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline double core_now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [base, base + bytes) of the arena, 256-byte granules.
class Arena {
 public:
  void init(size_t base, size_t bytes) {
    free_.clear();
    if (bytes > 0) free_[base] = bytes;
    total_ = bytes;
    used_ = peak_ = 0;
  }
  bool alloc(size_t n, size_t* off) {
    n = core_align_up(n, 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = core_align_up(n, 256);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t total() const { return total_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t total_ = 0, used_ = 0, peak_ = 0;
};

// The core's part of a request; the server's job type derives from it.
struct CoreJob {
  uint64_t id = 0;
  double t_submit = 0.0;
  size_t desc_bytes = 0;  // staging bytes of its descriptors in one step
  size_t ws_bytes = 0;    // arena bytes of its workspace
  size_t ws_off = 0;      // its workspace's offset in the arena once admitted
  virtual ~CoreJob() = default;
};

struct CoreConfig {
  size_t arena_base = 0, arena_bytes = 0;  // the admission arena
  int max_slots = 1;                       // requests in flight at most
  int queue_cap = 1;                       // requests waiting at most
  size_t step_budget = 0;                  // staging bytes of one step
  size_t step_overhead = 0;                // of which the step's own header takes this much
  size_t latency_window = 1 << 16;         // latency samples kept (the most recent)
};

struct CoreCounters {
  uint64_t submitted = 0, admitted = 0, completed = 0, failed = 0, steps = 0;
  double step_ms_total = 0.0;
};

template <class JobT, int kDepth = 2>
class SchedulerCore {
 public:
  void configure(const CoreConfig& c) {
    cfg_ = c;
    arena_.init(c.arena_base, c.arena_bytes);
    lat_.assign(c.latency_window, 0.0);
  }

  // Start the scheduler thread over an executor that outlives the core's run.
  template <class Exec>
  void start(Exec* ex) {
    worker_ = std::thread([this, ex] { run(ex); });
  }

  // Queue a request: BLFLS_E_NOMEM if its workspace can never fit the arena,
  // BLFLS_E_AGAIN if the queue is full, BLFLS_E_INVALID once stopping.
  // On success the core owns jb and *ticket identifies it.
  blfls_status submit(JobT* jb, uint64_t* ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    if (stopping_) return BLFLS_E_INVALID;
    if (jb->ws_bytes > arena_.total()) return BLFLS_E_NOMEM;
    if (static_cast<int>(queue_.size()) >= cfg_.queue_cap) return BLFLS_E_AGAIN;
    jb->id = next_id_++;
    jb->t_submit = core_now_ms();
    queue_.push_back(jb);
    tickets_[jb->id] = {BLFLS_QUEUED, BLFLS_OK};
    counters_.submitted++;
    *ticket = jb->id;
    cv_.notify_all();
    return BLFLS_OK;
  }

  // State of a ticket; DONE / FAILED retire it.  BLFLS_E_UNKNOWN_TICKET otherwise.
  blfls_status poll(uint64_t ticket, int32_t* state, blfls_status* result) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end()) return BLFLS_E_UNKNOWN_TICKET;
    *state = it->second.first;
    *result = it->second.second;
    if (*state == BLFLS_DONE || *state == BLFLS_FAILED) tickets_.erase(it);
    return BLFLS_OK;
  }

  // Counters, queue and arena state, and p50 / p99 / max over the latency window.
  void fill_stats(blfls_stats* out) {
    std::lock_guard<std::mutex> lk(mu_);
    out->submitted = counters_.submitted;
    out->admitted = counters_.admitted;
    out->completed = counters_.completed;
    out->failed = counters_.failed;
    out->steps = counters_.steps;
    out->queued_now = queue_.size();
    out->running_now = static_cast<uint64_t>(running_);
    out->arena_bytes = arena_.total();
    out->arena_in_use = arena_.used();
    out->arena_peak = arena_.peak();
    out->step_ms_mean = counters_.steps ? counters_.step_ms_total / static_cast<double>(counters_.steps) : 0.0;
    const size_t n = std::min<uint64_t>(lat_count_, lat_.size());
    std::vector<double> lat(lat_.begin(), lat_.begin() + static_cast<std::ptrdiff_t>(n));
    out->latency_samples = n;
    out->latency_p50_ms = out->latency_p99_ms = out->latency_max_ms = 0.0;
    if (!lat.empty()) {
      std::sort(lat.begin(), lat.end());
      auto pct = [&](double q) {
        const size_t i = static_cast<size_t>(std::ceil(q * static_cast<double>(lat.size()))) - 1;
        return lat[std::min(i, lat.size() - 1)];
      };
      out->latency_p50_ms = pct(0.50);
      out->latency_p99_ms = pct(0.99);
      out->latency_max_ms = lat.back();
    }
  }

  // Stop accepting work, run everything queued or in flight to completion,
  // join the scheduler thread, and free jobs never admitted (none, after the
  // drain).  Idempotent.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stopping_ = true;
    }
    cv_.notify_all();
    if (worker_.joinable()) worker_.join();
    for (JobT* jb : queue_) delete jb;
    queue_.clear();
  }

  // Monotone count of retired steps (for users that must not free what a
  // step in flight may still read).
  uint64_t retired_steps() const { return retired_.load(); }
  uint64_t launched_steps() const { return launched_.load(); }

 private:
  struct Step {
    std::vector<JobT*> jobs;
    int err = 0;
    double t_launch = 0.0;
    bool busy = false;
  };

  template <class Exec>
  void retire(Exec* ex, Step& st, int slot) {
    const int e = st.err;
    ex->drain(slot, e);  // launched work finishes before its memory is reused
    const double ms = core_now_ms() - st.t_launch;
    std::lock_guard<std::mutex> lk(mu_);
    for (JobT* jb : st.jobs) {
      auto it = tickets_.find(jb->id);
      if (it != tickets_.end()) {
        it->second.first = e == 0 ? BLFLS_DONE : BLFLS_FAILED;
        it->second.second = e == 0 ? BLFLS_OK : BLFLS_E_HIP;
      }
      if (e == 0) {
        counters_.completed++;
        lat_[lat_count_ % lat_.size()] = core_now_ms() - jb->t_submit;
        lat_count_++;
      } else {
        counters_.failed++;
      }
      arena_.release(jb->ws_off, jb->ws_bytes);
      running_--;
      delete jb;
    }
    st.jobs.clear();
    st.busy = false;
    counters_.step_ms_total += ms;
    retired_++;
    cv_.notify_all();
  }

  void admit(std::vector<JobT*>* admitted) {
    size_t desc = cfg_.step_overhead;
    while (!queue_.empty() && running_ < cfg_.max_slots) {
      JobT* jb = queue_.front();
      if (desc + jb->desc_bytes > cfg_.step_budget) break;  // the rest waits for the next step
      size_t off = 0;
      if (!arena_.alloc(jb->ws_bytes, &off)) break;           // FIFO: the head waits for space
      desc += jb->desc_bytes;
      jb->ws_off = off;
      queue_.pop_front();
      tickets_[jb->id].first = BLFLS_RUNNING;
      running_++;
      counters_.admitted++;
      admitted->push_back(jb);
    }
  }

  template <class Exec>
  void run(Exec* ex) {
    int next = 0;    // slot the next step launches into
    int oldest = 0;  // oldest in-flight step (steps complete in launch order)
    for (;;) {
      while (steps_[oldest].busy) {
        Step& st = steps_[oldest];
        if (st.err == 0) {
          const int q = ex->query(oldest);
          if (q > 0) break;
          if (q < 0) st.err = q;
        }
        retire(ex, st, oldest);
        oldest = (oldest + 1) % kDepth;
      }
      std::unique_lock<std::mutex> lk(mu_);
      bool any_busy = false;
      for (auto& x : steps_) any_busy = any_busy || x.busy;
      if (stopping_ && queue_.empty() && !any_busy) break;
      Step& st = steps_[next];
      std::vector<JobT*> admitted;
      if (!st.busy) admit(&admitted);
      if (!admitted.empty()) {
        counters_.steps++;
        lk.unlock();
        st.jobs = std::move(admitted);
        st.busy = true;
        st.t_launch = core_now_ms();
        st.err = ex->launch(st.jobs, next);
        launched_++;
        next = (next + 1) % kDepth;
        continue;
      }
      if (any_busy)  // poll the in-flight step (a timed wait on the system clock: pthread_cond_timedwait)
        cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::microseconds(50));
      else
        cv_.wait(lk, [&] { return stopping_ || !queue_.empty(); });
    }
  }

  CoreConfig cfg_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stopping_ = false;
  std::deque<JobT*> queue_;
  std::unordered_map<uint64_t, std::pair<int32_t, blfls_status>> tickets_;
  uint64_t next_id_ = 1;
  int running_ = 0;
  Arena arena_;
  Step steps_[kDepth];
  CoreCounters counters_;
  std::vector<double> lat_;
  uint64_t lat_count_ = 0;
  std::atomic<uint64_t> retired_{0}, launched_{0};
  std::thread worker_;
};

}  // namespace blfls
