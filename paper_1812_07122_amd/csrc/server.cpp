// Continuous-batching server for BLF-LS requests of uneven sizes.
//
// Requests are validated at submit and queued.  A scheduler thread runs
// steps: each step admits queued requests (FIFO) while a slot is free and the
// request's workspace fits in the caller's device arena (admission by HBM
// footprint), builds the descriptors of every admitted request into one
// pinned staging buffer, uploads it with one copy, and launches each kernel
// family ONCE for all admitted requests (the kernels look up their request by
// workgroup index).  Two steps are in flight: the host prepares and queues
// step k+1 while step k runs, then retires step k when its event completes.
// Requests that arrive while a step runs are admitted into the next one.
// Every request's arithmetic is independent of its neighbours in a batch, so
// a result is bitwise the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/blfls.h"
#include "blfls_internal.h"
#include "blfls_launch.h"
#include "blfls_plan.h"

namespace blfls {
namespace {

constexpr size_t kStageBytes = 8u << 20;  // descriptor staging per in-flight step
constexpr int kDepth = 2;                 // steps in flight

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

double now_ms() {
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
    n = align_up(n, 256);
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
    n = align_up(n, 256);
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

struct Job {
  uint64_t id = 0;
  double t_submit = 0.0;
  blfls_request req{};
  int radius = 0;
  blfls_plan_s* plan = nullptr;
  size_t ws_off = 0;
  RequestDesc rd;
};

struct Step {
  std::vector<Job*> jobs;
  hipEvent_t done = nullptr;
  hipError_t err = hipSuccess;
  double t_launch = 0.0;
  bool busy = false;
};

}  // namespace
}  // namespace blfls

using namespace blfls;

struct blfls_server_s {
  uint8_t* arena = nullptr;
  size_t arena_bytes = 0;
  size_t desc_region = 0;  // bytes of arena reserved for device descriptors (kDepth * kStageBytes)
  int max_slots = 1;
  int queue_cap = 1;
  blfls_precision precision = BLFLS_FP32;
  hipStream_t stream = nullptr;
  int device = 0;

  std::mutex mu;
  std::condition_variable cv;
  bool stopping = false;
  std::deque<Job*> queue;
  std::unordered_map<uint64_t, std::pair<int, blfls_status>> tickets;
  uint64_t next_id = 1;
  int running = 0;
  Arena arena_alloc;
  std::map<std::tuple<int, int, int>, blfls_plan_s*> plans;
  uint8_t* staging[kDepth] = {nullptr, nullptr};
  Step steps[kDepth];
  blfls_stats stats{};
  double step_ms_total = 0.0;
  std::vector<double> latencies;  // submit -> done, ms
  std::thread worker;

  void run();
  void retire(Step& st);
  void admit(std::vector<Job*>* admitted);
  hipError_t launch_step(Step& st, int slot);
};

namespace {

// Append `n` bytes to the staging buffer at 256-byte alignment; returns the offset.
struct Stager {
  uint8_t* host;
  uint8_t* dev;
  size_t cap;
  size_t used = 0;
  bool overflow = false;
  size_t put(const void* src, size_t n) {
    const size_t off = align_up(used, 256);
    if (off + n > cap) {
      overflow = true;
      return 0;
    }
    std::memcpy(host + off, src, n);
    used = off + n;
    return off;
  }
  size_t reserve(size_t n) {
    const size_t off = align_up(used, 256);
    if (off + n > cap) {
      overflow = true;
      return 0;
    }
    used = off + n;
    return off;
  }
};

}  // namespace

hipError_t blfls_server_s::launch_step(Step& st, int slot) {
  const int ft = precision == BLFLS_FP32 ? kF32 : precision == BLFLS_MIXED_BF16 ? kBF16 : kF16;
  Stager sg{staging[slot], arena + slot * kStageBytes, kStageBytes};
  // request tables first: the BLF and Gaussian descriptors point at them
  std::vector<size_t> tab_off(st.jobs.size());
  for (size_t j = 0; j < st.jobs.size(); ++j) tab_off[j] = sg.reserve(sizeof(RequestTables));
  int max_iter = 0;
  for (size_t j = 0; j < st.jobs.size(); ++j) {
    Job* jb = st.jobs[j];
    const blfls_request& q = jb->req;
    build_request(jb->plan, q.params, jb->radius, q.f, q.guide, q.u, q.pitch, arena + jb->ws_off,
                  sg.dev + tab_off[j], &jb->rd);
    std::memcpy(sg.host + tab_off[j], &jb->rd.tables, sizeof(RequestTables));
    max_iter = std::max(max_iter, jb->rd.iterations);
  }
  hipError_t e = hipSuccess;
  struct Launch {
    int kind;  // 0 gauss, 1 minmax, 2 blf, 3 fft
    int R;
    bool joint;
    size_t off;
    int n;
    int items;
    int rows, cols;
    size_t lds_rows, lds_cols;
    int64_t max_pix;
  };
  std::vector<Launch> launches;
  // Gaussian guide smoothing (before the first iteration)
  {
    std::vector<AuxPlane> g;
    int64_t max_pix = 0;
    for (Job* jb : st.jobs)
      if (jb->rd.smooth_guide)
        for (auto& a : jb->rd.gauss) {
          g.push_back(a);
          max_pix = std::max<int64_t>(max_pix, static_cast<int64_t>(a.H) * a.W);
        }
    if (!g.empty()) launches.push_back({0, 0, false, sg.put(g.data(), g.size() * sizeof(AuxPlane)),
                                        static_cast<int>(g.size()), 0, 0, 0, 0, 0, max_pix});
  }
  for (int it = 0; it < max_iter; ++it) {
    const bool first = it == 0;
    std::vector<AuxPlane> mm;
    std::map<std::pair<int, bool>, std::vector<BlfPlane>> blf;
    std::vector<FftPlane> fft;
    int rows = 0, cols = 0;
    size_t lds_rows = 0, lds_cols = 0;
    for (Job* jb : st.jobs) {
      RequestDesc& rd = jb->rd;
      if (it >= rd.iterations) continue;
      if (rd.normalize) for (auto& a : (first ? rd.mm_first : rd.mm_next)) mm.push_back(a);
      auto& bucket = blf[{rd.R, first ? rd.joint_first : true}];
      for (auto b : (first ? rd.blf_first : rd.blf_next)) {
        int tiles = 0;
        for (auto& x : bucket) tiles += x.tile_count;
        b.tile_begin = tiles;
        bucket.push_back(b);
      }
      for (auto fp : rd.fft) {
        fp.row_begin = rows;
        fp.col_begin = cols;
        rows += fp.row_count;
        cols += fp.col_count;
        fft.push_back(fp);
      }
      lds_rows = std::max(lds_rows, jb->plan->lds_rows);
      lds_cols = std::max(lds_cols, jb->plan->lds_cols);
    }
    if (!mm.empty())
      launches.push_back({1, 0, false, sg.put(mm.data(), mm.size() * sizeof(AuxPlane)),
                          static_cast<int>(mm.size()), 0, 0, 0, 0, 0, 0});
    for (auto& kv : blf) {
      int items = 0;
      for (auto& b : kv.second) items += 2 * b.tile_count;
      launches.push_back({2, kv.first.first, kv.first.second,
                          sg.put(kv.second.data(), kv.second.size() * sizeof(BlfPlane)),
                          static_cast<int>(kv.second.size()), items, 0, 0, 0, 0, 0});
    }
    if (!fft.empty())
      launches.push_back({3, 0, false, sg.put(fft.data(), fft.size() * sizeof(FftPlane)),
                          static_cast<int>(fft.size()), 0, rows, cols, lds_rows, lds_cols, 0});
  }
  if (sg.overflow) return hipErrorOutOfMemory;
  e = hipMemcpyAsync(sg.dev, sg.host, sg.used, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  for (const Launch& L : launches) {
    const uint8_t* d = sg.dev + L.off;
    switch (L.kind) {
      case 0: e = launch_gauss(reinterpret_cast<const AuxPlane*>(d), L.n, L.max_pix, stream); break;
      case 1: e = launch_minmax(reinterpret_cast<const AuxPlane*>(d), L.n, stream); break;
      case 2: e = launch_blf(L.R, reinterpret_cast<const BlfPlane*>(d), L.n, L.items, L.joint, ft, stream); break;
      default: {
        const FftPlane* fp = reinterpret_cast<const FftPlane*>(d);
        e = launch_fft_rows_fwd(fp, L.n, L.rows, L.lds_rows, ft, stream);
        if (e == hipSuccess) e = launch_fft_cols(fp, L.n, L.cols, L.lds_cols, stream);
        if (e == hipSuccess) e = launch_fft_rows_inv(fp, L.n, L.rows, L.lds_rows, stream);
      }
    }
    if (e != hipSuccess) return e;
  }
  return hipEventRecord(st.done, stream);
}

void blfls_server_s::retire(Step& st) {
  hipError_t e = st.err;
  if (e == hipSuccess) e = hipEventSynchronize(st.done);
  else (void)hipStreamSynchronize(stream);  // let launched kernels drain before their memory is reused
  const double ms = now_ms() - st.t_launch;
  std::lock_guard<std::mutex> lk(mu);
  for (Job* jb : st.jobs) {
    auto it = tickets.find(jb->id);
    if (it != tickets.end()) {
      it->second.first = e == hipSuccess ? BLFLS_DONE : BLFLS_FAILED;
      it->second.second = e == hipSuccess ? BLFLS_OK : BLFLS_E_HIP;
    }
    if (e == hipSuccess) {
      stats.completed++;
      latencies.push_back(now_ms() - jb->t_submit);
    } else {
      stats.failed++;
    }
    arena_alloc.release(jb->ws_off, jb->plan->ws_bytes);
    running--;
    delete jb;
  }
  st.jobs.clear();
  st.busy = false;
  step_ms_total += ms;
  cv.notify_all();
}

void blfls_server_s::admit(std::vector<Job*>* admitted) {
  while (!queue.empty() && running < max_slots) {
    Job* jb = queue.front();
    size_t off = 0;
    if (!arena_alloc.alloc(jb->plan->ws_bytes, &off)) break;  // FIFO: the head waits for space
    jb->ws_off = off;
    queue.pop_front();
    tickets[jb->id].first = BLFLS_RUNNING;
    running++;
    stats.admitted++;
    admitted->push_back(jb);
  }
}

void blfls_server_s::run() {
  (void)hipSetDevice(device);
  int next = 0;    // slot the next step launches into
  int oldest = 0;  // oldest in-flight step (steps complete in launch order: one stream)
  for (;;) {
    while (steps[oldest].busy) {
      Step& st = steps[oldest];
      if (st.err == hipSuccess) {
        const hipError_t q = hipEventQuery(st.done);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) st.err = q;
      }
      retire(st);
      oldest = (oldest + 1) % kDepth;
    }
    std::unique_lock<std::mutex> lk(mu);
    bool any_busy = false;
    for (auto& x : steps) any_busy = any_busy || x.busy;
    if (stopping && queue.empty() && !any_busy) break;
    Step& st = steps[next];
    std::vector<Job*> admitted;
    if (!st.busy) admit(&admitted);
    if (!admitted.empty()) {
      stats.steps++;
      lk.unlock();
      st.jobs = std::move(admitted);
      st.busy = true;
      st.t_launch = now_ms();
      st.err = launch_step(st, next);
      next = (next + 1) % kDepth;
      continue;
    }
    if (any_busy)
      cv.wait_for(lk, std::chrono::microseconds(50));  // poll the in-flight step's event
    else
      cv.wait(lk, [&] { return stopping || !queue.empty(); });
  }
}

extern "C" {

blfls_status blfls_server_create(blfls_server_t* out, void* arena, size_t arena_bytes, int32_t max_slots,
                                 int32_t queue_capacity, blfls_precision precision, void* stream) {
  if (out == nullptr) return set_error(BLFLS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (arena == nullptr || reinterpret_cast<uintptr_t>(arena) % 256 != 0)
    return set_error(BLFLS_E_INVALID, "arena must be a non-NULL 256-byte aligned device pointer");
  if (max_slots < 1 || queue_capacity < 1) return set_error(BLFLS_E_INVALID, "max_slots and queue_capacity must be >= 1");
  if (precision != BLFLS_FP32 && precision != BLFLS_MIXED_BF16 && precision != BLFLS_MIXED_FP16)
    return set_error(BLFLS_E_INVALID, "unknown precision");
  const size_t reserved = kDepth * kStageBytes;
  if (arena_bytes <= reserved) return set_error(BLFLS_E_NOMEM, "arena smaller than the descriptor region (16 MiB)");
  auto* s = new (std::nothrow) blfls_server_s();
  if (!s) return set_error(BLFLS_E_NOMEM, "host allocation failed");
  s->arena = static_cast<uint8_t*>(arena);
  s->arena_bytes = arena_bytes;
  s->desc_region = reserved;
  s->max_slots = max_slots;
  s->queue_cap = queue_capacity;
  s->precision = precision;
  s->stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) { delete s; return hip_error(e, "hipGetDevice"); }
  s->arena_alloc.init(reserved, arena_bytes - reserved);
  s->stats.arena_bytes = arena_bytes - reserved;
  for (int i = 0; i < kDepth; ++i) {
    e = hipHostMalloc(reinterpret_cast<void**>(&s->staging[i]), kStageBytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->steps[i].done, hipEventDisableTiming);
    if (e != hipSuccess) {
      for (int j = 0; j <= i; ++j) {
        if (s->staging[j]) (void)hipHostFree(s->staging[j]);
        if (s->steps[j].done) (void)hipEventDestroy(s->steps[j].done);
      }
      delete s;
      return hip_error(e, "server setup");
    }
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return BLFLS_OK;
}

blfls_status blfls_submit(blfls_server_t s, const blfls_request* r, uint64_t* ticket) {
  if (s == nullptr || r == nullptr || ticket == nullptr) return set_error(BLFLS_E_INVALID, "NULL argument");
  blfls_status st = check_shape(r->H, r->W, r->C);
  if (st != BLFLS_OK) return st;
  int radius = 0;
  st = check_params(&r->params, &radius);
  if (st != BLFLS_OK) return st;
  if (r->f == nullptr || r->u == nullptr) return set_error(BLFLS_E_INVALID, "f and u must not be NULL");
  if (r->pitch < r->W) return set_error(BLFLS_E_INVALID, "pitch must be >= W");
  const size_t img = static_cast<size_t>(r->C) * r->H * r->pitch * sizeof(float);
  auto ov = [](const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
  };
  if (ov(r->u, img, r->f, img) || (r->guide && ov(r->u, img, r->guide, img)) || ov(r->u, img, s->arena, s->arena_bytes))
    return set_error(BLFLS_E_INVALID, "u must not overlap f, guide or the arena");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->stopping) return set_error(BLFLS_E_INVALID, "server is shutting down");
  if (static_cast<int>(s->queue.size()) >= s->queue_cap) return set_error(BLFLS_E_AGAIN, "queue full");
  const auto key = std::make_tuple(r->H, r->W, r->C);
  blfls_plan_s* plan = nullptr;
  auto it = s->plans.find(key);
  if (it == s->plans.end()) {
    st = plan_create(r->H, r->W, r->C, s->precision, &plan);
    if (st != BLFLS_OK) return st;
    s->plans[key] = plan;
  } else {
    plan = it->second;
  }
  if (plan->ws_bytes > s->arena_bytes - s->desc_region)
    return set_error(BLFLS_E_NOMEM, "request workspace exceeds the arena");
  auto* jb = new (std::nothrow) Job();
  if (!jb) return set_error(BLFLS_E_NOMEM, "host allocation failed");
  jb->id = s->next_id++;
  jb->t_submit = now_ms();
  jb->req = *r;
  jb->radius = radius;
  jb->plan = plan;
  s->queue.push_back(jb);
  s->tickets[jb->id] = {BLFLS_QUEUED, BLFLS_OK};
  s->stats.submitted++;
  *ticket = jb->id;
  s->cv.notify_all();
  return BLFLS_OK;
}

blfls_status blfls_poll(blfls_server_t s, uint64_t ticket, int32_t* state, blfls_status* result) {
  if (s == nullptr || state == nullptr || result == nullptr) return set_error(BLFLS_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return set_error(BLFLS_E_UNKNOWN_TICKET, "unknown or retired ticket");
  *state = it->second.first;
  *result = it->second.second;
  if (*state == BLFLS_DONE || *state == BLFLS_FAILED) s->tickets.erase(it);
  return BLFLS_OK;
}

blfls_status blfls_server_stats(blfls_server_t s, blfls_stats* out) {
  if (s == nullptr || out == nullptr) return set_error(BLFLS_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->queued_now = s->queue.size();
  out->running_now = static_cast<uint64_t>(s->running);
  out->arena_in_use = s->arena_alloc.used();
  out->arena_peak = s->arena_alloc.peak();
  out->step_ms_mean = s->stats.steps ? s->step_ms_total / static_cast<double>(s->stats.steps) : 0.0;
  std::vector<double> lat = s->latencies;
  out->latency_samples = lat.size();
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
  return BLFLS_OK;
}

blfls_status blfls_server_destroy(blfls_server_t s) {
  if (s == nullptr) return set_error(BLFLS_E_INVALID, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->plans) plan_free(kv.second);
  for (int i = 0; i < kDepth; ++i) {
    if (s->staging[i]) (void)hipHostFree(s->staging[i]);
    if (s->steps[i].done) (void)hipEventDestroy(s->steps[i].done);
  }
  for (Job* jb : s->queue) delete jb;
  delete s;
  return BLFLS_OK;
}

}  // extern "C"
