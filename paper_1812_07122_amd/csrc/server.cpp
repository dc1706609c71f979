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
#include <atomic>
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
  size_t desc_bytes = 0;  // staging bytes of this request's tables and descriptors
  size_t ws_bytes = 0;    // arena bytes of its workspace (the AMF's is larger than the plan's)
  blfls_request req{};
  int radius = 0;
  blfls_plan_s* plan = nullptr;
  size_t ws_off = 0;
  RequestDesc rd;
};

// One launch group of a step: a kernel family over an array of plane descriptors.
// Kind 4 is one request's NC, grid or AMF filter stage, launched directly.
struct Group {
  int kind;  // 0 gauss, 1 minmax, 2 blf, 3 fft, 4 other filter (one request)
  int R = 0;
  bool joint = false;
  const Job* job = nullptr;     // kind 4: the request
  std::vector<uint8_t> planes;  // descriptor array bytes
  int n = 0;                    // planes
  int items = 0, items2 = 0;    // work items (fft: rows, cols)
  size_t lds_rows = 0, lds_cols = 0;
  int64_t max_pix = 0;
  bool wave_cols = false;       // fft: a plane's passes hold one column or row per wave
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

  // staging layout of one slot: [work header][request tables][descriptor arrays]
  static constexpr size_t kHeaderBytes = 16384;
  static constexpr int kMaxGroups = static_cast<int>(kHeaderBytes / sizeof(WorkHeader));
  static constexpr int kBlfGrid = 2048;  // persistent grids of the captured kernels
  static constexpr int kFftGrid = 1024;
  static constexpr int kAuxGrid = 1024;
  size_t stage_bytes = 0;
  size_t kFftLdsMax = 0;
  hipStream_t capture_stream = nullptr;
  std::map<std::pair<std::vector<int>, int>, hipGraphExec_t> graphs;
  // written by the scheduler thread outside the lock, read by blfls_server_stats
  std::atomic<uint64_t> stats_graph_steps{0}, stats_direct_steps{0};

  void run();
  void retire(Step& st);
  void admit(std::vector<Job*>* admitted);
  hipError_t launch_step(Step& st, int slot);
  hipError_t launch_direct(std::vector<Group>& groups, int slot, int ft, size_t tables_used);
  hipError_t launch_other_filter(const Job& jb, const uint8_t* planes, bool joint, int ft);
  hipError_t build_graph(const std::vector<Group>& groups, int slot, int ft, hipGraphExec_t* out);
};


template <class D>
static void push_desc(Group& g, const D& d) {
  const size_t off = g.planes.size();
  g.planes.resize(off + sizeof(D));
  std::memcpy(g.planes.data() + off, &d, sizeof(D));
  g.n++;
}

static std::vector<Group> build_groups(std::vector<Job*>& jobs) {
  std::vector<Group> groups;
  int max_iter = 0;
  for (Job* jb : jobs) max_iter = std::max(max_iter, jb->rd.iterations);
  {
    Group g{0};
    for (Job* jb : jobs)
      if (jb->rd.smooth_guide)
        for (auto& a : jb->rd.gauss) {
          push_desc(g, a);
          g.max_pix = std::max<int64_t>(g.max_pix, static_cast<int64_t>(a.H) * a.W);
        }
    g.items = g.n * gauss_chunks();
    if (g.n) groups.push_back(std::move(g));
  }
  for (int it = 0; it < max_iter; ++it) {
    const bool first = it == 0;
    Group mm{1};
    std::map<std::pair<int, bool>, Group> blf;
    std::vector<Group> other;
    Group fft{3};
    for (Job* jb : jobs) {
      RequestDesc& rd = jb->rd;
      if (it >= rd.iterations) continue;
      if (rd.normalize || rd.filter == BLFLS_FILTER_GRID)
        for (auto& a : (first ? rd.mm_first : rd.mm_next)) push_desc(mm, a);
      if (first && rd.fp16_scale)   // FP16 fields: the image's gradient extrema (store scales)
        for (auto& a : rd.mm_f) push_desc(mm, a);
      if (rd.filter != BLFLS_FILTER_BLF) {
        Group g{4};
        g.job = jb;
        g.joint = first ? rd.joint_first : true;   // the range source differs from the image
        if (rd.filter == BLFLS_FILTER_NC)
          for (const auto& d : (first ? rd.nc_first : rd.nc_next)) push_desc(g, d);
        else if (rd.filter == BLFLS_FILTER_GRID)
          for (const auto& d : (first ? rd.grid_first : rd.grid_next)) push_desc(g, d);
        else
          for (const auto& d : (first ? rd.amf_first : rd.amf_next)) push_desc(g, d);
        other.push_back(std::move(g));
      }
      const std::pair<int, bool> key{rd.R, first ? rd.joint_first : true};
      auto found = blf.find(key);
      if (found == blf.end()) {
        Group g{2};
        g.R = key.first;
        g.joint = key.second;
        found = blf.emplace(key, std::move(g)).first;
      }
      Group& bg = found->second;
      if (rd.filter == BLFLS_FILTER_BLF) {
        for (auto b : (first ? rd.blf_first : rd.blf_next)) {
          b.tile_begin = bg.items / 2;
          bg.items += 2 * b.tile_count;
          push_desc(bg, b);
        }
      }
      for (auto fp : (it + 1 == rd.iterations ? rd.fft_last : rd.fft)) {
        fp.row_begin = fft.items;
        fp.col_begin = fft.items2;
        fft.items += fp.row_count;
        fft.items2 += fp.col_count;
        fft.wave_cols = fft.wave_cols || fp.colw != 0 || fp.roww != 0;
        push_desc(fft, fp);
      }
      fft.lds_rows = std::max(fft.lds_rows, jb->plan->lds_rows);
      fft.lds_cols = std::max(fft.lds_cols, jb->plan->lds_cols);
    }
    mm.items = mm.n * kMinmaxBlocks;
    if (mm.n) groups.push_back(std::move(mm));
    for (auto& kv : blf)
      if (kv.second.n) groups.push_back(std::move(kv.second));
    for (auto& g : other) groups.push_back(std::move(g));
    if (fft.n) groups.push_back(std::move(fft));
  }
  return groups;
}

// LDS of the captured FFT launches: steps whose images all fit the small class
// keep four FFT workgroups per CU instead of the worst case's two.  The class
// stays 256 bytes under a quarter of the CU's 160 KiB, which leaves room for
// the kernels' static LDS (the item counter).
constexpr size_t kFftLdsSmall = 40960 - 256;

static size_t fft_lds_class(const Group& g, size_t lds_max) {
  return std::max(g.lds_rows, g.lds_cols) <= kFftLdsSmall ? kFftLdsSmall : lds_max;
}

static std::vector<int> signature(const std::vector<Group>& groups) {
  std::vector<int> sig;
  for (const Group& g : groups) {
    sig.push_back(g.kind);
    if (g.kind == 2) sig.push_back(g.R * 2 + (g.joint ? 1 : 0));
    else if (g.kind == 3) sig.push_back(std::max(g.lds_rows, g.lds_cols) <= kFftLdsSmall ? 1 : 2);
    else sig.push_back(0);
  }
  return sig;
}

// Direct launches (each kernel sized to its work), for steps that do not fit the
// fixed descriptor layout of a captured graph.
hipError_t blfls_server_s::launch_direct(std::vector<Group>& groups, int slot, int ft, size_t tables_used) {
  uint8_t* host = staging[slot];
  uint8_t* dev = arena + slot * stage_bytes;
  size_t used = tables_used;
  std::vector<size_t> offs;
  for (Group& g : groups) {
    used = align_up(used, 256);
    if (used + g.planes.size() > stage_bytes) return hipErrorOutOfMemory;
    std::memcpy(host + used, g.planes.data(), g.planes.size());
    offs.push_back(used);
    used += g.planes.size();
  }
  hipError_t e = hipMemcpyAsync(dev, host, used, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  for (size_t i = 0; i < groups.size(); ++i) {
    const Group& g = groups[i];
    const uint8_t* d = dev + offs[i];
    switch (g.kind) {
      case 0: e = launch_gauss(reinterpret_cast<const AuxPlane*>(d), g.n, g.max_pix, stream); break;
      case 1: e = launch_minmax(reinterpret_cast<const AuxPlane*>(d), g.n, stream); break;
      case 2: e = launch_blf(g.R, reinterpret_cast<const BlfPlane*>(d), g.n, g.items, g.joint, ft, stream); break;
      case 4: e = launch_other_filter(*g.job, d, g.joint, ft); break;
      default: {
        const FftPlane* fp = reinterpret_cast<const FftPlane*>(d);
        e = launch_fft_rows_fwd(fp, g.n, g.items, g.lds_rows, ft, stream);
        if (e == hipSuccess) e = launch_fft_cols(fp, g.n, g.items2, g.lds_cols, stream);
        if (e == hipSuccess) e = launch_fft_rows_inv(fp, g.n, g.items, g.lds_rows, stream);
      }
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One request's NC, grid or AMF stage, as blfls_smooth queues it, reading the
// descriptors staged at `planes`.
hipError_t blfls_server_s::launch_other_filter(const Job& jb, const uint8_t* planes, bool joint, int ft) {
  const RequestDesc& rd = jb.rd;
  const blfls_plan_s* plan = jb.plan;
  const int C = plan->C;
  if (rd.filter == BLFLS_FILTER_NC) {
    const NcPlane* np = reinterpret_cast<const NcPlane*>(planes);
    const int passes = 2 * rd.nc_rounds;
    for (int pass = 0; pass < passes; ++pass) {
      const int k = pass / 2;
      const int n_items = (pass & 1) ? C * nc_col_items(plan->H, plan->W) : C * nc_row_items(plan->H, plan->W);
      const hipError_t e = launch_nc_pass(np, C, n_items, pass, passes, rd.nc_r[k], rd.nc_R[k], ft, stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (rd.filter == BLFLS_FILTER_GRID)
    return launch_grid(reinterpret_cast<const GridPlane*>(planes), C, 2 * C * rd.grid_first[0].tile_count,
                       grid_z_stride(rd.grid_first[0]), !joint, ft, stream);
  AmfGeom G = rd.amf_geom;
  G.planes = reinterpret_cast<const AmfPlane*>(planes);
  return launch_amf(G, rd.amf_slots, rd.amf_height, stream);
}

// Capture the persistent launches of one step signature for one staging slot.
// Every kernel reads its items and its descriptor array from the slot's work
// header in device memory, so the graph replays unchanged with new work.
hipError_t blfls_server_s::build_graph(const std::vector<Group>& groups, int slot, int ft, hipGraphExec_t* out) {
  WorkHeader* header = reinterpret_cast<WorkHeader*>(arena + slot * stage_bytes);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (size_t i = 0; i < groups.size() && le == hipSuccess; ++i) {
    const Group& g = groups[i];
    WorkHeader* w = header + i;
    switch (g.kind) {
      case 0: le = launch_gauss(nullptr, 0, 0, capture_stream, w, kAuxGrid); break;
      case 1: le = launch_minmax(nullptr, 0, capture_stream, w, kAuxGrid); break;
      case 2: le = launch_blf(g.R, nullptr, 0, kBlfGrid, g.joint, ft, capture_stream, w); break;
      default: {
        const size_t lds = fft_lds_class(g, kFftLdsMax);
        le = launch_fft_rows_fwd(nullptr, 0, kFftGrid, lds, ft, capture_stream, w);
        if (le == hipSuccess) le = launch_fft_cols(nullptr, 0, kFftGrid, lds, capture_stream, w);
        if (le == hipSuccess) le = launch_fft_rows_inv(nullptr, 0, kFftGrid, lds, capture_stream, w);
      }
    }
  }
  e = hipStreamEndCapture(capture_stream, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return le;
  }
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  return e;
}

hipError_t blfls_server_s::launch_step(Step& st, int slot) {
  const int ft = precision == BLFLS_FP32 ? kF32 : precision == BLFLS_MIXED_BF16 ? kBF16 : kF16;
  uint8_t* host = staging[slot];
  uint8_t* dev = arena + slot * stage_bytes;
  // slot layout: [work header][request tables][packed descriptor arrays]; the
  // BLF and Gaussian descriptors point at their request's tables
  const size_t tables_base = kHeaderBytes;
  for (size_t j = 0; j < st.jobs.size(); ++j) {
    Job* jb = st.jobs[j];
    const blfls_request& q = jb->req;
    const size_t toff = tables_base + j * sizeof(RequestTables);
    build_request(jb->plan, q.params, jb->radius, q.f, q.guide, q.u, q.pitch, arena + jb->ws_off, dev + toff, &jb->rd);
    std::memcpy(host + toff, &jb->rd.tables, sizeof(RequestTables));
  }
  size_t used = tables_base + st.jobs.size() * sizeof(RequestTables);
  std::vector<Group> groups = build_groups(st.jobs);
  bool direct = static_cast<int>(groups.size()) > kMaxGroups;
  // per-request filters launch directly, and so do Fourier passes that hold one
  // column or row per wave (the captured persistent kernels have no such path)
  for (const Group& g : groups) direct = direct || g.kind == 4 || g.wave_cols;
  if (direct) {
    stats_direct_steps++;
    const hipError_t e = launch_direct(groups, slot, ft, used);
    return e == hipSuccess ? hipEventRecord(st.done, stream) : e;
  }
  WorkHeader* header = reinterpret_cast<WorkHeader*>(host);
  std::memset(header, 0, kHeaderBytes);
  for (size_t i = 0; i < groups.size(); ++i) {
    used = align_up(used, 256);
    if (used + groups[i].planes.size() > stage_bytes) return hipErrorOutOfMemory;
    std::memcpy(host + used, groups[i].planes.data(), groups[i].planes.size());
    header[i].items = groups[i].items;
    header[i].nplanes = groups[i].n;
    header[i].items2 = groups[i].items2;
    header[i].planes = dev + used;
    used += groups[i].planes.size();
  }
  const auto key = std::make_pair(signature(groups), slot);
  auto it = graphs.find(key);
  if (it == graphs.end()) {
    hipGraphExec_t exec = nullptr;
    const hipError_t e = build_graph(groups, slot, ft, &exec);
    if (e != hipSuccess) return e;
    it = graphs.emplace(key, exec).first;
  }
  hipError_t e = hipMemcpyAsync(dev, host, used, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  e = hipGraphLaunch(it->second, stream);
  if (e != hipSuccess) return e;
  stats_graph_steps++;
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
    arena_alloc.release(jb->ws_off, jb->ws_bytes);
    running--;
    delete jb;
  }
  st.jobs.clear();
  st.busy = false;
  step_ms_total += ms;
  cv.notify_all();
}

void blfls_server_s::admit(std::vector<Job*>* admitted) {
  // descriptor budget of one step: header, per-group alignment, then requests
  size_t desc = kHeaderBytes + static_cast<size_t>(kMaxGroups) * 256;
  while (!queue.empty() && running < max_slots) {
    Job* jb = queue.front();
    if (desc + jb->desc_bytes > stage_bytes) break;  // the rest waits for the next step
    size_t off = 0;
    if (!arena_alloc.alloc(jb->ws_bytes, &off)) break;  // FIFO: the head waits for space
    desc += jb->desc_bytes;
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
  const size_t stage_bytes = kStageBytes;  // descriptor staging per in-flight step
  const size_t reserved = kDepth * stage_bytes;
  if (arena_bytes <= reserved) return set_error(BLFLS_E_NOMEM, "arena smaller than the descriptor region");
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
  s->stage_bytes = stage_bytes;
  s->kFftLdsMax = std::max(fft_rows_lds_bytes(kFftLdsComplex - 1, 1), fft_cols_lds_bytes(kFftLdsComplex, 1));
  e = hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) { delete s; return hip_error(e, "capture stream"); }
  s->arena_alloc.init(reserved, arena_bytes - reserved);
  s->stats.arena_bytes = arena_bytes - reserved;
  for (int i = 0; i < kDepth; ++i) {
    e = hipHostMalloc(reinterpret_cast<void**>(&s->staging[i]), stage_bytes, hipHostMallocDefault);
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
  const size_t ws_bytes = request_workspace_bytes(plan, r->params);
  if (ws_bytes > s->arena_bytes - s->desc_region)
    return set_error(BLFLS_E_NOMEM, "request workspace exceeds the arena");
  // staging bytes: tables, the Gaussian descriptors, and per iteration the
  // filter's descriptors (one group of its own, aligned, for the filters other
  // than the BLF), one FFT and one extrema descriptor per channel
  const int filt = r->params.filter;
  const size_t C = static_cast<size_t>(r->C);
  const size_t filter_group = filt == BLFLS_FILTER_NC     ? C * sizeof(NcPlane) + 256
                              : filt == BLFLS_FILTER_GRID ? C * sizeof(GridPlane) + 256
                              : filt == BLFLS_FILTER_AMF  ? 2 * C * sizeof(AmfPlane) + 256
                                                          : C * sizeof(BlfPlane);
  const size_t desc_bytes = sizeof(RequestTables) + 16 + 2 * C * sizeof(AuxPlane) +
                            static_cast<size_t>(r->params.iterations) *
                                (filter_group + C * (sizeof(FftPlane) + sizeof(AuxPlane)));
  if (desc_bytes + blfls_server_s::kHeaderBytes + blfls_server_s::kMaxGroups * 256 > s->stage_bytes)
    return set_error(BLFLS_E_NOMEM, "too many iterations for one server step");
  auto* jb = new (std::nothrow) Job();
  if (!jb) return set_error(BLFLS_E_NOMEM, "host allocation failed");
  jb->desc_bytes = desc_bytes;
  jb->ws_bytes = ws_bytes;
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
  out->graph_steps = s->stats_graph_steps.load(std::memory_order_relaxed);
  out->direct_steps = s->stats_direct_steps.load(std::memory_order_relaxed);
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
  for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
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
