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
// a result is bitwise the same alone and in any mix.  Queueing, admission,
// tickets, retirement and latencies live in the GPU-independent scheduling
// core (server_core.h); this file is its HIP executor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/blfls.h"
#include "blfls_internal.h"
#include "blfls_launch.h"
#include "blfls_plan.h"
#include "server_core.h"

namespace blfls {
namespace {

constexpr size_t kStageBytes = 8u << 20;  // descriptor staging per in-flight step
constexpr int kDepth = 2;                 // steps in flight

size_t align_up(size_t v, size_t a) { return core_align_up(v, a); }

constexpr int kMaxGraphs = 32;            // captured step graphs kept (least recently used evicted)

struct Job : CoreJob {
  blfls_request req{};
  int radius = 0;
  blfls_plan_s* plan = nullptr;
  RequestDesc rd;
};

// One launch group of a step: a kernel family over an array of plane descriptors.
// Kind 4 is one request's NC, grid or AMF filter stage, launched directly.
struct Group {
  int kind;  // 0 gauss, 1 minmax, 2 blf, 3 fft, 4 other filter (one request)
  int R = 0;
  bool joint = false;
  bool pair = false;            // kind 2: the symmetric-pair filter (items: bands, items2: merge items)
  const Job* job = nullptr;     // kind 4: the request
  std::vector<uint8_t> planes;  // descriptor array bytes
  int n = 0;                    // planes
  int items = 0, items2 = 0;    // work items (fft: rows, cols)
  size_t lds_rows = 0, lds_cols = 0;
  int64_t max_pix = 0;
  bool wave_cols = false;       // fft: a plane's passes hold one column or row per wave
};

}  // namespace
}  // namespace blfls

using namespace blfls;

struct blfls_server_s {
  uint8_t* arena = nullptr;
  size_t arena_bytes = 0;
  size_t desc_region = 0;  // bytes of arena reserved for device descriptors (kDepth * kStageBytes)
  blfls_precision precision = BLFLS_FP32;
  hipStream_t stream = nullptr;
  int device = 0;

  SchedulerCore<Job, kDepth> core;
  std::mutex plans_mu;
  std::map<std::tuple<int, int, int>, blfls_plan_s*> plans;
  uint8_t* staging[kDepth] = {nullptr, nullptr};
  hipEvent_t done[kDepth] = {nullptr, nullptr};

  // staging layout of one slot: [work header][request tables][descriptor arrays]
  static constexpr size_t kHeaderBytes = 16384;
  static constexpr int kMaxGroups = static_cast<int>(kHeaderBytes / sizeof(WorkHeader));
  static constexpr int kBlfGrid = 2048;  // persistent grids of the captured kernels
  static constexpr int kPairGrid = 3072;  // one-wave workgroups of the pair filter
  static constexpr int kMergeGrid = 1024;
  static constexpr int kFftGrid = 1024;
  static constexpr int kAuxGrid = 1024;
  size_t stage_bytes = 0;
  size_t kFftLdsMax = 0;
  hipStream_t capture_stream = nullptr;
  struct CachedGraph {
    hipGraphExec_t exec = nullptr;
    uint64_t last_step = 0;  // launch index of the last step that replayed it
  };
  std::map<std::pair<std::vector<int>, int>, CachedGraph> graphs;
  // read by blfls_server_stats from other threads
  std::atomic<uint64_t> stats_graph_steps{0}, stats_direct_steps{0};

  // executor of the scheduling core (called on its scheduler thread)
  int launch(std::vector<Job*>& jobs, int slot);
  int query(int slot);
  void drain(int slot, int err);

  hipError_t launch_step(std::vector<Job*>& jobs, int slot);
  hipError_t launch_direct(std::vector<Group>& groups, int slot, int ft, size_t tables_used);
  hipError_t launch_other_filter(const Job& jb, const uint8_t* planes, bool joint, int ft);
  hipError_t build_graph(const std::vector<Group>& groups, int slot, int ft, hipGraphExec_t* out);
  void evict_graph();
  std::shared_ptr<void> exec_holder;   // the core's executor (owned here, outlives the core's thread)
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
    std::map<std::tuple<int, bool, bool>, Group> blf;
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
      if (rd.filter == BLFLS_FILTER_BLF) {
        const std::tuple<int, bool, bool> key{rd.R, first ? rd.joint_first : true, rd.pair};
        auto found = blf.find(key);
        if (found == blf.end()) {
          Group g{2};
          g.R = std::get<0>(key);
          g.joint = std::get<1>(key);
          g.pair = std::get<2>(key);
          found = blf.emplace(key, std::move(g)).first;
        }
        Group& bg = found->second;
        for (auto b : (first ? rd.blf_first : rd.blf_next)) {
          b.tile_begin = bg.items / 2;
          bg.items += 2 * b.tile_count;
          if (rd.pair) {
            b.merge_begin = bg.items2 / 2;
            bg.items2 += 2 * b.merge_count;
          }
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
    if (g.kind == 2) sig.push_back(g.R * 4 + (g.pair ? 2 : 0) + (g.joint ? 1 : 0));
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
      case 2:
        e = g.pair ? launch_blf_pair(g.R, reinterpret_cast<const BlfPlane*>(d), g.n, g.items, g.items2, g.joint, ft,
                                     stream)
                   : launch_blf(g.R, reinterpret_cast<const BlfPlane*>(d), g.n, g.items, g.joint, ft, stream);
        break;
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
      case 2:
        le = g.pair ? launch_blf_pair(g.R, nullptr, 0, kPairGrid, kMergeGrid, g.joint, ft, capture_stream, w)
                    : launch_blf(g.R, nullptr, 0, kBlfGrid, g.joint, ft, capture_stream, w);
        break;
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

hipError_t blfls_server_s::launch_step(std::vector<Job*>& jobs, int slot) {
  const int ft = precision == BLFLS_FP32 ? kF32 : precision == BLFLS_MIXED_BF16 ? kBF16 : kF16;
  uint8_t* host = staging[slot];
  uint8_t* dev = arena + slot * stage_bytes;
  // slot layout: [work header][request tables][packed descriptor arrays]; the
  // BLF and Gaussian descriptors point at their request's tables
  const size_t tables_base = kHeaderBytes;
  for (size_t j = 0; j < jobs.size(); ++j) {
    Job* jb = jobs[j];
    const blfls_request& q = jb->req;
    const size_t toff = tables_base + j * sizeof(RequestTables);
    build_request(jb->plan, q.params, jb->radius, q.f, q.guide, q.u, q.pitch, arena + jb->ws_off, dev + toff, &jb->rd);
    std::memcpy(host + toff, &jb->rd.tables, sizeof(RequestTables));
  }
  size_t used = tables_base + jobs.size() * sizeof(RequestTables);
  std::vector<Group> groups = build_groups(jobs);
  bool direct = static_cast<int>(groups.size()) > kMaxGroups;
  // per-request filters launch directly, and so do Fourier passes that hold one
  // column or row per wave (the captured persistent kernels have no such path)
  for (const Group& g : groups) direct = direct || g.kind == 4 || g.wave_cols;
  if (direct) {
    stats_direct_steps++;
    const hipError_t e = launch_direct(groups, slot, ft, used);
    return e == hipSuccess ? hipEventRecord(done[slot], stream) : e;
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
    if (graphs.size() >= static_cast<size_t>(kMaxGraphs)) evict_graph();
    hipGraphExec_t exec = nullptr;
    const hipError_t e = build_graph(groups, slot, ft, &exec);
    if (e != hipSuccess) return e;
    it = graphs.emplace(key, CachedGraph{exec, 0}).first;
  }
  hipError_t e = hipMemcpyAsync(dev, host, used, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  e = hipGraphLaunch(it->second.exec, stream);
  if (e != hipSuccess) return e;
  it->second.last_step = core.launched_steps() + 1;   // this step's launch index
  stats_graph_steps++;
  return hipEventRecord(done[slot], stream);
}

// Destroy the least recently used graph that no step in flight replays: its
// last step has retired (steps retire in launch order).
void blfls_server_s::evict_graph() {
  const uint64_t retired = core.retired_steps();
  auto victim = graphs.end();
  for (auto it = graphs.begin(); it != graphs.end(); ++it)
    if (it->second.last_step <= retired && (victim == graphs.end() || it->second.last_step < victim->second.last_step))
      victim = it;
  if (victim == graphs.end()) return;
  (void)hipGraphExecDestroy(victim->second.exec);
  graphs.erase(victim);
}

int blfls_server_s::launch(std::vector<Job*>& jobs, int slot) {
  const hipError_t e = launch_step(jobs, slot);
  return e == hipSuccess ? 0 : -static_cast<int>(e);
}

int blfls_server_s::query(int slot) {
  const hipError_t q = hipEventQuery(done[slot]);
  if (q == hipErrorNotReady) return 1;
  return q == hipSuccess ? 0 : -static_cast<int>(q);
}

void blfls_server_s::drain(int slot, int err) {
  if (err == 0) (void)hipEventSynchronize(done[slot]);
  else (void)hipStreamSynchronize(stream);  // kernels launched before the error finish first
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
  s->precision = precision;
  s->stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) { delete s; return hip_error(e, "hipGetDevice"); }
  s->stage_bytes = stage_bytes;
  s->kFftLdsMax = std::max(fft_rows_lds_bytes(kFftLdsComplex - 1, 1), fft_cols_lds_bytes(kFftLdsComplex, 1));
  e = hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) { delete s; return hip_error(e, "capture stream"); }
  for (int i = 0; i < kDepth; ++i) {
    e = hipHostMalloc(reinterpret_cast<void**>(&s->staging[i]), stage_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->done[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      for (int j = 0; j <= i; ++j) {
        if (s->staging[j]) (void)hipHostFree(s->staging[j]);
        if (s->done[j]) (void)hipEventDestroy(s->done[j]);
      }
      (void)hipStreamDestroy(s->capture_stream);
      delete s;
      return hip_error(e, "server setup");
    }
  }
  CoreConfig cfg;
  cfg.arena_base = reserved;
  cfg.arena_bytes = arena_bytes - reserved;
  cfg.max_slots = max_slots;
  cfg.queue_cap = queue_capacity;
  cfg.step_budget = stage_bytes;
  // descriptor budget of one step: header, per-group alignment, then requests
  cfg.step_overhead = blfls_server_s::kHeaderBytes + static_cast<size_t>(blfls_server_s::kMaxGroups) * 256;
  s->core.configure(cfg);
  const int dev = s->device;
  struct Exec {
    blfls_server_s* s;
    int dev;
    bool bound = false;
    int launch(std::vector<Job*>& jobs, int slot) {
      if (!bound) { (void)hipSetDevice(dev); bound = true; }
      return s->launch(jobs, slot);
    }
    int query(int slot) { return s->query(slot); }
    void drain(int slot, int err) { s->drain(slot, err); }
  };
  static_assert(sizeof(Exec) <= 64, "executor state");
  auto* ex = new (std::nothrow) Exec{s, dev};
  if (!ex) { blfls_server_destroy(s); return set_error(BLFLS_E_NOMEM, "host allocation failed"); }
  s->exec_holder.reset(ex, [](void* p) { delete static_cast<Exec*>(p); });
  s->core.start(ex);
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
  const auto key = std::make_tuple(r->H, r->W, r->C);
  blfls_plan_s* plan = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->plans_mu);
    auto it = s->plans.find(key);
    if (it == s->plans.end()) {
      st = plan_create(r->H, r->W, r->C, s->precision, &plan);
      if (st != BLFLS_OK) return st;
      s->plans[key] = plan;
    } else {
      plan = it->second;
    }
  }
  const size_t ws_bytes = request_workspace_bytes(plan, r->params);
  // staging bytes: tables, the Gaussian and image-extrema descriptors, and per
  // iteration the filter's descriptors (one group of its own, aligned, for the
  // filters other than the BLF), one FFT and one extrema descriptor per channel
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
  jb->req = *r;
  jb->radius = radius;
  jb->plan = plan;
  st = s->core.submit(jb, ticket);
  if (st != BLFLS_OK) {
    delete jb;
    if (st == BLFLS_E_NOMEM) return set_error(st, "request workspace exceeds the arena");
    if (st == BLFLS_E_AGAIN) return set_error(st, "queue full");
    return set_error(st, "server is shutting down");
  }
  return BLFLS_OK;
}

blfls_status blfls_poll(blfls_server_t s, uint64_t ticket, int32_t* state, blfls_status* result) {
  if (s == nullptr || state == nullptr || result == nullptr) return set_error(BLFLS_E_INVALID, "NULL argument");
  const blfls_status st = s->core.poll(ticket, state, result);
  if (st != BLFLS_OK) return set_error(st, "unknown or retired ticket");
  return BLFLS_OK;
}

blfls_status blfls_server_stats(blfls_server_t s, blfls_stats* out) {
  if (s == nullptr || out == nullptr) return set_error(BLFLS_E_INVALID, "NULL argument");
  *out = blfls_stats{};
  s->core.fill_stats(out);
  out->graph_steps = s->stats_graph_steps.load(std::memory_order_relaxed);
  out->direct_steps = s->stats_direct_steps.load(std::memory_order_relaxed);
  return BLFLS_OK;
}

blfls_status blfls_server_destroy(blfls_server_t s) {
  if (s == nullptr) return set_error(BLFLS_E_INVALID, "server is NULL");
  s->core.stop();   // drains everything queued or in flight
  for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
  for (auto& kv : s->plans) plan_free(kv.second);
  for (int i = 0; i < kDepth; ++i) {
    if (s->staging[i]) (void)hipHostFree(s->staging[i]);
    if (s->done[i]) (void)hipEventDestroy(s->done[i]);
  }
  delete s;
  return BLFLS_OK;
}

}  // extern "C"
