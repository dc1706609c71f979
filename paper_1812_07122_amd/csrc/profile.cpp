// Per-stage GPU timing of the synchronous path with HIP events recorded on
// the caller's stream (no synchronisation while recording).
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/blfls.h"
#include "blfls_plan.h"
#include "blfls_profile.h"

namespace blfls {
namespace {
struct Record {
  int stage;
  hipEvent_t a, b;
};
std::atomic<bool> g_enabled{false};
std::mutex g_mu;
std::vector<Record> g_records;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool profile_enabled() { return g_enabled.load(std::memory_order_relaxed); }

StageTimer::StageTimer(int stage, hipStream_t s) : stage_(stage), s_(s) {
  if (!profile_enabled()) return;
  std::lock_guard<std::mutex> lk(g_mu);
  a_ = take_event();
  b_ = take_event();
  if (a_ && b_) (void)hipEventRecord(a_, s_);
}

StageTimer::~StageTimer() {
  if (!a_ || !b_) return;
  (void)hipEventRecord(b_, s_);
  std::lock_guard<std::mutex> lk(g_mu);
  g_records.push_back({stage_, a_, b_});
}

}  // namespace blfls

using namespace blfls;

extern "C" {

blfls_status blfls_profile_enable(int enable) {
  g_enabled.store(enable != 0);
  return BLFLS_OK;
}

blfls_status blfls_profile_read(blfls_profile* out, int reset) {
  if (out == nullptr) return set_error(BLFLS_E_INVALID, "out is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  for (const Record& r : g_records) {
    hipError_t e = hipEventSynchronize(r.b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return hip_error(e, "profile event");
    if (r.stage >= 0 && r.stage < BLFLS_STAGE_COUNT) {
      out->ms[r.stage] += ms;
      out->launches[r.stage] += 1;
    }
  }
  if (reset) {
    for (const Record& r : g_records) {
      g_pool.push_back(r.a);
      g_pool.push_back(r.b);
    }
    g_records.clear();
  }
  return BLFLS_OK;
}

}  // extern "C"
