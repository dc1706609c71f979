// Scoped recorder of one kernel family's bracketing events (active only while
// blfls_profile_enable(1) is in effect).
#pragma once

#include <hip/hip_runtime.h>

namespace blfls {

bool profile_enabled();

class StageTimer {
 public:
  StageTimer(int stage, hipStream_t s);
  ~StageTimer();
  StageTimer(const StageTimer&) = delete;
  StageTimer& operator=(const StageTimer&) = delete;

 private:
  int stage_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace blfls
