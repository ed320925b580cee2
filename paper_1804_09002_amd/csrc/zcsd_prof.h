// Per-kernel event timing (prof.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace zcsd {

bool prof_on();

// RAII: records an event pair around the launches made while it is alive.
// With ext = true it records nothing itself: the launch site passes
// ext_start() and ext_stop() to hipExtLaunchKernelGGL, which attaches them to
// the dispatches (the kernels' own start and end, without marker packets);
// both are null while profiling is off or filtered out.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t s, double flops, double bytes, bool ext = false);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;
  hipEvent_t ext_start() const { return static_cast<hipEvent_t>(ext_ ? e0_ : nullptr); }
  hipEvent_t ext_stop() const { return static_cast<hipEvent_t>(ext_ ? e1_ : nullptr); }

 private:
  const char* name_;
  hipStream_t s_;
  double flops_, bytes_;
  bool active_ = false;
  bool ext_ = false;
  void* e0_ = nullptr;
  void* e1_ = nullptr;
};

}  // namespace zcsd
