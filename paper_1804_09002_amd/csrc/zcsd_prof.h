// Per-kernel event timing (prof.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace zcsd {

bool prof_on();

// RAII: records an event pair around the launches made while it is alive.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t s, double flops, double bytes);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  double flops_, bytes_;
  bool active_ = false;
  void* e0_ = nullptr;
  void* e1_ = nullptr;
};

}  // namespace zcsd
