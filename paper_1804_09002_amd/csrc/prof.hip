// Per-kernel timing with HIP events on the launching stream.
//
// When enabled (zcsd_profile_begin), instrumented launch sites bracket each
// launch with a pair of events recorded on the stream the kernel runs on (the
// matrix products attach them to the dispatch itself through
// hipExtLaunchKernelGGL) and add its algorithmic flop and byte counts to a
// per-kernel record; queries synchronise on the events and sum
// hipEventElapsedTime.  Disabled, a launch site costs one branch.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "zcsd_internal.h"
#include "zcsd_prof.h"

namespace zcsd {

namespace {
struct Rec {
  long long launches = 0;
  double flops = 0.0, bytes = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double ms_done = 0.0;
};
struct State {
  bool on = false;
  std::string filter;  // empty: every record
  std::map<std::string, Rec> recs;
  std::vector<hipEvent_t> pool;
  std::mutex mu;
};
State& st() {
  static State s;
  return s;
}
hipEvent_t get_event() {
  State& s = st();
  if (!s.pool.empty()) {
    hipEvent_t e = s.pool.back();
    s.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  ZCSD_HIP(hipEventCreate(&e));
  return e;
}
void settle(Rec& r) {
  for (auto& p : r.ev) {
    ZCSD_HIP(hipEventSynchronize(p.second));
    float ms = 0.f;
    ZCSD_HIP(hipEventElapsedTime(&ms, p.first, p.second));
    r.ms_done += ms;
    st().pool.push_back(p.first);
    st().pool.push_back(p.second);
  }
  r.ev.clear();
}
}  // namespace

bool prof_on() { return st().on; }

ProfScope::ProfScope(const char* name, hipStream_t s, double flops, double bytes, bool ext)
    : name_(name), s_(s), flops_(flops), bytes_(bytes) {
  if (!st().on) return;
  if (!st().filter.empty() && st().filter != name_) return;
  active_ = true;
  ext_ = ext;
  std::lock_guard<std::mutex> g(st().mu);
  e0_ = get_event();
  e1_ = get_event();
  if (!ext_) ZCSD_HIP(hipEventRecord(static_cast<hipEvent_t>(e0_), s_));
}

ProfScope::~ProfScope() {
  if (!active_) return;
  std::lock_guard<std::mutex> g(st().mu);
  if (!ext_) (void)hipEventRecord(static_cast<hipEvent_t>(e1_), s_);
  Rec& r = st().recs[name_];
  r.launches += 1;
  r.flops += flops_;
  r.bytes += bytes_;
  r.ev.emplace_back(static_cast<hipEvent_t>(e0_), static_cast<hipEvent_t>(e1_));
}

}  // namespace zcsd

using namespace zcsd;

extern "C" {

void zcsd_profile_begin(void) {
  std::lock_guard<std::mutex> g(st().mu);
  for (auto& kv : st().recs) {
    try {
      settle(kv.second);
    } catch (...) {
    }
  }
  st().recs.clear();
  st().on = true;
}

void zcsd_profile_end(void) { st().on = false; }

void zcsd_profile_filter(const char* name) {
  std::lock_guard<std::mutex> g(st().mu);
  st().filter = name ? name : "";
}

int zcsd_profile_query(const char* name, long long* launches, double* flops, double* bytes,
                       double* ms) {
  std::lock_guard<std::mutex> g(st().mu);
  auto it = st().recs.find(name ? name : "");
  if (it == st().recs.end()) return 0;
  try {
    settle(it->second);
  } catch (...) {
    return 0;
  }
  if (launches) *launches = it->second.launches;
  if (flops) *flops = it->second.flops;
  if (bytes) *bytes = it->second.bytes;
  if (ms) *ms = it->second.ms_done;
  return 1;
}

int zcsd_profile_names(char* buf, int len) {
  std::lock_guard<std::mutex> g(st().mu);
  std::string all;
  for (auto& kv : st().recs) {
    all += kv.first;
    all += '\n';
  }
  if (buf && len > 0) {
    const int c = (int)std::min<size_t>(all.size(), (size_t)len - 1);
    all.copy(buf, c);
    buf[c] = 0;
  }
  return (int)all.size();
}

}  // extern "C"
