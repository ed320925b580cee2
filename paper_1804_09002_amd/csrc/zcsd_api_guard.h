// Exception -> zcsd_status boundary used by every extern "C" entry point.
#pragma once
#include <cstdio>
#include <cstdlib>

#include "zcsd_internal.h"

namespace zcsd {

inline bool log_enabled() {
  static const bool v = [] {
    const char* e = std::getenv("ZCSD_LOG");
    return e && e[0] && e[0] != '0';
  }();
  return v;
}

template <class F>
zcsd_status guarded(F&& f) {
  try {
    f();
    return ZCSD_OK;
  } catch (const ArgError& e) {
    if (log_enabled()) std::fprintf(stderr, "[zcsd] %s\n", e.what());
    return ZCSD_EINVAL;
  } catch (const NumError& e) {
    if (log_enabled()) std::fprintf(stderr, "[zcsd] %s\n", e.what());
    return e.code;
  } catch (const HipError& e) {
    std::fprintf(stderr, "[zcsd] HIP error: %s\n", e.what());
    return ZCSD_EHIP;
  } catch (const std::bad_alloc&) {
    return ZCSD_ENOMEM;
  } catch (const std::exception& e) {
    std::fprintf(stderr, "[zcsd] error: %s\n", e.what());
    return ZCSD_EHIP;
  }
}

}  // namespace zcsd
