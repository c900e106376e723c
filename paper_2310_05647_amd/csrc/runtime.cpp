// Status strings, thread-local error messages and the version query of libmrf.
#include <string>

#include "../../include/mrf.h"

namespace {
thread_local std::string g_last_error;
}

namespace mrf {

mrf_status fail(mrf_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

void clear_error() { g_last_error.clear(); }

}  // namespace mrf

extern "C" const char* mrf_status_string(mrf_status st) {
  switch (st) {
    case MRF_OK: return "MRF_OK";
    case MRF_INVALID_ARG: return "MRF_INVALID_ARG";
    case MRF_SHAPE: return "MRF_SHAPE";
    case MRF_WORKSPACE: return "MRF_WORKSPACE";
    case MRF_DEVICE: return "MRF_DEVICE";
    case MRF_OOM: return "MRF_OOM";
    case MRF_NONFINITE: return "MRF_NONFINITE";
    case MRF_NOT_SUPPORTED: return "MRF_NOT_SUPPORTED";
  }
  return "MRF_UNKNOWN";
}

extern "C" const char* mrf_last_error(void) { return g_last_error.c_str(); }

extern "C" int mrf_version(void) { return 100; }
