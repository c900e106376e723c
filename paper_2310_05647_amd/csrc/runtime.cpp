// Status strings, thread-local error messages, the version query and per-kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

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

// The build step passes the SHA-256 of the sources it compiled and the build time, so that a
// caller can tell whether the loaded library was built from the sources beside it.
#ifndef MRF_SOURCE_SHA
#define MRF_SOURCE_SHA "unknown"
#endif
#ifndef MRF_BUILD_TIME
#define MRF_BUILD_TIME "unknown"
#endif
extern "C" const char* mrf_build_info(void) {
  return "sources-sha256=" MRF_SOURCE_SHA " built=" MRF_BUILD_TIME " arch=gfx950";
}

// ------------------------------------------------------------------ timing
namespace {
struct Rec {
  const char* name;
  hipEvent_t a, b;
};
std::atomic<bool> g_timing{false};
std::mutex g_tmu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<std::pair<const char*, hipEvent_t>> g_open;

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

namespace mrf {
bool timing_on() { return g_timing.load(std::memory_order_relaxed); }

void timing_mark(const char* name, hipStream_t s, bool begin) {
  std::lock_guard<std::mutex> lk(g_tmu);
  hipEvent_t e = take_event();
  if (!e) return;
  hipEventRecord(e, s);
  if (begin) {
    g_open.emplace_back(name, e);
  } else {
    for (size_t i = g_open.size(); i-- > 0;) {
      if (std::strcmp(g_open[i].first, name) == 0) {
        g_recs.push_back(Rec{name, g_open[i].second, e});
        g_open.erase(g_open.begin() + (long)i);
        return;
      }
    }
    g_pool.push_back(e);
  }
}
}  // namespace mrf

extern "C" mrf_status mrf_timing_enable(int on) {
  mrf::clear_error();
  g_timing.store(on != 0);
  return MRF_OK;
}

extern "C" mrf_status mrf_timing_report(char* buf, size_t len) {
  mrf::clear_error();
  if (!buf || len == 0) return mrf::fail(MRF_INVALID_ARG, "timing_report: null buffer");
  std::lock_guard<std::mutex> lk(g_tmu);
  struct Agg { long n = 0; double tot = 0, mn = 1e300, mx = 0; };
  std::map<std::string, Agg> agg;
  mrf_status st = MRF_OK;
  for (auto& r : g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      st = mrf::fail(MRF_DEVICE, "timing_report: event query failed");
    } else {
      Agg& a = agg[r.name];
      a.n += 1; a.tot += ms; a.mn = std::min(a.mn, (double)ms); a.mx = std::max(a.mx, (double)ms);
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  std::string out;
  char line[256];
  for (auto& kv : agg) {
    std::snprintf(line, sizeof line, "%s %ld %.6f %.6f %.6f\n", kv.first.c_str(), kv.second.n, kv.second.tot,
                  kv.second.mn, kv.second.mx);
    out += line;
  }
  const size_t n = std::min(len - 1, out.size());
  std::copy(out.begin(), out.begin() + (long)n, buf);
  buf[n] = 0;
  return st;
}
