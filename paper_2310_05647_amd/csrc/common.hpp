// Shared host/device helpers of libmrf: status handling, complex arithmetic, launch checks.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/mrf.h"

namespace mrf {

// Records a message for mrf_last_error() (thread-local) and returns the status.
mrf_status fail(mrf_status st, const std::string& msg);
void clear_error();

#define MRF_CHECK_HIP(expr)                                                        \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::mrf::fail(MRF_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define MRF_CHECK_LAUNCH()                                                         \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess)                                                          \
      return ::mrf::fail(MRF_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

#define MRF_REQUIRE(cond, st, msg)                                                 \
  do {                                                                             \
    if (!(cond)) return ::mrf::fail((st), (msg));                                  \
  } while (0)

// ------------------------------------------------------------------ complex
struct cf {
  float x, y;
};

__host__ __device__ inline cf cmake(float a, float b) { return cf{a, b}; }
__host__ __device__ inline cf cadd(cf a, cf b) { return cf{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cf csub(cf a, cf b) { return cf{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cf cmul(cf a, cf b) { return cf{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__host__ __device__ inline cf cconjmul(cf a, cf b) {  // conj(a) * b
  return cf{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__host__ __device__ inline cf cscale(cf a, float s) { return cf{a.x * s, a.y * s}; }
__host__ __device__ inline cf cconj(cf a) { return cf{a.x, -a.y}; }

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------------ per-kernel timing
// While enabled (mrf_timing_enable), each launch wrapped by MRF_LAUNCH is bracketed by two
// HIP events recorded on its own stream; mrf_timing_report aggregates them by name.
bool timing_on();
void timing_mark(const char* name, hipStream_t s, bool begin);

#define MRF_LAUNCH(name, stream, ...)                                  \
  do {                                                                 \
    const bool t_ = ::mrf::timing_on();                                \
    if (t_) ::mrf::timing_mark(name, stream, true);                    \
    __VA_ARGS__;                                                       \
    if (t_) ::mrf::timing_mark(name, stream, false);                   \
  } while (0)

}  // namespace mrf
