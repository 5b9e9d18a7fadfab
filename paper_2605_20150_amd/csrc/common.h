// Shared host/device helpers of the HIP library: error reporting, math
// traits for the float/double instantiations and wave64 primitives.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "tide.h"

namespace tide {

// ------------------------------------------------------------ error state
void set_error(const char* fmt, ...);
tide_status hip_fail(hipError_t e, const char* what);
// Records the events armed for `kernel` (tide_timer_arm) on `st`.
void timer_mark(const char* kernel, hipStream_t st, bool begin);
// N (rows) and B (rows per block) of a tier.
void residency_shape(const tide_residency* res, int64_t* n_rows, int32_t* block_rows);

#define TIDE_CHECK_ARG(cond, ...)          \
  do {                                     \
    if (!(cond)) {                         \
      ::tide::set_error(__VA_ARGS__);      \
      return TIDE_EINVAL;                  \
    }                                      \
  } while (0)

#define TIDE_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return ::tide::hip_fail(e_, #call); \
  } while (0)

// Launch wrapped by the timing hook: TIDE_TIMED("name", stream, launch...).
#define TIDE_TIMED(name, st, ...)                \
  do {                                           \
    ::tide::timer_mark(name, st, true);          \
    __VA_ARGS__;                                 \
    ::tide::timer_mark(name, st, false);         \
  } while (0)

#define TIDE_LAUNCH_CHECK(what)                               \
  do {                                                        \
    hipError_t e_ = hipGetLastError();                        \
    if (e_ != hipSuccess) return ::tide::hip_fail(e_, what);  \
  } while (0)

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Carves aligned sub-buffers out of one caller workspace.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename X>
  X* take(size_t count) {
    X* p = base ? reinterpret_cast<X*>(base + used) : nullptr;
    used = align_up(used + count * sizeof(X));
    return p;
  }
};

// ---------------------------------------------------------------- math
template <typename T>
struct Mth;

template <>
struct Mth<float> {
  __device__ static float exp(float x) { return __expf(x); }
  __device__ static float sqrt(float x) { return sqrtf(x); }
  __device__ static float rcp(float x) { return __frcp_rn(x); }
  __device__ static float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
  __device__ static float log(float x) { return __logf(x); }
  __device__ static float ceil(float x) { return ceilf(x); }
  __device__ static float floor(float x) { return floorf(x); }
};

template <>
struct Mth<double> {
  __device__ static double exp(double x) { return ::exp(x); }
  __device__ static double sqrt(double x) { return ::sqrt(x); }
  __device__ static double rcp(double x) { return 1.0 / x; }
  __device__ static double rcp_fast(double x) { return 1.0 / x; }
  __device__ static double log(double x) { return ::log(x); }
  __device__ static double ceil(double x) { return ::ceil(x); }
  __device__ static double floor(double x) { return ::floor(x); }
};

// ------------------------------------------------------------ wave64
constexpr int kWave = 64;

__device__ inline uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Sum over the 64 lanes; the result is valid in every lane.
template <typename T>
__device__ inline T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// Inclusive prefix sum over the 64 lanes (Hillis-Steele on shuffles).
__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  const int lane = __lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  return x;
}

}  // namespace tide
