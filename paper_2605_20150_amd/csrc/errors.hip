// Thread-local error message behind tide_last_error(), and the kernel timing
// hook behind tide_timer_arm().
#include <atomic>
#include <cstdarg>
#include <cstring>
#include <mutex>

#include "common.h"

namespace tide {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

tide_status hip_fail(hipError_t e, const char* what) {
  set_error("%s failed: %s", what, hipGetErrorString(e));
  return TIDE_EHIP;
}

namespace {
struct Armed {
  char name[32];
  hipEvent_t start, stop;
};
std::mutex g_mu;
Armed g_armed[16];
std::atomic<int> g_narmed{0};
}  // namespace

void timer_mark(const char* kernel, hipStream_t st, bool begin) {
  if (g_narmed.load(std::memory_order_relaxed) == 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  const int n = g_narmed.load();
  for (int i = 0; i < n; ++i)
    if (std::strcmp(g_armed[i].name, kernel) == 0)
      (void)hipEventRecord(begin ? g_armed[i].start : g_armed[i].stop, st);
}

}  // namespace tide

extern "C" const char* tide_last_error(void) { return tide::g_err; }
extern "C" int32_t tide_abi_version(void) { return 1; }

extern "C" tide_status tide_timer_arm(const char* kernel, void* ev_start, void* ev_stop) {
  using namespace tide;
  TIDE_CHECK_ARG(kernel && ev_start && ev_stop, "null argument");
  TIDE_CHECK_ARG(std::strlen(kernel) < sizeof(g_armed[0].name), "kernel name too long");
  std::lock_guard<std::mutex> lk(g_mu);
  const int n = g_narmed.load();
  for (int i = 0; i < n; ++i)
    if (std::strcmp(g_armed[i].name, kernel) == 0) {
      g_armed[i].start = (hipEvent_t)ev_start;
      g_armed[i].stop = (hipEvent_t)ev_stop;
      return TIDE_OK;
    }
  TIDE_CHECK_ARG(n < 16, "at most 16 kernels can be armed");
  std::strcpy(g_armed[n].name, kernel);
  g_armed[n].start = (hipEvent_t)ev_start;
  g_armed[n].stop = (hipEvent_t)ev_stop;
  g_narmed.store(n + 1);
  return TIDE_OK;
}

extern "C" tide_status tide_timer_clear(void) {
  std::lock_guard<std::mutex> lk(tide::g_mu);
  tide::g_narmed.store(0);
  return TIDE_OK;
}
