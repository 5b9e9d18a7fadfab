// Thread-local error message behind tide_last_error().
#include <cstdarg>

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

}  // namespace tide

extern "C" const char* tide_last_error(void) { return tide::g_err; }
extern "C" int32_t tide_abi_version(void) { return 1; }
