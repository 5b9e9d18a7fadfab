// Layout build (Sec. 3.3): Morton order of the Gaussian centres, so that
// contiguous runs of B rows (the blocks) are spatially compact.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>
#include <vector>

#include "common.h"

using namespace tide;

namespace {

// Spreads the low 21 bits of v so that bit i lands on bit 3 i.
inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

}  // namespace

extern "C" tide_status tide_morton_order(const float* xyz, int64_t n, int64_t stride, int64_t* perm) {
  TIDE_CHECK_ARG(n >= 0 && stride >= 3, "need n >= 0 and stride >= 3");
  if (n == 0) return TIDE_OK;
  TIDE_CHECK_ARG(xyz && perm, "null argument");
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) lo[a] = hi[a] = xyz[a];
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      const double v = xyz[i * stride + a];
      TIDE_CHECK_ARG(std::isfinite(v), "non-finite centre at row %lld", (long long)i);
      lo[a] = std::min(lo[a], v);
      hi[a] = std::max(hi[a], v);
    }
  const double cells = 2097152.0;   // 2^21 per axis
  double scale[3];
  for (int a = 0; a < 3; ++a) scale[a] = hi[a] > lo[a] ? cells / (hi[a] - lo[a]) : 0.0;
  std::vector<uint64_t> code((size_t)n);
  auto fill = [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      uint64_t c = 0;
      for (int a = 0; a < 3; ++a) {
        const double q = std::floor((xyz[i * stride + a] - lo[a]) * scale[a]);
        const uint64_t u = (uint64_t)std::min(cells - 1.0, std::max(0.0, q));
        c |= spread3(u) << a;
      }
      code[(size_t)i] = c;
    }
  };
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(16, n / 65536));
  std::vector<std::thread> th;
  for (int k = 0; k < nt; ++k) th.emplace_back(fill, n * k / nt, n * (k + 1) / nt);
  for (auto& t : th) t.join();
  std::iota(perm, perm + n, (int64_t)0);
  std::stable_sort(perm, perm + n, [&](int64_t a, int64_t b) { return code[(size_t)a] < code[(size_t)b]; });
  return TIDE_OK;
}
