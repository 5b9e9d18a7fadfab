// Layout build (Sec. 3.3): Morton order of the Gaussian centres, so that
// contiguous runs of B rows (the blocks) are spatially compact.
#include <algorithm>
#include <cmath>
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
  // (code, row) pairs are unique, so an unstable sort of the pairs is the
  // stable order by code; chunks are sorted on threads and merged pairwise.
  std::vector<std::pair<uint64_t, int64_t>> kv((size_t)n);
  auto fill = [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      uint64_t c = 0;
      for (int a = 0; a < 3; ++a) {
        const double q = std::floor((xyz[i * stride + a] - lo[a]) * scale[a]);
        const uint64_t u = (uint64_t)std::min(cells - 1.0, std::max(0.0, q));
        c |= spread3(u) << a;
      }
      kv[(size_t)i] = {c, i};
    }
  };
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(16, n / 65536));
  std::vector<int64_t> cut(nt + 1);
  for (int k = 0; k <= nt; ++k) cut[k] = n * k / nt;
  {
    std::vector<std::thread> th;
    for (int k = 0; k < nt; ++k)
      th.emplace_back([&, k] {
        fill(cut[k], cut[k + 1]);
        std::sort(kv.begin() + cut[k], kv.begin() + cut[k + 1]);
      });
    for (auto& t : th) t.join();
  }
  for (int width = 1; width < nt; width *= 2) {
    std::vector<std::thread> th;
    for (int k = 0; k + width < nt; k += 2 * width) {
      const int64_t a = cut[k], m = cut[k + width], b = cut[std::min(nt, k + 2 * width)];
      th.emplace_back([&, a, m, b] { std::inplace_merge(kv.begin() + a, kv.begin() + m, kv.begin() + b); });
    }
    for (auto& t : th) t.join();
  }
  for (int64_t i = 0; i < n; ++i) perm[i] = kv[(size_t)i].second;
  return TIDE_OK;
}
