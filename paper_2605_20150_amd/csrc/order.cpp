// View ordering (Sec. 3.5, App. A): a clustered travelling-salesperson
// order of the training cameras, so that consecutive batches see
// overlapping block sets.  Host code; the views are few (hundreds to
// thousands) and the order is computed once per pass.
//
// Steps (the paper names the method, not its parts; this is the reading the
// library implements):
//   1. d(i, j) = |p_i - p_j| + w |f_i - f_j|, p the camera centre, f the unit
//      viewing direction, w in metres (0: positions only).
//   2. k = ceil(n / cluster_size) clusters of the centres: farthest-point
//      seeds from view 0, then Lloyd iterations until no view changes
//      cluster (at most 100).
//   3. The non-empty clusters are visited along an open path over their
//      centroids that starts at view 0's cluster: nearest neighbour, then
//      2-opt.
//   4. Inside each cluster, an open path over its views with d, entered at
//      the view nearest the previous cluster's last view (view 0 for the
//      first cluster): nearest neighbour, then 2-opt.
// Ties go to the lower index everywhere; a 2-opt move is taken when it
// shortens the path by more than 1e-9.
#include <cmath>
#include <vector>

#include "common.h"

using namespace tide;

namespace {

struct V3 {
  double x, y, z;
};

double dist(const V3& a, const V3& b) {
  const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  return std::sqrt(dx * dx + dy * dy + dz * dz);
}

double dist2(const V3& a, const V3& b) {
  const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  return dx * dx + dy * dy + dz * dz;
}

// 2-opt on an open path whose first element stays first.  D(a, b) is the
// cost between two elements of x.
template <class Dist>
void two_opt(std::vector<int32_t>& x, Dist D) {
  const size_t m = x.size();
  if (m < 3) return;
  bool improved = true;
  while (improved) {
    improved = false;
    for (size_t i = 1; i + 1 < m; ++i)
      for (size_t j = i + 1; j < m; ++j) {
        const bool tail = j + 1 < m;
        const double before = D(x[i - 1], x[i]) + (tail ? D(x[j], x[j + 1]) : 0.0);
        const double after = D(x[i - 1], x[j]) + (tail ? D(x[i], x[j + 1]) : 0.0);
        if (after < before - 1e-9) {
          for (size_t a = i, b = j; a < b; ++a, --b) std::swap(x[a], x[b]);
          improved = true;
        }
      }
  }
}

// Nearest-neighbour open path over `items` starting at `start`.
template <class Dist>
std::vector<int32_t> nn_path(const std::vector<int32_t>& items, int32_t start, Dist D) {
  std::vector<int32_t> path{start};
  std::vector<char> used(items.size(), 0);
  for (size_t a = 0; a < items.size(); ++a)
    if (items[a] == start) used[a] = 1;
  for (size_t step = 1; step < items.size(); ++step) {
    const int32_t cur = path.back();
    int best = -1;
    double bd = 0.0;
    for (size_t a = 0; a < items.size(); ++a) {
      if (used[a]) continue;
      const double v = D(cur, items[a]);
      if (best < 0 || v < bd) { best = (int)a; bd = v; }   // items ascend: ties keep the lower
    }
    used[best] = 1;
    path.push_back(items[best]);
  }
  return path;
}

}  // namespace

extern "C" tide_status tide_view_order(const tide_camera* cams, int64_t n, int32_t cluster_size,
                                       double dir_weight, int32_t* perm) {
  TIDE_CHECK_ARG(n >= 0 && n <= (int64_t)INT32_MAX, "bad view count");
  if (n == 0) return TIDE_OK;
  TIDE_CHECK_ARG(cams && perm, "null argument");
  TIDE_CHECK_ARG(cluster_size >= 1, "cluster_size must be >= 1");
  TIDE_CHECK_ARG(dir_weight >= 0.0 && std::isfinite(dir_weight), "dir_weight must be finite and >= 0");
  std::vector<V3> p((size_t)n), f((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    const double* R = cams[i].R;
    const double* t = cams[i].t;
    // centre -R^T t; the viewing direction is R's third row (camera +z)
    p[i] = {-(R[0] * t[0] + R[3] * t[1] + R[6] * t[2]), -(R[1] * t[0] + R[4] * t[1] + R[7] * t[2]),
            -(R[2] * t[0] + R[5] * t[1] + R[8] * t[2])};
    f[i] = {R[6], R[7], R[8]};
    TIDE_CHECK_ARG(std::isfinite(p[i].x) && std::isfinite(p[i].y) && std::isfinite(p[i].z),
                   "non-finite camera %lld", (long long)i);
  }
  auto d = [&](int32_t i, int32_t j) { return dist(p[i], p[j]) + dir_weight * dist(f[i], f[j]); };

  // 2. clusters of the centres
  const int64_t k = (n + cluster_size - 1) / cluster_size;
  std::vector<V3> c((size_t)k);
  c[0] = p[0];
  std::vector<double> near((size_t)n);
  for (int64_t i = 0; i < n; ++i) near[i] = dist2(p[i], c[0]);
  for (int64_t m = 1; m < k; ++m) {
    int64_t best = 0;
    for (int64_t i = 1; i < n; ++i)
      if (near[i] > near[best]) best = i;
    c[m] = p[best];
    for (int64_t i = 0; i < n; ++i) near[i] = std::min(near[i], dist2(p[i], c[m]));
  }
  std::vector<int32_t> asg((size_t)n, -1);
  for (int it = 0; it < 100; ++it) {
    bool changed = false;
    for (int64_t i = 0; i < n; ++i) {
      int32_t bm = 0;
      double bd = dist2(p[i], c[0]);
      for (int64_t m = 1; m < k; ++m) {
        const double v = dist2(p[i], c[m]);
        if (v < bd) { bd = v; bm = (int32_t)m; }
      }
      if (asg[i] != bm) { asg[i] = bm; changed = true; }
    }
    if (!changed) break;
    std::vector<V3> sum((size_t)k, V3{0.0, 0.0, 0.0});
    std::vector<int64_t> cnt((size_t)k, 0);
    for (int64_t i = 0; i < n; ++i) {
      V3& s = sum[asg[i]];
      s.x += p[i].x;
      s.y += p[i].y;
      s.z += p[i].z;
      ++cnt[asg[i]];
    }
    for (int64_t m = 0; m < k; ++m)
      if (cnt[m] > 0) c[m] = {sum[m].x / (double)cnt[m], sum[m].y / (double)cnt[m], sum[m].z / (double)cnt[m]};
  }
  std::vector<std::vector<int32_t>> members((size_t)k);
  for (int64_t i = 0; i < n; ++i) members[asg[i]].push_back((int32_t)i);

  // 3. path over the non-empty clusters from view 0's
  std::vector<int32_t> nonempty;
  for (int64_t m = 0; m < k; ++m)
    if (!members[m].empty()) nonempty.push_back((int32_t)m);
  auto dc = [&](int32_t a, int32_t b) { return dist(c[a], c[b]); };
  std::vector<int32_t> tour = nn_path(nonempty, asg[0], dc);
  two_opt(tour, dc);

  // 4. paths inside the clusters
  int64_t out = 0;
  int32_t last = -1;
  for (int32_t m : tour) {
    const std::vector<int32_t>& mem = members[m];
    int32_t entry = mem[0];
    if (last < 0) {
      entry = 0;
    } else {
      double bd = d(last, mem[0]);
      for (size_t a = 1; a < mem.size(); ++a) {
        const double v = d(last, mem[a]);
        if (v < bd) { bd = v; entry = mem[a]; }
      }
    }
    std::vector<int32_t> path = nn_path(mem, entry, d);
    two_opt(path, d);
    for (int32_t v : path) perm[out++] = v;
    last = path.back();
  }
  return TIDE_OK;
}
