// FP64 CPU oracle of the block tier's bookkeeping: block bounding spheres,
// Level-1 frustum culling of block spheres (Sec. 3.3, Eq. Kt_def and the
// d < -r_k rule) and Alg. 1 (Sec. 3.5: recency, residency score, camera-
// balanced Top-C, set-difference streaming).
//
// TEST INFRASTRUCTURE ONLY; shares no code with the product library.
//
// Readings applied here (the paper leaves them open):
//   * sphere centre c_k = mean of the member means (fixed at layout time);
//     r_k = max_i |mu_i - c_k| + 3 kappa max_j exp(log-scale_ij), with
//     kappa = max over cameras of sqrt(1 + lx^2 + ly^2), lx = 1.3 (W/2)/fx:
//     the largest stretch the clamped EWA Jacobian can give, so the sphere
//     covers every 3-sigma footprint the exact rasterizer can keep.
//   * six planes per camera: near z = z_near, far z = z_far, and four side
//     planes through the camera centre and the edges of the pixel rectangle
//     widened by 3 px beyond the tile grid, [-3, 16 Tx + 3] x [-3, 16 Ty + 3]
//     (3 px > 3 sqrt(0.3) + 1, the dilation plus the radius ceiling).
//   * Alg. 1: Recency(k) = gamma^age_k, age reset to 0 when k is in
//     R_t intersect K_t and incremented otherwise; s(k) = lambda 1[k in K_{t+1}]
//     + (1 - lambda) Recency(k); camera quota q = floor(C / (4 J)); ties by
//     ascending block id.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <set>
#include <vector>

namespace {

struct Cam {
  double R[9], t[3], fx, fy, cx, cy;
  int W, H;
  double znear, zfar;
};

Cam load_cam(const double* c) {
  Cam k;
  for (int i = 0; i < 9; ++i) k.R[i] = c[i];
  for (int i = 0; i < 3; ++i) k.t[i] = c[9 + i];
  k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15];
  k.W = (int)c[16]; k.H = (int)c[17];
  k.znear = c[18]; k.zfar = c[19];
  return k;
}

// Signed distances (positive inside) of camera-space point p to the six planes.
void plane_distances(const Cam& c, const double p[3], double d[6]) {
  const double Tx = std::ceil(c.W / 16.0), Ty = std::ceil(c.H / 16.0);
  const double xl = -3.0, xr = 16.0 * Tx + 3.0, yt = -3.0, yb = 16.0 * Ty + 3.0;
  d[0] = p[2] - c.znear;
  d[1] = c.zfar - p[2];
  // u >= xl  <=>  fx x + (cx - xl) z >= 0
  d[2] = (c.fx * p[0] + (c.cx - xl) * p[2]) / std::sqrt(c.fx * c.fx + (c.cx - xl) * (c.cx - xl));
  // u <= xr  <=>  (xr - cx) z - fx x >= 0
  d[3] = ((xr - c.cx) * p[2] - c.fx * p[0]) / std::sqrt(c.fx * c.fx + (xr - c.cx) * (xr - c.cx));
  d[4] = (c.fy * p[1] + (c.cy - yt) * p[2]) / std::sqrt(c.fy * c.fy + (c.cy - yt) * (c.cy - yt));
  d[5] = ((yb - c.cy) * p[2] - c.fy * p[1]) / std::sqrt(c.fy * c.fy + (yb - c.cy) * (yb - c.cy));
}

}  // namespace

extern "C" {

double orc_kappa(const double* cams, int n_cams) {
  double k = 1.0;
  for (int i = 0; i < n_cams; ++i) {
    const Cam c = load_cam(cams + 20 * i);
    const double lx = 1.3 * 0.5 * c.W / c.fx, ly = 1.3 * 0.5 * c.H / c.fy;
    k = std::max(k, std::sqrt(1.0 + lx * lx + ly * ly));
  }
  return k;
}

// Morton layout order (Sec. 3.3): quantise each axis of the centres to 2^21
// cells over their bounding box (cell = floor((x - lo) * (2^21 / (hi - lo))),
// clamped to [0, 2^21 - 1], in double), interleave the cell bits with bit i
// of axis a at position 3 i + a, and sort the rows stably by that code.
void orc_morton_order(const double* xyz, int64_t n, int64_t stride, int64_t* perm) {
  if (n <= 0) return;
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) lo[a] = hi[a] = xyz[a];
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], xyz[i * stride + a]);
      hi[a] = std::max(hi[a], xyz[i * stride + a]);
    }
  std::vector<uint64_t> code(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      const double s = hi[a] > lo[a] ? 2097152.0 / (hi[a] - lo[a]) : 0.0;
      double q = std::floor((xyz[i * stride + a] - lo[a]) * s);
      q = std::min(2097151.0, std::max(0.0, q));
      const uint64_t cell = (uint64_t)q;
      for (int b = 0; b < 21; ++b)
        if ((cell >> b) & 1u) code[i] |= 1ull << (3 * b + a);
    }
  }
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  std::stable_sort(perm, perm + n, [&](int64_t x, int64_t y) { return code[x] < code[y]; });
}

// spheres[k] = (cx, cy, cz, r) for blocks of B consecutive rows of theta[n][59].
void orc_block_spheres(const double* theta, int64_t n, int64_t B, double kappa, double* spheres) {
  const int64_t K = (n + B - 1) / B;
  for (int64_t k = 0; k < K; ++k) {
    const int64_t a = k * B, b = std::min(n, a + B);
    double c[3] = {0, 0, 0};
    for (int64_t i = a; i < b; ++i)
      for (int j = 0; j < 3; ++j) c[j] += theta[59 * i + j];
    for (int j = 0; j < 3; ++j) c[j] /= (double)(b - a);
    double r = 0;
    for (int64_t i = a; i < b; ++i) {
      const double* th = theta + 59 * i;
      const double dx = th[0] - c[0], dy = th[1] - c[1], dz = th[2] - c[2];
      const double smax = std::exp(std::max(th[3], std::max(th[4], th[5])));
      r = std::max(r, std::sqrt(dx * dx + dy * dy + dz * dz) + 3.0 * kappa * smax);
    }
    for (int j = 0; j < 3; ++j) spheres[4 * k + j] = c[j];
    spheres[4 * k + 3] = r;
  }
}

// vis[c][k] = 1 unless some plane has d < -r_k (Eq. Kt_def; the d < -r_k rule).
void orc_cull_blocks(const double* spheres, int64_t K, const double* cams, int n_cams, uint8_t* vis) {
  for (int ci = 0; ci < n_cams; ++ci) {
    const Cam c = load_cam(cams + 20 * ci);
    for (int64_t k = 0; k < K; ++k) {
      const double* s = spheres + 4 * k;
      double p[3];
      for (int i = 0; i < 3; ++i) p[i] = c.R[3 * i] * s[0] + c.R[3 * i + 1] * s[1] + c.R[3 * i + 2] * s[2] + c.t[i];
      double d[6];
      plane_distances(c, p, d);
      bool keep = true;
      for (int q = 0; q < 6; ++q) keep = keep && !(d[q] < -s[3]);
      vis[ci * K + k] = keep ? 1 : 0;
    }
  }
}

// Alg. 1.  R (nR), Kcur (nK): current resident and visible blocks; Knext is
// the concatenation of the J per-camera next sets (counts[j] each).  age[K]
// is updated in place.  Writes R_{t+1} in ascending order into out_R and
// returns its size.  out_rank (optional, size C) receives the selection
// order (quota picks first, then the global fill) for inspection.
int orc_alg1(const int32_t* R, int nR, const int32_t* Kcur, int nK, const int32_t* Knext, const int32_t* counts,
             int J, double* age_io, int64_t n_blocks, double lambda, double gamma, int C, int32_t* out_R,
             int32_t* out_rank) {
  std::set<int32_t> Rt(R, R + nR), Kt(Kcur, Kcur + nK);
  std::vector<std::vector<int32_t>> Kj(J);
  std::set<int32_t> Kn;
  int off = 0;
  for (int j = 0; j < J; ++j) {
    Kj[j].assign(Knext + off, Knext + off + counts[j]);
    Kn.insert(Kj[j].begin(), Kj[j].end());
    off += counts[j];
  }
  // recency from the accessed resident blocks R_t intersect K_t
  for (int64_t k = 0; k < n_blocks; ++k) {
    const bool accessed = Rt.count((int32_t)k) && Kt.count((int32_t)k);
    age_io[k] = accessed ? 0.0 : age_io[k] + 1.0;
  }
  std::set<int32_t> Ct = Rt;
  Ct.insert(Kn.begin(), Kn.end());
  auto score = [&](int32_t k) {
    return lambda * (Kn.count(k) ? 1.0 : 0.0) + (1.0 - lambda) * std::pow(gamma, age_io[k]);
  };
  auto better = [&](int32_t a, int32_t b) {
    const double sa = score(a), sb = score(b);
    if (sa != sb) return sa > sb;
    return a < b;
  };
  std::set<int32_t> chosen;
  std::vector<int32_t> order;
  const int q = J > 0 ? C / (4 * J) : 0;
  for (int j = 0; j < J; ++j) {
    std::vector<int32_t> cand;
    for (int32_t k : Kj[j])
      if (!chosen.count(k)) cand.push_back(k);
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    std::stable_sort(cand.begin(), cand.end(), better);
    for (int i = 0; i < (int)cand.size() && i < q && (int)chosen.size() < C; ++i) {
      chosen.insert(cand[i]);
      order.push_back(cand[i]);
    }
  }
  std::vector<int32_t> rest;
  for (int32_t k : Ct)
    if (!chosen.count(k)) rest.push_back(k);
  std::stable_sort(rest.begin(), rest.end(), better);
  for (size_t i = 0; i < rest.size() && (int)chosen.size() < C; ++i) {
    chosen.insert(rest[i]);
    order.push_back(rest[i]);
  }
  int n = 0;
  for (int32_t k : chosen) out_R[n++] = k;
  if (out_rank)
    for (size_t i = 0; i < order.size(); ++i) out_rank[i] = order[i];
  return n;
}

}  // extern "C"
