// Host-side block geometry shared by the tier and the predictor's data path:
// the bounding sphere of a block (Sec. 3.3) and the six-plane Level-1 test.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "tide.h"

namespace tide {

// Bounding sphere of a block's Gaussians: centre = mean of the member means
// (fixed at layout time), radius = max over members of |mu_i - c| plus
// 3 kappa times the largest axis scale, rounded up.  P holds at least the
// first six parameter columns (mean xyz, log-scale xyz), column j at P + j*ld.
inline void block_sphere(const float* P, int64_t ld, int64_t rows, double kappa, float out[4]) {
  double c[3] = {0, 0, 0};
  for (int64_t i = 0; i < rows; ++i)
    for (int a = 0; a < 3; ++a) c[a] += P[(size_t)a * ld + i];
  for (int a = 0; a < 3; ++a) c[a] /= (double)std::max<int64_t>(rows, 1);
  double rad = 0;
  for (int64_t i = 0; i < rows; ++i) {
    double d2 = 0;
    for (int a = 0; a < 3; ++a) {
      const double d = P[(size_t)a * ld + i] - c[a];
      d2 += d * d;
    }
    const double ls = std::max(P[3 * (size_t)ld + i], std::max(P[4 * (size_t)ld + i], P[5 * (size_t)ld + i]));
    rad = std::max(rad, std::sqrt(d2) + 3.0 * kappa * std::exp(ls));
  }
  for (int a = 0; a < 3; ++a) out[a] = (float)c[a];
  out[3] = (float)(rad * (1.0 + 1e-6) + 1e-6);
}

// Level 1 (Sec. 3.3): the camera frustum widened to the tile-padded image
// plus 3 px on every side, as six planes; a sphere (c, r) is culled when its
// signed distance to some plane is below -r.
struct CullCam {
  const tide_camera* c;
  double xl, xr, yt, yb, nl, nr, nt, nb;
  explicit CullCam(const tide_camera& cam) : c(&cam) {
    const double Tx = std::ceil(cam.width / 16.0), Ty = std::ceil(cam.height / 16.0);
    xl = -3.0;
    xr = 16.0 * Tx + 3.0;
    yt = -3.0;
    yb = 16.0 * Ty + 3.0;
    nl = std::sqrt(cam.fx * cam.fx + (cam.cx - xl) * (cam.cx - xl));
    nr = std::sqrt(cam.fx * cam.fx + (xr - cam.cx) * (xr - cam.cx));
    nt = std::sqrt(cam.fy * cam.fy + (cam.cy - yt) * (cam.cy - yt));
    nb = std::sqrt(cam.fy * cam.fy + (yb - cam.cy) * (yb - cam.cy));
  }
  bool keep(const float* s) const {
    double p[3];
    for (int i = 0; i < 3; ++i) p[i] = c->R[3 * i] * s[0] + c->R[3 * i + 1] * s[1] + c->R[3 * i + 2] * s[2] + c->t[i];
    const double r = s[3];
    return !(p[2] - c->z_near < -r) && !(c->z_far - p[2] < -r) &&
           !((c->fx * p[0] + (c->cx - xl) * p[2]) / nl < -r) && !(((xr - c->cx) * p[2] - c->fx * p[0]) / nr < -r) &&
           !((c->fy * p[1] + (c->cy - yt) * p[2]) / nt < -r) && !(((yb - c->cy) * p[2] - c->fy * p[1]) / nb < -r);
  }
};

}  // namespace tide
