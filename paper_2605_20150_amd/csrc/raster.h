// Device-side camera set and record layout shared by the rasterizer kernels.
#pragma once

#include "common.h"

namespace tide {

constexpr int kD = TIDE_D;
constexpr int kTile = TIDE_TILE;
constexpr int kRec = 12;  // u, v, A, B, C, opacity, r, g, b, depth, radius, 0

template <typename T>
struct DevCam {
  double Rd[9], td[3], fxd, fyd, cxd, cyd;  // projection of the mean runs in double
  T R[9], t[3];
  T fx, fy, cx, cy;
  T znear, zfar;
  T limx, limy;   // tangent clamp: 1.3 x half-fov tangent
  T pos[3];       // camera centre -R^T t
  int32_t W, H, Tx, Ty;
};

// Degree-3 real SH constants (3DGS sign convention), filled on the host from
// their closed forms: c0 = 1/(2 sqrt(pi)), c1 = sqrt(3/(4 pi)), ...
template <typename T>
struct ShK {
  T c0, c1, c2a, c2b, c2c, c3a, c3b, c3c, c3d, c3e;
};

template <typename T>
struct CamSet {
  DevCam<T> c[TIDE_MAX_CAMS];
  ShK<T> sh;
  int32_t n;
};

template <typename T>
CamSet<T> make_camset(const tide_camera* cams, int n);

// Tile rectangle with exact integer-vs-real comparisons: tile tx is covered
// iff 16 tx - r <= u and 16 (tx+1) + r > u (same in y), clamped to the grid.
// Returns false for an empty rectangle.
template <typename T>
__device__ inline bool tile_rect(T u, T v, int r, int Tx, int Ty, int& x0, int& y0, int& x1, int& y1) {
  if ((T)(-r) > u || (T)(kTile * Tx + r) <= u) return false;
  if ((T)(-r) > v || (T)(kTile * Ty + r) <= v) return false;
  // u, v are now within [-r, 16 T + r): the floors below fit an int and are
  // off by at most one, which the exact tests correct.
  int lo = (int)Mth<T>::floor((u - (T)r) * (T)(1.0 / kTile));
  if ((T)(kTile * lo + r) > u) lo -= 1;               // condition holds at lo-1
  else if (!((T)(kTile * (lo + 1) + r) > u)) lo += 1;  // fails at lo
  int hi = (int)Mth<T>::floor((u + (T)r) * (T)(1.0 / kTile));
  if ((T)(kTile * (hi + 1) - r) <= u) hi += 1;
  else if (!((T)(kTile * hi - r) <= u)) hi -= 1;
  x0 = lo < 0 ? 0 : lo;
  x1 = hi + 1 > Tx ? Tx : hi + 1;
  lo = (int)Mth<T>::floor((v - (T)r) * (T)(1.0 / kTile));
  if ((T)(kTile * lo + r) > v) lo -= 1;
  else if (!((T)(kTile * (lo + 1) + r) > v)) lo += 1;
  hi = (int)Mth<T>::floor((v + (T)r) * (T)(1.0 / kTile));
  if ((T)(kTile * (hi + 1) - r) <= v) hi += 1;
  else if (!((T)(kTile * hi - r) <= v)) hi -= 1;
  y0 = lo < 0 ? 0 : lo;
  y1 = hi + 1 > Ty ? Ty : hi + 1;
  return x1 > x0 && y1 > y0;
}

// Real SH basis (degree 3) at unit direction (x, y, z).
template <typename T>
__device__ inline void sh_eval(const ShK<T>& k, T x, T y, T z, T Y[16]) {
  const T xx = x * x, yy = y * y, zz = z * z;
  Y[0] = k.c0;
  Y[1] = -k.c1 * y;
  Y[2] = k.c1 * z;
  Y[3] = -k.c1 * x;
  Y[4] = k.c2a * x * y;
  Y[5] = -k.c2a * y * z;
  Y[6] = k.c2b * (2 * zz - xx - yy);
  Y[7] = -k.c2a * x * z;
  Y[8] = k.c2c * (xx - yy);
  Y[9] = -k.c3a * y * (3 * xx - yy);
  Y[10] = k.c3b * x * y * z;
  Y[11] = -k.c3c * y * (4 * zz - xx - yy);
  Y[12] = k.c3d * z * (2 * zz - 3 * xx - 3 * yy);
  Y[13] = -k.c3c * x * (4 * zz - xx - yy);
  Y[14] = k.c3e * z * (xx - yy);
  Y[15] = -k.c3a * x * (xx - 3 * yy);
}

// Opacity-weighted Gaussian of one list entry at one pixel, shared by the
// forward and backward kernels so that both take identical skip decisions.
// Ah = -A/2, Bh = -B, Ch = -C/2 (pre-scaled conic).  Returns false when the
// entry is skipped (power > 0 or alpha < 1/255); otherwise G = exp(power),
// araw = opacity * G and alpha = min(0.99, araw).
template <typename T>
__device__ __forceinline__ bool entry_alpha(T Ah, T Bh, T Ch, T op, T dx, T dy, T& G, T& araw, T& alpha) {
  const T power = Ah * dx * dx + Ch * dy * dy + Bh * dx * dy;
  if (power > 0) return false;
  G = Mth<T>::exp(power);
  araw = op * G;
  alpha = araw < (T)0.99 ? araw : (T)0.99;
  return !(alpha < (T)(1.0 / 255.0));
}

}  // namespace tide
