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

// Masked Adam constants (Appendix A, the masked update equation).
template <typename T>
struct AdamK {
  T lr[kD];
  T b1, b2, eps, kappa;
};

// One column of the masked Adam update of an active row: first and second
// moments, then the parameter, with the row's bias corrections
// bcx = 1/(1 - b1^t) and bcy = 1/sqrt(1 - b2^t).  The Adam sweep and the
// backward with the update fused both apply this function, so the two give
// the same bits.
template <typename T>
__device__ __forceinline__ void adam_col(T& p, T& m, T& v, T g, T lr, T b1, T b2, T eps, T bcx, T bcy) {
  m = b1 * m + ((T)1 - b1) * g;
  v = b2 * v + ((T)1 - b2) * g * g;
  p = p - lr * (m * bcx) / (Mth<T>::sqrt(v) * bcy + eps);
}

// A row's step counter += 1 and its bias corrections 1/(1 - b1^t),
// 1/sqrt(1 - b2^t), evaluated in double precision (lb1 = log2 b1,
// lb2 = log2 b2) and rounded to T.
template <typename T>
__device__ __forceinline__ void adam_step_bias(uint32_t* step, double lb1, double lb2, T& bcx, T& bcy) {
  const uint32_t t = *step + 1u;
  *step = t;
  const double c1 = 1.0 - exp2((double)t * lb1), c2 = 1.0 - exp2((double)t * lb2);
  bcx = (T)(1.0 / c1);
  bcy = (T)(1.0 / sqrt(c2));
}

template <typename T>
inline AdamK<T> make_adam_k(const tide_adam_cfg* cfg) {
  AdamK<T> K;
  for (int j = 0; j < kD; ++j) K.lr[j] = cfg->lr[j];
  K.b1 = cfg->beta1; K.b2 = cfg->beta2; K.eps = cfg->eps; K.kappa = cfg->kappa;
  return K;
}

// The dirty marks and the bounding-sphere refresh that follow an Adam update
// of the active rows (either pointer may be null).
void launch_adam_bounds(const tide_pool* pool, const tide_proj* proj, float kappa, float* spheres, uint8_t* dirty,
                        hipStream_t st);

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

// Exponent scale of the compositing kernels: FP32 folds log2(e) into the
// conic and evaluates exp2 with the hardware v_exp_f32; FP64 keeps exp.
template <typename T>
struct Ex;
template <>
struct Ex<float> {
  static constexpr double k = 1.4426950408889634;  // log2(e)
  __device__ static float eval(float x) { return __builtin_amdgcn_exp2f(x); }
};
template <>
struct Ex<double> {
  static constexpr double k = 1.0;
  __device__ static double eval(double x) { return ::exp(x); }
};

// Opacity-weighted Gaussian of one list entry at one pixel, shared by the
// forward and backward kernels so that both take identical skip decisions.
// A pixel row at +infinity is reached by no entry: the power is -infinity
// (G = 0) or NaN (both tests fail).
// The per-entry terms are prepared once per lane column: with the scaled
// conic Ah = -A k/2, Bh = -B k, Ch = -C k/2 (k = Ex<T>::k) and dx the pixel
// offset, adx2 = Ah dx dx and bdx = Bh dx; then power = adx2 + bdx dy +
// Ch dy dy.  ok is false when the entry is skipped (power > 0 or
// alpha < 1/255); G = exp(power / k), araw = opacity G, alpha = min(0.99, araw).
template <typename T>
__device__ __forceinline__ void entry_alpha_tests(T adx2, T bdx, T Ch, T op, T dy, T& G, T& araw, T& alpha,
                                                  bool& in_power, bool& in_alpha) {
  const T power = adx2 + dy * (bdx + Ch * dy);
  G = Ex<T>::eval(power);
  araw = op * G;
  alpha = araw < (T)0.99 ? araw : (T)0.99;
  in_power = power <= (T)0;
  // alpha >= 1/255 exactly when araw >= 1/255 (0.99 > 1/255; a NaN araw
  // comes from a NaN power, which fails in_power)
  in_alpha = araw >= (T)(1.0 / 255.0);
}
// alpha = below ? araw : 0.99 (below = araw < 0.99) as a select on the bit
// patterns: the same value as min(araw, 0.99), without the canonicalisation
// a floating-point minimum of a reused value costs.
__device__ __forceinline__ float alpha_clamped(float araw, bool below) {
  return __uint_as_float(below ? __float_as_uint(araw) : __float_as_uint(0.99f));
}
__device__ __forceinline__ double alpha_clamped(double araw, bool below) {
  return __longlong_as_double(below ? __double_as_longlong(araw) : __double_as_longlong(0.99));
}

template <typename T>
__device__ __forceinline__ bool entry_alpha(T adx2, T bdx, T Ch, T op, T dy, T& G, T& araw, T& alpha) {
  bool in_power, in_alpha;
  entry_alpha_tests<T>(adx2, bdx, Ch, op, dy, G, araw, alpha, in_power, in_alpha);
  return in_power && in_alpha;
}

// Tile-level test of one list entry, conservative: false only when no pixel
// centre of tile (tx, ty) can take the entry, i.e. when opacity * G < 1/255
// at every centre, G = exp(-Q/2), Q = A dx^2 + 2 B dx dy + C dy^2 (the conic
// is positive definite).  The minimum of Q over the continuous box of the
// tile's pixel centres bounds it over the centres: 0 if the mean is inside,
// else the least of the four edge minima (on an edge, Q is a 1-D quadratic
// minimised at the clamped stationary point).  A slack of 1e-3 (relative and
// absolute) covers the rounding of this test and of the per-pixel one.
template <typename T>
__device__ __forceinline__ bool tile_may_take(T u, T v, T A, T B, T C, T op, int tx, int ty) {
  const T xa = (T)(kTile * tx) + (T)0.5 - u, xb = xa + (T)(kTile - 1);
  const T ya = (T)(kTile * ty) + (T)0.5 - v, yb = ya + (T)(kTile - 1);
  T qmin = 0;
  if (!(xa <= (T)0 && xb >= (T)0 && ya <= (T)0 && yb >= (T)0)) {
    auto q = [&](T dx, T dy) { return A * dx * dx + (T)2 * B * dx * dy + C * dy * dy; };
    auto cl = [](T x, T lo, T hi) { return x < lo ? lo : (x > hi ? hi : x); };
    const T e0 = q(xa, cl(-B * xa / C, ya, yb)), e1 = q(xb, cl(-B * xb / C, ya, yb));
    const T e2 = q(cl(-B * ya / A, xa, xb), ya), e3 = q(cl(-B * yb / A, xa, xb), yb);
    qmin = e0 < e1 ? e0 : e1;
    qmin = qmin < e2 ? qmin : e2;
    qmin = qmin < e3 ? qmin : e3;
  }
  return (T)0.5 * qmin * (T)(1.0 - 1e-3) <= Mth<T>::log((T)255 * op) + (T)1e-3;
}

// Wave64 sum with DPP row shifts and row broadcasts; the total lands in
// lane 63 (other lanes hold partial sums).
template <int CTRL, int ROWS, bool BC>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, BC));
}
__device__ __forceinline__ float wave_sum_to_63(float x) {
  x += dpp_f32<0x111, 0xF, true>(x);   // row_shr:1
  x += dpp_f32<0x112, 0xF, true>(x);   // row_shr:2
  x += dpp_f32<0x114, 0xF, true>(x);   // row_shr:4
  x += dpp_f32<0x118, 0xF, true>(x);   // row_shr:8  -> lane 15 of each row holds its row sum
  x += dpp_f32<0x142, 0xA, false>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_f32<0x143, 0xC, false>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}
__device__ __forceinline__ double wave_sum_to_63(double x) { return wave_sum(x); }

// Sum over each row of 16 lanes; lane 16 r + 15 holds row r's total.
__device__ __forceinline__ float row_sum_to_15(float x) {
  x += dpp_f32<0x111, 0xF, true>(x);
  x += dpp_f32<0x112, 0xF, true>(x);
  x += dpp_f32<0x114, 0xF, true>(x);
  x += dpp_f32<0x118, 0xF, true>(x);
  // the sum is only read in lane 15; without this the compiler sinks the
  // last add under that lane's branch and pays a DPP move plus an add for it
  asm volatile("" : "+v"(x));
  return x;
}
// Row sums of two quantities in one reduction.  Lane l holds x, its own
// share of quantity (l & 1), and y, its share of the other one.  After the
// exchange with the neighbour (quad_perm [1,0,3,2]) each lane holds a lane
// pair's total of quantity (l & 1); the even and the odd lanes of the row
// are then summed apart.  In lane 15, q1 is quantity 1's row sum and q0
// quantity 0's (taken from lane 14).
__device__ __forceinline__ void row_pair_sum_to_15(float x, float y, float& q0, float& q1) {
  float z = x + dpp_f32<0xB1, 0xF, false>(y);
  z += dpp_f32<0x112, 0xF, true>(z);
  z += dpp_f32<0x114, 0xF, true>(z);
  z += dpp_f32<0x118, 0xF, true>(z);
  asm volatile("" : "+v"(z));
  q1 = z;
  q0 = dpp_f32<0x111, 0xF, true>(z);
}
__device__ __forceinline__ double row_sum_to_15(double x) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) {
    const double y = __shfl_up(x, off, 16);
    if ((__lane_id() & 15) >= off) x += y;
  }
  return x;
}
__device__ __forceinline__ void row_pair_sum_to_15(double x, double y, double& q0, double& q1) {
  double z = x + __shfl_xor(y, 1, 16);
#pragma unroll
  for (int off = 2; off < 16; off <<= 1) {
    const double w = __shfl_up(z, off, 16);
    if ((__lane_id() & 15) >= off) z += w;
  }
  q1 = z;
  q0 = __shfl_up(z, 1, 16);
}


}  // namespace tide
