// FP64 CPU oracle of the differentiable 3DGS rasterizer, its loss, its
// adjoint and the masked Adam update.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
// or calls this file; only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load it.  It shares no code with the GPU
// path.
//
// What it follows.  The paper keeps "the standard 3DGS forward/backward
// semantics on the resident primitives" (Sec. 1; Sec. 3.3, Level 2) and
// defers the rasterizer itself to Kerbl et al. 2023, so every function here
// is the plain published 3DGS / EWA mathematics, evaluated in double
// precision, with the readings that the paper leaves open written next to the
// code that uses them:
//   * 59 columns: mean(3), log-scale(3), quaternion wxyz(4), opacity logit(1),
//     SH coefficients 16 x rgb, coefficient-major (Sec. 2, D = 59).
//   * activations exp / sigmoid / normalise.
//   * pinhole camera, OpenCV axes, pixel centres at +0.5.
//   * near plane 0.2 and a far plane, both culling (camera-space depth).
//   * tangent clamp at 1.3 x the half-field-of-view tangent, 0.3 px^2 dilation.
//   * radius ceil(3 sqrt(lambda_max)); 16x16 tiles; a Gaussian covers tile
//     (tx, ty) iff 16 tx <= u + r and 16 (tx+1) > u - r (same in y), clamped.
//   * colour = max(0, SH(d) + 0.5).
//   * alpha = min(0.99, opacity * G); skip alpha < 1/255; stop before an entry
//     that would take transmittance below 1e-4.
//   * per-tile order (tile, depth, global id).
//   * loss 0.8 L1 + 0.2 (1 - SSIM), 11x11 Gaussian window sigma 1.5, zero
//     padding, C1 = 0.01^2, C2 = 0.03^2, mean over views.
//   * Adam with a per-row step, bias correction, per-column learning rate,
//     inactive rows unchanged (Appendix A, masked update equation).
//
// All loops are plain: projection per (camera, Gaussian), binning by direct
// enumeration of every tile against the coverage rule, std::stable_sort,
// per-pixel compositing, direct 11x11 convolution.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr int kD = 59;
constexpr int kTile = 16;

struct Cam {
  double R[9], t[3];
  double fx, fy, cx, cy;
  int W, H;
  double znear, zfar;
  int tx() const { return (W + kTile - 1) / kTile; }
  int ty() const { return (H + kTile - 1) / kTile; }
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

// ---------------------------------------------------------------- SH basis
// Real spherical harmonics up to degree 3, in the sign convention of the
// 3DGS reference renderer; constants are evaluated from their closed forms.
struct ShConst {
  double c0, c1, c2a, c2b, c2c, c3a, c3b, c3c, c3d, c3e;
  ShConst() {
    const double pi = M_PI;
    c0 = 0.5 * std::sqrt(1.0 / pi);
    c1 = std::sqrt(3.0 / (4.0 * pi));
    c2a = 0.5 * std::sqrt(15.0 / pi);       // xy, yz, xz terms
    c2b = 0.25 * std::sqrt(5.0 / pi);       // 2z^2 - x^2 - y^2
    c2c = 0.25 * std::sqrt(15.0 / pi);      // x^2 - y^2
    c3a = 0.25 * std::sqrt(35.0 / (2.0 * pi));
    c3b = 0.5 * std::sqrt(105.0 / pi);
    c3c = 0.25 * std::sqrt(21.0 / (2.0 * pi));
    c3d = 0.25 * std::sqrt(7.0 / pi);
    c3e = 0.25 * std::sqrt(105.0 / pi);
  }
};
const ShConst& shc() { static ShConst k; return k; }

void sh_basis(const double d[3], double Y[16]) {
  const ShConst& k = shc();
  const double x = d[0], y = d[1], z = d[2];
  Y[0] = k.c0;
  Y[1] = -k.c1 * y;
  Y[2] = k.c1 * z;
  Y[3] = -k.c1 * x;
  Y[4] = k.c2a * x * y;
  Y[5] = -k.c2a * y * z;
  Y[6] = k.c2b * (2 * z * z - x * x - y * y);
  Y[7] = -k.c2a * x * z;
  Y[8] = k.c2c * (x * x - y * y);
  Y[9] = -k.c3a * y * (3 * x * x - y * y);
  Y[10] = k.c3b * x * y * z;
  Y[11] = -k.c3c * y * (4 * z * z - x * x - y * y);
  Y[12] = k.c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
  Y[13] = -k.c3c * x * (4 * z * z - x * x - y * y);
  Y[14] = k.c3e * z * (x * x - y * y);
  Y[15] = -k.c3a * x * (x * x - 3 * y * y);
}

// dY[k][0..2] = partial derivatives of Y_k with respect to (x, y, z), with
// the three components treated as independent variables.
void sh_basis_grad(const double d[3], double dY[16][3]) {
  const ShConst& k = shc();
  const double x = d[0], y = d[1], z = d[2];
  for (int i = 0; i < 16; ++i) dY[i][0] = dY[i][1] = dY[i][2] = 0.0;
  dY[1][1] = -k.c1;
  dY[2][2] = k.c1;
  dY[3][0] = -k.c1;
  dY[4][0] = k.c2a * y; dY[4][1] = k.c2a * x;
  dY[5][1] = -k.c2a * z; dY[5][2] = -k.c2a * y;
  dY[6][0] = -2 * k.c2b * x; dY[6][1] = -2 * k.c2b * y; dY[6][2] = 4 * k.c2b * z;
  dY[7][0] = -k.c2a * z; dY[7][2] = -k.c2a * x;
  dY[8][0] = 2 * k.c2c * x; dY[8][1] = -2 * k.c2c * y;
  dY[9][0] = -k.c3a * 6 * x * y; dY[9][1] = -k.c3a * (3 * x * x - 3 * y * y);
  dY[10][0] = k.c3b * y * z; dY[10][1] = k.c3b * x * z; dY[10][2] = k.c3b * x * y;
  dY[11][0] = 2 * k.c3c * x * y; dY[11][1] = -k.c3c * (4 * z * z - x * x - 3 * y * y);
  dY[11][2] = -8 * k.c3c * y * z;
  dY[12][0] = -6 * k.c3d * x * z; dY[12][1] = -6 * k.c3d * y * z;
  dY[12][2] = k.c3d * (6 * z * z - 3 * x * x - 3 * y * y);
  dY[13][0] = -k.c3c * (4 * z * z - 3 * x * x - y * y); dY[13][1] = 2 * k.c3c * x * y;
  dY[13][2] = -8 * k.c3c * x * z;
  dY[14][0] = 2 * k.c3e * x * z; dY[14][1] = -2 * k.c3e * y * z; dY[14][2] = k.c3e * (x * x - y * y);
  dY[15][0] = -k.c3a * (3 * x * x - 3 * y * y); dY[15][1] = 6 * k.c3a * x * y;
}

// --------------------------------------------------------------- projection
struct Fwd {
  bool keep = false;
  double p[3];
  double u = 0, v = 0, depth = 0;
  double s00 = 0, s01 = 0, s11 = 0, det = 0;
  double A = 0, B = 0, C = 0;
  double op = 0;
  double raw[3], rgb[3];
  double dir[3], vlen = 0;
  int r = 0, rect[4] = {0, 0, 0, 0}, tt = 0;
  double rr = 0;              // 3 sqrt(lambda_max) before the ceiling
  bool clampx = false, clampy = false;
  double xi = 0, eta = 0;
  double J[6], T[6];          // J (2x3), T = J W (2x3)
  double Sig[9], M[9], Rq[9];
  double s[3], qh[4], qn = 0;
  double perr = 0, derr = 0;  // first-order FP32 uncertainty of (u, v) in px and of depth
  double margin = 1e300;      // smallest decision margin / its FP32 uncertainty (< 1: near tie)
};

inline double rel_int_dist(double x) {  // distance of x to the nearest integer
  return std::fabs(x - std::nearbyint(x));
}

// Near-tie model.  A discrete decision taken in single precision can differ
// from the double-precision one when its margin is within the rounding error
// its inputs carry.  Every margin below is divided by a first-order estimate
// of that error (16 units of the precision the decision is evaluated in), so
// a ratio below 1 marks a near tie.  The camera-space mean, the pixel
// position and the near/far tests are double-precision quantities rounded
// once to single precision (u, v, depth); everything else is single:
//   position  perr = 2^-20 (|u| + |v| + |cx| + |cy|) + 2^-48 f (|mu| + |t|) / p_z   pixels
//   depth     the sort key is single precision on both sides; its only risk
//             is a rounding midpoint within 2^-48 (|mu| + |t|) of p_z
//   near/far  2^-48 (|mu| + |t|)
//   any other quantity x: 2^-20 |x| (relative).
constexpr double kTieRel = 1.0 / 1048576.0;
constexpr double kTieRel64 = 1.0 / 281474976710656.0;   // 2^-48

// Depth sort key (reading of the total order (tile, depth, gid) with the
// depth taken in single precision, as the binning keys are).
inline double sort_key(double depth) { return (double)(float)depth; }

// Distance of x to the nearest single-precision rounding midpoint.
inline double key_midpoint_distance(double x) {
  const float f = (float)x;
  const double lo = 0.5 * ((double)f + (double)std::nextafter(f, -INFINITY));
  const double hi = 0.5 * ((double)f + (double)std::nextafter(f, INFINITY));
  return std::min(std::fabs(x - lo), std::fabs(hi - x));
}

// Tile-coverage rectangle of O4 with exact integer-vs-real comparisons:
// x0 = smallest tx with 16(tx+1) + r > u, x1 = 1 + largest tx with 16 tx - r <= u,
// both clamped to [0, Tx]; same in y.
void tile_rect(double u, double v, int r, int Tx, int Ty, int rect[4]) {
  int x0 = Tx, x1 = 0, y0 = Ty, y1 = 0;
  for (int tx = 0; tx < Tx; ++tx) {
    const bool cov = (double)(kTile * tx - r) <= u && (double)(kTile * (tx + 1) + r) > u;
    if (cov) { x0 = std::min(x0, tx); x1 = std::max(x1, tx + 1); }
  }
  for (int ty = 0; ty < Ty; ++ty) {
    const bool cov = (double)(kTile * ty - r) <= v && (double)(kTile * (ty + 1) + r) > v;
    if (cov) { y0 = std::min(y0, ty); y1 = std::max(y1, ty + 1); }
  }
  if (x1 <= x0 || y1 <= y0) { x0 = x1 = y0 = y1 = 0; }
  rect[0] = x0; rect[1] = y0; rect[2] = x1; rect[3] = y1;
}

double rect_margin(double u, double v, int r) {
  // distance (px) of u +- r, v +- r to the nearest tile boundary
  auto dm = [](double a) { return std::fabs(a / kTile - std::nearbyint(a / kTile)) * kTile; };
  return std::min(std::min(dm(u + r), dm(u - r)), std::min(dm(v + r), dm(v - r)));
}

// Whether p_z = R_20 mu_0 + R_21 mu_1 + R_22 mu_2 + t_2, evaluated left to
// right in double precision, is exact: every product and every partial sum
// carries no rounding error (error-free transformations: the product's error
// is fma(a, b, -ab), the sum's that of Knuth's two-sum).  An exact p_z is the
// same whatever evaluation order or fused multiply-adds another double
// evaluation uses, so its depth decisions carry no uncertainty.
bool depth_exact(const Cam& c, const double* mu) {
  double s = 0;
  for (int k = 0; k < 3; ++k) {
    const double a = c.R[6 + k], b = mu[k];
    const double p = a * b;
    if (std::fma(a, b, -p) != 0) return false;
    const double t = s + p, bp = t - s;
    if ((s - (t - bp)) + (p - bp) != 0) return false;
    s = t;
  }
  const double t = s + c.t[2], bp = t - s;
  return (s - (t - bp)) + (c.t[2] - bp) == 0;
}

void project_one(const double* th, const Cam& c, Fwd& f) {
  const double* mu = th;
  f.keep = false;
  f.margin = 1e300;
  // camera-space position
  for (int i = 0; i < 3; ++i)
    f.p[i] = c.R[3 * i] * mu[0] + c.R[3 * i + 1] * mu[1] + c.R[3 * i + 2] * mu[2] + c.t[i];
  const double pz = f.p[2];
  f.depth = pz;
  const double mun = std::sqrt(mu[0] * mu[0] + mu[1] * mu[1] + mu[2] * mu[2]);
  const double tn = std::sqrt(c.t[0] * c.t[0] + c.t[1] * c.t[1] + c.t[2] * c.t[2]);
  const double nf_err = kTieRel64 * (mun + tn);
  // The sort key is the single-precision depth (ties by gid): the only way
  // an order can differ is a double-precision depth so close to a rounding
  // midpoint of single precision that another evaluation order of p_z
  // rounds it the other way.
  f.derr = 0;
  if (!depth_exact(c, mu)) {
    f.margin = std::min(f.margin, key_midpoint_distance(pz) / nf_err);
    f.margin = std::min(f.margin, std::fabs(pz - c.znear) / nf_err);
    f.margin = std::min(f.margin, std::fabs(pz - c.zfar) / nf_err);
  }
  if (!(pz > c.znear) || pz > c.zfar) return;

  // activations
  for (int i = 0; i < 3; ++i) f.s[i] = std::exp(th[3 + i]);
  f.qn = std::sqrt(th[6] * th[6] + th[7] * th[7] + th[8] * th[8] + th[9] * th[9]);
  for (int i = 0; i < 4; ++i) f.qh[i] = th[6 + i] / f.qn;
  const double w = f.qh[0], x = f.qh[1], y = f.qh[2], z = f.qh[3];
  double* Rq = f.Rq;
  Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z);     Rq[2] = 2 * (x * z + w * y);
  Rq[3] = 2 * (x * y + w * z);     Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
  Rq[6] = 2 * (x * z - w * y);     Rq[7] = 2 * (y * z + w * x);     Rq[8] = 1 - 2 * (x * x + y * y);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) f.M[3 * i + j] = Rq[3 * i + j] * f.s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k) a += f.M[3 * i + k] * f.M[3 * j + k];
      f.Sig[3 * i + j] = a;
    }
  f.op = 1.0 / (1.0 + std::exp(-th[10]));

  // pinhole projection
  f.u = c.fx * f.p[0] / pz + c.cx;
  f.v = c.fy * f.p[1] / pz + c.cy;
  f.perr = kTieRel * (std::fabs(f.u) + std::fabs(f.v) + std::fabs(c.cx) + std::fabs(c.cy)) +
           kTieRel64 * std::max(c.fx, c.fy) * (mun + tn) / std::fabs(pz);

  // EWA: J evaluated at the clamped tangents
  const double limx = 1.3 * (0.5 * c.W) / c.fx, limy = 1.3 * (0.5 * c.H) / c.fy;
  const double tx = f.p[0] / pz, ty = f.p[1] / pz;
  f.clampx = tx < -limx || tx > limx;
  f.clampy = ty < -limy || ty > limy;
  f.xi = std::min(limx, std::max(-limx, tx));
  f.eta = std::min(limy, std::max(-limy, ty));
  double* J = f.J;
  J[0] = c.fx / pz; J[1] = 0; J[2] = -c.fx * f.xi / pz;
  J[3] = 0; J[4] = c.fy / pz; J[5] = -c.fy * f.eta / pz;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k) a += J[3 * i + k] * c.R[3 * k + j];
      f.T[3 * i + j] = a;
    }
  double S2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) a += f.T[3 * i + k] * f.Sig[3 * k + l] * f.T[3 * j + l];
      S2[2 * i + j] = a;
    }
  f.s00 = S2[0] + 0.3;
  f.s01 = 0.5 * (S2[1] + S2[2]);
  f.s11 = S2[3] + 0.3;
  f.det = f.s00 * f.s11 - f.s01 * f.s01;
  f.margin = std::min(f.margin, std::fabs(f.det) / (f.s00 * f.s11) / kTieRel);
  if (!(f.det > 0)) return;
  f.A = f.s11 / f.det;
  f.B = -f.s01 / f.det;
  f.C = f.s00 / f.det;
  const double m = 0.5 * (f.s00 + f.s11);
  const double lam1 = m + std::sqrt(std::max(0.0, m * m - f.det));
  const double rr = 3.0 * std::sqrt(lam1);
  f.rr = rr;
  // radius cap of 2^21 px (a footprint that large covers any image; it keeps
  // 16 t +- r exactly representable in single precision on the GPU side)
  f.r = (int)std::ceil(std::min(rr, 2097152.0));
  f.margin = std::min(f.margin, rel_int_dist(rr) / (kTieRel * std::max(rr, 1.0)));
  tile_rect(f.u, f.v, f.r, c.tx(), c.ty(), f.rect);
  f.margin = std::min(f.margin, rect_margin(f.u, f.v, f.r) / f.perr);
  f.tt = (f.rect[2] - f.rect[0]) * (f.rect[3] - f.rect[1]);
  if (f.tt == 0) return;

  // view-dependent colour
  double o[3];
  for (int i = 0; i < 3; ++i)
    o[i] = -(c.R[i] * c.t[0] + c.R[3 + i] * c.t[1] + c.R[6 + i] * c.t[2]);
  double dv[3] = {mu[0] - o[0], mu[1] - o[1], mu[2] - o[2]};
  f.vlen = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  for (int i = 0; i < 3; ++i) f.dir[i] = dv[i] / f.vlen;
  double Y[16];
  sh_basis(f.dir, Y);
  for (int ch = 0; ch < 3; ++ch) {
    double a = 0.5;
    for (int k = 0; k < 16; ++k) a += Y[k] * th[11 + 3 * k + ch];
    f.raw[ch] = a;
    f.rgb[ch] = std::max(0.0, a);
  }
  f.keep = true;
}

// ----------------------------------------------------------------- binning
struct Inst { int64_t tile; double depth; int64_t gid; };

// Emits every (tile, depth, gid) instance of the kept pairs of camera c in
// ascending gid, tiles row-major, then stable-sorts by (tile, depth, gid).
void bin_camera(const Cam& c, int64_t n, const double* u, const double* v, const double* depth,
                const int32_t* radius, const int32_t* keep, std::vector<Inst>& out) {
  out.clear();
  const int Tx = c.tx(), Ty = c.ty();
  for (int64_t i = 0; i < n; ++i) {
    if (!keep[i]) continue;
    int rect[4];
    tile_rect(u[i], v[i], radius[i], Tx, Ty, rect);
    for (int ty = rect[1]; ty < rect[3]; ++ty)
      for (int tx = rect[0]; tx < rect[2]; ++tx)
        out.push_back(Inst{(int64_t)ty * Tx + tx, depth[i], i});
  }
  std::stable_sort(out.begin(), out.end(), [](const Inst& a, const Inst& b) {
    if (a.tile != b.tile) return a.tile < b.tile;
    if (a.depth != b.depth) return a.depth < b.depth;
    return a.gid < b.gid;
  });
}

// ------------------------------------------------------------- compositing
struct Rec { double u, v, A, B, C, op, rgb[3], depth, perr, derr; };

// Composites one tile of camera c. Writes image/t_final/last/visits for the
// pixels of the tile.  `list` holds the tile's gids in order.
void composite_tile(const Cam& c, int tx, int ty, const int64_t* list, int64_t len, const Rec* rec,
                    const double* bg, double* image, double* tfin, int32_t* last, int64_t* visits,
                    double* pmargin) {
  const int W = c.W, H = c.H;
  for (int py = ty * kTile; py < std::min(H, (ty + 1) * kTile); ++py)
    for (int px = tx * kTile; px < std::min(W, (tx + 1) * kTile); ++px) {
      double T = 1.0, col[3] = {0, 0, 0}, mg = 1e300;
      int32_t lst = 0;
      int64_t vis = 0;
      double eT = 0;  // uncertainty of ln T
      for (int64_t j = 0; j < len; ++j) {
        const Rec& g = rec[list[j]];
        ++vis;
        if (j > 0 && g.derr + rec[list[j - 1]].derr > 0)  // depth order against the previous entry
          mg = std::min(mg, std::fabs(g.depth - rec[list[j - 1]].depth) / (g.derr + rec[list[j - 1]].derr));
        const double dx = px + 0.5 - g.u, dy = py + 0.5 - g.v;
        const double power = -0.5 * (g.A * dx * dx + g.C * dy * dy) - g.B * dx * dy;
        if (power > 0) continue;
        const double a_raw = g.op * std::exp(power);
        const double alpha = std::min(0.99, a_raw);
        const double gx = g.A * dx + g.B * dy, gy = g.B * dx + g.C * dy;
        // single-precision rounding acts on the three terms of the quadratic
        // form, which can be far larger than their sum (an elongated
        // footprint away from its centre), so the bound is relative to
        // their magnitudes, not to the power
        const double terms = 0.5 * (g.A * dx * dx + g.C * dy * dy) + std::fabs(g.B * dx * dy);
        const double epow = std::sqrt(gx * gx + gy * gy) * g.perr + kTieRel * (terms + 1.0);
        mg = std::min(mg, std::fabs(power + std::log(255.0 * g.op)) / epow);
        if (alpha < 1.0 / 255.0) continue;
        const double ea = (a_raw < 0.99 ? alpha / (1 - alpha) * epow : 0.0) + kTieRel;
        const double Tn = T * (1 - alpha);
        mg = std::min(mg, std::fabs(std::log(Tn / 1e-4)) / (eT + ea));
        if (Tn < 1e-4) break;
        eT += ea;
        for (int ch = 0; ch < 3; ++ch) col[ch] += g.rgb[ch] * alpha * T;
        T = Tn;
        lst = (int32_t)(j + 1);
      }
      const int64_t pix = (int64_t)py * W + px;
      for (int ch = 0; ch < 3; ++ch) image[(int64_t)ch * H * W + pix] = col[ch] + T * bg[ch];
      tfin[pix] = T;
      last[pix] = lst;
      visits[pix] = vis;
      if (pmargin) pmargin[pix] = mg;
    }
}

// ------------------------------------------------------------------- loss
std::vector<double> gauss_window() {
  std::vector<double> g(11);
  double s = 0;
  for (int i = 0; i < 11; ++i) { g[i] = std::exp(-((i - 5) * (i - 5)) / (2 * 1.5 * 1.5)); s += g[i]; }
  for (int i = 0; i < 11; ++i) g[i] /= s;
  return g;
}

// Direct 2-D convolution with the 11x11 window w(i)w(j), zero padding,
// same-size output.
void conv11(const double* x, int H, int W, const std::vector<double>& g, double* y) {
  for (int r = 0; r < H; ++r)
    for (int c = 0; c < W; ++c) {
      double a = 0;
      for (int i = -5; i <= 5; ++i) {
        const int rr = r + i;
        if (rr < 0 || rr >= H) continue;
        for (int j = -5; j <= 5; ++j) {
          const int cc = c + j;
          if (cc < 0 || cc >= W) continue;
          a += g[i + 5] * g[j + 5] * x[(int64_t)rr * W + cc];
        }
      }
      y[(int64_t)r * W + c] = a;
    }
}

}  // namespace

// =========================================================================
extern "C" {

void orc_sh_basis(const double* dir, double* Y) { sh_basis(dir, Y); }
void orc_sh_basis_grad(const double* dir, double* dY) {
  double g[16][3];
  sh_basis_grad(dir, g);
  for (int k = 0; k < 16; ++k)
    for (int i = 0; i < 3; ++i) dY[3 * k + i] = g[k][i];
}

// Per (camera, Gaussian) projection, O2-O5.
//   out_f[c][i][16]: u, v, depth, A, B, C, opacity, r, g, b, s00, s01, s11, 3 sqrt(lambda_max),
//                    position uncertainty (px), depth uncertainty
//   out_i[c][i][7]:  keep, radius, x0, y0, x1, y1, tiles_touched
//   margin[c][i]:    smallest margin / uncertainty ratio of the pair's decisions (< 1: near tie)
int orc_project(const double* theta, int64_t n, const double* cams, int n_cams, double* out_f,
                int32_t* out_i, double* margin) {
  for (int ci = 0; ci < n_cams; ++ci) {
    const Cam c = load_cam(cams + 20 * ci);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      Fwd f;
      project_one(theta + kD * i, c, f);
      double* of = out_f + ((int64_t)ci * n + i) * 16;
      int32_t* oi = out_i + ((int64_t)ci * n + i) * 7;
      of[0] = f.u; of[1] = f.v; of[2] = f.depth; of[3] = f.A; of[4] = f.B; of[5] = f.C;
      of[6] = f.op; of[7] = f.rgb[0]; of[8] = f.rgb[1]; of[9] = f.rgb[2];
      of[10] = f.s00; of[11] = f.s01; of[12] = f.s11;
      of[13] = f.rr;
      of[14] = f.perr;
      of[15] = f.derr;
      oi[0] = f.keep; oi[1] = f.r; oi[2] = f.rect[0]; oi[3] = f.rect[1]; oi[4] = f.rect[2];
      oi[5] = f.rect[3]; oi[6] = f.keep ? f.tt : 0;
      if (margin) margin[(int64_t)ci * n + i] = f.margin;
    }
  }
  return 0;
}

// Tile-coverage rectangle (O4) for one footprint.
void orc_tile_rect(double u, double v, int r, int Tx, int Ty, int32_t* rect) {
  int q[4];
  tile_rect(u, v, r, Tx, Ty, q);
  for (int k = 0; k < 4; ++k) rect[k] = q[k];
}

// Threads the OpenMP loops of the oracle use (timing runs only; results do
// not depend on it).  Returns the count in effect.
int orc_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}

// O4's tile rectangle for n (u, v, r) triples on one camera's Tx x Ty grid
// (the same rule as orc_tile_rect, one call per triple).
void orc_tile_rects(const double* u, const double* v, const int32_t* r, int64_t n, int Tx, int Ty,
                    int32_t* rect) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int q[4];
    tile_rect(u[i], v[i], r[i], Tx, Ty, q);
    for (int k = 0; k < 4; ++k) rect[4 * i + k] = q[k];
  }
}

// Binning and sort, O6, for all cameras.  Inputs are per (camera, Gaussian):
// u, v, depth, integer radius and keep flag.  Returns the number of
// instances; fills the outputs only when it does not exceed `cap`.
//   out_gid[m]   gid of instance m, cameras concatenated, each (tile, depth, gid) ordered
//   ranges[2*(tile_base[c] + tile)] = [start, end) into out_gid (tile_base = running sum of Tx*Ty)
int64_t orc_bin(const double* u, const double* v, const double* depth, const int32_t* radius,
                const int32_t* keep, int64_t n, const double* cams, int n_cams, int64_t* out_gid,
                int64_t cap, int64_t* ranges) {
  int64_t total = 0, tile_base = 0;
  std::vector<Inst> insts;
  for (int ci = 0; ci < n_cams; ++ci) {
    const Cam c = load_cam(cams + 20 * ci);
    const int64_t off = (int64_t)ci * n;
    bin_camera(c, n, u + off, v + off, depth + off, radius + off, keep + off, insts);
    const int64_t T = (int64_t)c.tx() * c.ty();
    if (total + (int64_t)insts.size() <= cap) {
      for (int64_t t = 0; t < T; ++t) { ranges[2 * (tile_base + t)] = total; ranges[2 * (tile_base + t) + 1] = total; }
      for (size_t m = 0; m < insts.size(); ++m) {
        out_gid[total + m] = insts[m].gid;
        const int64_t t = tile_base + insts[m].tile;
        if (m == 0 || insts[m - 1].tile != insts[m].tile) ranges[2 * t] = total + m;
        ranges[2 * t + 1] = total + m + 1;
      }
    }
    total += insts.size();
    tile_base += T;
  }
  return total;
}

// Compositing, O7, over given per-tile lists.  rec[c][i][9] = u, v, A, B, C,
// opacity, r, g, b; unc[c][i][3] = depth, position uncertainty (px), depth
// uncertainty (used only for the near-tie margins).  All cameras share W
// and H.  Outputs per camera: image[c][3][H][W], t_final[c][H][W],
// last[c][H][W], visits[c][H][W] (entries evaluated per pixel, including the
// one that stops it), and the smallest margin / uncertainty ratio of the
// pixel's depth-order, alpha and transmittance decisions (< 1: near tie).
int orc_composite(const int64_t* gid, const int64_t* ranges, const double* rec, int64_t n,
                  const double* cams, int n_cams, const double* bg, double* image, double* t_final,
                  int32_t* last, int64_t* visits, double* pmargin, const double* unc) {
  int64_t tile_base = 0;
  for (int ci = 0; ci < n_cams; ++ci) {
    const Cam c = load_cam(cams + 20 * ci);
    const int Tx = c.tx(), Ty = c.ty();
    const int64_t HW = (int64_t)c.H * c.W;
    std::vector<Rec> R(n);
    for (int64_t i = 0; i < n; ++i) {
      const double* q = rec + ((int64_t)ci * n + i) * 9;
      const double* e = unc + ((int64_t)ci * n + i) * 3;   // depth, perr, derr
      R[i] = Rec{q[0], q[1], q[2], q[3], q[4], q[5], {q[6], q[7], q[8]}, e[0], e[1], e[2]};
    }
#pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < Tx * Ty; ++t) {
      const int64_t s = ranges[2 * (tile_base + t)], e = ranges[2 * (tile_base + t) + 1];
      composite_tile(c, t % Tx, t / Tx, gid + s, e - s, R.data(), bg, image + ci * 3 * HW,
                     t_final + ci * HW, last + ci * HW, visits + ci * HW,
                     pmargin ? pmargin + ci * HW : nullptr);
    }
    tile_base += (int64_t)Tx * Ty;
  }
  return 0;
}

// Full forward render from parameters: O2-O7.  Also returns, per pair, the
// keep flag (active set) and the smallest decision margin.
int orc_render(const double* theta, int64_t n, const double* cams, int n_cams, const double* bg,
               double* image, double* t_final, int32_t* last, int64_t* visits, double* pair_margin,
               double* pix_margin, int32_t* keep_out) {
  std::vector<double> pf((size_t)n_cams * n * 16);
  std::vector<int32_t> pi((size_t)n_cams * n * 7);
  orc_project(theta, n, cams, n_cams, pf.data(), pi.data(), pair_margin);
  std::vector<double> u(n_cams * n), v(n_cams * n), d(n_cams * n), rec(n_cams * n * 9), unc(n_cams * n * 3);
  std::vector<int32_t> r(n_cams * n), k(n_cams * n);
  for (int64_t q = 0; q < n_cams * n; ++q) {
    u[q] = pf[16 * q]; v[q] = pf[16 * q + 1]; d[q] = sort_key(pf[16 * q + 2]);
    r[q] = pi[7 * q + 1]; k[q] = pi[7 * q];
    for (int j = 0; j < 9; ++j) rec[9 * q + j] = pf[16 * q + (j < 2 ? j : j + 1)];
    unc[3 * q] = d[q]; unc[3 * q + 1] = pf[16 * q + 14]; unc[3 * q + 2] = pf[16 * q + 15];
    if (keep_out) keep_out[q] = k[q];
  }
  int64_t tiles = 0;
  for (int ci = 0; ci < n_cams; ++ci) {
    const Cam c = load_cam(cams + 20 * ci);
    tiles += (int64_t)c.tx() * c.ty();
  }
  std::vector<int64_t> ranges(2 * tiles);
  const int64_t m = orc_bin(u.data(), v.data(), d.data(), r.data(), k.data(), n, cams, n_cams, nullptr, 0,
                            ranges.data());
  std::vector<int64_t> gid(std::max<int64_t>(m, 1));
  orc_bin(u.data(), v.data(), d.data(), r.data(), k.data(), n, cams, n_cams, gid.data(), m, ranges.data());
  orc_composite(gid.data(), ranges.data(), rec.data(), n, cams, n_cams, bg, image, t_final, last, visits,
                pix_margin, unc.data());
  return 0;
}

// Loss, O8: L = mean_v [0.8 mean|I-T| + 0.2 (1 - mean SSIM)], and dL/dI.
int orc_loss(const double* img, const double* target, int n_views, int H, int W, double* loss,
             double* dimg) {
  const std::vector<double> g = gauss_window();
  const int64_t HW = (int64_t)H * W;
  const double n_el = 3.0 * HW;
  const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
  double total = 0;
  std::vector<double> x2(HW), y2(HW), xy(HW), mx(HW), my(HW), mxx(HW), myy(HW), mxy(HW);
  std::vector<double> d1(HW), d2(HW), d12(HW), b1(HW), b2(HW), b12(HW);
  for (int vi = 0; vi < n_views; ++vi) {
    double l1 = 0, ss = 0;
    for (int ch = 0; ch < 3; ++ch) {
      const double* X = img + ((int64_t)vi * 3 + ch) * HW;
      const double* Y = target + ((int64_t)vi * 3 + ch) * HW;
      double* G = dimg + ((int64_t)vi * 3 + ch) * HW;
      for (int64_t p = 0; p < HW; ++p) {
        x2[p] = X[p] * X[p]; y2[p] = Y[p] * Y[p]; xy[p] = X[p] * Y[p];
      }
      conv11(X, H, W, g, mx.data());
      conv11(Y, H, W, g, my.data());
      conv11(x2.data(), H, W, g, mxx.data());
      conv11(y2.data(), H, W, g, myy.data());
      conv11(xy.data(), H, W, g, mxy.data());
      for (int64_t p = 0; p < HW; ++p) {
        const double mux = mx[p], muy = my[p];
        const double sx = mxx[p] - mux * mux, sy = myy[p] - muy * muy, sxy = mxy[p] - mux * muy;
        const double Np = 2 * mux * muy + C1, Ns = 2 * sxy + C2;
        const double Dp = mux * mux + muy * muy + C1, Ds = sx + sy + C2;
        const double s = (Np * Ns) / (Dp * Ds);
        ss += s;
        // partial derivatives of s with respect to mu_x, sigma_x^2, sigma_xy
        const double ds_dmux = (2 * muy * Ns) / (Dp * Ds) - s * (2 * mux) / Dp;
        const double ds_dsx = -s / Ds;
        const double ds_dsxy = 2 * Np / (Dp * Ds);
        // chain to the window moments m1 = w*x, m2 = w*x^2, m12 = w*(xy)
        d1[p] = ds_dmux - 2 * mux * ds_dsx - muy * ds_dsxy;
        d2[p] = ds_dsx;
        d12[p] = ds_dsxy;
        const double diff = X[p] - Y[p];
        l1 += std::fabs(diff);
        G[p] = 0.8 * (diff > 0 ? 1.0 : (diff < 0 ? -1.0 : 0.0)) / n_el;
      }
      // the window operator is symmetric, so its adjoint is the same convolution
      conv11(d1.data(), H, W, g, b1.data());
      conv11(d2.data(), H, W, g, b2.data());
      conv11(d12.data(), H, W, g, b12.data());
      for (int64_t p = 0; p < HW; ++p) {
        const double dsdx = b1[p] + 2 * X[p] * b2[p] + Y[p] * b12[p];
        G[p] = (G[p] - 0.2 * dsdx / n_el) / n_views;
      }
    }
    total += 0.8 * l1 / n_el + 0.2 * (1.0 - ss / n_el);
  }
  *loss = total / n_views;
  return 0;
}

// Backward, O9-O10.  dimg = dL/dI [V][3][H][W].  grad[n][59] is overwritten.
// g2d (optional) [V][n][9] receives the per-pair 2-D gradients
// (du, dv, dA, dB, dC, dopacity, dr, dg, db).
int orc_backward(const double* theta, int64_t n, const double* cams, int n_cams, const double* bg,
                 const double* dimg, double* grad, double* g2d_out) {
  std::memset(grad, 0, sizeof(double) * kD * n);
  for (int ci = 0; ci < n_cams; ++ci) {
    const Cam c = load_cam(cams + 20 * ci);
    const int Tx = c.tx(), Ty = c.ty();
    const int64_t HW = (int64_t)c.H * c.W;
    std::vector<Fwd> F(n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) project_one(theta + kD * i, c, F[i]);
    std::vector<double> u(n), v(n), d(n);
    std::vector<int32_t> r(n), k(n);
    std::vector<Rec> R(n);
    for (int64_t i = 0; i < n; ++i) {
      u[i] = F[i].u; v[i] = F[i].v; d[i] = sort_key(F[i].depth); r[i] = F[i].r; k[i] = F[i].keep;
      R[i] = Rec{F[i].u, F[i].v, F[i].A, F[i].B, F[i].C, F[i].op, {F[i].rgb[0], F[i].rgb[1], F[i].rgb[2]},
                 F[i].depth, F[i].perr, F[i].derr};
    }
    std::vector<Inst> insts;
    bin_camera(c, n, u.data(), v.data(), d.data(), r.data(), k.data(), insts);
    const int64_t M = insts.size();
    std::vector<int64_t> start(Tx * Ty, 0), end(Tx * Ty, 0);
    for (int64_t m = 0; m < M; ++m) {
      if (m == 0 || insts[m - 1].tile != insts[m].tile) start[insts[m].tile] = m;
      end[insts[m].tile] = m + 1;
    }
    // per-instance 2-D partials; every instance belongs to exactly one tile
    std::vector<double> part(9 * M, 0.0);
    const double* G = dimg + (int64_t)ci * 3 * HW;
#pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < Tx * Ty; ++t) {
      const int tx = t % Tx, ty = t / Tx;
      const int64_t s0 = start[t], len = end[t] - start[t];
      for (int py = ty * kTile; py < std::min(c.H, (ty + 1) * kTile); ++py)
        for (int px = tx * kTile; px < std::min(c.W, (tx + 1) * kTile); ++px) {
          // forward pass for this pixel: final T and last contributor
          double T = 1.0;
          int64_t lst = 0;
          for (int64_t j = 0; j < len; ++j) {
            const Rec& q = R[insts[s0 + j].gid];
            const double dx = px + 0.5 - q.u, dy = py + 0.5 - q.v;
            const double power = -0.5 * (q.A * dx * dx + q.C * dy * dy) - q.B * dx * dy;
            if (power > 0) continue;
            const double alpha = std::min(0.99, q.op * std::exp(power));
            if (alpha < 1.0 / 255.0) continue;
            const double Tn = T * (1 - alpha);
            if (Tn < 1e-4) break;
            T = Tn;
            lst = j + 1;
          }
          const int64_t pix = (int64_t)py * c.W + px;
          const double g[3] = {G[pix], G[HW + pix], G[2 * HW + pix]};
          double rb[3] = {bg[0], bg[1], bg[2]};  // normalised colour behind the entry
          for (int64_t j = lst - 1; j >= 0; --j) {
            const Rec& q = R[insts[s0 + j].gid];
            const double dx = px + 0.5 - q.u, dy = py + 0.5 - q.v;
            const double power = -0.5 * (q.A * dx * dx + q.C * dy * dy) - q.B * dx * dy;
            if (power > 0) continue;
            const double Gv = std::exp(power);
            const double a_raw = q.op * Gv;
            const double alpha = std::min(0.99, a_raw);
            if (alpha < 1.0 / 255.0) continue;
            T = T / (1 - alpha);               // transmittance in front of entry j
            double* P = &part[9 * (s0 + j)];
            double dalpha = 0;
            for (int ch = 0; ch < 3; ++ch) {
              P[6 + ch] += alpha * T * g[ch];
              dalpha += T * (q.rgb[ch] - rb[ch]) * g[ch];
            }
            for (int ch = 0; ch < 3; ++ch) rb[ch] = alpha * q.rgb[ch] + (1 - alpha) * rb[ch];
            if (a_raw >= 0.99) continue;       // clamped: alpha does not depend on the inputs
            P[5] += dalpha * Gv;               // d/d opacity
            const double dpow = dalpha * a_raw;
            P[0] += dpow * (q.A * dx + q.B * dy);  // d/du
            P[1] += dpow * (q.B * dx + q.C * dy);  // d/dv
            P[2] += dpow * (-0.5 * dx * dx);
            P[3] += dpow * (-dx * dy);
            P[4] += dpow * (-0.5 * dy * dy);
          }
        }
    }
    // per-pair 2-D gradients, summed over instances in list order
    std::vector<double> g2(9 * n, 0.0);
    for (int64_t m = 0; m < M; ++m)
      for (int k2 = 0; k2 < 9; ++k2) g2[9 * insts[m].gid + k2] += part[9 * m + k2];
    if (g2d_out) std::memcpy(g2d_out + (int64_t)ci * n * 9, g2.data(), sizeof(double) * 9 * n);

    // preprocess adjoint
    for (int64_t i = 0; i < n; ++i) {
      const Fwd& f = F[i];
      if (!f.keep) continue;
      const double* th = theta + kD * i;
      double* gr = grad + kD * i;
      const double* q2 = &g2[9 * i];
      const double gu = q2[0], gv = q2[1], gA = q2[2], gB = q2[3], gC = q2[4], gop = q2[5];
      double dmu[3] = {0, 0, 0};
      // colour: SH coefficients and view direction
      double graw[3];
      for (int ch = 0; ch < 3; ++ch) graw[ch] = f.raw[ch] < 0 ? 0.0 : q2[6 + ch];
      double Y[16], dY[16][3];
      sh_basis(f.dir, Y);
      sh_basis_grad(f.dir, dY);
      double gdir[3] = {0, 0, 0};
      for (int k2 = 0; k2 < 16; ++k2)
        for (int ch = 0; ch < 3; ++ch) {
          gr[11 + 3 * k2 + ch] += Y[k2] * graw[ch];
          const double fk = th[11 + 3 * k2 + ch];
          for (int a = 0; a < 3; ++a) gdir[a] += fk * graw[ch] * dY[k2][a];
        }
      const double dd = gdir[0] * f.dir[0] + gdir[1] * f.dir[1] + gdir[2] * f.dir[2];
      for (int a = 0; a < 3; ++a) dmu[a] += (gdir[a] - dd * f.dir[a]) / f.vlen;
      // opacity
      gr[10] += gop * f.op * (1 - f.op);
      // conic -> Sigma' : dL/dSigma' = -Q Gq Q with Gq the symmetric-matrix gradient
      const double Q[4] = {f.A, f.B, f.B, f.C};
      const double Gq[4] = {gA, 0.5 * gB, 0.5 * gB, gC};
      double QG[4], dS2[4];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) QG[2 * a + b] = Q[2 * a] * Gq[b] + Q[2 * a + 1] * Gq[2 + b];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) dS2[2 * a + b] = -(QG[2 * a] * Q[b] + QG[2 * a + 1] * Q[2 + b]);
      // Sigma' = T Sigma T^T (+0.3 I): dL/dSigma = T^T dS2 T, dL/dT = 2 dS2 T Sigma
      double dSig[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0;
          for (int k2 = 0; k2 < 2; ++k2)
            for (int l = 0; l < 2; ++l) s += f.T[3 * k2 + a] * dS2[2 * k2 + l] * f.T[3 * l + b];
          dSig[3 * a + b] = s;
        }
      double dT[6];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0;
          for (int l = 0; l < 2; ++l)
            for (int k2 = 0; k2 < 3; ++k2) s += dS2[2 * a + l] * f.T[3 * l + k2] * f.Sig[3 * k2 + b];
          dT[3 * a + b] = 2 * s;
        }
      // T = J W -> dL/dJ = dT W^T
      double dJ[6];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0;
          for (int k2 = 0; k2 < 3; ++k2) s += dT[3 * a + k2] * c.R[3 * b + k2];
          dJ[3 * a + b] = s;
        }
      // J(p) and (u, v)(p) -> dL/dp
      const double px = f.p[0], py = f.p[1], pz = f.p[2];
      double dp[3] = {0, 0, 0};
      dp[0] += gu * c.fx / pz;
      dp[1] += gv * c.fy / pz;
      dp[2] += -(gu * c.fx * px + gv * c.fy * py) / (pz * pz);
      dp[2] += -dJ[0] * c.fx / (pz * pz) - dJ[4] * c.fy / (pz * pz);
      if (!f.clampx) {  // J02 = -fx px / pz^2
        dp[0] += dJ[2] * (-c.fx / (pz * pz));
        dp[2] += dJ[2] * (2 * c.fx * px / (pz * pz * pz));
      } else {          // J02 = -fx xi / pz with xi fixed
        dp[2] += dJ[2] * (c.fx * f.xi / (pz * pz));
      }
      if (!f.clampy) {
        dp[1] += dJ[5] * (-c.fy / (pz * pz));
        dp[2] += dJ[5] * (2 * c.fy * py / (pz * pz * pz));
      } else {
        dp[2] += dJ[5] * (c.fy * f.eta / (pz * pz));
      }
      // p = W mu + t
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) dmu[a] += c.R[3 * b + a] * dp[b];
      for (int a = 0; a < 3; ++a) gr[a] += dmu[a];
      // Sigma = M M^T, M = Rq diag(s)
      double dM[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0;
          for (int k2 = 0; k2 < 3; ++k2) s += (dSig[3 * a + k2] + dSig[3 * k2 + a]) * f.M[3 * k2 + b];
          dM[3 * a + b] = s;
        }
      double dRq[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) dRq[3 * a + b] = dM[3 * a + b] * f.s[b];
      for (int b = 0; b < 3; ++b) {
        double s = 0;
        for (int a = 0; a < 3; ++a) s += dM[3 * a + b] * f.Rq[3 * a + b];
        gr[3 + b] += s * f.s[b];  // d/d log-scale
      }
      const double w = f.qh[0], x = f.qh[1], y = f.qh[2], z = f.qh[3];
      const double* g9 = dRq;
      double dq[4];
      dq[0] = 2 * (-z * g9[1] + y * g9[2] + z * g9[3] - x * g9[5] - y * g9[6] + x * g9[7]);
      dq[1] = 2 * (y * g9[1] + z * g9[2] + y * g9[3] - 2 * x * g9[4] - w * g9[5] + z * g9[6] + w * g9[7] -
                   2 * x * g9[8]);
      dq[2] = 2 * (-2 * y * g9[0] + x * g9[1] + w * g9[2] + x * g9[3] + z * g9[5] - w * g9[6] + z * g9[7] -
                   2 * y * g9[8]);
      dq[3] = 2 * (-2 * z * g9[0] - w * g9[1] + x * g9[2] + w * g9[3] - 2 * z * g9[4] + y * g9[5] + x * g9[6] +
                   y * g9[7]);
      const double dqq = dq[0] * f.qh[0] + dq[1] * f.qh[1] + dq[2] * f.qh[2] + dq[3] * f.qh[3];
      for (int a = 0; a < 4; ++a) gr[6 + a] += (dq[a] - dqq * f.qh[a]) / f.qn;
    }
  }
  return 0;
}

// Masked Adam, O11 (Appendix A, masked update equation).  Rows with
// active[i] == 0 are left untouched, bit for bit.
int orc_adam(double* theta, double* m, double* v, int64_t* step, const double* grad, const uint8_t* active,
             int64_t n, const double* lr, double b1, double b2, double eps) {
  for (int64_t i = 0; i < n; ++i) {
    if (!active[i]) continue;
    const int64_t t = ++step[i];
    const double bc1 = 1.0 - std::pow(b1, (double)t), bc2 = 1.0 - std::pow(b2, (double)t);
    for (int j = 0; j < kD; ++j) {
      const int64_t k = kD * i + j;
      const double g = grad[k];
      m[k] = b1 * m[k] + (1 - b1) * g;
      v[k] = b2 * v[k] + (1 - b2) * g * g;
      theta[k] -= lr[j] * (m[k] / bc1) / (std::sqrt(v[k] / bc2) + eps);
    }
  }
  return 0;
}

}  // extern "C"
