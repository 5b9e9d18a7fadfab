// Photometric loss 0.8 L1 + 0.2 (1 - SSIM) and its gradient.  SSIM windows
// are separable 11-tap Gaussians (sigma 1.5, zero padding).
//
// One wave sweeps a strip of 64 columns (one per lane) down a strip of
// output rows.  Each input row is staged in LDS with a 5-column halo on both sides;
// a lane's horizontal 11-tap sums go into a register ring holding the last 11
// rows, and the vertical sum over the ring gives the output row 5 rows above
// the newest input row.  LDS carries only the horizontal exchange (two values
// per pixel in the forward, three in the backward), and the next input row is
// in flight while the current one is processed.
#include <cmath>

#include "common.h"

namespace tide {

constexpr int kHalo = 5, kTaps = 2 * kHalo + 1;
constexpr int kSpan = kWave + 2 * kHalo;   // 74 staged columns
// Ring turns per wave and the output rows they give (11 turns - 10 halo
// rows).  Set for 1080-row frames: the forward's 11 strips of 100 rows are
// 3960 waves, one round at its four waves per SIMD; the backward (68 VGPRs)
// does best with 14 strips of 78 rows (measured: 100 rows 204 us against
// 45 rows 213 us for the forward, 78 rows 164 us against 181 us for the
// backward, 4 x 3 x 1080 x 1920).
constexpr int kTurnsFwd = 10, kTurnsBwd = 8;
constexpr int rows_of(int turns) { return kTaps * turns - 2 * kHalo; }
constexpr int kRowsFwd = rows_of(kTurnsFwd), kRowsBwd = rows_of(kTurnsBwd);

template <typename T>
struct Win {
  T w[kTaps];
};

// Pass 1: per output pixel the five window moments, SSIM and the three
// derivative maps d1 = ds/dm1, d2 = ds/dm2, d12 = ds/dm12 (m1 = w*x,
// m2 = w*x^2, m12 = w*xy).  Per-wave partial sums of |x - y| and SSIM go to
// part[wave][2] for a fixed-order final sum.
template <typename T>
__global__ void __launch_bounds__(kWave) k_ssim_fwd(const T* __restrict__ X, const T* __restrict__ Y, int32_t H,
                                                    int32_t W, Win<T> win, T* __restrict__ dmaps,
                                                    double* __restrict__ part) {
  __shared__ T sx[2][kSpan], sy[2][kSpan];
  const int lane = threadIdx.x;
  const int64_t plane = blockIdx.z;
  const int64_t HW = (int64_t)H * W, PS = (int64_t)gridDim.z * HW;
  const T* x = X + plane * HW;
  const T* y = Y + plane * HW;
  const int c = blockIdx.x * kWave + lane;      // output column of this lane
  const int ca = c - kHalo;                     // column staged in slot lane
  const int cb = c + kWave - kHalo;             // column staged in slot 64 + lane (lane < 10)
  const bool ina = ca >= 0 && ca < W, inb = lane < 2 * kHalo && cb < W, inc = c < W;
  const int r0 = blockIdx.y * kRowsFwd;
  T xa, ya, xb, yb;   // the next input row
  auto fetch = [&](int ir) {
    const bool rin = ir >= 0 && ir < H;
    const int64_t o = (int64_t)ir * W;
    xa = rin && ina ? x[o + ca] : (T)0;
    ya = rin && ina ? y[o + ca] : (T)0;
    xb = rin && inb ? x[o + cb] : (T)0;
    yb = rin && inb ? y[o + cb] : (T)0;
  };
  fetch(r0 - kHalo);
  T ring[kTaps][5];
  const T C1 = (T)1e-4, C2 = (T)9e-4;
  double l1 = 0, ss = 0;
  for (int turn = 0; turn < kTurnsFwd; ++turn) {
#pragma unroll
    for (int j = 0; j < kTaps; ++j) {
      const int n = turn * kTaps + j;   // input rows staged before this one
      const int ir = r0 - kHalo + n;
      const int q = n & 1;
      sx[q][lane] = xa;
      sy[q][lane] = ya;
      if (lane < 2 * kHalo) {
        sx[q][kWave + lane] = xb;
        sy[q][kWave + lane] = yb;
      }
      if (n + 1 < kTaps * kTurnsFwd) fetch(ir + 1);
      __syncthreads();
      T a = 0, b = 0, aa = 0, bb = 0, ab = 0, xc = 0, yc = 0;
#pragma unroll
      for (int t = 0; t < kTaps; ++t) {
        const T xv = sx[q][lane + t], yv = sy[q][lane + t];
        const T wx = win.w[t] * xv, wy = win.w[t] * yv;
        a += wx; b += wy; aa += wx * xv; bb += wy * yv; ab += wx * yv;
        if (t == kHalo) { xc = xv; yc = yv; }
      }
      ring[j][0] = a; ring[j][1] = b; ring[j][2] = aa; ring[j][3] = bb; ring[j][4] = ab;
      // this input row is an output row of the wave: its L1 term
      if (n >= kHalo && n < kHalo + kRowsFwd && ir < H && inc) l1 += (double)(xc > yc ? xc - yc : yc - xc);
      if (n >= 2 * kHalo) {
        // ring slot (j + 1 + t) mod 11 holds input row ir - 10 + t
        T mx = 0, my = 0, mxx = 0, myy = 0, mxy = 0;
#pragma unroll
        for (int t = 0; t < kTaps; ++t) {
          const int s = (j + 1 + t) % kTaps;
          const T wt = win.w[t];
          mx += wt * ring[s][0]; my += wt * ring[s][1]; mxx += wt * ring[s][2];
          myy += wt * ring[s][3]; mxy += wt * ring[s][4];
        }
        const int o = ir - kHalo;
        if (o < H && inc) {
          const T sxx = mxx - mx * mx, syy = myy - my * my, sxy = mxy - mx * my;
          const T Np = 2 * mx * my + C1, Ns = 2 * sxy + C2, Dp = mx * mx + my * my + C1, Ds = sxx + syy + C2;
          // two reciprocals (the hardware's, within an ulp in FP32) in place
          // of three divisions: Dp >= C1 and Ds is about C2 or more
          const T iDp = Mth<T>::rcp_fast(Dp), iDs = Mth<T>::rcp_fast(Ds);
          const T iD = iDp * iDs;
          const T sv = Np * Ns * iD;
          const T ds_dmx = 2 * my * Ns * iD - sv * 2 * mx * iDp;
          const T ds_dsx = -sv * iDs;
          const T ds_dsxy = 2 * Np * iD;
          const int64_t p = plane * HW + (int64_t)o * W + c;
          dmaps[p] = ds_dmx - 2 * mx * ds_dsx - my * ds_dsxy;
          dmaps[p + PS] = ds_dsx;
          dmaps[p + 2 * PS] = ds_dsxy;
          ss += (double)sv;
        }
      }
    }
  }
  l1 = wave_sum(l1);
  ss = wave_sum(ss);
  if (lane == 0) {
    const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[2 * blk] = l1;
    part[2 * blk + 1] = ss;
  }
}

// Pass 2: dL/dx = (0.8 sign(x - y) - 0.2 (w*d1 + 2 x w*d2 + y w*d12)) / (3 H W V).
template <typename T>
__global__ void __launch_bounds__(kWave) k_ssim_bwd(const T* __restrict__ X, const T* __restrict__ Y,
                                                    const T* __restrict__ dmaps, int32_t H, int32_t W, Win<T> win,
                                                    T scale, T* __restrict__ dx_out) {
  __shared__ T sd[2][3][kSpan];
  const int lane = threadIdx.x;
  const int64_t plane = blockIdx.z;
  const int64_t HW = (int64_t)H * W, PS = (int64_t)gridDim.z * HW;
  const T* d = dmaps + plane * HW;
  const int c = blockIdx.x * kWave + lane;
  const int ca = c - kHalo, cb = c + kWave - kHalo;
  const bool ina = ca >= 0 && ca < W, inb = lane < 2 * kHalo && cb < W, inc = c < W;
  const int r0 = blockIdx.y * kRowsBwd;
  T da[3], db[3], xo, yo;   // the next input row of the maps; x, y of the next output row
  auto fetch = [&](int ir) {
    const bool rin = ir >= 0 && ir < H;
    const int64_t o = (int64_t)ir * W;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      da[m] = rin && ina ? d[m * PS + o + ca] : (T)0;
      db[m] = rin && inb ? d[m * PS + o + cb] : (T)0;
    }
    const int orow = ir - kHalo;
    const bool oin = orow >= 0 && orow < H && inc;
    xo = oin ? X[plane * HW + (int64_t)orow * W + c] : (T)0;
    yo = oin ? Y[plane * HW + (int64_t)orow * W + c] : (T)0;
  };
  fetch(r0 - kHalo);
  T ring[kTaps][3];
  for (int turn = 0; turn < kTurnsBwd; ++turn) {
#pragma unroll
    for (int j = 0; j < kTaps; ++j) {
      const int n = turn * kTaps + j;
      const int ir = r0 - kHalo + n;
      const int q = n & 1;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        sd[q][m][lane] = da[m];
        if (lane < 2 * kHalo) sd[q][m][kWave + lane] = db[m];
      }
      const T xv = xo, yv = yo;
      if (n + 1 < kTaps * kTurnsBwd) fetch(ir + 1);
      __syncthreads();
      T a = 0, b = 0, e = 0;
#pragma unroll
      for (int t = 0; t < kTaps; ++t) {
        const T wt = win.w[t];
        a += wt * sd[q][0][lane + t]; b += wt * sd[q][1][lane + t]; e += wt * sd[q][2][lane + t];
      }
      ring[j][0] = a; ring[j][1] = b; ring[j][2] = e;
      if (n >= 2 * kHalo) {
        T va = 0, vb = 0, ve = 0;
#pragma unroll
        for (int t = 0; t < kTaps; ++t) {
          const int s = (j + 1 + t) % kTaps;
          const T wt = win.w[t];
          va += wt * ring[s][0]; vb += wt * ring[s][1]; ve += wt * ring[s][2];
        }
        const int o = ir - kHalo;
        if (o < H && inc) {
          const T sg = xv > yv ? (T)1 : (xv < yv ? (T)-1 : (T)0);
          dx_out[plane * HW + (int64_t)o * W + c] = ((T)0.8 * sg - (T)0.2 * (va + 2 * xv * vb + yv * ve)) * scale;
        }
      }
    }
  }
}

// Fixed-order sum of the block partials: lane-strided partial sums, then a
// tree in LDS (deterministic for a given grid).
__global__ void __launch_bounds__(1024) k_loss_final(const double* part, int64_t nblk, double inv_n, double* loss) {
  __shared__ double r1[1024], r2[1024];
  double a = 0, b = 0;
  for (int64_t k = threadIdx.x; k < nblk; k += 1024) { a += part[2 * k]; b += part[2 * k + 1]; }
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) { r1[threadIdx.x] += r1[threadIdx.x + s]; r2[threadIdx.x] += r2[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = 0.8 * r1[0] * inv_n + 0.2 * (1.0 - r2[0] * inv_n);
}

template <typename T>
static Win<T> make_window() {
  Win<T> w;
  double g[kTaps], s = 0;
  for (int i = 0; i < kTaps; ++i) { g[i] = std::exp(-((i - 5) * (i - 5)) / (2 * 1.5 * 1.5)); s += g[i]; }
  for (int i = 0; i < kTaps; ++i) w.w[i] = (T)(g[i] / s);
  return w;
}

}  // namespace tide

using namespace tide;

extern "C" size_t tide_loss_ws_bytes(int32_t n_views, int32_t height, int32_t width, int32_t dtype) {
  const size_t es = dtype == TIDE_F64 ? 8 : 4;
  const size_t planes = (size_t)n_views * 3;
  const size_t nblk = planes * ceil_div(width, kWave) * ceil_div(height, kRowsFwd);
  return align_up(3 * planes * (size_t)height * width * es) + align_up(2 * nblk * sizeof(double)) + 256;
}

extern "C" tide_status tide_loss(const void* image, const void* target, int32_t n_views, int32_t height, int32_t width,
                                 int32_t dtype, double* d_loss, void* d_dimage, void* ws, size_t ws_bytes,
                                 void* stream) {
  TIDE_CHECK_ARG(image && target && d_loss && d_dimage && ws, "null argument");
  TIDE_CHECK_ARG(n_views > 0 && height > 0 && width > 0, "bad sizes");
  TIDE_CHECK_ARG((int64_t)n_views * 3 < 65536, "too many views");
  TIDE_CHECK_ARG(dtype == TIDE_F32 || dtype == TIDE_F64, "bad dtype");
  const size_t need = tide_loss_ws_bytes(n_views, height, width, dtype);
  if (ws_bytes < need) {
    set_error("loss workspace too small (%zu < %zu)", ws_bytes, need);
    return TIDE_ECAPACITY;
  }
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid((uint32_t)ceil_div(width, kWave), (uint32_t)ceil_div(height, kRowsFwd), (uint32_t)(n_views * 3));
  const dim3 gridb((uint32_t)ceil_div(width, kWave), (uint32_t)ceil_div(height, kRowsBwd), (uint32_t)(n_views * 3));
  const int64_t nblk = (int64_t)grid.x * grid.y * grid.z;
  const double n_all = 3.0 * height * width * n_views;
  Carver cv(ws);
  if (dtype == TIDE_F32) {
    float* dm = cv.take<float>(3 * (size_t)n_views * 3 * height * width);
    double* part = cv.take<double>(2 * nblk);
    const Win<float> w = make_window<float>();
    TIDE_TIMED("loss_fwd", st, hipLaunchKernelGGL(k_ssim_fwd<float>, grid, dim3(kWave), 0, st, (const float*)image, (const float*)target, height,
                       width, w, dm, part));
    TIDE_TIMED("loss_bwd", st, hipLaunchKernelGGL(k_ssim_bwd<float>, gridb, dim3(kWave), 0, st, (const float*)image, (const float*)target, dm,
                       height, width, w, (float)(1.0 / n_all), (float*)d_dimage));
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, st, part, nblk, 1.0 / n_all, d_loss);
  } else {
    double* dm = cv.take<double>(3 * (size_t)n_views * 3 * height * width);
    double* part = cv.take<double>(2 * nblk);
    const Win<double> w = make_window<double>();
    TIDE_TIMED("loss_fwd", st, hipLaunchKernelGGL(k_ssim_fwd<double>, grid, dim3(kWave), 0, st, (const double*)image, (const double*)target,
                       height, width, w, dm, part));
    TIDE_TIMED("loss_bwd", st, hipLaunchKernelGGL(k_ssim_bwd<double>, gridb, dim3(kWave), 0, st, (const double*)image, (const double*)target, dm,
                       height, width, w, 1.0 / n_all, (double*)d_dimage));
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, st, part, nblk, 1.0 / n_all, d_loss);
  }
  TIDE_LAUNCH_CHECK("tide_loss");
  return TIDE_OK;
}
