// Photometric loss 0.8 L1 + 0.2 (1 - SSIM) and its gradient.  SSIM windows
// are separable 11-tap Gaussians (sigma 1.5, zero padding); both passes run
// out of LDS on output tiles with a 5-pixel halo: 64 x 32 in single
// precision (halo re-reads 1.5x the tile, 79 KB of LDS, two workgroups per
// CU), 32 x 16 in double precision.
#include <cmath>

#include "common.h"

namespace tide {

constexpr int kHalo = 5;
template <typename T>
struct Tile {
  static constexpr int OW = sizeof(T) == 4 ? 64 : 32, OH = sizeof(T) == 4 ? 32 : 16;
  static constexpr int IW = OW + 2 * kHalo, IH = OH + 2 * kHalo;
  static constexpr int NT = sizeof(T) == 4 ? 512 : 256;   // threads per workgroup
};

template <typename T>
struct Win {
  T w[11];
};

// Pass 1: per output pixel the five window moments, SSIM and the three
// derivative maps d1 = ds/dm1, d2 = ds/dm2, d12 = ds/dm12 (m1 = w*x,
// m2 = w*x^2, m12 = w*xy).  Block partial sums of |x - y| and SSIM go to
// part[block][2] for a fixed-order final sum.
template <typename T>
__global__ void __launch_bounds__(Tile<T>::NT) k_ssim_fwd(const T* __restrict__ X, const T* __restrict__ Y, int32_t H,
                                                  int32_t W, Win<T> win, T* __restrict__ dmaps,
                                                  double* __restrict__ part) {
  constexpr int kOW = Tile<T>::OW, kOH = Tile<T>::OH, kIW = Tile<T>::IW, kIH = Tile<T>::IH, kNT = Tile<T>::NT;
  __shared__ T sx[kIH][kIW], sy[kIH][kIW];
  __shared__ T hc[5][kIH][kOW];
  __shared__ double red[2][kNT / kWave];
  const int64_t plane = blockIdx.z;
  const int64_t HW = (int64_t)H * W;
  const T* x = X + plane * HW;
  const T* y = Y + plane * HW;
  const int ox = blockIdx.x * kOW, oy = blockIdx.y * kOH;
  for (int k = threadIdx.x; k < kIH * kIW; k += kNT) {
    const int r = k / kIW, c = k % kIW;
    const int gy = oy - kHalo + r, gx = ox - kHalo + c;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    sx[r][c] = in ? x[(int64_t)gy * W + gx] : (T)0;
    sy[r][c] = in ? y[(int64_t)gy * W + gx] : (T)0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kIH * kOW; k += kNT) {
    const int r = k / kOW, c = k % kOW;
    T a = 0, b = 0, aa = 0, bb = 0, ab = 0;
#pragma unroll
    for (int t = 0; t < 11; ++t) {
      const T xv = sx[r][c + t], yv = sy[r][c + t], wt = win.w[t];
      a += wt * xv; b += wt * yv; aa += wt * xv * xv; bb += wt * yv * yv; ab += wt * xv * yv;
    }
    hc[0][r][c] = a; hc[1][r][c] = b; hc[2][r][c] = aa; hc[3][r][c] = bb; hc[4][r][c] = ab;
  }
  __syncthreads();
  const T C1 = (T)1e-4, C2 = (T)9e-4;
  double l1 = 0, ss = 0;
  for (int k = threadIdx.x; k < kOH * kOW; k += kNT) {
    const int r = k / kOW, c = k % kOW;
    const int gy = oy + r, gx = ox + c;
    if (gy >= H || gx >= W) continue;
    T mx = 0, my = 0, mxx = 0, myy = 0, mxy = 0;
#pragma unroll
    for (int t = 0; t < 11; ++t) {
      const T wt = win.w[t];
      mx += wt * hc[0][r + t][c]; my += wt * hc[1][r + t][c]; mxx += wt * hc[2][r + t][c];
      myy += wt * hc[3][r + t][c]; mxy += wt * hc[4][r + t][c];
    }
    const T sxx = mxx - mx * mx, syy = myy - my * my, sxy = mxy - mx * my;
    const T Np = 2 * mx * my + C1, Ns = 2 * sxy + C2, Dp = mx * mx + my * my + C1, Ds = sxx + syy + C2;
    const T iD = (T)1 / (Dp * Ds);
    const T s = Np * Ns * iD;
    const T ds_dmx = 2 * my * Ns * iD - s * 2 * mx / Dp;
    const T ds_dsx = -s / Ds;
    const T ds_dsxy = 2 * Np * iD;
    const int64_t p = plane * HW + (int64_t)gy * W + gx;
    dmaps[p] = ds_dmx - 2 * mx * ds_dsx - my * ds_dsxy;
    dmaps[p + 1 * (int64_t)gridDim.z * HW] = ds_dsx;
    dmaps[p + 2 * (int64_t)gridDim.z * HW] = ds_dsxy;
    const T xv = sx[r + kHalo][c + kHalo], yv = sy[r + kHalo][c + kHalo];
    l1 += (double)(xv > yv ? xv - yv : yv - xv);
    ss += (double)s;
  }
  l1 = wave_sum(l1);
  ss = wave_sum(ss);
  const int w = threadIdx.x / kWave;
  if (__lane_id() == 0) { red[0][w] = l1; red[1][w] = ss; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int q = 0; q < kNT / kWave; ++q) { a += red[0][q]; b += red[1][q]; }
    const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[2 * blk] = a;
    part[2 * blk + 1] = b;
  }
}

// Pass 2: dL/dx = (0.8 sign(x - y) - 0.2 (w*d1 + 2 x w*d2 + y w*d12)) / (3 H W V).
template <typename T>
__global__ void __launch_bounds__(Tile<T>::NT) k_ssim_bwd(const T* __restrict__ X, const T* __restrict__ Y,
                                                  const T* __restrict__ dmaps, int32_t H, int32_t W, Win<T> win,
                                                  T scale, T* __restrict__ dx_out) {
  constexpr int kOW = Tile<T>::OW, kOH = Tile<T>::OH, kIW = Tile<T>::IW, kIH = Tile<T>::IH, kNT = Tile<T>::NT;
  __shared__ T sd[3][kIH][kIW];
  __shared__ T hc[3][kIH][kOW];
  const int64_t plane = blockIdx.z;
  const int64_t HW = (int64_t)H * W, PS = (int64_t)gridDim.z * HW;
  const int ox = blockIdx.x * kOW, oy = blockIdx.y * kOH;
  for (int k = threadIdx.x; k < kIH * kIW; k += kNT) {
    const int r = k / kIW, c = k % kIW;
    const int gy = oy - kHalo + r, gx = ox - kHalo + c;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const int64_t p = plane * HW + (int64_t)gy * W + gx;
    sd[0][r][c] = in ? dmaps[p] : (T)0;
    sd[1][r][c] = in ? dmaps[p + PS] : (T)0;
    sd[2][r][c] = in ? dmaps[p + 2 * PS] : (T)0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kIH * kOW; k += kNT) {
    const int r = k / kOW, c = k % kOW;
    T a = 0, b = 0, e = 0;
#pragma unroll
    for (int t = 0; t < 11; ++t) {
      const T wt = win.w[t];
      a += wt * sd[0][r][c + t]; b += wt * sd[1][r][c + t]; e += wt * sd[2][r][c + t];
    }
    hc[0][r][c] = a; hc[1][r][c] = b; hc[2][r][c] = e;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kOH * kOW; k += kNT) {
    const int r = k / kOW, c = k % kOW;
    const int gy = oy + r, gx = ox + c;
    if (gy >= H || gx >= W) continue;
    T a = 0, b = 0, e = 0;
#pragma unroll
    for (int t = 0; t < 11; ++t) {
      const T wt = win.w[t];
      a += wt * hc[0][r + t][c]; b += wt * hc[1][r + t][c]; e += wt * hc[2][r + t][c];
    }
    const int64_t p = plane * HW + (int64_t)gy * W + gx;
    const T xv = X[p], yv = Y[p];
    const T sg = xv > yv ? (T)1 : (xv < yv ? (T)-1 : (T)0);
    dx_out[p] = ((T)0.8 * sg - (T)0.2 * (a + 2 * xv * b + yv * e)) * scale;
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
  double g[11], s = 0;
  for (int i = 0; i < 11; ++i) { g[i] = std::exp(-((i - 5) * (i - 5)) / (2 * 1.5 * 1.5)); s += g[i]; }
  for (int i = 0; i < 11; ++i) w.w[i] = (T)(g[i] / s);
  return w;
}

}  // namespace tide

using namespace tide;

extern "C" size_t tide_loss_ws_bytes(int32_t n_views, int32_t height, int32_t width, int32_t dtype) {
  const size_t es = dtype == TIDE_F64 ? 8 : 4;
  const size_t planes = (size_t)n_views * 3;
  const int ow = dtype == TIDE_F64 ? Tile<double>::OW : Tile<float>::OW;
  const int oh = dtype == TIDE_F64 ? Tile<double>::OH : Tile<float>::OH;
  const size_t nblk = planes * ceil_div(width, ow) * ceil_div(height, oh);
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
  const int ow = dtype == TIDE_F64 ? Tile<double>::OW : Tile<float>::OW;
  const int oh = dtype == TIDE_F64 ? Tile<double>::OH : Tile<float>::OH;
  const dim3 grid((uint32_t)ceil_div(width, ow), (uint32_t)ceil_div(height, oh), (uint32_t)(n_views * 3));
  const int64_t nblk = (int64_t)grid.x * grid.y * grid.z;
  const double n_all = 3.0 * height * width * n_views;
  Carver cv(ws);
  if (dtype == TIDE_F32) {
    float* dm = cv.take<float>(3 * (size_t)n_views * 3 * height * width);
    double* part = cv.take<double>(2 * nblk);
    const Win<float> w = make_window<float>();
    TIDE_TIMED("loss_fwd", st, hipLaunchKernelGGL(k_ssim_fwd<float>, grid, dim3(Tile<float>::NT), 0, st, (const float*)image, (const float*)target, height,
                       width, w, dm, part));
    TIDE_TIMED("loss_bwd", st, hipLaunchKernelGGL(k_ssim_bwd<float>, grid, dim3(Tile<float>::NT), 0, st, (const float*)image, (const float*)target, dm,
                       height, width, w, (float)(1.0 / n_all), (float*)d_dimage));
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, st, part, nblk, 1.0 / n_all, d_loss);
  } else {
    double* dm = cv.take<double>(3 * (size_t)n_views * 3 * height * width);
    double* part = cv.take<double>(2 * nblk);
    const Win<double> w = make_window<double>();
    TIDE_TIMED("loss_fwd", st, hipLaunchKernelGGL(k_ssim_fwd<double>, grid, dim3(Tile<double>::NT), 0, st, (const double*)image, (const double*)target,
                       height, width, w, dm, part));
    TIDE_TIMED("loss_bwd", st, hipLaunchKernelGGL(k_ssim_bwd<double>, grid, dim3(Tile<double>::NT), 0, st, (const double*)image, (const double*)target, dm,
                       height, width, w, 1.0 / n_all, (double*)d_dimage));
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, st, part, nblk, 1.0 / n_all, d_loss);
  }
  TIDE_LAUNCH_CHECK("tide_loss");
  return TIDE_OK;
}
