// Forward half of the rasterizer: preprocessing (projection, culling, EWA
// footprint, tile rectangle, SH colour), tile binning with the two-level
// depth/tile radix sort, and front-to-back compositing.
#include <cmath>
#include <cstring>
#include <mutex>

#include "onesweep.h"
#include "prims.h"
#include "raster.h"

namespace tide {

template <typename T>
CamSet<T> make_camset(const tide_camera* cams, int n) {
  CamSet<T> s;
  std::memset(&s, 0, sizeof(s));
  s.n = n;
  for (int i = 0; i < n; ++i) {
    const tide_camera& c = cams[i];
    DevCam<T>& d = s.c[i];
    for (int k = 0; k < 9; ++k) d.R[k] = (T)c.R[k];
    for (int k = 0; k < 3; ++k) d.t[k] = (T)c.t[k];
    for (int k = 0; k < 9; ++k) d.Rd[k] = c.R[k];
    for (int k = 0; k < 3; ++k) d.td[k] = c.t[k];
    d.fxd = c.fx; d.fyd = c.fy; d.cxd = c.cx; d.cyd = c.cy;
    d.fx = (T)c.fx; d.fy = (T)c.fy; d.cx = (T)c.cx; d.cy = (T)c.cy;
    d.znear = (T)c.z_near; d.zfar = (T)c.z_far;
    d.limx = (T)(1.3 * 0.5 * c.width / c.fx);
    d.limy = (T)(1.3 * 0.5 * c.height / c.fy);
    for (int k = 0; k < 3; ++k)
      d.pos[k] = (T)(-(c.R[k] * c.t[0] + c.R[3 + k] * c.t[1] + c.R[6 + k] * c.t[2]));
    d.W = c.width; d.H = c.height;
    d.Tx = (c.width + kTile - 1) / kTile;
    d.Ty = (c.height + kTile - 1) / kTile;
  }
  const double pi = M_PI;
  s.sh.c0 = (T)(0.5 * std::sqrt(1.0 / pi));
  s.sh.c1 = (T)std::sqrt(3.0 / (4.0 * pi));
  s.sh.c2a = (T)(0.5 * std::sqrt(15.0 / pi));
  s.sh.c2b = (T)(0.25 * std::sqrt(5.0 / pi));
  s.sh.c2c = (T)(0.25 * std::sqrt(15.0 / pi));
  s.sh.c3a = (T)(0.25 * std::sqrt(35.0 / (2.0 * pi)));
  s.sh.c3b = (T)(0.5 * std::sqrt(105.0 / pi));
  s.sh.c3c = (T)(0.25 * std::sqrt(21.0 / (2.0 * pi)));
  s.sh.c3d = (T)(0.25 * std::sqrt(7.0 / pi));
  s.sh.c3e = (T)(0.25 * std::sqrt(105.0 / pi));
  return s;
}
template CamSet<float> make_camset<float>(const tide_camera*, int);
template CamSet<double> make_camset<double>(const tide_camera*, int);

// ------------------------------------------------------------- preprocess
// One thread per processing index.  The mean (12 B) is read first and every
// camera's depth test runs on it; the other 56 columns are read only if some
// camera keeps the Gaussian.  Columns of a block are contiguous, so lanes
// (consecutive rows) read coalesced.  The camera-space position and the
// pixel position are computed in double: at aerial scales (|p| ~ 300 m,
// f ~ 1700 px) single precision would put ~3e-4 px of error on u, v, which a
// sub-pixel footprint turns into flipped alpha >= 1/255 decisions; rounding
// the double result once leaves at most half an ulp of u.  This costs a few
// FP64 operations per (Gaussian, camera) in a bandwidth-bound kernel.
__device__ inline double cam_depth(const double* Rd, const double* td, double m0, double m1, double m2) {
  return Rd[6] * m0 + Rd[7] * m1 + Rd[8] * m2 + td[2];
}
template <typename T>
__global__ void __launch_bounds__(256) k_preprocess(const T* __restrict__ params, const int32_t* __restrict__ order,
                                                    const int32_t* __restrict__ slot_rows, int32_t B,
                                                    int64_t n_pidx, CamSet<T> cs, T* __restrict__ rec,
                                                    float* __restrict__ depth, uint32_t* __restrict__ rect,
                                                    uint32_t* __restrict__ tt, uint32_t* __restrict__ active) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pidx) return;
  const int64_t k = i / B;
  const int32_t row = (int32_t)(i - k * B);
  const int32_t slot = order[k];
  const int ncam = cs.n;
  uint32_t keep = 0;
  T mu[3] = {0, 0, 0};
  const T* P = params + (int64_t)slot * kD * B + row;
  if (row < slot_rows[slot]) {
    mu[0] = P[0]; mu[1] = P[B]; mu[2] = P[2 * (int64_t)B];
#pragma unroll 1
    for (int c = 0; c < ncam; ++c) {
      const DevCam<T>& cm = cs.c[c];
      const double pz = cam_depth(cm.Rd, cm.td, (double)mu[0], (double)mu[1], (double)mu[2]);
      if (pz > (double)cm.znear && pz <= (double)cm.zfar) keep |= 1u << c;
    }
  }
  uint32_t any = 0;
  if (keep) {
    // activations
    const T s0 = Mth<T>::exp(P[3 * (int64_t)B]), s1 = Mth<T>::exp(P[4 * (int64_t)B]),
            s2 = Mth<T>::exp(P[5 * (int64_t)B]);
    T qw = P[6 * (int64_t)B], qx = P[7 * (int64_t)B], qy = P[8 * (int64_t)B], qz = P[9 * (int64_t)B];
    const T qn = Mth<T>::sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const T iq = (T)1 / qn;
    qw *= iq; qx *= iq; qy *= iq; qz *= iq;
    const T op = (T)1 / ((T)1 + Mth<T>::exp(-P[10 * (int64_t)B]));
    T sh[48];
#pragma unroll
    for (int m = 0; m < 48; ++m) sh[m] = P[(int64_t)(11 + m) * B];
    // Sigma = M M^T, M = R(q) diag(s)
    const T r00 = 1 - 2 * (qy * qy + qz * qz), r01 = 2 * (qx * qy - qw * qz), r02 = 2 * (qx * qz + qw * qy);
    const T r10 = 2 * (qx * qy + qw * qz), r11 = 1 - 2 * (qx * qx + qz * qz), r12 = 2 * (qy * qz - qw * qx);
    const T r20 = 2 * (qx * qz - qw * qy), r21 = 2 * (qy * qz + qw * qx), r22 = 1 - 2 * (qx * qx + qy * qy);
    const T m00 = r00 * s0, m01 = r01 * s1, m02 = r02 * s2;
    const T m10 = r10 * s0, m11 = r11 * s1, m12 = r12 * s2;
    const T m20 = r20 * s0, m21 = r21 * s1, m22 = r22 * s2;
    const T S00 = m00 * m00 + m01 * m01 + m02 * m02;
    const T S01 = m00 * m10 + m01 * m11 + m02 * m12;
    const T S02 = m00 * m20 + m01 * m21 + m02 * m22;
    const T S11 = m10 * m10 + m11 * m11 + m12 * m12;
    const T S12 = m10 * m20 + m11 * m21 + m12 * m22;
    const T S22 = m20 * m20 + m21 * m21 + m22 * m22;
#pragma unroll 1
    for (int c = 0; c < ncam; ++c) {
      const int64_t o = (int64_t)c * n_pidx + i;
      uint32_t ntt = 0;
      if (keep & (1u << c)) {
        const DevCam<T>& cm = cs.c[c];
        const double m0 = mu[0], m1 = mu[1], m2 = mu[2];
        const double pxd = cm.Rd[0] * m0 + cm.Rd[1] * m1 + cm.Rd[2] * m2 + cm.td[0];
        const double pyd = cm.Rd[3] * m0 + cm.Rd[4] * m1 + cm.Rd[5] * m2 + cm.td[1];
        const double pzd = cam_depth(cm.Rd, cm.td, m0, m1, m2);
        const double izd = 1.0 / pzd;
        const T u = (T)(cm.fxd * pxd * izd + cm.cxd);
        const T v = (T)(cm.fyd * pyd * izd + cm.cyd);
        const T px = (T)pxd, py = (T)pyd, pz = (T)pzd;
        const T iz = (T)izd;
        T xi = px * iz, eta = py * iz;
        xi = xi < -cm.limx ? -cm.limx : (xi > cm.limx ? cm.limx : xi);
        eta = eta < -cm.limy ? -cm.limy : (eta > cm.limy ? cm.limy : eta);
        const T j00 = cm.fx * iz, j02 = -cm.fx * xi * iz, j11 = cm.fy * iz, j12 = -cm.fy * eta * iz;
        // T = J W (2x3)
        const T t00 = j00 * cm.R[0] + j02 * cm.R[6], t01 = j00 * cm.R[1] + j02 * cm.R[7],
                t02 = j00 * cm.R[2] + j02 * cm.R[8];
        const T t10 = j11 * cm.R[3] + j12 * cm.R[6], t11 = j11 * cm.R[4] + j12 * cm.R[7],
                t12 = j11 * cm.R[5] + j12 * cm.R[8];
        const T a0 = t00 * S00 + t01 * S01 + t02 * S02, a1 = t00 * S01 + t01 * S11 + t02 * S12,
                a2 = t00 * S02 + t01 * S12 + t02 * S22;
        const T b0 = t10 * S00 + t11 * S01 + t12 * S02, b1 = t10 * S01 + t11 * S11 + t12 * S12,
                b2 = t10 * S02 + t11 * S12 + t12 * S22;
        const T c00 = a0 * t00 + a1 * t01 + a2 * t02 + (T)0.3;
        const T c01 = a0 * t10 + a1 * t11 + a2 * t12;
        const T c11 = b0 * t10 + b1 * t11 + b2 * t12 + (T)0.3;
        const T det = c00 * c11 - c01 * c01;
        if (det > 0) {
          const T idet = (T)1 / det;
          const T mid = (T)0.5 * (c00 + c11);
          T disc = mid * mid - det;
          disc = disc > 0 ? disc : (T)0;
          T rr = (T)3 * Mth<T>::sqrt(mid + Mth<T>::sqrt(disc));
          rr = rr < (T)2097152 ? rr : (T)2097152;
          const int r = (int)Mth<T>::ceil(rr);
          int x0, y0, x1, y1;
          if (tile_rect<T>(u, v, r, cm.Tx, cm.Ty, x0, y0, x1, y1)) {
            ntt = (uint32_t)((x1 - x0) * (y1 - y0));
            // view-dependent colour
            T dx = mu[0] - cm.pos[0], dy = mu[1] - cm.pos[1], dz = mu[2] - cm.pos[2];
            const T il = (T)1 / Mth<T>::sqrt(dx * dx + dy * dy + dz * dz);
            dx *= il; dy *= il; dz *= il;
            T Y[16];
            sh_eval<T>(cs.sh, dx, dy, dz, Y);
            T col[3] = {(T)0.5, (T)0.5, (T)0.5};
#pragma unroll
            for (int m = 0; m < 16; ++m) {
              col[0] += Y[m] * sh[3 * m];
              col[1] += Y[m] * sh[3 * m + 1];
              col[2] += Y[m] * sh[3 * m + 2];
            }
            T* R12 = rec + o * kRec;
            R12[0] = u; R12[1] = v;
            R12[2] = c11 * idet; R12[3] = -c01 * idet; R12[4] = c00 * idet;
            R12[5] = op;
            R12[6] = col[0] > 0 ? col[0] : (T)0;
            R12[7] = col[1] > 0 ? col[1] : (T)0;
            R12[8] = col[2] > 0 ? col[2] : (T)0;
            R12[9] = pz; R12[10] = (T)r; R12[11] = 0;
            depth[o] = (float)pzd;
            rect[2 * o] = (uint32_t)x0 | ((uint32_t)y0 << 16);
            rect[2 * o + 1] = (uint32_t)x1 | ((uint32_t)y1 << 16);
          }
        }
      }
      tt[o] = ntt;
      any |= ntt;
    }
  } else {
    for (int c = 0; c < ncam; ++c) tt[(int64_t)c * n_pidx + i] = 0;
  }
  active[i] = any ? 1u : 0u;
}

size_t preprocess_ws_bytes(int64_t n_pidx) {
  return align_up(scan_partial_count(n_pidx) * 8) + 256;
}

template <typename T>
static tide_status preprocess_t(const tide_pool* pool, const tide_camera* cams, int n_cams, tide_proj* out,
                                void* ws, hipStream_t st) {
  const CamSet<T> cs = make_camset<T>(cams, n_cams);
  const int64_t n = out->n_pidx;
  if (n > 0) {
    TIDE_TIMED("preprocess", st, hipLaunchKernelGGL(k_preprocess<T>, dim3((uint32_t)ceil_div(n, 256)), dim3(256), 0, st,
                       (const T*)pool->params, pool->order, pool->slot_rows, pool->block_rows, n, cs,
                       (T*)out->rec, out->depth, out->rect, out->tiles_touched, out->active));
    TIDE_LAUNCH_CHECK("k_preprocess");
  }
  Carver cv(ws);
  unsigned long long* partial = cv.take<unsigned long long>(scan_partial_count(n));
  unsigned long long* total = cv.take<unsigned long long>(1);
  // the count goes to the caller as u32 from the block that holds the total
  scan_exclusive(ArrayIn{out->active}, n, out->act_idx, partial, total, st, nullptr,
                 ScanTail{out->n_active, nullptr});
  TIDE_LAUNCH_CHECK("active scan");
  return TIDE_OK;
}

static tide_status check_pool(const tide_pool* pool) {
  TIDE_CHECK_ARG(pool, "pool is null");
  TIDE_CHECK_ARG(pool->params && pool->order && pool->slot_rows && pool->slot_block, "pool has a null pointer");
  TIDE_CHECK_ARG(pool->block_rows > 0 && pool->n_slots > 0 && pool->n_order >= 0 && pool->n_order <= pool->n_slots,
                 "bad pool sizes (block_rows %d, n_slots %d, n_order %d)", pool->block_rows, pool->n_slots,
                 pool->n_order);
  TIDE_CHECK_ARG(pool->dtype == TIDE_F32 || pool->dtype == TIDE_F64, "bad dtype %d", pool->dtype);
  TIDE_CHECK_ARG(aligned16(pool->params), "params must be 16-byte aligned");
  return TIDE_OK;
}

static tide_status check_cams(const tide_camera* cams, int n_cams) {
  TIDE_CHECK_ARG(cams, "cams is null");
  TIDE_CHECK_ARG(n_cams >= 1 && n_cams <= TIDE_MAX_CAMS, "n_cams must be in [1, %d]", TIDE_MAX_CAMS);
  for (int c = 0; c < n_cams; ++c) {
    TIDE_CHECK_ARG(cams[c].width > 0 && cams[c].height > 0 && cams[c].width <= 65535 * 16 &&
                       cams[c].height <= 65535 * 16,
                   "camera %d has a bad image size", c);
    TIDE_CHECK_ARG(cams[c].fx > 0 && cams[c].fy > 0, "camera %d has a non-positive focal length", c);
    TIDE_CHECK_ARG(cams[c].z_near > 0 && cams[c].z_far > cams[c].z_near, "camera %d has bad near/far planes", c);
  }
  return TIDE_OK;
}

static tide_status check_proj(const tide_proj* p) {
  TIDE_CHECK_ARG(p, "proj is null");
  TIDE_CHECK_ARG(p->rec && p->depth && p->rect && p->tiles_touched && p->active && p->act_idx && p->n_active,
                 "proj has a null pointer");
  TIDE_CHECK_ARG(aligned16(p->rec), "proj.rec must be 16-byte aligned");
  TIDE_CHECK_ARG(p->n_cams >= 1 && p->n_cams <= TIDE_MAX_CAMS, "proj.n_cams out of range");
  TIDE_CHECK_ARG(p->n_pidx >= 0 && (int64_t)p->n_cams * p->n_pidx < (int64_t)UINT32_MAX,
                 "n_cams * n_pidx must fit 32 bits");
  TIDE_CHECK_ARG(p->dtype == TIDE_F32 || p->dtype == TIDE_F64, "bad dtype");
  return TIDE_OK;
}

// ---------------------------------------------------------------- binning
// Down-sweep of the visibility scan fused with the compaction.  Thread t of
// block b owns elements [4096 b + 16 t, + 16) of the flattened (camera,
// pidx) array (read in 16-byte pieces when vec); a visible element's place
// among the block's visible elements (exclusive scan of the flags) puts its
// key (the depth's bit pattern: depth > 0, so it orders like the value) and
// its index in LDS, and the block's run is written out contiguously at the
// block's start, the sum of the earlier blocks' counts (kSums: added up here
// from the blocks' sums, one launch fewer; else partial holds their scan).
// Block 0 writes the count of visible pairs.  The grid also clears
// clear32[0, n_clear) (the depth sort's control words) and *clear64 (the
// binning's error word).
template <bool kSums>
__global__ void __launch_bounds__(kScanThreads) k_vis_compact(const uint32_t* __restrict__ tt,
                                                              const float* __restrict__ depth, int64_t n,
                                                              const unsigned long long* __restrict__ partial,
                                                              int64_t nb, unsigned long long* __restrict__ total,
                                                              uint32_t* __restrict__ key, uint32_t* __restrict__ val,
                                                              uint32_t* __restrict__ clear32, int64_t n_clear,
                                                              unsigned long long* __restrict__ clear64, int vec) {
  for (int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x; i < n_clear;
       i += (int64_t)gridDim.x * kScanThreads)
    clear32[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *clear64 = 0ull;
  constexpr int kW = kScanThreads / kWave;
  __shared__ unsigned long long bpre[kW + 1];
  __shared__ uint32_t wtot[kW];
  __shared__ uint32_t skey[kScanTile], sval[kScanTile];
  const int w = threadIdx.x / kWave, lane = __lane_id();
  if (kSums) {
    const int64_t upto = blockIdx.x == 0 ? nb : (int64_t)blockIdx.x;
    unsigned long long a = 0;
    for (int64_t q = threadIdx.x; q < upto; q += kScanThreads) a += partial[q];
    a = wave_sum(a);
    if (lane == 0) bpre[w] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long t = 0;
      for (int q = 0; q < kW; ++q) t += bpre[q];
      if (blockIdx.x == 0) *total = t;
      bpre[kW] = blockIdx.x == 0 ? 0ull : t;
    }
    __syncthreads();
  }
  const unsigned long long bp = kSums ? bpre[kW] : partial[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t f[kScanItems], d[kScanItems];
  if (vec && base + kScanItems <= n) {
#pragma unroll
    for (int j = 0; j < kScanItems; j += 4) {
      const uint4 a = *reinterpret_cast<const uint4*>(tt + base + j);
      const uint4 b = *reinterpret_cast<const uint4*>(depth + base + j);
      f[j] = a.x != 0u; f[j + 1] = a.y != 0u; f[j + 2] = a.z != 0u; f[j + 3] = a.w != 0u;
      d[j] = b.x; d[j + 1] = b.y; d[j + 2] = b.z; d[j + 3] = b.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const bool in = base + k < n;
      f[k] = in && tt[base + k] != 0u;
      d[k] = f[k] ? __float_as_uint(depth[base + k]) : 0u;
    }
  }
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) sum += f[k];
  const uint32_t inc = wave_incl_scan(sum);
  if (lane == kWave - 1) wtot[w] = inc;
  __syncthreads();
  uint32_t off = inc - sum, cnt = 0;
  for (int q = 0; q < kW; ++q) {
    off += q < w ? wtot[q] : 0u;
    cnt += wtot[q];
  }
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (f[k]) {
      skey[off] = d[k];
      sval[off] = (uint32_t)(base + k);
      ++off;
    }
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < cnt; j += kScanThreads) {
    key[bp + j] = skey[j];
    val[bp + j] = sval[j];
  }
}

// What the depth sort's last pass writes for each visible pair, in depth
// order: the key of its rectangle's first tile (camera-major tile id), its
// record index, the rectangle's width and its tile count.  The rectangle is
// gathered here, once per pair, so that the emit reads all of it coalesced.
struct PairRectOut {
  uint32_t* first;
  uint32_t* rec;
  uint32_t* width;
  uint32_t* count;
  const uint32_t* rect;
  int64_t nv_max, n_pidx;
  uint32_t n_tiles, tiles_x;
  __device__ void operator()(uint32_t pos, uint32_t, uint32_t r) const {
    r = (int64_t)r < nv_max ? r : 0u;   // in bounds even after a failed sort
    const uint2 q = *reinterpret_cast<const uint2*>(rect + 2 * (int64_t)r);
    const uint32_t x0 = q.x & 0xffff, y0 = q.x >> 16, x1 = q.y & 0xffff, y1 = q.y >> 16;
    const uint32_t c = (uint32_t)(r / (uint64_t)n_pidx);
    first[pos] = c * n_tiles + y0 * tiles_x + x0;
    rec[pos] = r;
    width[pos] = x1 - x0;
    count[pos] = (x1 - x0) * (y1 - y0);
  }
};

// Instances of the depth-ordered visible pairs, each pair's tiles in
// row-major order.  A wave64 workgroup takes 64 consecutive pairs at a time
// (grid-stride over the pair count read on the device) and walks their
// contiguous instance range [inst_off[s0], inst_off[s0 + 64])) 64 at a time
// (coalesced writes); a lane finds its pair by binary search over the 64
// offsets and its tile from the pair's first tile and width.  Balanced
// whatever the footprint sizes.  Instances at or past cap are not written
// (the call then reports the count it needs).  The grid also clears
// zero[0, n_zero) (the tile ranges, filled in later).
__global__ void __launch_bounds__(64) k_emit(const uint32_t* __restrict__ first, const uint32_t* __restrict__ width,
                                             const uint32_t* __restrict__ vis_rec,
                                             const uint32_t* __restrict__ inst_off, int64_t nv_max,
                                             const unsigned long long* __restrict__ d_nvis, int64_t cap, int32_t Tx,
                                             uint32_t* __restrict__ tkey, uint32_t* __restrict__ inst_rec,
                                             uint32_t* __restrict__ zero, int64_t n_zero) {
  const int lane = threadIdx.x;
  for (int64_t i = (int64_t)blockIdx.x * kWave + lane; i < n_zero; i += (int64_t)gridDim.x * kWave) zero[i] = 0u;
  const int64_t n_vis = dev_count(nv_max, d_nvis);
  __shared__ uint32_t s_off[kWave + 1];
  __shared__ uint32_t s_rec[kWave], s_first[kWave], s_w[kWave];
  for (int64_t s0 = (int64_t)blockIdx.x * kWave; s0 < n_vis; s0 += (int64_t)gridDim.x * kWave) {
    const int np = (int)(n_vis - s0 < kWave ? n_vis - s0 : kWave);
    if (lane <= np) s_off[lane] = inst_off[s0 + lane];
    if (lane == 0 && np == kWave) s_off[kWave] = inst_off[s0 + kWave];
    if (lane < np) {
      s_rec[lane] = vis_rec[s0 + lane];
      s_first[lane] = first[s0 + lane];
      s_w[lane] = width[s0 + lane];
    }
    __syncthreads();
    const uint32_t e0 = s_off[0];
    const uint32_t e1 = (int64_t)s_off[np] < cap ? s_off[np] : (uint32_t)cap;
    for (uint32_t e = e0 + (uint32_t)lane; e < e1; e += kWave) {
      int lo = 0, hi = np;   // s_off[lo] <= e < s_off[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_off[mid] <= e) lo = mid;
        else hi = mid;
      }
      const uint32_t k = e - s_off[lo], w = s_w[lo];
      // row = k / w: below 2^24 from the float reciprocal, corrected by one
      // step (the estimate is off by less than one: row < 2^16)
      uint32_t row;
      if (k < (1u << 24)) {
        row = (uint32_t)((float)k * __builtin_amdgcn_rcpf((float)w));
        row = row * w > k ? row - 1u : row;
        row = (row + 1u) * w <= k ? row + 1u : row;
      } else {
        row = k / w;
      }
      const uint32_t col = k - row * w;
      tkey[e] = s_first[lo] + row * (uint32_t)Tx + col;
      inst_rec[e] = s_rec[lo];
    }
    __syncthreads();
  }
}

// Per-tile [start, end) of the tile-sorted keys; the count is read on the
// device (grid-stride).  A thread takes four consecutive keys (one 16-byte
// load when kVec: the keys are 16-byte aligned) and compares each with its
// neighbours; ~0u stands in past either end (keys are below 2^31).
// After a failed depth sort (*err set) the ranges stay empty, so the
// compositing reads no entry.
template <bool kVec>
__global__ void k_ranges(const uint32_t* __restrict__ key, int64_t n_max, const unsigned long long* __restrict__ d_n,
                         uint32_t* __restrict__ ranges, const uint32_t* __restrict__ err) {
  if (*err) return;
  const int64_t n = dev_count(n_max, d_n);
  const int64_t stride = 4 * (int64_t)gridDim.x * blockDim.x;
  for (int64_t j0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x); j0 < n; j0 += stride) {
    uint32_t k[6];   // key[j0 - 1 .. j0 + 4]
    k[0] = j0 > 0 ? key[j0 - 1] : ~0u;
    if (kVec && j0 + 4 <= n) {
      const uint4 q = *reinterpret_cast<const uint4*>(key + j0);
      k[1] = q.x; k[2] = q.y; k[3] = q.z; k[4] = q.w;
    } else {
#pragma unroll
      for (int a = 0; a < 4; ++a) k[1 + a] = j0 + a < n ? key[j0 + a] : ~0u;
    }
    k[5] = j0 + 4 < n ? key[j0 + 4] : ~0u;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int64_t j = j0 + a;
      if (j < n) {
        if (k[a] != k[a + 1]) ranges[2 * (int64_t)k[a + 1]] = (uint32_t)j;
        if (k[a + 2] != k[a + 1]) ranges[2 * (int64_t)k[a + 1] + 1] = (uint32_t)(j + 1);
      }
    }
  }
}

// Launch order of the compositing kernels: tiles by descending list length
// (ties in tile order), so that the longest lists start first and the tail
// of the launch is made of short ones.  A tile's key is its list length on a
// log scale with 16 steps per octave (the leading bit's position and the
// next four bits of len + 1), longest first; lengths of 2^16 and more share
// the first bucket.
__device__ inline uint32_t tile_len_key(const uint32_t* __restrict__ ranges, int64_t g) {
  const uint32_t x = ranges[2 * g + 1] - ranges[2 * g] + 1u;
  const uint32_t e = 31u - (uint32_t)__clz(x);
  const uint32_t f = e >= 4u ? (x >> (e - 4u)) & 15u : (x << (4u - e)) & 15u;
  const uint32_t b = 16u * e + f;
  return 255u - (b < 255u ? b : 255u);
}

__global__ void k_tile_keys(const uint32_t* __restrict__ ranges, int64_t n, uint32_t* __restrict__ key) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) key[g] = tile_len_key(ranges, g);
}

// The tiles sorted by that key, stably, in two small launches over
// kOrderTiles-tile blocks (one thread per tile): k_order_hist counts each
// block's keys (hist[block 256 + key]); k_order_place adds up,
// per key, the counts of all blocks and of the blocks before its own, and
// places its tiles at that start plus their rank among the block's earlier
// tiles of the same key (earlier waves' counts, then ballot peer masks
// within the wave).  Used while nb <= kOrderMaxBlocks (every block reads
// all nb counts of each key); larger grids take the radix sort.
constexpr int kOrderTiles = 256;
constexpr int64_t kOrderMaxBlocks = 1024;

__device__ __forceinline__ uint64_t key_peers(uint32_t d, bool ok) {
  uint64_t peers = __ballot(ok);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t mk = __ballot(bit);
    peers &= bit ? mk : ~mk;
  }
  return peers;
}

// Per wave of the block: counts of each key among its 64 tiles, into
// cnt[wave][key] (zero on entry); returns the tile's key and peer mask.
__device__ __forceinline__ uint32_t order_count(const uint32_t* __restrict__ ranges, int64_t n,
                                                uint32_t (*cnt)[256], bool& ok, uint64_t& peers) {
  const int64_t g = (int64_t)blockIdx.x * kOrderTiles + threadIdx.x;
  ok = g < n;
  const uint32_t d = ok ? tile_len_key(ranges, g) : 0u;
  peers = key_peers(d, ok);
  if (ok && (peers & lanemask_lt()) == 0) cnt[threadIdx.x / kWave][d] = (uint32_t)__popcll(peers);
  return d;
}

__global__ void __launch_bounds__(kOrderTiles) k_order_hist(const uint32_t* __restrict__ ranges, int64_t n,
                                                            uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[kOrderTiles / kWave][256];
  for (int k = threadIdx.x; k < (kOrderTiles / kWave) * 256; k += kOrderTiles) (&cnt[0][0])[k] = 0;
  __syncthreads();
  bool ok;
  uint64_t peers;
  order_count(ranges, n, cnt, ok, peers);
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kOrderTiles / kWave; ++w) c += cnt[w][threadIdx.x];
  hist[(int64_t)blockIdx.x * 256 + threadIdx.x] = c;
}

__global__ void __launch_bounds__(kOrderTiles) k_order_place(const uint32_t* __restrict__ ranges, int64_t n,
                                                             const uint32_t* __restrict__ hist,
                                                             uint32_t* __restrict__ order) {
  __shared__ uint32_t cnt[kOrderTiles / kWave][256];
  __shared__ uint32_t start[256], wsum[kOrderTiles / kWave];
  for (int k = threadIdx.x; k < (kOrderTiles / kWave) * 256; k += kOrderTiles) (&cnt[0][0])[k] = 0;
  // key k = threadIdx.x: all blocks' count and the earlier blocks' count
  const int k = threadIdx.x, w = threadIdx.x / kWave, lane = __lane_id();
  uint32_t tot = 0, pre = 0;
  const uint32_t nbk = gridDim.x;
  uint32_t b = 0;
  for (; b + 8 <= nbk; b += 8) {   // eight coalesced rows in flight
    uint32_t c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = hist[(int64_t)(b + u) * 256 + k];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      tot += c[u];
      pre += b + u < blockIdx.x ? c[u] : 0u;
    }
  }
  for (; b < nbk; ++b) {
    const uint32_t c = hist[(int64_t)b * 256 + k];
    tot += c;
    pre += b < blockIdx.x ? c : 0u;
  }
  const uint32_t inc = wave_incl_scan(tot);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  uint32_t base = inc - tot + pre;
  for (int q = 0; q < w; ++q) base += wsum[q];
  start[k] = base;
  bool ok;
  uint64_t peers;
  const uint32_t d = order_count(ranges, n, cnt, ok, peers);
  __syncthreads();
  if (ok) {
    uint32_t pos = start[d] + (uint32_t)__popcll(peers & lanemask_lt());
    for (int q = 0; q < w; ++q) pos += cnt[q][d];
    order[pos] = (uint32_t)((int64_t)blockIdx.x * kOrderTiles + threadIdx.x);
  }
}

// The depth sort's tiles: kDepthWaves waves of kDepthRounds keys per lane.
// 4096-key tiles were faster than 2048 or 1024 (fewer look-back words to
// publish and read), and eight waves of eight rounds faster than four of
// sixteen (124 against 144 us for the four passes over 2.25 M keys: a
// tile's ranking is a chain of rounds), sixteen of four no faster.
constexpr int kDepthWaves = 8;
constexpr int kDepthRounds = 64 / kDepthWaves;

struct BinLayout {
  uint32_t *vis_off, *ka, *va, *kb, *vb, *inst_off, *tka, *tva, *tkb, *tvb, *inst_rec, *ranges, *order;
  uint32_t *oka, *ova, *okb, *ovb;   // launch-order radix sort (grids beyond kOrderMaxBlocks blocks)
  uint32_t* pwidth;                  // per visible pair in depth order, its rectangle's width
  uint32_t* ctl;                     // control words of the depth sort
  unsigned long long* status;        // its look-back words
  uint32_t* hist;                    // per-tile digit counts of the tile sort
  unsigned long long* tvis;          // per-tile visit counts of the compositing
  unsigned long long *partial, *totals;
  size_t bytes;
};

// Bits of the tile sort's key (camera-major tile id), at least one pass.
static int tile_key_bits(int n_cams, int64_t n_tiles) {
  int bits = 0;
  while ((1ll << bits) < (int64_t)n_cams * n_tiles) ++bits;
  return bits < 8 ? 8 : bits;
}

static BinLayout bin_layout(void* ws, int n_cams, int64_t n_pidx, int64_t n_tiles, int64_t cap) {
  const int64_t nv = (int64_t)n_cams * n_pidx;
  Carver cv(ws);
  BinLayout L;
  L.vis_off = cv.take<uint32_t>(nv);
  L.ka = cv.take<uint32_t>(nv);
  L.va = cv.take<uint32_t>(nv);
  L.kb = cv.take<uint32_t>(nv);
  L.vb = cv.take<uint32_t>(nv);
  L.inst_off = cv.take<uint32_t>(nv + 1);
  L.pwidth = cv.take<uint32_t>(nv);
  L.tka = cv.take<uint32_t>(cap);
  L.tva = cv.take<uint32_t>(cap);
  L.tkb = cv.take<uint32_t>(cap);
  L.tvb = cv.take<uint32_t>(cap);
  L.inst_rec = cv.take<uint32_t>(cap);
  const int64_t ntt = (int64_t)n_cams * n_tiles;
  L.ranges = cv.take<uint32_t>(2 * (size_t)ntt);
  L.order = cv.take<uint32_t>(ntt);
  L.tvis = cv.take<unsigned long long>(2 * ntt);
  L.ctl = cv.take<uint32_t>(kOsCtlLen);
  L.status = cv.take<unsigned long long>(onesweep_status_count(nv, 4, (int64_t)kWave * kDepthWaves * kDepthRounds));
  const int64_t nob = ceil_div(ntt, kOrderTiles);
  const bool order_radix = nob > kOrderMaxBlocks;
  L.oka = cv.take<uint32_t>(order_radix ? ntt : 0);
  L.ova = cv.take<uint32_t>(order_radix ? ntt : 0);
  L.okb = cv.take<uint32_t>(order_radix ? ntt : 0);
  L.ovb = cv.take<uint32_t>(order_radix ? ntt : 0);
  size_t nh = radix_hist_count(cap);
  const size_t nho = order_radix ? radix_hist_count(ntt) : 256 * (size_t)nob;
  nh = nh > nho ? nh : nho;
  L.hist = cv.take<uint32_t>(nh);
  L.partial = cv.take<unsigned long long>(scan_partial_count(nv > (int64_t)nh ? nv : (int64_t)nh));
  L.totals = cv.take<unsigned long long>(6);   // n_vis, -, n_inst, error word, tile sort's scan total and length
  L.bytes = cv.used;
  return L;
}

// ------------------------------------------------------------- compositing
// One wave64 per 16x16 tile; lane l owns the four pixels of column l % 16,
// rows l / 16 + {0, 4, 8, 12}.  The tile's list is streamed through LDS in
// batches of 64 records and read back as broadcasts.  The per-pixel update is
// branch-free (selects on the skip / stop / contribute predicates), and the
// terms that depend only on the lane's column are formed once per entry and
// shared by its four pixels.
template <typename T>
__global__ void __launch_bounds__(64) k_render_fwd(const uint32_t* __restrict__ order,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ inst_e,
                                                   const uint32_t* __restrict__ inst_rec, const T* __restrict__ rec,
                                                   int32_t Tx, int32_t Ty, int32_t W, int32_t H, T bg0, T bg1,
                                                   T bg2, T* __restrict__ image, T* __restrict__ tfin,
                                                   uint32_t* __restrict__ last_out,
                                                   unsigned long long* __restrict__ tile_visits) {
  const int nt = Tx * Ty;
  const int g = (int)order[blockIdx.x];
  const int c = g / nt, t = g - c * nt;
  const int tx = t % Tx, ty = t / Tx;
  const int lane = threadIdx.x;
  const int px = tx * kTile + (lane & 15);
  const int py0 = ty * kTile + (lane >> 4);
  const T fxp = (T)px + (T)0.5;
  // A pixel that stops (or lies outside the image) moves its row to
  // +infinity, where no entry reaches it, so the per-entry work needs no
  // liveness test; Tr then keeps its final T.
  const T kGone = __builtin_inf();
  T fyp[4], Tr[4], C0[4], C1[4], C2[4];
  uint32_t lst[4];
  // live pixels of the wave; every entry reached counts them as visits
  uint32_t nlive = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const bool in = px < W && py0 + 4 * q < H;
    fyp[q] = in ? (T)(py0 + 4 * q) + (T)0.5 : kGone;
    Tr[q] = 1;
    C0[q] = C1[q] = C2[q] = 0;
    lst[q] = 0;
    nlive += (uint32_t)__popcll(__ballot(in));
  }
  unsigned long long nvis = 0;   // wave-uniform: live pixels summed over entries
  const uint32_t start = ranges[2 * g], end = ranges[2 * g + 1];
  __shared__ T s_u[64], s_v[64], s_A[64], s_B[64], s_C[64], s_o[64], s_r[64], s_g[64], s_b[64];
  const T ks = (T)Ex<T>::k;
  bool any = nlive != 0;
  for (uint32_t b0 = start; b0 < end && any; b0 += 64) {
    const uint32_t j = b0 + lane;
    bool may = false;
    if (j < end) {
      const T* q = rec + (int64_t)inst_rec[inst_e[j]] * kRec;
      s_u[lane] = q[0]; s_v[lane] = q[1];
      s_A[lane] = (T)-0.5 * ks * q[2]; s_B[lane] = -ks * q[3]; s_C[lane] = (T)-0.5 * ks * q[4];
      s_o[lane] = q[5]; s_r[lane] = q[6]; s_g[lane] = q[7]; s_b[lane] = q[8];
      // entries whose footprint misses every pixel centre of the tile at
      // alpha >= 1/255 (about 40 % of the aerial scene's instances) are
      // passed over without any per-pixel work
      may = tile_may_take<T>(q[0], q[1], q[2], q[3], q[4], q[5], tx, ty);
    }
    // the batch's entries that some pixel centre may take, one bit each: the
    // walk below visits only those, and the others cost nothing
    uint64_t rest = __ballot(may);
    __syncthreads();
    const int nb = (int)(end - b0 < 64 ? end - b0 : 64);
    int counted = 0;   // entries of the batch whose visits are in nvis
    while (rest != 0) {
      const int k = __builtin_ctzll(rest);
      rest &= rest - 1;
      // every live pixel visits entries counted..k
      nvis += (unsigned long long)nlive * (unsigned long long)(k + 1 - counted);
      counted = k + 1;
      const T v = s_v[k], Ch = s_C[k], op = s_o[k];
      const T cr = s_r[k], cg = s_g[k], cb = s_b[k];
      const T dx = fxp - s_u[k];
      const T adx2 = s_A[k] * dx * dx, bdx = s_B[k] * dx;
      const uint32_t idx = b0 - start + (uint32_t)k + 1;
      // Alphas first: when no pixel takes the entry (the tile test is
      // conservative, and pixels stop), the update below would change
      // nothing, and the wave skips it.  Each comparison is balloted on its
      // own and the masks are combined on the scalar unit (a ballot of a
      // combined condition costs two vector instructions).
      T al[4];
      bool ps[4];
      uint64_t pm[4], take_m = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T G, araw;
        bool in_power, in_alpha;
        entry_alpha_tests<T>(adx2, bdx, Ch, op, fyp[q] - v, G, araw, al[q], in_power, in_alpha);
        ps[q] = in_power && in_alpha;
        pm[q] = __ballot(in_power) & __ballot(in_alpha);
        take_m |= pm[q];
      }
      if (take_m == 0) continue;
      uint32_t nstop = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (pm[q] == 0) continue;   // no pixel of row group q takes the entry: nothing changes
        const T alpha = al[q];
        const bool pass = ps[q];
        const T wr = alpha * Tr[q];
        const T tn = Tr[q] - wr;   // T (1 - alpha)
        const bool low = tn < (T)1e-4;
        const bool stop = pass && low;
        const bool take = pass && !low;
        const T w = take ? wr : (T)0;
        C0[q] += cr * w; C1[q] += cg * w; C2[q] += cb * w;
        Tr[q] = take ? tn : Tr[q];
        fyp[q] = stop ? kGone : fyp[q];
        lst[q] = take ? idx : lst[q];
        nstop += (uint32_t)__popcll(pm[q] & __ballot(low));
      }
      nlive -= nstop;
      if (nlive == 0) { any = false; break; }
    }
    nvis += (unsigned long long)nlive * (unsigned long long)(nb - counted);
    __syncthreads();
  }
  const int64_t HW = (int64_t)H * W;
  unsigned long long nback = 0;   // entries the backward walks for this lane's pixels
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int py = py0 + 4 * q;
    if (px < W && py < H) {
      const int64_t p = (int64_t)py * W + px;
      nback += lst[q];
      const T tf = Tr[q];
      image[((int64_t)c * 3 + 0) * HW + p] = C0[q] + tf * bg0;
      image[((int64_t)c * 3 + 1) * HW + p] = C1[q] + tf * bg1;
      image[((int64_t)c * 3 + 2) * HW + p] = C2[q] + tf * bg2;
      tfin[(int64_t)c * HW + p] = tf;
      last_out[(int64_t)c * HW + p] = lst[q];
    }
  }
  // per-tile counts, summed per view by k_sum_visits (no same-address
  // atomics: those cross the XCDs' separate L2s)
  nback = wave_sum(nback);
  if (lane == 0) {
    tile_visits[g] = nvis;
    tile_visits[gridDim.x + g] = nback;
  }
}

// visits[r][c] += sum over camera c's tiles of tile_visits[r][c * nt + t]:
// kVisitParts workgroups per (row, camera), each adding its share of the
// tiles with one 64-bit atomic (integer sums: exact in any order).
constexpr int kVisitParts = 16;
__global__ void __launch_bounds__(256) k_sum_visits(const unsigned long long* __restrict__ tile_visits,
                                                    int64_t nt, int32_t n_cams,
                                                    unsigned long long* __restrict__ visits) {
  const int rc = blockIdx.x / kVisitParts, part = blockIdx.x % kVisitParts;   // rc = r * n_cams + c
  const unsigned long long* p = tile_visits + (int64_t)rc * nt;
  unsigned long long s = 0;
  for (int64_t t = (int64_t)part * 256 + threadIdx.x; t < nt; t += 256 * kVisitParts) s += p[t];
  s = wave_sum(s);
  __shared__ unsigned long long ws[4];
  if (__lane_id() == 0) ws[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&visits[rc], ws[0] + ws[1] + ws[2] + ws[3]);
}

}  // namespace tide

using namespace tide;

// ------------------------------------------------- preprocess without allocation
// Device scratch of tide_preprocess_noalloc: the active scan's per-block sums
// (one u64 per 4096 pidx) and its total.  One copy per GPU, held until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (kept in g_noalloc_ptr).
constexpr size_t kNoallocScratchBytes = 256 * 1024;
static_assert(kNoallocScratchBytes == (size_t)TIDE_PREPROCESS_NOALLOC_SCRATCH, "header and scratch size differ");
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[64];

// Address of the current device's scratch, looked up once per device.
static tide_status noalloc_scratch(void** out) {
  int dev = 0;
  TIDE_HIP(hipGetDevice(&dev));
  TIDE_CHECK_ARG(dev >= 0 && dev < 64, "device ordinal %d beyond the 64 this library tracks", dev);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    TIDE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    TIDE_CHECK_ARG(p != nullptr, "hipGetSymbolAddress gave a null scratch address");
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return TIDE_OK;
}

extern "C" size_t tide_preprocess_ws_bytes(int64_t n_pidx) { return preprocess_ws_bytes(n_pidx); }

extern "C" tide_status tide_preprocess(const tide_pool* pool, const tide_camera* cams, int32_t n_cams,
                                       tide_proj* out, void* ws, size_t ws_bytes, void* stream) {
  tide_status s;
  if ((s = check_pool(pool)) != TIDE_OK) return s;
  if ((s = check_cams(cams, n_cams)) != TIDE_OK) return s;
  if ((s = check_proj(out)) != TIDE_OK) return s;
  TIDE_CHECK_ARG(out->n_cams == n_cams, "proj.n_cams (%d) != n_cams (%d)", out->n_cams, n_cams);
  TIDE_CHECK_ARG(out->dtype == pool->dtype, "proj and pool dtypes differ");
  TIDE_CHECK_ARG(out->n_pidx == (int64_t)pool->n_order * pool->block_rows, "proj.n_pidx must be n_order * block_rows");
  TIDE_CHECK_ARG(ws && ws_bytes >= preprocess_ws_bytes(out->n_pidx), "workspace too small (%zu < %zu)", ws_bytes,
                 preprocess_ws_bytes(out->n_pidx));
  hipStream_t st = (hipStream_t)stream;
  return pool->dtype == TIDE_F32 ? preprocess_t<float>(pool, cams, n_cams, out, ws, st)
                                 : preprocess_t<double>(pool, cams, n_cams, out, ws, st);
}

extern "C" tide_status tide_preprocess_noalloc(const tide_pool* pool, const tide_camera* cams, int32_t n_cams,
                                               tide_proj* out, void* stream) {
  tide_status s;
  if ((s = check_pool(pool)) != TIDE_OK) return s;
  if ((s = check_cams(cams, n_cams)) != TIDE_OK) return s;
  if ((s = check_proj(out)) != TIDE_OK) return s;
  TIDE_CHECK_ARG(out->n_cams == n_cams, "proj.n_cams (%d) != n_cams (%d)", out->n_cams, n_cams);
  TIDE_CHECK_ARG(out->dtype == pool->dtype, "proj and pool dtypes differ");
  TIDE_CHECK_ARG(out->n_pidx == (int64_t)pool->n_order * pool->block_rows, "proj.n_pidx must be n_order * block_rows");
  if (out->n_pidx > (int64_t)TIDE_PREPROCESS_NOALLOC_MAX_PIDX) {
    set_error("tide_preprocess_noalloc: n_pidx %lld exceeds the maximum %lld of its %zu-byte static scratch "
              "(use tide_preprocess with a workspace)",
              (long long)out->n_pidx, (long long)TIDE_PREPROCESS_NOALLOC_MAX_PIDX, kNoallocScratchBytes);
    return TIDE_ECAPACITY;
  }
  if (preprocess_ws_bytes(out->n_pidx) > kNoallocScratchBytes) {  // guards the constant above
    set_error("tide_preprocess_noalloc: scratch of %zu bytes is short of %zu", kNoallocScratchBytes,
              preprocess_ws_bytes(out->n_pidx));
    return TIDE_ECAPACITY;
  }
  void* ws = nullptr;
  if ((s = noalloc_scratch(&ws)) != TIDE_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  return pool->dtype == TIDE_F32 ? preprocess_t<float>(pool, cams, n_cams, out, ws, st)
                                 : preprocess_t<double>(pool, cams, n_cams, out, ws, st);
}

// Pinned host slot for the binning's counts and the event that marks their
// arrival, one per device; calls on one device take turns on it.  Allocated
// on first use and kept for the life of the process.
struct CountSlot {
  std::mutex mu;
  unsigned long long* host = nullptr;
  hipEvent_t ev = nullptr;
};

static CountSlot& count_slot() {
  static CountSlot slots[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  return slots[dev];
}

extern "C" size_t tide_bin_sort_ws_bytes(int32_t n_cams, int64_t n_pidx, int32_t tiles_x, int32_t tiles_y,
                                         int64_t n_inst_cap) {
  return bin_layout(nullptr, n_cams, n_pidx, (int64_t)tiles_x * tiles_y, n_inst_cap).bytes;
}

extern "C" tide_status tide_bin_sort(const tide_proj* proj, int32_t tiles_x, int32_t tiles_y, void* ws,
                                     size_t ws_bytes, tide_bins* out, void* stream) {
  tide_status s;
  if ((s = check_proj(proj)) != TIDE_OK) return s;
  TIDE_CHECK_ARG(out, "bins is null");
  TIDE_CHECK_ARG(tiles_x > 0 && tiles_y > 0 && tiles_x < 65536 && tiles_y < 65536, "bad tile grid");
  const int V = proj->n_cams;
  const int64_t N = proj->n_pidx, nv = (int64_t)V * N, nt = (int64_t)tiles_x * tiles_y;
  TIDE_CHECK_ARG((int64_t)V * nt < (1ll << 31), "too many tiles");
  hipStream_t st = (hipStream_t)stream;
  out->ws_required = 0;
  // capacity this workspace gives for instances
  const size_t fixed = bin_layout(nullptr, V, N, nt, 0).bytes;
  TIDE_CHECK_ARG(ws, "workspace is null");
  if (ws_bytes < fixed + 4096) {
    out->ws_required = tide_bin_sort_ws_bytes(V, N, tiles_x, tiles_y, nv * 4 + 1024);
    set_error("bin_sort workspace too small (%zu bytes; need at least %zu)", ws_bytes, out->ws_required);
    return TIDE_ECAPACITY;
  }
  int64_t cap = (int64_t)((ws_bytes - fixed) / (6 * sizeof(uint32_t))) - 1024;
  while (cap > 0 && bin_layout(nullptr, V, N, nt, cap).bytes > ws_bytes) cap -= (cap / 64 + 256);
  if (cap < 0) cap = 0;
  BinLayout L = bin_layout(ws, V, N, nt, cap);

  // 1. visible pairs, compacted in (camera, pidx) order, keyed by depth
  //    bits: the blocks' counts, then the down-sweep that writes each
  //    block's pairs through LDS (and clears the depth sort's control words
  //    and the error word)
  {
    const int64_t nbv = ceil_div(nv > 0 ? nv : 1, kScanTile);
    const bool vec = aligned16(proj->tiles_touched) && aligned16(proj->depth);
    if (vec)
      hipLaunchKernelGGL((k_scan_reduce<NonzeroIn, true>), dim3((uint32_t)nbv), dim3(kScanThreads), 0, st,
                         NonzeroIn{proj->tiles_touched}, nv, nullptr, L.partial);
    else
      hipLaunchKernelGGL((k_scan_reduce<NonzeroIn, false>), dim3((uint32_t)nbv), dim3(kScanThreads), 0, st,
                         NonzeroIn{proj->tiles_touched}, nv, nullptr, L.partial);
    if (nbv <= 1024) {
      TIDE_TIMED("compact_vis", st, hipLaunchKernelGGL(k_vis_compact<true>, dim3((uint32_t)nbv), dim3(kScanThreads), 0,
                                                       st, proj->tiles_touched, proj->depth, nv, L.partial, nbv,
                                                       &L.totals[0], L.ka, L.va, L.ctl, (int64_t)kOsCtlLen,
                                                       &L.totals[3], vec ? 1 : 0));
    } else {
      hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, L.partial, nbv, &L.totals[0], ScanTail{}, nv,
                         nullptr);
      TIDE_TIMED("compact_vis", st, hipLaunchKernelGGL(k_vis_compact<false>, dim3((uint32_t)nbv), dim3(kScanThreads),
                                                       0, st, proj->tiles_touched, proj->depth, nv, L.partial, nbv,
                                                       &L.totals[0], L.ka, L.va, L.ctl, (int64_t)kOsCtlLen,
                                                       &L.totals[3], vec ? 1 : 0));
    }
  }
  TIDE_LAUNCH_CHECK("visibility compaction");
  uint32_t* err = reinterpret_cast<uint32_t*>(&L.totals[3]);
  // 2. stable sort of the visible pairs by depth; grids are sized by the
  //    upper bound and the kernels read the visible count from the device;
  //    the last pass writes, per pair in depth order, its first tile's key
  //    (over the keys, not needed after the sort), its record index, its
  //    rectangle's width and its tile count (into vis_off, free once the
  //    compaction has run)
  uint32_t *pfirst, *vrec;
  onesweep_sort_pairs<kDepthRounds, kDepthWaves>(
      L.ka, L.va, L.kb, L.vb, nv, 32, false, OsWork{L.ctl, L.status, err}, st, &pfirst, &vrec, &L.totals[0],
      PairRectOut{L.ka, L.va, L.pwidth, L.vis_off, proj->rect, nv, N, (uint32_t)nt, (uint32_t)tiles_x});
  TIDE_LAUNCH_CHECK("depth sort");
  // 3. instance offsets in depth order, closed by inst_off[n_vis] = n_inst;
  //    the block that holds the total also copies the counts and the depth
  //    sort's error word into the pinned host slot, whose event the host
  //    waits on after queueing the rest of the binning (those kernels are
  //    sized by the instance capacity and read the counts on the device, so
  //    the GPU does not wait for the host)
  CountSlot& slot = count_slot();
  std::lock_guard<std::mutex> lk(slot.mu);
  if (!slot.host) {
    TIDE_HIP(hipHostMalloc((void**)&slot.host, 4 * sizeof(unsigned long long), hipHostMallocDefault));
    TIDE_HIP(hipEventCreateWithFlags(&slot.ev, hipEventDisableTiming));
  }
  {
    ScanTail tail;
    tail.end = L.inst_off;
    tail.copy_src = L.totals;
    tail.copy_dst = slot.host;
    tail.copy_n = 4;
    scan_exclusive(ArrayIn{L.vis_off}, nv, L.inst_off, L.partial, &L.totals[2], st, &L.totals[0], tail);
  }
  TIDE_LAUNCH_CHECK("instance scan");
  TIDE_HIP(hipEventRecord(slot.ev, st));
  // 5. emit instances in depth order, keyed by global tile id (and clear
  //    the tile ranges)
  const int64_t nr = 2 * (int64_t)V * nt;
  {
    const int64_t chunks = ceil_div(nv > 0 ? nv : 1, kWave);
    TIDE_TIMED("emit", st, hipLaunchKernelGGL(k_emit, dim3((uint32_t)(chunks < 32768 ? chunks : 32768)), dim3(kWave), 0,
                                              st, pfirst, L.pwidth, vrec, L.inst_off, nv, &L.totals[0], cap, tiles_x,
                                              L.tka, L.inst_rec, L.ranges, nr));
  }
  TIDE_LAUNCH_CHECK("k_emit");
  // 6. stable sort by tile; values are emission indices (histogram, scan
  //    and scatter per pass: with this many keys the look-back would cost
  //    more than the launches it saves)
  const int bits = tile_key_bits(V, nt);
  uint32_t *tk, *te;
  radix_sort_pairs(L.tka, L.tva, L.tkb, L.tvb, cap, bits, true, L.hist, L.partial, &L.totals[4], st, &tk, &te,
                   &L.totals[2], nullptr, nullptr, /*xcd_order=*/true);
  TIDE_LAUNCH_CHECK("tile sort");
  // 7. per-tile ranges (left empty if the depth sort gave up)
  if (cap > 0) {
    const int64_t nb = ceil_div(ceil_div(cap, 4), 256);
    const dim3 grid((uint32_t)(nb < 65536 ? nb : 65536));
    if (((uintptr_t)tk & 15) == 0)
      hipLaunchKernelGGL(k_ranges<true>, grid, dim3(256), 0, st, tk, cap, &L.totals[2], L.ranges, err);
    else
      hipLaunchKernelGGL(k_ranges<false>, grid, dim3(256), 0, st, tk, cap, &L.totals[2], L.ranges, err);
  }
  TIDE_LAUNCH_CHECK("k_ranges");
  // 8. launch order of the tiles: longest lists first
  const int64_t ntt = (int64_t)V * nt;
  const int64_t nob = ceil_div(ntt, kOrderTiles);
  if (nob <= kOrderMaxBlocks) {
    hipLaunchKernelGGL(k_order_hist, dim3((uint32_t)nob), dim3(kOrderTiles), 0, st, L.ranges, ntt, L.hist);
    hipLaunchKernelGGL(k_order_place, dim3((uint32_t)nob), dim3(kOrderTiles), 0, st, L.ranges, ntt, L.hist, L.order);
  } else {
    hipLaunchKernelGGL(k_tile_keys, dim3((uint32_t)ceil_div(ntt, 256)), dim3(256), 0, st, L.ranges, ntt, L.oka);
    uint32_t *ok, *ord;
    radix_sort_pairs(L.oka, L.ova, L.okb, L.ovb, ntt, 8, true, L.hist, L.partial, &L.totals[1], st, &ok, &ord);
    TIDE_HIP(hipMemcpyAsync(L.order, ord, ntt * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
  }
  TIDE_LAUNCH_CHECK("tile launch order");
  // 9. the counts, once they are on the host; a depth sort whose look-back
  //    gave up is an error (its lists are invalid and its ranges empty)
  TIDE_HIP(hipEventSynchronize(slot.ev));
  const int64_t n_vis = (int64_t)slot.host[0];
  const int64_t n_inst = (int64_t)slot.host[2];
  out->n_vis = n_vis;
  out->n_inst = n_inst;
  if (slot.host[3]) {
    set_error("binning: the depth sort's look-back exceeded its spin limit; the lists of this call are invalid");
    return TIDE_EHIP;
  }
  if (n_inst >= (int64_t)UINT32_MAX) {
    set_error("instance count %lld exceeds 32-bit indexing", (long long)n_inst);
    return TIDE_EINVAL;
  }
  if (n_inst > cap) {
    out->ws_required = tide_bin_sort_ws_bytes(V, N, tiles_x, tiles_y, n_inst + n_inst / 8 + 1024);
    set_error("bin_sort needs %lld instances, workspace holds %lld", (long long)n_inst, (long long)cap);
    return TIDE_ECAPACITY;
  }
  uint32_t* order = L.order;
  out->tile_order = order;
  out->tile_visits = L.tvis;
  out->vis_rec = vrec;
  out->inst_off = L.inst_off;
  out->inst_e = te;
  out->inst_rec = L.inst_rec;
  out->ranges = L.ranges;
  out->n_cams = V;
  out->tiles_x = tiles_x;
  out->tiles_y = tiles_y;
  out->n_pidx = N;
  return TIDE_OK;
}

extern "C" tide_status tide_render_fwd(const tide_proj* proj, const tide_bins* bins, const float* bg,
                                       tide_frame* fr, void* stream) {
  tide_status s;
  if ((s = check_proj(proj)) != TIDE_OK) return s;
  TIDE_CHECK_ARG(bins && fr && bg && bins->tile_visits, "null argument");
  TIDE_CHECK_ARG(fr->image && fr->t_final && fr->last && fr->visits, "frame has a null pointer");
  TIDE_CHECK_ARG(bins->n_cams == proj->n_cams && bins->n_pidx == proj->n_pidx, "bins do not match proj");
  TIDE_CHECK_ARG(fr->width > 0 && fr->height > 0 && (fr->width + kTile - 1) / kTile == bins->tiles_x &&
                     (fr->height + kTile - 1) / kTile == bins->tiles_y,
                 "frame size does not match the tile grid");
  hipStream_t st = (hipStream_t)stream;
  const uint32_t grid = (uint32_t)(bins->n_cams * bins->tiles_x * bins->tiles_y);
  if (proj->dtype == TIDE_F32)
    TIDE_TIMED("render_fwd", st, hipLaunchKernelGGL(k_render_fwd<float>, dim3(grid), dim3(64), 0, st, bins->tile_order, bins->ranges, bins->inst_e, bins->inst_rec,
                       (const float*)proj->rec, bins->tiles_x, bins->tiles_y, fr->width, fr->height, bg[0], bg[1],
                       bg[2], (float*)fr->image, (float*)fr->t_final, fr->last, bins->tile_visits));
  else
    TIDE_TIMED("render_fwd", st, hipLaunchKernelGGL(k_render_fwd<double>, dim3(grid), dim3(64), 0, st, bins->tile_order, bins->ranges, bins->inst_e,
                       bins->inst_rec, (const double*)proj->rec, bins->tiles_x, bins->tiles_y, fr->width,
                       fr->height, (double)bg[0], (double)bg[1], (double)bg[2], (double*)fr->image,
                       (double*)fr->t_final, fr->last, bins->tile_visits));
  TIDE_LAUNCH_CHECK("k_render_fwd");
  hipLaunchKernelGGL(k_sum_visits, dim3((uint32_t)(2 * bins->n_cams * kVisitParts)), dim3(256), 0, st, bins->tile_visits,
                     (int64_t)bins->tiles_x * bins->tiles_y, bins->n_cams, fr->visits);
  TIDE_LAUNCH_CHECK("k_sum_visits");
  return TIDE_OK;
}
