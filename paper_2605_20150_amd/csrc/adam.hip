// Fused masked Adam over the active rows of the resident pool, with the
// dirty-block mark and the conservative bounding-sphere refresh.
#include "raster.h"

namespace tide {

template <typename T>
struct AdamK {
  T lr[kD];
  T b1, b2, eps, kappa;
};

// Thread per processing index; inactive rows return at once and stay
// bit-identical.  For each of the 59 columns the lanes (consecutive rows)
// touch consecutive addresses of p, m, v and of the compact gradient.
template <typename T>
__global__ void __launch_bounds__(256) k_adam(T* __restrict__ params, T* __restrict__ m1, T* __restrict__ m2,
                                              uint32_t* __restrict__ step, const int32_t* __restrict__ order,
                                              const int32_t* __restrict__ slot_block, int32_t B, int64_t n_pidx,
                                              const uint32_t* __restrict__ active,
                                              const uint32_t* __restrict__ act_idx, const T* __restrict__ grad,
                                              int64_t ld, AdamK<T> K, float* __restrict__ spheres,
                                              uint8_t* __restrict__ dirty) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = i < n_pidx && active[i] != 0u;
  int32_t blk = -1;
  float reach = 0.f;
  if (act) {
    const int64_t k = i / B;
    const int32_t row = (int32_t)(i - k * B);
    const int32_t slot = order[k];
    blk = slot_block[slot];
    const int64_t base = (int64_t)slot * kD * B + row;
    const int64_t a = act_idx[i];
    const uint32_t t = step[(int64_t)slot * B + row] + 1u;
    step[(int64_t)slot * B + row] = t;
    const T bc1 = (T)1 - pow(K.b1, (T)t);
    const T bc2 = (T)1 - pow(K.b2, (T)t);
    const T ibc1 = (T)1 / bc1, isb2 = (T)1 / Mth<T>::sqrt(bc2);
    T pcol[6];
#pragma unroll 4
    for (int j = 0; j < kD; ++j) {
      const int64_t o = base + (int64_t)j * B;
      const T gj = grad[a + (int64_t)j * ld];
      const T m = K.b1 * m1[o] + ((T)1 - K.b1) * gj;
      const T v = K.b2 * m2[o] + ((T)1 - K.b2) * gj * gj;
      m1[o] = m;
      m2[o] = v;
      const T p = params[o] - K.lr[j] * (m * ibc1) / (Mth<T>::sqrt(v) * isb2 + K.eps);
      params[o] = p;
      if (j < 6) pcol[j] = p;
    }
    if (spheres) {
      const float* S = spheres + 4 * (int64_t)blk;
      const float dx = (float)pcol[0] - S[0], dy = (float)pcol[1] - S[1], dz = (float)pcol[2] - S[2];
      T ls = pcol[3] > pcol[4] ? pcol[3] : pcol[4];
      ls = ls > pcol[5] ? ls : pcol[5];
      reach = sqrtf(dx * dx + dy * dy + dz * dz) + 3.f * (float)K.kappa * expf((float)ls);
    }
  }
  if (!spheres && !dirty) return;
  // lanes of one wave usually share a block: reduce first, then one update
  const int32_t b0 = __shfl(blk, 0, kWave);
  const bool uniform = __ballot(blk != b0) == 0ull;
  if (uniform) {
    if (b0 < 0) return;
    float r = reach;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) r = fmaxf(r, __shfl_xor(r, off, kWave));
    if (__lane_id() == 0) {
      if (dirty) dirty[b0] = 1;
      if (spheres) atomicMax(reinterpret_cast<unsigned int*>(spheres + 4 * (int64_t)b0 + 3), __float_as_uint(r));
    }
  } else if (blk >= 0) {
    if (dirty) dirty[blk] = 1;
    if (spheres) atomicMax(reinterpret_cast<unsigned int*>(spheres + 4 * (int64_t)blk + 3), __float_as_uint(reach));
  }
}

}  // namespace tide

using namespace tide;

extern "C" tide_status tide_adam_sparse(tide_pool* pool, const tide_proj* proj, const void* grad, int64_t grad_ld,
                                        const tide_adam_cfg* cfg, float* spheres, uint8_t* dirty, int64_t n_blocks,
                                        void* stream) {
  TIDE_CHECK_ARG(pool && proj && grad && cfg, "null argument");
  TIDE_CHECK_ARG(pool->params && pool->exp_avg && pool->exp_avg_sq && pool->step && pool->order && pool->slot_block,
                 "pool has a null pointer");
  TIDE_CHECK_ARG(proj->dtype == pool->dtype, "dtype mismatch");
  TIDE_CHECK_ARG(proj->n_pidx == (int64_t)pool->n_order * pool->block_rows, "proj does not match pool");
  TIDE_CHECK_ARG(grad_ld >= proj->n_pidx, "grad_ld too small");
  TIDE_CHECK_ARG(cfg->beta1 >= 0 && cfg->beta1 < 1 && cfg->beta2 >= 0 && cfg->beta2 < 1 && cfg->eps >= 0,
                 "bad Adam constants");
  TIDE_CHECK_ARG((!spheres && !dirty) || n_blocks > 0, "n_blocks must be given with spheres/dirty");
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = proj->n_pidx;
  if (n == 0) return TIDE_OK;
  const dim3 grid((uint32_t)ceil_div(n, 256));
  if (pool->dtype == TIDE_F32) {
    AdamK<float> K;
    for (int j = 0; j < kD; ++j) K.lr[j] = cfg->lr[j];
    K.b1 = cfg->beta1; K.b2 = cfg->beta2; K.eps = cfg->eps; K.kappa = cfg->kappa;
    TIDE_TIMED("adam", st, hipLaunchKernelGGL(k_adam<float>, grid, dim3(256), 0, st, (float*)pool->params, (float*)pool->exp_avg,
                       (float*)pool->exp_avg_sq, pool->step, pool->order, pool->slot_block, pool->block_rows, n,
                       proj->active, proj->act_idx, (const float*)grad, grad_ld, K, spheres, dirty));
  } else {
    AdamK<double> K;
    for (int j = 0; j < kD; ++j) K.lr[j] = cfg->lr[j];
    K.b1 = cfg->beta1; K.b2 = cfg->beta2; K.eps = cfg->eps; K.kappa = cfg->kappa;
    TIDE_TIMED("adam", st, hipLaunchKernelGGL(k_adam<double>, grid, dim3(256), 0, st, (double*)pool->params, (double*)pool->exp_avg,
                       (double*)pool->exp_avg_sq, pool->step, pool->order, pool->slot_block, pool->block_rows, n,
                       proj->active, proj->act_idx, (const double*)grad, grad_ld, K, spheres, dirty));
  }
  TIDE_LAUNCH_CHECK("k_adam");
  return TIDE_OK;
}
