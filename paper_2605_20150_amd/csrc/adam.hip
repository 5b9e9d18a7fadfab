// Fused masked Adam over the active rows of the resident pool, with the
// dirty-block mark and the conservative bounding-sphere refresh.
#include <cmath>

#include "raster.h"

namespace tide {

// Passes over the active rows; inactive rows are never written, so they
// stay bit-identical.
//  1. Per row, step += 1 and the bias corrections 1/(1 - b1^t),
//     1/sqrt(1 - b2^t), evaluated in double precision: inside k_adam_sweep,
//     rounded to single precision for its update; k_adam_rows into a row
//     table of doubles for the double-precision update.
//  2. k_adam_sweep (single precision): one thread per row over its 59
//     columns; k_adam_cols (double precision): a 2-D grid (rows x 59
//     columns), one element per thread.
//  3. k_adam_bounds: per updated row, the dirty mark and the conservative
//     bounding-sphere refresh r_k = max(r_k, |mu - c_k| + 3 kappa max scale).
__global__ void __launch_bounds__(256) k_adam_rows(uint32_t* __restrict__ step, const int32_t* __restrict__ order,
                                                   int32_t B, int64_t n_pidx, const uint32_t* __restrict__ active,
                                                   double lb1, double lb2, double2* __restrict__ bias) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pidx || !active[i]) return;
  const int64_t k = i / B;
  const int32_t row = (int32_t)(i - k * B);
  double bcx, bcy;
  adam_step_bias<double>(step + (int64_t)order[k] * B + row, lb1, lb2, bcx, bcy);
  bias[i] = make_double2(bcx, bcy);
}

template <typename T>
__global__ void __launch_bounds__(256) k_adam_cols(T* __restrict__ params, T* __restrict__ m1, T* __restrict__ m2,
                                                   const int32_t* __restrict__ order, int32_t B, int64_t n_pidx,
                                                   const uint32_t* __restrict__ active,
                                                   const uint32_t* __restrict__ act_idx, const T* __restrict__ grad,
                                                   int64_t ld, AdamK<T> K, const double2* __restrict__ bias) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n_pidx || !active[i]) return;
  const int64_t k = i / B;
  const int32_t row = (int32_t)(i - k * B);
  const int64_t o = ((int64_t)order[k] * kD + j) * B + row;
  const T g = grad[(int64_t)act_idx[i] + (int64_t)j * ld];
  const double2 bc = bias[i];
  T p = params[o], m = m1[o], v = m2[o];
  adam_col<T>(p, m, v, g, K.lr[j], K.b1, K.b2, K.eps, (T)bc.x, (T)bc.y);
  m1[o] = m;
  m2[o] = v;
  params[o] = p;
}

// The same update with one thread per row sweeping its 59 columns: the
// row's flag, compact index and bias corrections are read once instead of
// once per column, and a workgroup covers 256 rows.  For a given column the
// lanes of a wave touch consecutive rows, so every access stays coalesced
// (lanes of inactive rows idle: compacting the active rows into a list was
// slower, 0.26 ms against 0.20 ms on the aerial step, as it spreads a
// wave's accesses over twice the address range).  Every access is
// non-temporal: the streams are touched once, and stores that do not stay
// dirty in the caches spare the next kernel their write-back (on the aerial
// step Adam 0.204 -> 0.187 ms and the following preprocess 0.109 ->
// 0.080 ms; non-temporal moment stores alone changed nothing).
template <typename T>
__global__ void __launch_bounds__(256) k_adam_sweep(T* __restrict__ params, T* __restrict__ m1, T* __restrict__ m2,
                                                    uint32_t* __restrict__ step, const int32_t* __restrict__ order,
                                                    int32_t B, int64_t n_pidx, const uint32_t* __restrict__ active,
                                                    const uint32_t* __restrict__ act_idx, const T* __restrict__ grad,
                                                    int64_t ld, AdamK<T> K, double lb1, double lb2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pidx || !active[i]) return;
  const int64_t k = i / B;
  const int32_t row = (int32_t)(i - k * B);
  const int64_t o0 = (int64_t)order[k] * kD * B + row;
  const T* gp = grad + (int64_t)act_idx[i];
  // the row's step and bias corrections (what k_adam_rows computes for the
  // column-grid update), in the same precision
  T bcx, bcy;
  adam_step_bias<T>(step + (int64_t)order[k] * B + row, lb1, lb2, bcx, bcy);
#pragma unroll 4
  for (int j = 0; j < kD; ++j) {
    const int64_t o = o0 + (int64_t)j * B;
    const T g = __builtin_nontemporal_load(gp + (int64_t)j * ld);
    T p = __builtin_nontemporal_load(params + o);
    T m = __builtin_nontemporal_load(m1 + o), v = __builtin_nontemporal_load(m2 + o);
    adam_col<T>(p, m, v, g, K.lr[j], K.b1, K.b2, K.eps, bcx, bcy);
    __builtin_nontemporal_store(m, m1 + o);
    __builtin_nontemporal_store(v, m2 + o);
    __builtin_nontemporal_store(p, params + o);
  }
}

// One workgroup covers up to kBoundRows consecutive rows of one block: the
// rows are reduced in registers and LDS, then a single atomic max per
// workgroup raises the block radius.  Four rows per thread: with 4096 rows
// per workgroup (16 dependent loads per thread, one workgroup per CU for 1M
// rows) the kernel took 25 us on the aerial step.
constexpr int kBoundRows = 1024;

template <typename T>
__global__ void __launch_bounds__(256) k_adam_bounds(const T* __restrict__ params, const int32_t* __restrict__ order,
                                                     const int32_t* __restrict__ slot_block, int32_t B, int64_t n_pidx,
                                                     const uint32_t* __restrict__ active, float kappa,
                                                     float* __restrict__ spheres, uint8_t* __restrict__ dirty) {
  // workgroup -> (block k in the order, chunk c of kBoundRows rows within it)
  const int64_t chunks = (B + kBoundRows - 1) / kBoundRows;
  const int64_t k = blockIdx.x / chunks, c = blockIdx.x - k * chunks;
  const int64_t i0 = k * (int64_t)B + c * kBoundRows;
  if (i0 >= n_pidx) return;
  const int32_t slot = order[k];
  const int32_t blk = slot_block[slot];
  const float* S = spheres ? spheres + 4 * (int64_t)blk : nullptr;
  float reach = 0.f;
  bool any = false;
  const int64_t iend = (k + 1) * (int64_t)B < i0 + kBoundRows ? (k + 1) * (int64_t)B : i0 + kBoundRows;
  for (int64_t i = i0 + threadIdx.x; i < iend && i < n_pidx; i += 256) {
    if (!active[i]) continue;
    any = true;
    if (S) {
      const int32_t row = (int32_t)(i - k * B);
      const T* P = params + (int64_t)slot * kD * B + row;
      const float dx = (float)P[0] - S[0], dy = (float)P[B] - S[1], dz = (float)P[2 * (int64_t)B] - S[2];
      const float ls = fmaxf((float)P[3 * (int64_t)B], fmaxf((float)P[4 * (int64_t)B], (float)P[5 * (int64_t)B]));
      // rounded up so that single-precision evaluation never undercuts the bound
      reach = fmaxf(reach, (sqrtf(dx * dx + dy * dy + dz * dz) + 3.f * kappa * expf(ls)) * 1.000001f + 1e-6f);
    }
  }
  __shared__ float s_r[256 / kWave];
  __shared__ int s_any[256 / kWave];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) reach = fmaxf(reach, __shfl_xor(reach, off, kWave));
  const bool wany = __ballot(any) != 0;
  if (__lane_id() == 0) { s_r[threadIdx.x / kWave] = reach; s_any[threadIdx.x / kWave] = wany; }
  __syncthreads();
  if (threadIdx.x == 0) {
    float r = 0.f;
    int a = 0;
    for (int w = 0; w < 256 / kWave; ++w) { r = fmaxf(r, s_r[w]); a |= s_any[w]; }
    if (a && blk >= 0) {
      if (dirty) dirty[blk] = 1;
      if (spheres) atomicMax(reinterpret_cast<unsigned int*>(spheres + 4 * (int64_t)blk + 3), __float_as_uint(r));
    }
  }
}

void launch_adam_bounds(const tide_pool* pool, const tide_proj* proj, float kappa, float* spheres, uint8_t* dirty,
                        hipStream_t st) {
  const int64_t n = proj->n_pidx;
  if (n == 0 || (!spheres && !dirty)) return;
  // workgroups of kBoundRows indices, never straddling a block
  const uint32_t gb = (uint32_t)((int64_t)pool->n_order * ceil_div(pool->block_rows, kBoundRows));
  if (pool->dtype == TIDE_F32)
    hipLaunchKernelGGL(k_adam_bounds<float>, dim3(gb), dim3(256), 0, st, (const float*)pool->params, pool->order,
                       pool->slot_block, pool->block_rows, n, proj->active, kappa, spheres, dirty);
  else
    hipLaunchKernelGGL(k_adam_bounds<double>, dim3(gb), dim3(256), 0, st, (const double*)pool->params, pool->order,
                       pool->slot_block, pool->block_rows, n, proj->active, kappa, spheres, dirty);
}

}  // namespace tide

using namespace tide;

extern "C" size_t tide_adam_ws_bytes(int64_t n_pidx) { return align_up((size_t)(n_pidx > 0 ? n_pidx : 1) * 16) + 256; }

extern "C" tide_status tide_adam_sparse(tide_pool* pool, const tide_proj* proj, const void* grad, int64_t grad_ld,
                                        const tide_adam_cfg* cfg, float* spheres, uint8_t* dirty, int64_t n_blocks,
                                        void* ws, size_t ws_bytes, void* stream) {
  TIDE_CHECK_ARG(pool && proj && grad && cfg && ws, "null argument");
  TIDE_CHECK_ARG(pool->params && pool->exp_avg && pool->exp_avg_sq && pool->step && pool->order && pool->slot_block,
                 "pool has a null pointer");
  TIDE_CHECK_ARG(proj->dtype == pool->dtype, "dtype mismatch");
  TIDE_CHECK_ARG(proj->n_pidx == (int64_t)pool->n_order * pool->block_rows, "proj does not match pool");
  TIDE_CHECK_ARG(grad_ld >= proj->n_pidx, "grad_ld too small");
  TIDE_CHECK_ARG(cfg->beta1 > 0 && cfg->beta1 < 1 && cfg->beta2 > 0 && cfg->beta2 < 1 && cfg->eps >= 0,
                 "bad Adam constants");
  TIDE_CHECK_ARG((!spheres && !dirty) || n_blocks > 0, "n_blocks must be given with spheres/dirty");
  TIDE_CHECK_ARG(ws_bytes >= tide_adam_ws_bytes(proj->n_pidx), "adam workspace too small");
  TIDE_CHECK_ARG(aligned16(ws), "adam workspace must be 16-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = proj->n_pidx;
  if (n == 0) return TIDE_OK;
  const uint32_t gx = (uint32_t)ceil_div(n, 256);
  double2* bias = (double2*)ws;
  const double lb1 = std::log2((double)cfg->beta1), lb2 = std::log2((double)cfg->beta2);
  if (pool->dtype == TIDE_F32) {
    const AdamK<float> K = make_adam_k<float>(cfg);
    // the row sweep takes the step and bias corrections itself
    TIDE_TIMED("adam", st, hipLaunchKernelGGL(k_adam_sweep<float>, dim3(gx), dim3(256), 0, st,
                                              (float*)pool->params, (float*)pool->exp_avg, (float*)pool->exp_avg_sq,
                                              pool->step, pool->order, pool->block_rows, n, proj->active,
                                              proj->act_idx, (const float*)grad, grad_ld, K, lb1, lb2));
  } else {
    hipLaunchKernelGGL(k_adam_rows, dim3(gx), dim3(256), 0, st, pool->step, pool->order, pool->block_rows, n,
                       proj->active, lb1, lb2, bias);
    TIDE_LAUNCH_CHECK("k_adam_rows");
    const AdamK<double> K = make_adam_k<double>(cfg);
    TIDE_TIMED("adam", st, hipLaunchKernelGGL(k_adam_cols<double>, dim3(gx, kD), dim3(256), 0, st,
                                              (double*)pool->params, (double*)pool->exp_avg,
                                              (double*)pool->exp_avg_sq, pool->order, pool->block_rows, n,
                                              proj->active, proj->act_idx, (const double*)grad, grad_ld, K, bias));
  }
  TIDE_LAUNCH_CHECK("k_adam");
  launch_adam_bounds(pool, proj, cfg->kappa, spheres, dirty, st);
  TIDE_LAUNCH_CHECK("k_adam_bounds");
  return TIDE_OK;
}
