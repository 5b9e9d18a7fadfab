// Prefetch-predictor MLP on gfx950: forward, backward and Adam.
//
// Every product is one LDS-tiled GEMM on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Weights are bf16.  An
// FP32 operand (activations, gradients) is split into hi = bf16(a) and
// lo = bf16(a - hi), and both halves are multiplied: W (hi + lo) keeps about
// 16 significant bits of a, against 8 for a plain bf16 cast, for twice the
// matrix-core work.  The weight-gradient product has FP32 on both sides and
// takes the three significant terms hi.hi + lo.hi + hi.lo.
//
// Tiles: 64 x 64 outputs per 256-thread workgroup (4 waves, 32 x 32 each =
// 2 x 2 MFMA tiles), K staged 32 at a time through LDS as bf16 rows
// [row][k] so that one 16-byte LDS read gives a lane its 8 operands.
#include <cmath>

#include "common.h"

namespace tide {
namespace {

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kLdk = kBK + 8;   // LDS row stride in bf16 (80 bytes, 16-byte aligned rows)

// Nearest bfloat16 (ties to even) of an FP32 value, as its 16-bit pattern.
__device__ inline uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline void split(float f, uint16_t& hi, uint16_t& lo) {
  hi = bf16_bits(f);
  lo = bf16_bits(f - bf16_float(hi));   // exact difference
}

enum AKind { kA_KC = 0, kA_MC = 1 };                 // FP32 A contiguous along K / along M
enum BKind { kB_WKC = 0, kB_WNC = 1, kB_FNC = 2 };   // bf16 W [n][k], bf16 W [k][n], FP32 X [k][n]
enum Epi { kE_BIAS = 0, kE_BIAS_RELU = 1, kE_MASK = 2, kE_STORE = 3 };

// C[m][n] = sum_k A(m, k) B(k, n), then the epilogue:
//   kE_BIAS       C = acc + bias[n]
//   kE_BIAS_RELU  C = max(acc + bias[n], 0)
//   kE_MASK       C = mask[m][n] > 0 ? acc : 0   (ReLU adjoint)
//   kE_STORE      C = acc
// Requirements (checked by the host): the contiguous extent of every
// operand (K for kA_KC / kB_WKC, M for kA_MC, N for kB_WNC / kB_FNC) and
// every leading dimension are multiples of 8, and base pointers are 16-byte
// aligned, so a 4- or 8-wide vector load is either wholly inside or wholly
// outside the operand.
template <int AK, int BK, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ A, int64_t lda, const void* __restrict__ Bv,
                                              int64_t ldb, float* __restrict__ C, int64_t ldc,
                                              const float* __restrict__ bias, const float* __restrict__ mask,
                                              int64_t ldm, int M, int N, int K) {
  constexpr bool kSplitB = BK == kB_FNC;
  __shared__ __attribute__((aligned(16))) uint16_t sAh[kBM][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sAl[kBM][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sBh[kBN][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sBl[kSplitB ? kBN : 1][kLdk];

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < K; k0 += kBK) {
    // ---- stage A (FP32 -> bf16 hi/lo), 64 x 32
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      const int idx = t + rep * 256;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (AK == kA_KC) {
        const int m = idx >> 3, kk = (idx & 7) * 4;
        if (m0 + m < M && k0 + kk < K) v = *reinterpret_cast<const float4*>(A + (int64_t)(m0 + m) * lda + k0 + kk);
        const float f[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) split(f[j], sAh[m][kk + j], sAl[m][kk + j]);
      } else {
        const int kk = idx >> 4, mm = (idx & 15) * 4;
        if (k0 + kk < K && m0 + mm < M) v = *reinterpret_cast<const float4*>(A + (int64_t)(k0 + kk) * lda + m0 + mm);
        const float f[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) split(f[j], sAh[mm + j][kk], sAl[mm + j][kk]);
      }
    }
    // ---- stage B, 32 x 64, stored [n][k]
    if (BK == kB_WKC) {
      const uint16_t* W = static_cast<const uint16_t*>(Bv);
      const int n = t >> 2, kk = (t & 3) * 8;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (n0 + n < N && k0 + kk < K) v = *reinterpret_cast<const uint4*>(W + (int64_t)(n0 + n) * ldb + k0 + kk);
      *reinterpret_cast<uint4*>(&sBh[n][kk]) = v;
    } else if (BK == kB_WNC) {
      const uint16_t* W = static_cast<const uint16_t*>(Bv);
      const int kk = t >> 3, nn = (t & 7) * 8;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (k0 + kk < K && n0 + nn < N) v = *reinterpret_cast<const uint4*>(W + (int64_t)(k0 + kk) * ldb + n0 + nn);
      const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        sBh[nn + 2 * j][kk] = (uint16_t)(u[j] & 0xffffu);
        sBh[nn + 2 * j + 1][kk] = (uint16_t)(u[j] >> 16);
      }
    } else {
      const float* X = static_cast<const float*>(Bv);
#pragma unroll
      for (int rep = 0; rep < 2; ++rep) {
        const int idx = t + rep * 256;
        const int kk = idx >> 4, nn = (idx & 15) * 4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k0 + kk < K && n0 + nn < N) v = *reinterpret_cast<const float4*>(X + (int64_t)(k0 + kk) * ldb + n0 + nn);
        const float f[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) split(f[j], sBh[nn + j][kk], sBl[kSplitB ? nn + j : 0][kk]);
      }
    }
    __syncthreads();

    // ---- matrix cores: lane holds row (lane % 16), k = 8 (lane / 16) .. +7
    const int r = lane & 15, kc = (lane >> 4) * 8;
    bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = *reinterpret_cast<const bf16x8*>(&sAh[wm + 16 * i + r][kc]);
      al[i] = *reinterpret_cast<const bf16x8*>(&sAl[wm + 16 * i + r][kc]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      bh[j] = *reinterpret_cast<const bf16x8*>(&sBh[wn + 16 * j + r][kc]);
      if (kSplitB) bl[j] = *reinterpret_cast<const bf16x8*>(&sBl[kSplitB ? wn + 16 * j + r : 0][kc]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        if (kSplitB) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
      }
    __syncthreads();
  }

  // ---- epilogue: accumulator lane layout row = 4 (lane / 16) + e, column = lane % 16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + e;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= M || n >= N) continue;
        float v = acc[i][j][e];
        if (EPI == kE_BIAS || EPI == kE_BIAS_RELU) v += bias[n];
        if (EPI == kE_BIAS_RELU) v = fmaxf(v, 0.f);
        if (EPI == kE_MASK) v = mask[(int64_t)m * ldm + n] > 0.f ? v : 0.f;
        C[(int64_t)m * ldc + n] = v;
      }
}

template <int AK, int BK, int EPI>
tide_status gemm(hipStream_t st, const float* A, int64_t lda, const void* B, int64_t ldb, float* C, int64_t ldc,
                 const float* bias, const float* mask, int64_t ldm, int M, int N, int K) {
  if (M <= 0 || N <= 0) return TIDE_OK;
  const dim3 grid((unsigned)ceil_div(N, kBN), (unsigned)ceil_div(M, kBM));
  hipLaunchKernelGGL((k_gemm<AK, BK, EPI>), grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, bias, mask, ldm, M, N,
                     K);
  TIDE_LAUNCH_CHECK("mlp gemm");
  return TIDE_OK;
}

// ------------------------------------------------------------------ loss
constexpr int kLossBlocks = 1024;

// Number of valid outputs -> 1 / (batch * n_valid) and the count itself.
__global__ __launch_bounds__(256) void k_count_valid(const uint32_t* __restrict__ valid, int n_words, int batch,
                                                     float* __restrict__ inv_denom, double* __restrict__ denom) {
  __shared__ int s[256];
  int c = 0;
  for (int i = threadIdx.x; i < n_words; i += 256) c += __popc(valid[i]);
  s[threadIdx.x] = c;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double d = (double)batch * (double)(s[0] > 0 ? s[0] : 1);
    *denom = d;
    *inv_denom = (float)(1.0 / d);
  }
}

// G = (sigmoid(z) - y) / denom on valid outputs (0 elsewhere); per-block
// partial sums of the element losses in double, fixed order.
__global__ __launch_bounds__(256) void k_bce(const float* __restrict__ Z, const uint32_t* __restrict__ lab,
                                             const uint32_t* __restrict__ valid, int64_t total, int nout,
                                             const float* __restrict__ inv_denom, float* __restrict__ G,
                                             double* __restrict__ partial) {
  __shared__ double s[256];
  const float inv = *inv_denom;
  const int words = nout >> 5;
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t b = i / nout;
    const int o = (int)(i - b * nout);
    const bool ok = (valid[o >> 5] >> (o & 31)) & 1u;
    const float y = ((lab[b * words + (o >> 5)] >> (o & 31)) & 1u) ? 1.f : 0.f;
    const float z = Z[i];
    const float e = __expf(-fabsf(z));
    const float sig = z >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
    G[i] = ok ? (sig - y) * inv : 0.f;
    if (ok) acc += (double)(fmaxf(z, 0.f) - z * y + log1pf(e));
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(1024) void k_loss_sum(const double* __restrict__ partial, int n,
                                                   const double* __restrict__ denom, double* __restrict__ out) {
  __shared__ double s[1024];
  s[threadIdx.x] = (int)threadIdx.x < n ? partial[threadIdx.x] : 0.0;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0] / *denom;
}

// db[o] = sum over the batch of G[b][o], in batch order.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ G, int batch, int n,
                                                float* __restrict__ db) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= n) return;
  float a = 0.f;
  for (int b = 0; b < batch; ++b) a += G[(int64_t)b * n + o];
  db[o] = a;
}

// ------------------------------------------------------------------ Adam
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ p, uint16_t* __restrict__ pb,
                                                  const float* __restrict__ g, float* __restrict__ m,
                                                  float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                                                  float eps, float bc1, float bc2s) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    const float pi = p[i] - lr * (mi * bc1) / (sqrtf(vi) * bc2s + eps);
    m[i] = mi;
    v[i] = vi;
    p[i] = pi;
    pb[i] = bf16_bits(pi);
  }
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ pb, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    pb[i] = bf16_bits(p[i]);
}

__global__ __launch_bounds__(256) void k_threshold(const float* __restrict__ Z, int64_t n_words, int nout, float thr,
                                                   uint32_t* __restrict__ out) {
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= n_words) return;
  const int wpr = nout >> 5;
  const int64_t b = w / wpr;
  const int o0 = (int)(w - b * wpr) * 32;
  const float* z = Z + b * nout + o0;
  uint32_t bits = 0;
#pragma unroll 8
  for (int j = 0; j < 32; ++j) bits |= (z[j] >= thr ? 1u : 0u) << j;
  out[w] = bits;
}

// ------------------------------------------------------------------ host
struct Layout {
  int L;
  const int32_t* d;
  int64_t w_off[TIDE_MLP_MAX_LAYERS], b_off[TIDE_MLP_MAX_LAYERS], P;
  int max_out;
};

bool layout(const int32_t* dims, int L, Layout& lay) {
  if (!dims || L < 1 || L > TIDE_MLP_MAX_LAYERS) return false;
  for (int l = 0; l <= L; ++l)
    if (dims[l] <= 0 || dims[l] % 8 != 0) return false;
  if (dims[L] % 32 != 0) return false;
  lay.L = L;
  lay.d = dims;
  int64_t off = 0;
  lay.max_out = 0;
  for (int l = 0; l < L; ++l) {
    lay.w_off[l] = off;
    off += (int64_t)dims[l] * dims[l + 1];
    lay.b_off[l] = off;
    off += dims[l + 1];
    lay.max_out = dims[l + 1] > lay.max_out ? dims[l + 1] : lay.max_out;
  }
  lay.P = off;
  return true;
}

struct Ws {
  float* act[TIDE_MLP_MAX_LAYERS];   // act[l], l = 1..L-1: [batch][dims[l]]
  float* g[2];                       // [batch][max_out]
  double* partial;                   // [kLossBlocks]
  double* denom;
  float* inv_denom;
  size_t bytes;
};

Ws carve(void* base, const Layout& lay, int batch) {
  Carver c(base);
  Ws w{};
  for (int l = 1; l < lay.L; ++l) w.act[l] = c.take<float>((size_t)batch * lay.d[l]);
  w.g[0] = c.take<float>((size_t)batch * lay.max_out);
  w.g[1] = c.take<float>((size_t)batch * lay.max_out);
  w.partial = c.take<double>(kLossBlocks);
  w.denom = c.take<double>(1);
  w.inv_denom = c.take<float>(1);
  w.bytes = c.used;
  return w;
}

tide_status check_mlp(const tide_mlp* mlp, Layout& lay) {
  TIDE_CHECK_ARG(mlp, "null mlp");
  TIDE_CHECK_ARG(layout(mlp->dims, mlp->n_layers, lay),
                 "bad MLP dims: 1..%d layers, widths positive multiples of 8, output a multiple of 32",
                 TIDE_MLP_MAX_LAYERS);
  TIDE_CHECK_ARG(mlp->params && mlp->params_bf16, "null parameter buffers");
  TIDE_CHECK_ARG(aligned16(mlp->params) && aligned16(mlp->params_bf16), "parameter buffers must be 16-byte aligned");
  return TIDE_OK;
}

int grid_for(int64_t n) { return (int)std::min<int64_t>(ceil_div(n, 256), 4096); }

}  // namespace
}  // namespace tide

using namespace tide;

extern "C" int64_t tide_mlp_param_count(const int32_t* dims, int32_t n_layers) {
  Layout lay;
  return layout(dims, n_layers, lay) ? lay.P : -1;
}

extern "C" size_t tide_mlp_ws_bytes(const tide_mlp* mlp, int32_t batch) {
  Layout lay;
  if (!mlp || !layout(mlp->dims, mlp->n_layers, lay) || batch < 0) return 0;
  return carve(nullptr, lay, batch).bytes;
}

extern "C" tide_status tide_mlp_sync_bf16(const tide_mlp* mlp, void* stream) {
  Layout lay;
  tide_status s = check_mlp(mlp, lay);
  if (s != TIDE_OK) return s;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(lay.P)), dim3(256), 0, (hipStream_t)stream, mlp->params,
                     mlp->params_bf16, lay.P);
  TIDE_LAUNCH_CHECK("mlp to_bf16");
  return TIDE_OK;
}

extern "C" tide_status tide_mlp_fwd(const tide_mlp* mlp, const float* x, int32_t batch, float* logits, void* ws,
                                    size_t ws_bytes, void* stream) {
  Layout lay;
  tide_status s = check_mlp(mlp, lay);
  if (s != TIDE_OK) return s;
  TIDE_CHECK_ARG(batch >= 0, "negative batch");
  if (batch == 0) return TIDE_OK;
  TIDE_CHECK_ARG(x && logits && ws, "null argument");
  TIDE_CHECK_ARG(aligned16(x) && aligned16(ws), "x and ws must be 16-byte aligned");
  const Ws w = carve(ws, lay, batch);
  if (ws_bytes < w.bytes) {
    set_error("mlp workspace too small: %zu < %zu bytes", ws_bytes, w.bytes);
    return TIDE_ECAPACITY;
  }
  hipStream_t st = (hipStream_t)stream;
  const int32_t* d = lay.d;
  const float* in = x;
  timer_mark("mlp_fwd", st, true);
  for (int l = 0; l < lay.L; ++l) {
    const uint16_t* W = mlp->params_bf16 + lay.w_off[l];
    const float* b = mlp->params + lay.b_off[l];
    if (l + 1 < lay.L) {
      s = gemm<kA_KC, kB_WKC, kE_BIAS_RELU>(st, in, d[l], W, d[l], w.act[l + 1], d[l + 1], b, nullptr, 0, batch,
                                            d[l + 1], d[l]);
      in = w.act[l + 1];
    } else {
      s = gemm<kA_KC, kB_WKC, kE_BIAS>(st, in, d[l], W, d[l], logits, d[l + 1], b, nullptr, 0, batch, d[l + 1],
                                       d[l]);
    }
    if (s != TIDE_OK) return s;
  }
  timer_mark("mlp_fwd", st, false);
  return TIDE_OK;
}

extern "C" tide_status tide_mlp_bwd(const tide_mlp* mlp, const float* x, const float* logits,
                                    const uint32_t* label_bits, const uint32_t* valid_bits, int32_t batch,
                                    double* d_loss, void* ws, size_t ws_bytes, void* stream) {
  Layout lay;
  tide_status s = check_mlp(mlp, lay);
  if (s != TIDE_OK) return s;
  TIDE_CHECK_ARG(batch >= 1, "batch must be positive");
  TIDE_CHECK_ARG(x && logits && label_bits && valid_bits && d_loss && ws && mlp->grad, "null argument");
  TIDE_CHECK_ARG(aligned16(x) && aligned16(ws) && aligned16(mlp->grad), "x, ws and grad must be 16-byte aligned");
  const Ws w = carve(ws, lay, batch);
  if (ws_bytes < w.bytes) {
    set_error("mlp workspace too small: %zu < %zu bytes", ws_bytes, w.bytes);
    return TIDE_ECAPACITY;
  }
  hipStream_t st = (hipStream_t)stream;
  const int32_t* d = lay.d;
  const int L = lay.L, nout = d[L];
  const int64_t total = (int64_t)batch * nout;
  hipLaunchKernelGGL(k_count_valid, dim3(1), dim3(256), 0, st, valid_bits, nout / 32, batch, w.inv_denom, w.denom);
  TIDE_LAUNCH_CHECK("mlp count_valid");
  const int nb = (int)std::min<int64_t>(kLossBlocks, ceil_div(total, 256));
  TIDE_TIMED("mlp_bce", st,
             hipLaunchKernelGGL(k_bce, dim3(nb), dim3(256), 0, st, logits, label_bits, valid_bits, total, nout,
                                w.inv_denom, w.g[0], w.partial));
  TIDE_LAUNCH_CHECK("mlp bce");
  hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(1024), 0, st, w.partial, nb, w.denom, d_loss);
  TIDE_LAUNCH_CHECK("mlp loss_sum");
  int cur = 0;
  timer_mark("mlp_bwd", st, true);
  for (int l = L - 1; l >= 0; --l) {
    const float* G = w.g[cur];                      // dL/d(pre-activation of layer l's output) [batch][d[l+1]]
    const float* a = l == 0 ? x : w.act[l];         // layer input [batch][d[l]]
    float* gW = mlp->grad + lay.w_off[l];
    float* gb = mlp->grad + lay.b_off[l];
    s = gemm<kA_MC, kB_FNC, kE_STORE>(st, G, d[l + 1], a, d[l], gW, d[l], nullptr, nullptr, 0, d[l + 1], d[l],
                                      batch);
    if (s != TIDE_OK) return s;
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)ceil_div(d[l + 1], 256)), dim3(256), 0, st, G, batch, d[l + 1], gb);
    TIDE_LAUNCH_CHECK("mlp colsum");
    if (l > 0) {
      s = gemm<kA_KC, kB_WNC, kE_MASK>(st, G, d[l + 1], mlp->params_bf16 + lay.w_off[l], d[l], w.g[cur ^ 1], d[l],
                                       nullptr, w.act[l], d[l], batch, d[l], d[l + 1]);
      if (s != TIDE_OK) return s;
      cur ^= 1;
    }
  }
  timer_mark("mlp_bwd", st, false);
  return TIDE_OK;
}

extern "C" tide_status tide_mlp_adam(tide_mlp* mlp, float lr, float beta1, float beta2, float eps, void* stream) {
  Layout lay;
  tide_status s = check_mlp(mlp, lay);
  if (s != TIDE_OK) return s;
  TIDE_CHECK_ARG(mlp->grad && mlp->exp_avg && mlp->exp_avg_sq, "null Adam buffers");
  TIDE_CHECK_ARG(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f, "bad Adam constants");
  const int64_t t = mlp->step + 1;
  const float bc1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)t)));
  const float bc2s = (float)(1.0 / std::sqrt(1.0 - std::pow((double)beta2, (double)t)));
  hipStream_t st = (hipStream_t)stream;
  TIDE_TIMED("mlp_adam", st,
             hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(lay.P)), dim3(256), 0, st, mlp->params, mlp->params_bf16,
                                mlp->grad, mlp->exp_avg, mlp->exp_avg_sq, lay.P, lr, beta1, beta2, eps, bc1, bc2s));
  TIDE_LAUNCH_CHECK("mlp adam");
  mlp->step = t;
  return TIDE_OK;
}

extern "C" tide_status tide_mlp_predict_bits(const float* logits, int32_t batch, int32_t n_out, float threshold_logit,
                                             uint32_t* out_bits, void* stream) {
  TIDE_CHECK_ARG(batch >= 0 && n_out > 0 && n_out % 32 == 0, "n_out must be a positive multiple of 32");
  if (batch == 0) return TIDE_OK;
  TIDE_CHECK_ARG(logits && out_bits, "null argument");
  const int64_t words = (int64_t)batch * (n_out / 32);
  hipLaunchKernelGGL(k_threshold, dim3((unsigned)ceil_div(words, 256)), dim3(256), 0, (hipStream_t)stream, logits,
                     words, n_out, threshold_logit, out_bits);
  TIDE_LAUNCH_CHECK("mlp threshold");
  return TIDE_OK;
}
