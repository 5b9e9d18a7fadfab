// Non-template parts of the scan and radix sort (see prims.h).
#include "prims.h"

namespace tide {

__global__ void __launch_bounds__(1024) k_scan_partials(unsigned long long* partial, int64_t nb,
                                                        unsigned long long* total, ScanTail tail, int64_t n_max,
                                                        const unsigned long long* d_n) {
  __shared__ unsigned long long wtot[1024 / kWave];
  __shared__ unsigned long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = __lane_id(), w = threadIdx.x / kWave;
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    const int64_t i = b0 + threadIdx.x;
    const unsigned long long x = i < nb ? partial[i] : 0ull;
    unsigned long long inc = x;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const unsigned long long y = __shfl_up(inc, off, kWave);
      if (lane >= off) inc += y;
    }
    if (lane == kWave - 1) wtot[w] = inc;
    __syncthreads();
    unsigned long long pre = carry;
    for (int q = 0; q < w; ++q) pre += wtot[q];
    if (i < nb) partial[i] = pre + inc - x;
    __syncthreads();
    if (threadIdx.x == 1023) carry = pre + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *total = carry;
    write_tail(tail, carry, dev_count(n_max, d_n));
  }
}

// Adds this lane's run (digit d, count c) to the wave's bins: one add for
// the whole wave when every lane holds the same digit (the top digits of
// sorted or narrow-range keys), else one LDS atomic per lane.
__device__ __forceinline__ void hist_add(uint32_t* hw, uint32_t d, uint32_t c) {
  const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
  if (__all(d == d0)) {
    const uint32_t t = wave_sum(c);
    if (__lane_id() == 0) atomicAdd(&hw[d0], t);   // atomic: other lanes' earlier runs may add to it too
  } else {
    atomicAdd(&hw[d], c);
  }
}

// Per-block digit histogram.  Each wave counts into bins of its own, a
// thread takes four consecutive keys per load (16 bytes when kVec: the keys
// are 16-byte aligned) and adds equal neighbouring digits as one run, and the
// waves' bins are added at the end.
template <bool kVec>
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint32_t* keys, int64_t n_max,
                                                             const unsigned long long* d_n, int shift,
                                                             uint32_t* ghist, int64_t nb) {
  const int64_t n = dev_count(n_max, d_n);
  __shared__ uint32_t h[kSortWaves][256];
  for (int k = threadIdx.x; k < kSortWaves * 256; k += kSortThreads) (&h[0][0])[k] = 0;
  __syncthreads();
  uint32_t* hw = h[threadIdx.x / kWave];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int r = 0; r < kSortRounds / 4; ++r) {
    const int64_t i = base + 4 * ((int64_t)r * kSortThreads + threadIdx.x);
    uint32_t d[4];
    int cnt = 0;   // valid keys of the four (a prefix)
    if (kVec && i + 4 <= n) {
      const uint4 q = *reinterpret_cast<const uint4*>(keys + i);
      d[0] = q.x; d[1] = q.y; d[2] = q.z; d[3] = q.w;
      cnt = 4;
    } else {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        d[a] = i + a < n ? keys[i + a] : 0u;
        cnt += i + a < n ? 1 : 0;
      }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) d[a] = (d[a] >> shift) & 255u;
    // runs of equal digits among the valid keys; lanes with none add 0 to
    // their first digit's bin
    uint32_t cur = d[0], run = cnt > 0 ? 1u : 0u;
#pragma unroll
    for (int a = 1; a < 4; ++a) {
      if (a < cnt) {
        if (d[a] == cur) {
          ++run;
        } else {
          atomicAdd(&hw[cur], run);
          cur = d[a];
          run = 1;
        }
      }
    }
    hist_add(hw, cur, run);
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kSortWaves; ++w) c += h[w][threadIdx.x];
  ghist[(int64_t)threadIdx.x * nb + blockIdx.x] = c;
}

__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(const uint32_t* keys_in,
                                                                const uint32_t* vals_in, int64_t n_max,
                                                                const unsigned long long* d_n, int shift,
                                                                const uint32_t* gofs, int64_t nb,
                                                                uint32_t* keys_out, uint32_t* vals_out,
                                                                const uint32_t* gather_src, uint32_t* gather_out) {
  const int64_t n = dev_count(n_max, d_n);
  const int64_t b0 = (int64_t)blockIdx.x * kSortTile;
  if (b0 >= n) return;
  const int m = (int)(n - b0 < kSortTile ? n - b0 : kSortTile);   // elements of this block
  __shared__ uint32_t wcnt[kSortWaves][256];
  __shared__ uint32_t gbase[256], lstart[256], wsum[kSortWaves];
  __shared__ uint32_t skey[kSortTile], sval[kSortTile];
  for (int k = threadIdx.x; k < kSortWaves * 256; k += kSortThreads) (&wcnt[0][0])[k] = 0;
  gbase[threadIdx.x] = gofs[(int64_t)threadIdx.x * nb + blockIdx.x];
  __syncthreads();
  const int w = threadIdx.x / kWave, lane = __lane_id();
  const uint64_t lt = lanemask_lt();
  const int64_t base = b0 + (int64_t)w * (kWave * kSortRounds);
  uint32_t key[kSortRounds], val[kSortRounds], rank[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + (int64_t)r * kWave + lane;
    const bool ok = i < n;
    key[r] = ok ? keys_in[i] : 0u;
    val[r] = ok ? (vals_in ? vals_in[i] : (uint32_t)i) : 0u;
    const uint32_t d = (key[r] >> shift) & 255u;
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t mk = __ballot(bit);
      peers &= bit ? mk : ~mk;
    }
    uint32_t r0 = 0;
    if (ok) r0 = wcnt[w][d];
    rank[r] = r0 + (uint32_t)__popcll(peers & lt);
    // the lowest lane of each digit group advances the wave's counter
    if (ok && (peers & lt) == 0) wcnt[w][d] = r0 + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // per digit: the waves' offsets within the digit, and the digit's start in
  // the block (exclusive scan of the block's digit counts)
  const int d = threadIdx.x;
  uint32_t cnt = 0;
#pragma unroll
  for (int q = 0; q < kSortWaves; ++q) {
    const uint32_t c = wcnt[q][d];
    wcnt[q][d] = cnt;
    cnt += c;
  }
  const uint32_t inc = wave_incl_scan(cnt);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (int q = 0; q < w; ++q) pre += wsum[q];
  lstart[d] = pre + inc - cnt;
  __syncthreads();
  // the block's elements in (digit, rank) order in LDS ...
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + (int64_t)r * kWave + lane;
    if (i < n) {
      const uint32_t dd = (key[r] >> shift) & 255u;
      const uint32_t j = lstart[dd] + wcnt[w][dd] + rank[r];
      skey[j] = key[r];
      sval[j] = val[r];
    }
  }
  __syncthreads();
  // ... written out in that order: runs of one digit land on consecutive
  // addresses
  for (int j = threadIdx.x; j < m; j += kSortThreads) {
    const uint32_t k = skey[j];
    const uint32_t dd = (k >> shift) & 255u;
    const uint32_t pos = gbase[dd] + (uint32_t)j - lstart[dd];
    const uint32_t v = sval[j];
    keys_out[pos] = k;
    vals_out[pos] = v;
    if (gather_src) gather_out[pos] = gather_src[v];
  }
}

void radix_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t n, int bits,
                      bool identity_vals, uint32_t* hist, unsigned long long* partial,
                      unsigned long long* total, hipStream_t st, uint32_t** keys_res,
                      uint32_t** vals_res, const unsigned long long* d_n, const uint32_t* gather_src,
                      uint32_t* gather_out) {
  uint32_t *ki = ka, *vi = va, *ko = kb, *vo = vb;
  bool ident = identity_vals;
  const int64_t nb = ceil_div(n > 0 ? n : 1, kSortTile);
  if (n > 0) {
    for (int shift = 0; shift < bits; shift += 8) {
      if (((uintptr_t)ki & 15) == 0)
        hipLaunchKernelGGL(k_radix_hist<true>, dim3((uint32_t)nb), dim3(kSortThreads), 0, st, ki, n, d_n, shift, hist, nb);
      else
        hipLaunchKernelGGL(k_radix_hist<false>, dim3((uint32_t)nb), dim3(kSortThreads), 0, st, ki, n, d_n, shift, hist,
                           nb);
      scan_exclusive(ArrayIn{hist}, 256 * nb, hist, partial, total, st);
      const bool last = shift + 8 >= bits;
      TIDE_TIMED("radix_scatter", st, hipLaunchKernelGGL(k_radix_scatter, dim3((uint32_t)nb), dim3(kSortThreads), 0, st, ki,
                         ident ? nullptr : vi, n, d_n, shift, hist, nb, ko, vo, last ? gather_src : nullptr,
                         last ? gather_out : nullptr));
      ident = false;
      uint32_t* t = ki; ki = ko; ko = t;
      t = vi; vi = vo; vo = t;
    }
  }
  *keys_res = ki;
  *vals_res = vi;
}

}  // namespace tide
