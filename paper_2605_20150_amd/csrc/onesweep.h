// One-sweep LSD radix sort (see prims.h for the method): the histogram and
// pass kernels as templates, so that the caller chooses what the last pass
// writes for each sorted key.
#pragma once

#include "prims.h"

namespace tide {

// ------------------------------------------------- one-sweep radix sort
// Every pass's digit counts over all keys (see prims.h).  Block b takes
// tiles b, b + G, ... of the actual count, clears their status words for
// every pass, counts into LDS bins and adds its nonzero bins to its copy of
// the global counts (device-scope atomics, at most 256 per pass and block).
template <bool kVec>
__global__ void __launch_bounds__(kSortThreads) k_os_hist(const uint32_t* keys, int64_t n_max,
                                                          const unsigned long long* d_n, int passes,
                                                          int64_t nb_max, int64_t tile_keys, uint32_t* ctl,
                                                          unsigned long long* status) {
  const int64_t n = dev_count(n_max, d_n);
  // the look-back words of the passes' tiles (tile_keys keys each) below the count
  const int64_t nbp = (n + tile_keys - 1) / tile_keys;
  for (int64_t t = blockIdx.x; t < nbp; t += gridDim.x)
    for (int p = 0; p < passes; ++p) status[((int64_t)p * nb_max + t) * 256 + threadIdx.x] = 0ull;
  // the counts, over chunks of 4096 keys
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  __shared__ uint32_t h[kOsMaxPasses][256];
  for (int k = threadIdx.x; k < kOsMaxPasses * 256; k += kSortThreads) (&h[0][0])[k] = 0;
  __syncthreads();
  for (int64_t t = blockIdx.x; t < nb; t += gridDim.x) {
    const int64_t base = t * kSortTile;
#pragma unroll
    for (int r = 0; r < kSortRounds / 4; ++r) {
      const int64_t i = base + 4 * ((int64_t)r * kSortThreads + threadIdx.x);
      uint32_t k4[4];
      int cnt = 0;   // valid keys of the four (a prefix)
      if (kVec && i + 4 <= n) {
        const uint4 q = *reinterpret_cast<const uint4*>(keys + i);
        k4[0] = q.x; k4[1] = q.y; k4[2] = q.z; k4[3] = q.w;
        cnt = 4;
      } else {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          k4[a] = i + a < n ? keys[i + a] : 0u;
          cnt += i + a < n ? 1 : 0;
        }
      }
      for (int p = 0; p < passes; ++p) {
        uint32_t d[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) d[a] = (k4[a] >> (8 * p)) & 255u;
        uint32_t cur = d[0], run = cnt > 0 ? 1u : 0u;
#pragma unroll
        for (int a = 1; a < 4; ++a) {
          if (a < cnt) {
            if (d[a] == cur) {
              ++run;
            } else {
              atomicAdd(&h[p][cur], run);
              cur = d[a];
              run = 1;
            }
          }
        }
        hist_add(h[p], cur, run);
      }
    }
  }
  __syncthreads();
  uint32_t* g = ctl + kOsCtlWords + (blockIdx.x % kOsCopies) * kOsMaxPasses * 256;
  for (int p = 0; p < passes; ++p) {
    const uint32_t c = h[p][threadIdx.x];
    if (c) atomicAdd(&g[p * 256 + threadIdx.x], c);
  }
}

// One pass: tile t (the block index) is ranked, its digit counts are
// published (inclusive at once for tile 0, else as an aggregate), the tile
// is staged in LDS, thread d walks back over earlier tiles' words of digit d
// until an inclusive one, publishes its own inclusive count, and the tile is
// written to the digit's start plus the counts before it.
//
// Why every wait ends: the dispatcher starts a kernel's workgroups in
// index order on each XCD, so when the lowest unfinished tile m is not
// running, its XCD holds only lower tiles, which have finished, and m
// starts; once running it waits only on lower tiles, which have finished.
// (An atomic ticket would not need that order, but same-address device
// atomics serialise at about 12 ns each: 0.15 ms per binning.)
constexpr unsigned long long kOsAgg = 1ull << 32, kOsIncl = 2ull << 32;

template <int R, int W, typename Out>
__global__ void __launch_bounds__(kWave * W) k_os_pass(const uint32_t* keys_in, const uint32_t* vals_in,
                                                       int64_t n_max, const unsigned long long* d_n, int shift,
                                                       unsigned long long* status, uint32_t* ctl, int pass,
                                                       uint32_t* err, Out out) {
  constexpr int kTile = kWave * W * R;
  __shared__ TileLds<R, W> L;
  for (int k = threadIdx.x; k < W * 256; k += kWave * W) (&L.wcnt[0][0])[k] = 0;
  __syncthreads();
  const int64_t t = blockIdx.x;
  const int64_t n = dev_count(n_max, d_n);
  const int64_t b0 = t * kTile;
  if (b0 >= n) return;
  const int m = (int)(n - b0 < kTile ? n - b0 : kTile);
  uint32_t key[R], val[R], rank[R];
  tile_rank(keys_in, vals_in, n, b0, shift, L, key, val, rank);
  __syncthreads();
  const uint32_t cnt = tile_digit_offsets(L);
  // threads 0..255 own one digit each from here on
  const int d = threadIdx.x;
  const bool dig = d < 256;
  unsigned long long* mine = status + t * 256 + d;
  if (dig) __hip_atomic_store(mine, (t == 0 ? kOsIncl : kOsAgg) | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // the tile goes to LDS before the look-back, so its registers are free
  // while the look-back waits
  __syncthreads();
  tile_stage(n, b0, shift, L, key, val, rank);
  // this digit's count over all keys (its copies added up): a digit no key
  // holds needs no start, so its words stay aggregates of zero and no tile
  // walks back for it (most of the top byte's digits, say)
  uint32_t gc = 0;
  if (dig) {
#pragma unroll
    for (int c = 0; c < kOsCopies; ++c) gc += ctl[kOsCtlWords + (c * kOsMaxPasses + pass) * 256 + d];
  }
  // look-back: kOsWindow earlier tiles' words per poll, nearest first; the
  // aggregates before the first inclusive word are added, and a word not
  // yet published is polled again (after the aggregates before it)
  uint32_t excl = 0;
  if (dig && t > 0 && gc > 0) {
    int64_t j = t - 1;
    uint32_t spins = 0;
    for (;;) {
      unsigned long long s[kOsWindow];
#pragma unroll
      for (int k = 0; k < kOsWindow; ++k)
        s[k] = j - k >= 0 ? __hip_atomic_load(status + (j - k) * 256 + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                          : kOsIncl;   // before tile 0: an inclusive zero
      int k = 0;
      bool done = false;
      for (; k < kOsWindow; ++k) {
        const unsigned long long f = s[k] & ~0xffffffffull;
        if (f == 0ull) break;
        excl += (uint32_t)s[k];
        if (f == kOsIncl) {
          done = true;
          break;
        }
      }
      if (done) break;
      j -= k;
      if (k < kOsWindow) {   // tile j has not published yet: poll that word alone
        unsigned long long x;
        while (((x = __hip_atomic_load(status + j * 256 + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 32) ==
                   0ull &&
               ++spins < kOsSpinLimit)
          __builtin_amdgcn_s_sleep(8);
        if (spins >= kOsSpinLimit) {
          atomicOr(err, 1u);
          break;
        }
        excl += (uint32_t)x;
        if ((x & ~0xffffffffull) == kOsIncl) break;
        --j;
      }
    }
    __hip_atomic_store(mine, kOsIncl | (excl + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // the digit's start: exclusive scan of the global digit counts (waves 0..3)
  const uint32_t ginc = wave_incl_scan(gc);
  const int w = threadIdx.x / kWave;
  __syncthreads();   // L.wsum is free again
  if (dig && __lane_id() == kWave - 1) L.wsum[w] = ginc;
  __syncthreads();
  if (dig) {
    uint32_t gpre = 0;
    for (int q = 0; q < w; ++q) gpre += L.wsum[q];
    L.gbase[d] = gpre + ginc - gc + excl;
  }
  __syncthreads();
  tile_write(m, shift, L, out);
}

template <int R, int W, typename LastOut>
void onesweep_run(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t n, int passes, bool identity_vals,
                  const OsWork& w, hipStream_t st, uint32_t** keys_res, uint32_t** vals_res,
                  const unsigned long long* d_n, const LastOut& last_out) {
  uint32_t *ki = ka, *vi = va, *ko = kb, *vo = vb;
  constexpr int64_t kTile = kWave * W * R;
  const int64_t nb = ceil_div(n, kTile);
  const int64_t nc = ceil_div(n, kSortTile);
  const uint32_t g = (uint32_t)(nc < kOsHistBlocks ? nc : kOsHistBlocks);
  if (((uintptr_t)ki & 15) == 0)
    hipLaunchKernelGGL(k_os_hist<true>, dim3(g), dim3(kSortThreads), 0, st, ki, n, d_n, passes, nb, kTile, w.ctl,
                       w.status);
  else
    hipLaunchKernelGGL(k_os_hist<false>, dim3(g), dim3(kSortThreads), 0, st, ki, n, d_n, passes, nb, kTile, w.ctl,
                       w.status);
  for (int p = 0; p < passes; ++p) {
    const uint32_t* vin = (identity_vals && p == 0) ? nullptr : vi;
    unsigned long long* sp = w.status + (size_t)p * nb * 256;
    if (p + 1 == passes)
      hipLaunchKernelGGL((k_os_pass<R, W, LastOut>), dim3((uint32_t)nb), dim3(kWave * W), 0, st, ki, vin, n, d_n,
                         8 * p, sp, w.ctl, p, w.err, last_out);
    else
      hipLaunchKernelGGL((k_os_pass<R, W, PairsOut>), dim3((uint32_t)nb), dim3(kWave * W), 0, st, ki, vin, n, d_n,
                         8 * p, sp, w.ctl, p, w.err, PairsOut{ko, vo, nullptr, nullptr});
    uint32_t* t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
  }
  *keys_res = ki;
  *vals_res = vi;
}

// As radix_sort_pairs (bits <= 32, at most kOsMaxPasses passes) over tiles
// of 64 W R keys (W waves of R rounds, W >= 4); n is the launch bound and
// d_n, when given, the count on the device.  The last pass writes through
// last_out(position, key, value) instead of the ping-pong buffer it would
// fill (PairsOut over that buffer gives the sorted keys and values; another
// functor can write what the caller needs of each sorted pair instead), and
// *keys_res / *vals_res name that buffer as if it had.
template <int R, int W, typename LastOut>
void onesweep_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t n, int bits,
                         bool identity_vals, const OsWork& w, hipStream_t st, uint32_t** keys_res,
                         uint32_t** vals_res, const unsigned long long* d_n, const LastOut& last_out) {
  static_assert(W >= 4, "256 threads own the digits");
  const int passes = (bits + 7) / 8;
  if (n <= 0 || passes <= 0) {
    *keys_res = ka;
    *vals_res = va;
    return;
  }
  onesweep_run<R, W>(ka, va, kb, vb, n, passes, identity_vals, w, st, keys_res, vals_res, d_n, last_out);
}

}  // namespace tide
