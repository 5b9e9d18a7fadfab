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

// Shared LDS of a sort tile's ranking and scatter (tiles of 256 R keys).
template <int R>
struct TileLds {
  uint32_t wcnt[kSortWaves][256];
  uint32_t gbase[256], lstart[256], wsum[kSortWaves];
  uint32_t skey[kSortThreads * R], sval[kSortThreads * R];
};

// Ranks the keys of tile [b0, b0 + 256 R) ∩ [0, n) by digit (key >> shift) &
// 255: wave w holds R rounds of 64 consecutive keys; rank[r] is the key's
// rank among the keys of its digit held by the wave in earlier rounds and
// lower lanes, and L.wcnt[w][d] ends as the wave's count of digit d.
// L.wcnt must be zero on entry; the caller synchronises afterwards.
template <int R>
__device__ __forceinline__ void tile_rank(const uint32_t* keys_in, const uint32_t* vals_in, int64_t n, int64_t b0,
                                          int shift, TileLds<R>& L, uint32_t* key, uint32_t* val, uint32_t* rank) {
  const int w = threadIdx.x / kWave, lane = __lane_id();
  const uint64_t lt = lanemask_lt();
  const int64_t base = b0 + (int64_t)w * (kWave * R);
#pragma unroll
  for (int r = 0; r < R; ++r) {
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
    if (ok) r0 = L.wcnt[w][d];
    rank[r] = r0 + (uint32_t)__popcll(peers & lt);
    // the lowest lane of each digit group advances the wave's counter
    if (ok && (peers & lt) == 0) L.wcnt[w][d] = r0 + (uint32_t)__popcll(peers);
  }
}

// Thread d: turns L.wcnt[.][d] into the waves' offsets within digit d,
// writes the digit's start in the tile to L.lstart[d] and returns the
// tile's count of digit d.  Synchronises.
template <int R>
__device__ __forceinline__ uint32_t tile_digit_offsets(TileLds<R>& L) {
  const int d = threadIdx.x, w = threadIdx.x / kWave, lane = __lane_id();
  uint32_t cnt = 0;
#pragma unroll
  for (int q = 0; q < kSortWaves; ++q) {
    const uint32_t c = L.wcnt[q][d];
    L.wcnt[q][d] = cnt;
    cnt += c;
  }
  const uint32_t inc = wave_incl_scan(cnt);
  if (lane == kWave - 1) L.wsum[w] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (int q = 0; q < w; ++q) pre += L.wsum[q];
  L.lstart[d] = pre + inc - cnt;
  return cnt;
}

// Places the ranked keys in LDS in (digit, rank) order (L.lstart and L.wcnt
// must be visible).
template <int R>
__device__ __forceinline__ void tile_stage(int64_t n, int64_t b0, int shift, TileLds<R>& L, const uint32_t* key,
                                           const uint32_t* val, const uint32_t* rank) {
  const int w = threadIdx.x / kWave, lane = __lane_id();
  const int64_t base = b0 + (int64_t)w * (kWave * R);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = base + (int64_t)r * kWave + lane;
    if (i < n) {
      const uint32_t dd = (key[r] >> shift) & 255u;
      const uint32_t j = L.lstart[dd] + L.wcnt[w][dd] + rank[r];
      L.skey[j] = key[r];
      L.sval[j] = val[r];
    }
  }
}

// Writes the staged keys out to L.gbase[digit] + their place in the digit's
// run, so a digit's run lands on consecutive addresses (L.gbase and the
// staged keys must be visible).
template <int R>
__device__ __forceinline__ void tile_write(int m, int shift, const TileLds<R>& L, uint32_t* keys_out, uint32_t* vals_out,
                                           const uint32_t* gather_src, uint32_t* gather_out) {
  for (int j = threadIdx.x; j < m; j += kSortThreads) {
    const uint32_t k = L.skey[j];
    const uint32_t dd = (k >> shift) & 255u;
    const uint32_t pos = L.gbase[dd] + (uint32_t)j - L.lstart[dd];
    const uint32_t v = L.sval[j];
    keys_out[pos] = k;
    vals_out[pos] = v;
    if (gather_src) gather_out[pos] = gather_src[v];
  }
}

__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(const uint32_t* keys_in,
                                                                const uint32_t* vals_in, int64_t n_max,
                                                                const unsigned long long* d_n, int shift,
                                                                const uint32_t* gofs, int64_t nb,
                                                                uint32_t* keys_out, uint32_t* vals_out,
                                                                const uint32_t* gather_src, uint32_t* gather_out,
                                                                int xcd_order) {
  const int64_t n = dev_count(n_max, d_n);
  // with xcd_order, workgroup b (which starts on XCD b % 8) takes tile
  // x q + min(x, r) + b / 8 of nb = 8 q + r tiles, x = b % 8: each XCD
  // sorts a contiguous eighth of the tiles, so the runs of one digit that
  // consecutive tiles write side by side meet in the same L2
  int64_t tile = blockIdx.x;
  if (xcd_order) {
    const int64_t q = nb / kXcds, r = nb % kXcds, x = blockIdx.x % kXcds;
    tile = x * q + (x < r ? x : r) + blockIdx.x / kXcds;
  }
  const int64_t b0 = tile * kSortTile;
  if (b0 >= n) return;
  const int m = (int)(n - b0 < kSortTile ? n - b0 : kSortTile);   // elements of this block
  __shared__ TileLds<kSortRounds> L;
  for (int k = threadIdx.x; k < kSortWaves * 256; k += kSortThreads) (&L.wcnt[0][0])[k] = 0;
  L.gbase[threadIdx.x] = gofs[(int64_t)threadIdx.x * nb + tile];
  __syncthreads();
  uint32_t key[kSortRounds], val[kSortRounds], rank[kSortRounds];
  tile_rank(keys_in, vals_in, n, b0, shift, L, key, val, rank);
  __syncthreads();
  tile_digit_offsets(L);
  __syncthreads();
  tile_stage(n, b0, shift, L, key, val, rank);
  __syncthreads();
  tile_write(m, shift, L, keys_out, vals_out, gather_src, gather_out);
}

void radix_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t n, int bits,
                      bool identity_vals, uint32_t* hist, unsigned long long* partial,
                      unsigned long long* total, hipStream_t st, uint32_t** keys_res,
                      uint32_t** vals_res, const unsigned long long* d_n, const uint32_t* gather_src,
                      uint32_t* gather_out, bool xcd_order) {
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
      hipLaunchKernelGGL(k_radix_scatter, dim3((uint32_t)nb), dim3(kSortThreads), 0, st, ki, ident ? nullptr : vi, n,
                         d_n, shift, hist, nb, ko, vo, last ? gather_src : nullptr, last ? gather_out : nullptr,
                         xcd_order ? 1 : 0);
      ident = false;
      uint32_t* t = ki; ki = ko; ko = t;
      t = vi; vi = vo; vo = t;
    }
  }
  *keys_res = ki;
  *vals_res = vi;
}

// ------------------------------------------------- one-sweep radix sort
// Every pass's digit counts over all keys (see prims.h).  Block b takes
// tiles b, b + G, ... of the actual count, clears their status words for
// every pass, counts into LDS bins and adds its nonzero bins to its copy of
// the global counts (device-scope atomics, at most 256 per pass and block).
template <bool kVec, int R>
__global__ void __launch_bounds__(kSortThreads) k_os_hist(const uint32_t* keys, int64_t n_max,
                                                          const unsigned long long* d_n, int passes,
                                                          int64_t nb_max, uint32_t* ctl,
                                                          unsigned long long* status) {
  const int64_t n = dev_count(n_max, d_n);
  const int64_t nb = (n + kSortThreads * R - 1) / (kSortThreads * R);
  __shared__ uint32_t h[kOsMaxPasses][256];
  for (int k = threadIdx.x; k < kOsMaxPasses * 256; k += kSortThreads) (&h[0][0])[k] = 0;
  __syncthreads();
  for (int64_t t = blockIdx.x; t < nb; t += gridDim.x) {
    for (int p = 0; p < passes; ++p) status[((int64_t)p * nb_max + t) * 256 + threadIdx.x] = 0ull;
    const int64_t base = t * (kSortThreads * R);
#pragma unroll
    for (int r = 0; r < R / 4; ++r) {
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

template <int R>
__global__ void __launch_bounds__(kSortThreads) k_os_pass(const uint32_t* keys_in, const uint32_t* vals_in,
                                                          int64_t n_max, const unsigned long long* d_n, int shift,
                                                          unsigned long long* status,
                                                          uint32_t* ctl, int pass, uint32_t* err,
                                                          uint32_t* keys_out, uint32_t* vals_out,
                                                          const uint32_t* gather_src, uint32_t* gather_out) {
  __shared__ TileLds<R> L;
  for (int k = threadIdx.x; k < kSortWaves * 256; k += kSortThreads) (&L.wcnt[0][0])[k] = 0;
  __syncthreads();
  const int64_t t = blockIdx.x;
  const int64_t n = dev_count(n_max, d_n);
  const int64_t b0 = t * (kSortThreads * R);
  if (b0 >= n) return;
  const int m = (int)(n - b0 < kSortThreads * R ? n - b0 : kSortThreads * R);
  uint32_t key[R], val[R], rank[R];
  tile_rank(keys_in, vals_in, n, b0, shift, L, key, val, rank);
  __syncthreads();
  const uint32_t cnt = tile_digit_offsets(L);
  const int d = threadIdx.x;
  unsigned long long* mine = status + t * 256 + d;
  __hip_atomic_store(mine, (t == 0 ? kOsIncl : kOsAgg) | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // the tile goes to LDS before the look-back, so its registers are free
  // while the look-back waits
  __syncthreads();
  tile_stage(n, b0, shift, L, key, val, rank);
  // look-back: kOsWindow earlier tiles' words per poll, nearest first; the
  // aggregates before the first inclusive word are added, and a word not
  // yet published is polled again (after the aggregates before it)
  // this digit's count over all keys (its copies added up): a digit no key
  // holds needs no start, so its words stay aggregates of zero and no tile
  // walks back for it (most of the top byte's digits, say)
  uint32_t gc = 0;
#pragma unroll
  for (int c = 0; c < kOsCopies; ++c) gc += ctl[kOsCtlWords + (c * kOsMaxPasses + pass) * 256 + d];
  uint32_t excl = 0;
  if (t > 0 && gc > 0) {
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
  // the digit's start: exclusive scan of the global digit counts
  const uint32_t ginc = wave_incl_scan(gc);
  const int w = threadIdx.x / kWave;
  __syncthreads();   // L.wsum is free again
  if (__lane_id() == kWave - 1) L.wsum[w] = ginc;
  __syncthreads();
  uint32_t gpre = 0;
  for (int q = 0; q < w; ++q) gpre += L.wsum[q];
  L.gbase[d] = gpre + ginc - gc + excl;
  __syncthreads();
  tile_write(m, shift, L, keys_out, vals_out, gather_src, gather_out);
}

template <int R>
static void onesweep_run(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t n, int passes,
                         bool identity_vals, const OsWork& w, hipStream_t st, uint32_t** keys_res, uint32_t** vals_res,
                         const unsigned long long* d_n, const uint32_t* gather_src, uint32_t* gather_out) {
  uint32_t *ki = ka, *vi = va, *ko = kb, *vo = vb;
  const int64_t nb = ceil_div(n, kSortThreads * R);
  const uint32_t g = (uint32_t)(nb < kOsHistBlocks ? nb : kOsHistBlocks);
  if (((uintptr_t)ki & 15) == 0)
    hipLaunchKernelGGL((k_os_hist<true, R>), dim3(g), dim3(kSortThreads), 0, st, ki, n, d_n, passes, nb, w.ctl,
                       w.status);
  else
    hipLaunchKernelGGL((k_os_hist<false, R>), dim3(g), dim3(kSortThreads), 0, st, ki, n, d_n, passes, nb, w.ctl,
                       w.status);
  for (int p = 0; p < passes; ++p) {
    const bool last = p + 1 == passes;
    hipLaunchKernelGGL(k_os_pass<R>, dim3((uint32_t)nb), dim3(kSortThreads), 0, st, ki,
                       (identity_vals && p == 0) ? nullptr : vi, n, d_n, 8 * p, w.status + (size_t)p * nb * 256,
                       w.ctl, p, w.err, ko, vo, last ? gather_src : nullptr, last ? gather_out : nullptr);
    uint32_t* t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
  }
  *keys_res = ki;
  *vals_res = vi;
}

void onesweep_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t n, int bits, int rounds,
                         bool identity_vals, const OsWork& w, hipStream_t st, uint32_t** keys_res,
                         uint32_t** vals_res, const unsigned long long* d_n, const uint32_t* gather_src,
                         uint32_t* gather_out) {
  const int passes = (bits + 7) / 8;
  if (n <= 0 || passes <= 0) {
    *keys_res = ka;
    *vals_res = va;
    return;
  }
  if (rounds == 4)
    onesweep_run<4>(ka, va, kb, vb, n, passes, identity_vals, w, st, keys_res, vals_res, d_n, gather_src, gather_out);
  else if (rounds == 8)
    onesweep_run<8>(ka, va, kb, vb, n, passes, identity_vals, w, st, keys_res, vals_res, d_n, gather_src, gather_out);
  else
    onesweep_run<16>(ka, va, kb, vb, n, passes, identity_vals, w, st, keys_res, vals_res, d_n, gather_src, gather_out);
}

}  // namespace tide
