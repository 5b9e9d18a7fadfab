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

// Per-tile digit histogram.  Each wave counts into bins of its own, a
// thread takes four consecutive keys per load (16 bytes when kVec: the keys
// are 16-byte aligned) and adds equal neighbouring digits as one run, and the
// waves' bins are added at the end.  Workgroup b takes tiles b, b + G, ...
// (G the grid), so a grid sized for a large capacity costs little when the
// count on the device is small.
template <bool kVec>
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint32_t* keys, int64_t n_max,
                                                             const unsigned long long* d_n, int shift,
                                                             uint32_t* ghist, int64_t nb,
                                                             unsigned long long* nscan) {
  const int64_t n = dev_count(n_max, d_n);
  // with the count on the device, only its tiles count (the layout's stride
  // is their number, and the scan reads its length from nscan)
  const int64_t nba = d_n ? (n + kSortTile - 1) / kSortTile : nb;
  if (nscan && blockIdx.x == 0 && threadIdx.x == 0) *nscan = 256ull * (unsigned long long)nba;
  __shared__ uint32_t h[kSortWaves][256];
  uint32_t* hw = h[threadIdx.x / kWave];
  for (int64_t tile = blockIdx.x; tile < nba; tile += gridDim.x) {
    for (int k = threadIdx.x; k < kSortWaves * 256; k += kSortThreads) (&h[0][0])[k] = 0;
    __syncthreads();
    const int64_t base = tile * kSortTile;
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
    ghist[(int64_t)threadIdx.x * nba + tile] = c;
    __syncthreads();
  }
}

// The scatter's 4096-key tiles as eight waves of eight rounds: a tile's
// ranking is a chain of rounds, and eight waves ran the two tile-sort passes
// over 14 M keys in 56.5 + 60.6 us against 61.4 + 66.8 us with four.
constexpr int kScatterWaves = 8;
constexpr int kScatterRounds = kSortTile / (kWave * kScatterWaves);

__global__ void __launch_bounds__(kWave * kScatterWaves) k_radix_scatter(const uint32_t* keys_in,
                                                                const uint32_t* vals_in, int64_t n_max,
                                                                const unsigned long long* d_n, int shift,
                                                                const uint32_t* gofs, int64_t nb,
                                                                uint32_t* keys_out, uint32_t* vals_out,
                                                                const uint32_t* gather_src, uint32_t* gather_out,
                                                                int xcd_order) {
  const int64_t n = dev_count(n_max, d_n);
  const int64_t nba = d_n ? (n + kSortTile - 1) / kSortTile : nb;   // the tiles that hold keys
  // with xcd_order, workgroup b (which starts on XCD x = b % 8) takes tile
  // x q + min(x, r) + b / 8 of the nba = 8 q + r tiles that hold keys, if
  // b / 8 is below XCD x's share (q, plus one for x < r; every such b is
  // below nba): each XCD sorts a contiguous eighth of the tiles, so the runs
  // of one digit that consecutive tiles write side by side meet in the same
  // L2.  (One workgroup per tile: taking several tiles per workgroup from a
  // smaller grid was slower, 576 against 663 us per pass over 101 M keys.)
  int64_t tile = blockIdx.x;
  if (xcd_order) {
    const int64_t q = nba / kXcds, r = nba % kXcds, x = blockIdx.x % kXcds, k = blockIdx.x / kXcds;
    if (k >= q + (x < r ? 1 : 0)) return;
    tile = x * q + (x < r ? x : r) + k;
  }
  if (tile >= nba) return;
  const int64_t b0 = tile * kSortTile;
  const int m = (int)(n - b0 < kSortTile ? n - b0 : kSortTile);   // elements of this tile
  __shared__ TileLds<kScatterRounds, kScatterWaves> L;
  for (int k = threadIdx.x; k < kScatterWaves * 256; k += kWave * kScatterWaves) (&L.wcnt[0][0])[k] = 0;
  if (threadIdx.x < 256) L.gbase[threadIdx.x] = gofs[(int64_t)threadIdx.x * nba + tile];
  __syncthreads();
  uint32_t key[kScatterRounds], val[kScatterRounds], rank[kScatterRounds];
  tile_rank(keys_in, vals_in, n, b0, shift, L, key, val, rank);
  __syncthreads();
  tile_digit_offsets(L);
  __syncthreads();
  tile_stage(n, b0, shift, L, key, val, rank);
  __syncthreads();
  tile_write(m, shift, L, PairsOut{keys_out, vals_out, gather_src, gather_out});
}

void radix_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t n, int bits,
                      bool identity_vals, uint32_t* hist, unsigned long long* partial,
                      unsigned long long* total, hipStream_t st, uint32_t** keys_res,
                      uint32_t** vals_res, const unsigned long long* d_n, const uint32_t* gather_src,
                      uint32_t* gather_out, bool xcd_order) {
  uint32_t *ki = ka, *vi = va, *ko = kb, *vo = vb;
  bool ident = identity_vals;
  const int64_t nb = ceil_div(n > 0 ? n : 1, kSortTile);
  // the histogram's grid: one workgroup per tile up to kRadixMaxGrid,
  // beyond that tiles per workgroup (the scatter keeps one per tile)
  const int64_t grid = nb < kRadixMaxGrid ? nb : kRadixMaxGrid;
  if (n > 0) {
    for (int shift = 0; shift < bits; shift += 8) {
      unsigned long long* nscan = d_n ? total + 1 : nullptr;
      if (((uintptr_t)ki & 15) == 0)
        hipLaunchKernelGGL(k_radix_hist<true>, dim3((uint32_t)grid), dim3(kSortThreads), 0, st, ki, n, d_n, shift, hist,
                           nb, nscan);
      else
        hipLaunchKernelGGL(k_radix_hist<false>, dim3((uint32_t)grid), dim3(kSortThreads), 0, st, ki, n, d_n, shift, hist,
                           nb, nscan);
      scan_exclusive(ArrayIn{hist}, 256 * nb, hist, partial, total, st, nscan);
      const bool last = shift + 8 >= bits;
      hipLaunchKernelGGL(k_radix_scatter, dim3((uint32_t)nb), dim3(kWave * kScatterWaves), 0, st, ki,
                         ident ? nullptr : vi, n,
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

}  // namespace tide
