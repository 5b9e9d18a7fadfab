// Device-wide exclusive scan and stable LSD radix sort for wave64 (gfx950).
//
// Scan: reduce-then-scan over tiles of 4096 elements (256 lanes x 16
// consecutive items, moved in 16-byte pieces when the arrays are 16-byte
// aligned); with at most 1024 tiles each tile adds up its
// predecessors' sums itself, else one workgroup scans the tile sums.
// Radix sort: 8-bit digits; per tile 256-bin LDS histograms (one per wave,
// added at the end), a bin-major scan of the per-tile histograms, then a
// stable scatter whose in-tile ranks
// come from ballot-based peer masks (a wave sees 64 consecutive keys per
// round, so rank = keys of the same digit in earlier waves + earlier rounds +
// lower lanes).  Equal keys keep their input order, which is what makes the
// (tile, depth, pidx) order of the binning total.
#pragma once

#include "common.h"

namespace tide {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;       // 4
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;  // 4096
constexpr int kXcds = 8;                               // workgroup b starts on XCD b % 8
constexpr int64_t kRadixMaxGrid = 8192;                // radix histogram workgroups at most

// ------------------------------------------------------------------ scan
// Input functors: value of element i as u32; load4 reads elements i..i+3
// with one 16-byte load (i a multiple of 4, used only when aligned() holds).
__device__ inline uint4 ld4(const uint32_t* p) { return *reinterpret_cast<const uint4*>(p); }
struct ArrayIn {
  const uint32_t* a;
  __device__ uint32_t operator()(int64_t i) const { return a[i]; }
  __device__ void load4(int64_t i, uint32_t* v) const {
    const uint4 q = ld4(a + i);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  bool aligned() const { return ((uintptr_t)a & 15) == 0; }
};
struct NonzeroIn {
  const uint32_t* a;
  __device__ uint32_t operator()(int64_t i) const { return a[i] != 0u ? 1u : 0u; }
  __device__ void load4(int64_t i, uint32_t* v) const {
    const uint4 q = ld4(a + i);
    v[0] = q.x != 0u; v[1] = q.y != 0u; v[2] = q.z != 0u; v[3] = q.w != 0u;
  }
  bool aligned() const { return ((uintptr_t)a & 15) == 0; }
};

// Output sinks: element i with exclusive prefix `off` and value v; store4
// writes elements i..i+3 (as load4).
struct OffsetsOut {   // out[i] = off
  uint32_t* out;
  __device__ void operator()(int64_t i, uint32_t off, uint32_t) const { out[i] = off; }
  __device__ void store4(int64_t i, const uint32_t* off, const uint32_t*) const {
    *reinterpret_cast<uint4*>(out + i) = make_uint4(off[0], off[1], off[2], off[3]);
  }
  bool aligned() const { return ((uintptr_t)out & 15) == 0; }
};

// Extras written by whichever block holds the total: a u32 copy of it,
// end[n] = total (the closing offset of an offsets array), and a copy of
// copy_n u64 words from copy_src (read after the total is stored, so it may
// include it) to copy_dst (say, pinned host memory the host reads after an
// event: no copy kernel needed).
struct ScanTail {
  uint32_t* total32 = nullptr;
  uint32_t* end = nullptr;
  const unsigned long long* copy_src = nullptr;
  unsigned long long* copy_dst = nullptr;
  int copy_n = 0;
};

// Element counts: n_max bounds the launch; when d_n is given the kernels
// read the actual count from device memory (n = min(n_max, *d_n)), which
// lets a pipeline size its grids without a host round trip.
__device__ inline int64_t dev_count(int64_t n_max, const unsigned long long* d_n) {
  if (!d_n) return n_max;
  const int64_t n = (int64_t)*d_n;
  return n < n_max ? n : n_max;
}

// A thread's kScanItems consecutive elements: 16-byte loads when kVec and
// the whole run lies below n, else one element at a time (zero past n).
template <bool kVec, typename In>
__device__ inline void scan_items(const In& in, int64_t base, int64_t n, uint32_t* v) {
  if (kVec && base + kScanItems <= n) {
#pragma unroll
    for (int j = 0; j < kScanItems; j += 4) in.load4(base + j, v + j);
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? in(base + k) : 0u;
  }
}

template <typename In, bool kVec>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(In in, int64_t n_max, const unsigned long long* d_n,
                                                              unsigned long long* partial) {
  const int64_t n = dev_count(n_max, d_n);
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  scan_items<kVec>(in, base, n, v);
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) s += v[k];
  s = wave_sum(s);
  __shared__ unsigned long long ws[kScanThreads / kWave];
  if (__lane_id() == 0) ws[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += ws[w];
    partial[blockIdx.x] = t;
  }
}

// One workgroup scans partial[0..nb) in place (exclusive) and writes the
// total and the tail (n as for dev_count).
__global__ void __launch_bounds__(1024) k_scan_partials(unsigned long long* partial, int64_t nb,
                                                        unsigned long long* total, ScanTail tail, int64_t n_max,
                                                        const unsigned long long* d_n);

__device__ inline void write_tail(const ScanTail& tail, unsigned long long t, int64_t n) {
  if (tail.total32) *tail.total32 = (uint32_t)t;
  if (tail.end) tail.end[n] = (uint32_t)t;
  for (int k = 0; k < tail.copy_n; ++k) tail.copy_dst[k] = tail.copy_src[k];
}

// kSums: partial holds the blocks' sums (not yet scanned); each block adds
// up its predecessors' itself and block 0 writes the total (one launch
// fewer; used when there are at most 1024 blocks).
template <typename In, bool kSums, typename Out, bool kVec>
__global__ void __launch_bounds__(kScanThreads) k_scan_down(In in, int64_t n_max, const unsigned long long* d_n,
                                                            const unsigned long long* partial,
                                                            Out out, int64_t nb,
                                                            unsigned long long* total, ScanTail tail) {
  const int64_t n = dev_count(n_max, d_n);
  __shared__ unsigned long long bpre[kScanThreads / kWave + 1];
  if (kSums) {
    // predecessors' sums (and, in block 0, all the sums for the total)
    const int64_t upto = blockIdx.x == 0 ? nb : (int64_t)blockIdx.x;
    unsigned long long a = 0;
    for (int64_t q = threadIdx.x; q < upto; q += kScanThreads) a += partial[q];
    a = wave_sum(a);
    if (__lane_id() == 0) bpre[threadIdx.x / kWave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long t = 0;
      for (int q = 0; q < kScanThreads / kWave; ++q) t += bpre[q];
      if (blockIdx.x == 0) {
        *total = t;
        write_tail(tail, t, n);
      }
      bpre[kScanThreads / kWave] = blockIdx.x == 0 ? 0ull : t;
    }
    __syncthreads();
  }
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  scan_items<kVec>(in, base, n, v);
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) s += v[k];
  // exclusive scan of the 256 thread sums
  const uint32_t inc = wave_incl_scan(s);
  __shared__ uint32_t wtot[kScanThreads / kWave];
  const int w = threadIdx.x / kWave;
  if (__lane_id() == kWave - 1) wtot[w] = inc;
  __syncthreads();
  uint32_t wpre = 0;
  for (int q = 0; q < w; ++q) wpre += wtot[q];
  const unsigned long long bp = kSums ? bpre[kScanThreads / kWave] : partial[blockIdx.x];
  uint32_t run = (uint32_t)bp + wpre + inc - s;
  if (kVec && base + kScanItems <= n) {
    uint32_t o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      o[k] = run;
      run += v[k];
    }
#pragma unroll
    for (int j = 0; j < kScanItems; j += 4) out.store4(base + j, o + j, v + j);
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (base + k < n) out(base + k, run, v[k]);
      run += v[k];
    }
  }
}

// Exclusive scan of in(0..n) into the sink out; total (u64, device)
// receives the sum, and the tail its extras.  partial needs
// ceil(n_max/4096) u64 entries; d_n as for dev_count.
template <typename In, typename Out>
inline void scan_to(In in, int64_t n, Out out, unsigned long long* partial, unsigned long long* total,
                    hipStream_t st, const unsigned long long* d_n = nullptr, ScanTail tail = ScanTail{}) {
  const int64_t nb = ceil_div(n > 0 ? n : 1, kScanTile);
  const bool vec = in.aligned() && out.aligned();
  if (vec)
    hipLaunchKernelGGL((k_scan_reduce<In, true>), dim3((uint32_t)nb), dim3(kScanThreads), 0, st, in, n, d_n, partial);
  else
    hipLaunchKernelGGL((k_scan_reduce<In, false>), dim3((uint32_t)nb), dim3(kScanThreads), 0, st, in, n, d_n, partial);
  if (nb <= 1024) {
    if (vec)
      hipLaunchKernelGGL((k_scan_down<In, true, Out, true>), dim3((uint32_t)nb), dim3(kScanThreads), 0, st, in, n, d_n,
                         (const unsigned long long*)partial, out, nb, total, tail);
    else
      hipLaunchKernelGGL((k_scan_down<In, true, Out, false>), dim3((uint32_t)nb), dim3(kScanThreads), 0, st, in, n,
                         d_n, (const unsigned long long*)partial, out, nb, total, tail);
    return;
  }
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, partial, nb, total, tail, n, d_n);
  if (vec)
    hipLaunchKernelGGL((k_scan_down<In, false, Out, true>), dim3((uint32_t)nb), dim3(kScanThreads), 0, st, in, n, d_n,
                       (const unsigned long long*)partial, out, nb, total, tail);
  else
    hipLaunchKernelGGL((k_scan_down<In, false, Out, false>), dim3((uint32_t)nb), dim3(kScanThreads), 0, st, in, n,
                       d_n, (const unsigned long long*)partial, out, nb, total, tail);
}

// Exclusive scan into an offsets array.
template <typename In>
inline void scan_exclusive(In in, int64_t n, uint32_t* out, unsigned long long* partial,
                           unsigned long long* total, hipStream_t st, const unsigned long long* d_n = nullptr,
                           ScanTail tail = ScanTail{}) {
  scan_to(in, n, OffsetsOut{out}, partial, total, st, d_n, tail);
}

inline size_t scan_partial_count(int64_t n) { return (size_t)ceil_div(n > 0 ? n : 1, kScanTile); }

// ------------------------------------------------------------- radix sort
inline size_t radix_hist_count(int64_t n) { return 256 * (size_t)ceil_div(n > 0 ? n : 1, kSortTile); }

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

// Shared LDS of a sort tile's ranking and scatter (tiles of 64 W R keys:
// W waves of R rounds).
template <int R, int W = kSortWaves>
struct TileLds {
  uint32_t wcnt[W][256];
  uint32_t gbase[256], lstart[256], wsum[4];
  uint32_t skey[kWave * W * R], sval[kWave * W * R];
};

// Ranks the keys of tile [b0, b0 + 64 W R) ∩ [0, n) by digit (key >> shift)
// & 255: wave w holds R rounds of 64 consecutive keys; rank[r] is the key's
// rank among the keys of its digit held by the wave in earlier rounds and
// lower lanes, and L.wcnt[w][d] ends as the wave's count of digit d.
// L.wcnt must be zero on entry; the caller synchronises afterwards.
template <int R, int W>
__device__ __forceinline__ void tile_rank(const uint32_t* keys_in, const uint32_t* vals_in, int64_t n, int64_t b0,
                                          int shift, TileLds<R, W>& L, uint32_t* key, uint32_t* val, uint32_t* rank) {
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

// Thread d < 256: turns L.wcnt[.][d] into the waves' offsets within digit
// d, writes the digit's start in the tile to L.lstart[d] and returns the
// tile's count of digit d (threads from 256 on return 0).  Synchronises.
template <int R, int W>
__device__ __forceinline__ uint32_t tile_digit_offsets(TileLds<R, W>& L) {
  const int d = threadIdx.x, w = threadIdx.x / kWave, lane = __lane_id();
  const bool dig = d < 256;
  uint32_t cnt = 0;
  if (dig) {
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const uint32_t c = L.wcnt[q][d];
      L.wcnt[q][d] = cnt;
      cnt += c;
    }
  }
  const uint32_t inc = wave_incl_scan(cnt);
  if (dig && lane == kWave - 1) L.wsum[w] = inc;
  __syncthreads();
  if (dig) {
    uint32_t pre = 0;
    for (int q = 0; q < w; ++q) pre += L.wsum[q];
    L.lstart[d] = pre + inc - cnt;
  }
  return cnt;
}

// Places the ranked keys in LDS in (digit, rank) order (L.lstart and L.wcnt
// must be visible).
template <int R, int W>
__device__ __forceinline__ void tile_stage(int64_t n, int64_t b0, int shift, TileLds<R, W>& L, const uint32_t* key,
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
// staged keys must be visible): out(position, key, value) stores one.
template <int R, int W, typename Out>
__device__ __forceinline__ void tile_write(int m, int shift, const TileLds<R, W>& L, const Out& out) {
  for (int j = threadIdx.x; j < m; j += kWave * W) {
    const uint32_t k = L.skey[j];
    const uint32_t dd = (k >> shift) & 255u;
    out(L.gbase[dd] + (uint32_t)j - L.lstart[dd], k, L.sval[j]);
  }
}

// The plain output of a pass: key and value, and with gather_src also
// gather_out[position] = gather_src[value].
struct PairsOut {
  uint32_t* keys;
  uint32_t* vals;
  const uint32_t* gather_src;
  uint32_t* gather_out;
  __device__ void operator()(uint32_t pos, uint32_t k, uint32_t v) const {
    keys[pos] = k;
    vals[pos] = v;
    if (gather_src) gather_out[pos] = gather_src[v];
  }
};

// Sorts (keys, vals) stably by bits [0, bits) of the key, 8 bits per pass.
// Input in (ka, va); with identity_vals the input values are taken to be
// the input indices and va is only used as storage.  Buffers (ka, va) and
// (kb, vb) ping-pong; the sorted result pointers are returned through
// *keys_res / *vals_res.  hist needs radix_hist_count(n) u32, partial
// scan_partial_count(radix_hist_count(n)) u64, total one u64 (two with d_n:
// then only the tiles that hold the device count's keys are counted,
// scanned and scattered, the second u64 holding the scan's length).  With
// gather_src, the last pass also writes gather_out[j] = gather_src[value j]
// for every sorted position j.  With xcd_order the scatter's tiles are
// assigned so that each XCD writes a contiguous eighth of them.
void radix_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t n, int bits,
                      bool identity_vals, uint32_t* hist, unsigned long long* partial,
                      unsigned long long* total, hipStream_t st, uint32_t** keys_res,
                      uint32_t** vals_res, const unsigned long long* d_n = nullptr,
                      const uint32_t* gather_src = nullptr, uint32_t* gather_out = nullptr,
                      bool xcd_order = false);

// ------------------------------------------------- one-sweep radix sort
// The same stable LSD sort with one kernel per 8-bit pass.  A first kernel
// counts every pass's digits over all keys at once (LDS bins per block,
// added to global counts with device-scope atomics).  Each pass kernel then
// ranks its 4096-key tile as k_radix_scatter does, publishes its digit
// counts, and finds the counts of all earlier tiles by walking back over
// their published words until one holds an inclusive prefix (decoupled
// look-back, kOsWindow words per poll).  A tile publishes its own counts
// before it waits on anyone and workgroups start in index order on each
// XCD, so every wait ends; the walk also gives up after kOsSpinLimit polls
// of one word and sets an error word (the output is then wrong, but every
// write stays in bounds), so no kernel spins without end.  Used where the
// keys are few (the depth sort of the visible pairs): there the two
// launches per pass that it saves weigh more than the look-back.
//
// Control words: kOsCtlLen u32 that must read zero when the sort starts
// (an earlier kernel on the stream clears them).  The global digit counts
// are kept in kOsCopies copies (histogram block b adds to copy
// b % kOsCopies, which spreads the atomics), ctl[kOsCtlWords +
// (kOsMaxPasses c + p) 256 + d] being copy c of pass p's count of digit d.
constexpr int kOsCtlWords = 8;
constexpr int kOsMaxPasses = 4;
constexpr int kOsCopies = 8;
constexpr int kOsCtlLen = kOsCtlWords + kOsCopies * kOsMaxPasses * 256;
constexpr int kOsHistBlocks = 1024;
constexpr int kOsWindow = 4;
constexpr uint32_t kOsSpinLimit = 1u << 20;

struct OsWork {
  uint32_t* ctl;                  // kOsCtlLen u32, zero at the start
  unsigned long long* status;     // onesweep_status_count(n, passes)
  uint32_t* err;                  // set to nonzero if a look-back gave up
};

// Look-back words of a sort of n keys in tiles of tile_keys keys.
inline size_t onesweep_status_count(int64_t n, int passes, int64_t tile_keys) {
  return (size_t)passes * 256 * (size_t)ceil_div(n > 0 ? n : 1, tile_keys);
}

// The sort itself: onesweep_sort_pairs in onesweep.h.

}  // namespace tide
