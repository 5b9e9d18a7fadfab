// Backward half of the rasterizer: compositing adjoint per tile, per-pair
// reduction of the per-instance 2-D gradients in a fixed order, and the
// adjoint of projection / EWA / activations / SH.  No floating-point atomics:
// every sum has one fixed order, so two runs give identical bits.
#include "prims.h"
#include "raster.h"

namespace tide {

constexpr int kG2 = 9;  // du, dv, dA, dB, dC, dopacity, dr, dg, db
// Colour columns whose Adam state the fused update loads together: four keep
// the kernel within 128 registers (four waves per SIMD) with no spills, and
// ran the fused kernel in 0.183 ms against 0.212 ms one column at a time.
constexpr int kMvGroup = 4;

// A per-instance record of the kG2 partials, aligned only to its element:
// accessed as one object, the compiler moves it in 16-byte pieces.
template <typename T>
struct __attribute__((aligned(sizeof(T)))) Rec9 {
  T v[kG2];
};

// ----------------------------------------------------- compositing adjoint
// Same lane/pixel layout as the forward.  Each pixel walks back from its
// last contributor, recovering T_i = T_{i+1} / (1 - alpha_i) and the
// normalised colour behind the entry (r_{i-1} = alpha_i c_i + (1-alpha_i) r_i,
// starting from the background).  The per-pixel update is branch-free; the
// four pixels of a lane are summed in registers, each row of 16 lanes is
// reduced with DPP and the four row sums are parked in LDS; once a batch of
// 32 entries is done, lane k adds entry k's four row sums, applies the
// entry's factors (opacity, conic) and stores its partial.  (Batches of 32 keep the parked sums at the LDS size that 64
// entries with rows added in pairs took, so occupancy is unchanged, and each
// taken entry saves the nine pair additions.)  Entries no pixel reaches get
// zero partials.
template <typename T>
__global__ void __launch_bounds__(64) k_render_bwd(const uint32_t* __restrict__ order,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ inst_e,
                                                   const uint32_t* __restrict__ inst_rec, const T* __restrict__ rec,
                                                   int32_t Tx, int32_t Ty, int32_t W, int32_t H, T bg0, T bg1,
                                                   T bg2, const T* __restrict__ tfin,
                                                   const uint32_t* __restrict__ last_in,
                                                   const T* __restrict__ dimg, T* __restrict__ partial) {
  const int nt = Tx * Ty;
  const int g = (int)order[blockIdx.x];
  const int c = g / nt, t = g - c * nt;
  const int tx = t % Tx, ty = t / Tx;
  const int lane = threadIdx.x;
  const int px = tx * kTile + (lane & 15);
  const int py0 = ty * kTile + (lane >> 4);
  const T fxp = (T)px + (T)0.5;
  const int64_t HW = (int64_t)H * W;
  // Pb = -(colour behind the current entry) . dL/dpixel, per pixel: the only
  // way the backward needs the colour behind, so it is carried as one scalar.
  T fyp[4], Tr[4], g0[4], g1[4], g2[4], Pb[4];
  uint32_t lst[4];
  uint32_t maxl = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int py = py0 + 4 * q;
    fyp[q] = (T)py + (T)0.5;
    if (px < W && py < H) {
      const int64_t p = (int64_t)py * W + px;
      Tr[q] = tfin[(int64_t)c * HW + p];
      lst[q] = last_in[(int64_t)c * HW + p];
      g0[q] = dimg[((int64_t)c * 3 + 0) * HW + p];
      g1[q] = dimg[((int64_t)c * 3 + 1) * HW + p];
      g2[q] = dimg[((int64_t)c * 3 + 2) * HW + p];
    } else {
      Tr[q] = 1; lst[q] = 0; g0[q] = g1[q] = g2[q] = 0;
    }
    Pb[q] = -(bg0 * g0[q] + bg1 * g1[q] + bg2 * g2[q]);
    maxl = lst[q] > maxl ? lst[q] : maxl;
  }
  // red and green are reduced together (row_pair_sum_to_15): an odd lane
  // carries green in g0 and red in g1, so its first accumulator sums green
  const bool odd = (lane & 1) != 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const T a = g0[q], b = g1[q];
    g0[q] = odd ? b : a;
    g1[q] = odd ? a : b;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t o = __shfl_xor(maxl, off, kWave);
    maxl = o > maxl ? o : maxl;
  }
  const uint32_t start = ranges[2 * g], end = ranges[2 * g + 1];
  for (uint32_t j = start + maxl + lane; j < end; j += 64) {
    Rec9<T> z;
#pragma unroll
    for (int m = 0; m < kG2; ++m) z.v[m] = 0;
    *reinterpret_cast<Rec9<T>*>(partial + (int64_t)inst_e[j] * kG2) = z;
  }
  __shared__ T s_u[64], s_v[64], s_Ah[64], s_Bh[64], s_Ch[64], s_A[64], s_B[64], s_C[64], s_o[64], s_r[64],
      s_g[64], s_b[64];
  __shared__ T s_part[32][4][kG2];   // per entry, the sums of the four rows

  const T ks = (T)Ex<T>::k;
  // The batch ending at h covers entries [max(h - 32, 0), h).  An entry's
  // record lies two indices deep (its emission index, then that emission's
  // record); both are loaded a batch ahead (e_c, r_c for this batch, e_n,
  // r_n for the next), so a batch waits only for its records' fields.
  uint32_t e_c = 0, r_c = 0, e_n = 0, r_n = 0;
  {
    const int32_t h0 = (int32_t)maxl, h1 = h0 - 32;
    const int32_t l0 = h0 - 32 > 0 ? h0 - 32 : 0, l1 = h1 - 32 > 0 ? h1 - 32 : 0;
    const bool v0 = h0 > 0 && lane < h0 - l0, v1 = h1 > 0 && lane < h1 - l1;
    if (v0) e_c = inst_e[start + l0 + lane];
    if (v1) e_n = inst_e[start + l1 + lane];
    if (v0) r_c = inst_rec[e_c];
    if (v1) r_n = inst_rec[e_n];
  }
  for (int32_t hi = (int32_t)maxl; hi > 0; hi -= 32) {
    const int32_t lo = hi - 32 > 0 ? hi - 32 : 0;
    const int32_t n = hi - lo;
    const int32_t h2 = hi - 64, l2 = h2 - 32 > 0 ? h2 - 32 : 0;
    const bool v2 = h2 > 0 && lane < h2 - l2;
    uint32_t e2 = 0;
    if (v2) e2 = inst_e[start + l2 + lane];
    uint32_t my_e = 0;
    bool may = false;
    if (lane < n) {
      my_e = e_c;
      const T* q = rec + (int64_t)r_c * kRec;
      s_u[lane] = q[0]; s_v[lane] = q[1];
      s_A[lane] = q[2]; s_B[lane] = q[3]; s_C[lane] = q[4];
      s_Ah[lane] = (T)-0.5 * ks * q[2]; s_Bh[lane] = -ks * q[3]; s_Ch[lane] = (T)-0.5 * ks * q[4];
      s_o[lane] = q[5]; s_r[lane] = q[6]; s_g[lane] = q[7]; s_b[lane] = q[8];
      may = tile_may_take<T>(q[0], q[1], q[2], q[3], q[4], q[5], tx, ty);
    }
    // entries some pixel centre of the tile may take (the forward's test),
    // walked from the back; hit: the entries some pixel took
    uint64_t rest = __ballot(may), hit = 0;
    __syncthreads();
    while (rest != 0) {
      const int k = 63 - __builtin_clzll(rest);
      rest &= ~(1ull << k);
      const uint32_t pos = (uint32_t)(lo + k);
      const T v = s_v[k], Ch = s_Ch[k], op = s_o[k];
      const T cr = s_r[k], cg = s_g[k], cb = s_b[k];
      const T c0 = odd ? cg : cr, c1 = odd ? cr : cg;   // in the lane's g0/g1 order
      const T dx = fxp - s_u[k];
      const T adx2 = s_Ah[k] * dx * dx, bdx = s_Bh[k] * dx;
      // G first: an entry no pixel takes (pass and before the pixel's last
      // contributor) leaves every pixel's state and the entry's partial at
      // zero, so the wave skips the rest.
      // (each comparison balloted on its own: see the forward)
      T Gq[4];
      bool okq[4];
      uint64_t qm[4], hit_m = 0;   // per pixel row q, the lanes whose pixel takes the entry
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T araw, alpha;
        bool in_power, in_alpha;
        entry_alpha_tests<T>(adx2, bdx, Ch, op, fyp[q] - v, Gq[q], araw, alpha, in_power, in_alpha);
        const bool before_last = pos < lst[q];
        okq[q] = in_power && in_alpha && before_last;
        qm[q] = __ballot(in_power) & __ballot(in_alpha) & __ballot(before_last);
        hit_m |= qm[q];
      }
      if (hit_m == 0) continue;
      hit |= 1ull << k;
      // Per pixel, t = dL/dalpha G is the opacity gradient's share and
      // opacity t = dL/dpower (alpha below the clamp), so the power's
      // moments over dy are summed without the opacity and the entry's
      // factors are applied once, in the batch's store below.  A lane's four
      // pixels share dx: d/du = op (A dx S0 + B S1), d/dv = op (B dx S0 + C S1),
      // d/dA = -op dx^2 S0 / 2, d/dB = -op dx S1, d/dC = -op S2 / 2, with
      // S0 = sum t, S1 = sum t dy, S2 = sum t dy^2.
      // A pixel row (q: rows q*4 .. q*4+3 of the tile, one per lane row) in
      // which no pixel takes the entry is passed over: its update would
      // leave every state as it is (a_ok = 0, t = 0).
      T S0 = 0, S1 = 0, S2 = 0, a_0 = 0, a_1 = 0, a_b = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (qm[q] == 0) continue;
        const T dy = fyp[q] - v;
        const T G = Gq[q];
        const T araw = op * G;
        const bool below = araw < (T)0.99;
        const T alpha = alpha_clamped(araw, below);
        const bool ok = okq[q];
        const bool okg = ok && below;   // alpha clamped at 0.99: no input dependence
        const T a_ok = ok ? alpha : (T)0;
        const T G_ok = okg ? G : (T)0;
        // a pixel the entry does not reach keeps its T: a_ok = 0 and the
        // hardware reciprocal of 1 is exactly 1 (exact at powers of two), so
        // no select is needed after the product
        const T Tn = Tr[q] * Mth<T>::rcp_fast((T)1 - a_ok);
        Tr[q] = Tn;
        const T w = a_ok * Tn;
        a_0 += w * g0[q]; a_1 += w * g1[q]; a_b += w * g2[q];
        const T e = c0 * g0[q] + (c1 * g1[q] + (cb * g2[q] + Pb[q]));   // (c - behind) . dL/dpixel
        const T dal = Tn * e;
        Pb[q] -= a_ok * e;
        const T t = dal * G_ok;
        S0 += t;
        const T tdy = t * dy;
        S1 += tdy; S2 += tdy * dy;
      }
      T p1 = dx * S0;
      T a_A = dx * p1, a_B = dx * S1, a_C = S2;
      T q_r, q_g;
      p1 = row_sum_to_15(p1); S1 = row_sum_to_15(S1); a_A = row_sum_to_15(a_A);
      a_B = row_sum_to_15(a_B); a_C = row_sum_to_15(a_C); S0 = row_sum_to_15(S0);
      row_pair_sum_to_15(a_0, a_1, q_r, q_g);
      a_b = row_sum_to_15(a_b);
      if ((lane & 15) == 15) {
        T* S = s_part[k][lane >> 4];
        S[0] = p1; S[1] = S1; S[2] = a_A; S[3] = a_B; S[4] = a_C;
        S[5] = S0; S[6] = q_r; S[7] = q_g; S[8] = a_b;
      }
    }
    __syncthreads();
    if (lane < n) {
      Rec9<T> r;
      if ((hit >> lane) & 1u) {
#pragma unroll
        for (int m = 0; m < kG2; ++m)
          r.v[m] = (s_part[lane][0][m] + s_part[lane][1][m]) + (s_part[lane][2][m] + s_part[lane][3][m]);
        // dpower/du = A dx + B dy, dpower/dv = B dx + C dy, dpower/dA =
        // -dx^2/2, dpower/dB = -dx dy, dpower/dC = -dy^2/2; dL/dpower =
        // opacity t
        const T op = s_o[lane], p1 = r.v[0], s1 = r.v[1];
        r.v[0] = op * (s_A[lane] * p1 + s_B[lane] * s1);
        r.v[1] = op * (s_B[lane] * p1 + s_C[lane] * s1);
        r.v[2] *= (T)-0.5 * op;
        r.v[3] *= -op;
        r.v[4] *= (T)-0.5 * op;
      } else {
#pragma unroll
        for (int m = 0; m < kG2; ++m) r.v[m] = 0;
      }
      *reinterpret_cast<Rec9<T>*>(partial + (int64_t)my_e * kG2) = r;
    }
    uint32_t r2 = 0;
    if (v2) r2 = inst_rec[e2];
    e_c = e_n; r_c = r_n;
    e_n = e2; r_n = r2;
    __syncthreads();
  }
}

// ---------------------------------------------- per-pair reduction (fixed order)
// One DPP step of a segmented inclusive scan: each lane adds the source
// lane's values where that lane is in the same segment (segments are runs of
// equal p; a source the pattern leaves out reads -2, which no p equals).
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_val(float x) {
  return __uint_as_float(dpp_u32<CTRL, ROWS>(0u, __float_as_uint(x)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_val(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const uint32_t lo = dpp_u32<CTRL, ROWS>(0u, (uint32_t)b), hi = dpp_u32<CTRL, ROWS>(0u, (uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ void seg_step(int p, T (&v)[kG2]) {
  const bool same = (int)dpp_u32<CTRL, ROWS>((uint32_t)-2, (uint32_t)p) == p;
#pragma unroll
  for (int m = 0; m < kG2; ++m) {
    const T y = dpp_val<CTRL, ROWS>(v[m]);
    v[m] = same ? v[m] + y : v[m];
  }
}

// Per visible pair, the sum of its instances' partials; one wave64 workgroup
// per 64 consecutive depth-ordered visible pairs.  Their partials are
// contiguous ([inst_off[s0], inst_off[s0 + 64])), so the wave
// walks them 64 instances at a time with coalesced loads; each lane finds its
// pair by binary search over the 64 offsets, a segmented inclusive scan in
// DPP (row shifts 1, 2, 4, 8, then the broadcasts of lanes 15 and 31; no LDS
// round trips) sums equal-pair lanes, and the last lane of each segment adds
// into that pair's LDS accumulator.  A pair gets at most one add per step and
// steps run in order, so the sums are deterministic.  Balanced whatever the
// footprint sizes.
template <typename T>
__global__ void __launch_bounds__(64) k_reduce_pairs(const uint32_t* __restrict__ vis_rec,
                                                     const uint32_t* __restrict__ inst_off, int64_t n_vis,
                                                     int64_t n_rec, const T* __restrict__ partial,
                                                     T* __restrict__ g2d) {
  const int lane = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * kWave;
  const int np = (int)(n_vis - s0 < kWave ? n_vis - s0 : kWave);
  __shared__ uint32_t s_off[kWave + 1];
  __shared__ T s_acc[kWave][kG2];
  if (lane <= np) s_off[lane] = inst_off[s0 + lane];
  if (lane == 0 && np == kWave) s_off[kWave] = inst_off[s0 + kWave];
#pragma unroll
  for (int m = 0; m < kG2; ++m) s_acc[lane][m] = 0;
  __syncthreads();
  const uint32_t e0 = s_off[0], e1 = s_off[np];
  for (uint32_t base = e0; base < e1; base += kWave) {
    const uint32_t e = base + (uint32_t)lane;
    const bool valid = e < e1;
    int lo = 0, hi = np;   // s_off[lo] <= e < s_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_off[mid] <= e) lo = mid;
      else hi = mid;
    }
    const int p = valid ? lo : -1;
    // one record load (a lane's 36 bytes as two 16-byte loads and one
    // 4-byte load: nine single loads at a 36-byte stride made every load
    // instruction touch 36 cache segments)
    const Rec9<T> rec = *reinterpret_cast<const Rec9<T>*>(partial + (int64_t)(valid ? e : e0) * kG2);
    T v[kG2];
#pragma unroll
    for (int m = 0; m < kG2; ++m) v[m] = valid ? rec.v[m] : (T)0;
    seg_step<0x111, 0xF>(p, v);   // row_shr:1
    seg_step<0x112, 0xF>(p, v);   // row_shr:2
    seg_step<0x114, 0xF>(p, v);   // row_shr:4
    seg_step<0x118, 0xF>(p, v);   // row_shr:8
    seg_step<0x142, 0xA>(p, v);   // row_bcast:15 into rows 1 and 3
    seg_step<0x143, 0xC>(p, v);   // row_bcast:31 into rows 2 and 3
    const bool seg_end = valid && (lane == kWave - 1 || e + 1 == s_off[lo + 1]);
    if (seg_end) {
#pragma unroll
      for (int m = 0; m < kG2; ++m) s_acc[p][m] += v[m];
    }
    __syncthreads();
  }
  if (lane < np) {
    const uint32_t r = vis_rec[s0 + lane];
#pragma unroll
    for (int m = 0; m < kG2; ++m) g2d[(int64_t)r * kG2 + m] = s_acc[lane][m];
  }
}

// --------------------------------------------------- preprocess adjoint
template <typename T, int N>
struct __attribute__((aligned(sizeof(T)))) VecN {
  T v[N];
};

// Per camera: the geometry adjoint (mean through the projection, covariance
// through EWA) for one (Gaussian, camera) pair's 2-D gradients.
template <typename T>
__device__ __forceinline__ void adj_geom_cam(const DevCam<T>& cm, T mu0, T mu1, T mu2, const T (&Sg)[9], T gu, T gv,
                                             T gA, T gB, T gC, T (&dSig)[9], T& dmu0, T& dmu1, T& dmu2) {
  // recompute p, J, T, Sigma', conic
  const T px = cm.R[0] * mu0 + cm.R[1] * mu1 + cm.R[2] * mu2 + cm.t[0];
  const T py = cm.R[3] * mu0 + cm.R[4] * mu1 + cm.R[5] * mu2 + cm.t[1];
  const T pz = cm.R[6] * mu0 + cm.R[7] * mu1 + cm.R[8] * mu2 + cm.t[2];
  const T iz = (T)1 / pz;
  const T txz = px * iz, tyz = py * iz;
  const bool clx = txz < -cm.limx || txz > cm.limx;
  const bool cly = tyz < -cm.limy || tyz > cm.limy;
  const T xi = txz < -cm.limx ? -cm.limx : (txz > cm.limx ? cm.limx : txz);
  const T eta = tyz < -cm.limy ? -cm.limy : (tyz > cm.limy ? cm.limy : tyz);
  const T J00 = cm.fx * iz, J02 = -cm.fx * xi * iz, J11 = cm.fy * iz, J12 = -cm.fy * eta * iz;
  T Tm[6];
  Tm[0] = J00 * cm.R[0] + J02 * cm.R[6]; Tm[1] = J00 * cm.R[1] + J02 * cm.R[7]; Tm[2] = J00 * cm.R[2] + J02 * cm.R[8];
  Tm[3] = J11 * cm.R[3] + J12 * cm.R[6]; Tm[4] = J11 * cm.R[4] + J12 * cm.R[7]; Tm[5] = J11 * cm.R[5] + J12 * cm.R[8];
  T TS[6];  // T Sigma (2x3)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      TS[3 * a + b] = Tm[3 * a] * Sg[b] + Tm[3 * a + 1] * Sg[3 + b] + Tm[3 * a + 2] * Sg[6 + b];
  const T c00 = TS[0] * Tm[0] + TS[1] * Tm[1] + TS[2] * Tm[2] + (T)0.3;
  const T c01 = TS[0] * Tm[3] + TS[1] * Tm[4] + TS[2] * Tm[5];
  const T c11 = TS[3] * Tm[3] + TS[4] * Tm[4] + TS[5] * Tm[5] + (T)0.3;
  const T idet = (T)1 / (c00 * c11 - c01 * c01);
  const T A = c11 * idet, Bc = -c01 * idet, C = c00 * idet;
  // dL/dSigma' = -Q Gq Q, Q = [[A, B], [B, C]], Gq = [[gA, gB/2], [gB/2, gC]]
  const T hB = (T)0.5 * gB;
  const T q00 = A * gA + Bc * hB, q01 = A * hB + Bc * gC, q10 = Bc * gA + C * hB, q11 = Bc * hB + C * gC;
  const T d00 = -(q00 * A + q01 * Bc), d01 = -(q00 * Bc + q01 * C), d11 = -(q10 * Bc + q11 * C);
  const T dS[4] = {d00, d01, d01, d11};
  // dL/dSigma += T^T dS T
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      dSig[3 * a + b] += Tm[a] * (dS[0] * Tm[b] + dS[1] * Tm[3 + b]) + Tm[3 + a] * (dS[2] * Tm[b] + dS[3] * Tm[3 + b]);
  // dL/dT = 2 dS T Sigma = 2 dS TS
  T dT[6];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    dT[b] = 2 * (dS[0] * TS[b] + dS[1] * TS[3 + b]);
    dT[3 + b] = 2 * (dS[2] * TS[b] + dS[3] * TS[3 + b]);
  }
  // dL/dJ = dT W^T (entries 00, 02, 11, 12)
  const T dJ00 = dT[0] * cm.R[0] + dT[1] * cm.R[1] + dT[2] * cm.R[2];
  const T dJ02 = dT[0] * cm.R[6] + dT[1] * cm.R[7] + dT[2] * cm.R[8];
  const T dJ11 = dT[3] * cm.R[3] + dT[4] * cm.R[4] + dT[5] * cm.R[5];
  const T dJ12 = dT[3] * cm.R[6] + dT[4] * cm.R[7] + dT[5] * cm.R[8];
  const T iz2 = iz * iz;
  T dpx = gu * cm.fx * iz, dpy = gv * cm.fy * iz;
  T dpz = -(gu * cm.fx * px + gv * cm.fy * py) * iz2;
  dpz += -dJ00 * cm.fx * iz2 - dJ11 * cm.fy * iz2;
  if (!clx) {
    dpx += dJ02 * (-cm.fx * iz2);
    dpz += dJ02 * ((T)2 * cm.fx * px * iz2 * iz);
  } else {
    dpz += dJ02 * (cm.fx * xi * iz2);
  }
  if (!cly) {
    dpy += dJ12 * (-cm.fy * iz2);
    dpz += dJ12 * ((T)2 * cm.fy * py * iz2 * iz);
  } else {
    dpz += dJ12 * (cm.fy * eta * iz2);
  }
  dmu0 += cm.R[0] * dpx + cm.R[3] * dpy + cm.R[6] * dpz;
  dmu1 += cm.R[1] * dpx + cm.R[4] * dpy + cm.R[7] * dpz;
  dmu2 += cm.R[2] * dpx + cm.R[5] * dpy + cm.R[8] * dpz;
}

// Per (camera, colour channel): the colour adjoint of SH degree 3 for the
// channel's 16 coefficients, and the viewing direction's share of the mean
// gradient (linear in the channel's contribution).
template <typename T>
__device__ __forceinline__ void adj_colour_cam(const ShK<T>& K, const DevCam<T>& cm, T mu0, T mu1, T mu2,
                                               const T (&sh)[16], T gcol, T (&gs)[16], T& dmu0, T& dmu1, T& dmu2) {
  T dx = mu0 - cm.pos[0], dy = mu1 - cm.pos[1], dz = mu2 - cm.pos[2];
  const T len = Mth<T>::sqrt(dx * dx + dy * dy + dz * dz);
  const T il = (T)1 / len;
  dx *= il; dy *= il; dz *= il;
  T Y[16];
  sh_eval<T>(K, dx, dy, dz, Y);
  T raw = (T)0.5;
#pragma unroll
  for (int m = 0; m < 16; ++m) raw += Y[m] * sh[m];
  const T graw = raw < 0 ? (T)0 : gcol;
  T wk[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    gs[m] += Y[m] * graw;
    wk[m] = sh[m] * graw;
  }
  {
    const T x = dx, y = dy, z = dz, xx = x * x, yy = y * y, zz = z * z;
    T gx = 0, gy = 0, gz = 0;
    gy += -K.c1 * wk[1];
    gz += K.c1 * wk[2];
    gx += -K.c1 * wk[3];
    gx += K.c2a * y * wk[4]; gy += K.c2a * x * wk[4];
    gy += -K.c2a * z * wk[5]; gz += -K.c2a * y * wk[5];
    gx += -2 * K.c2b * x * wk[6]; gy += -2 * K.c2b * y * wk[6]; gz += 4 * K.c2b * z * wk[6];
    gx += -K.c2a * z * wk[7]; gz += -K.c2a * x * wk[7];
    gx += 2 * K.c2c * x * wk[8]; gy += -2 * K.c2c * y * wk[8];
    gx += -K.c3a * 6 * x * y * wk[9]; gy += -K.c3a * (3 * xx - 3 * yy) * wk[9];
    gx += K.c3b * y * z * wk[10]; gy += K.c3b * x * z * wk[10]; gz += K.c3b * x * y * wk[10];
    gx += 2 * K.c3c * x * y * wk[11]; gy += -K.c3c * (4 * zz - xx - 3 * yy) * wk[11];
    gz += -8 * K.c3c * y * z * wk[11];
    gx += -6 * K.c3d * x * z * wk[12]; gy += -6 * K.c3d * y * z * wk[12];
    gz += K.c3d * (6 * zz - 3 * xx - 3 * yy) * wk[12];
    gx += -K.c3c * (4 * zz - 3 * xx - yy) * wk[13]; gy += 2 * K.c3c * x * y * wk[13];
    gz += -8 * K.c3c * x * z * wk[13];
    gx += 2 * K.c3e * x * z * wk[14]; gy += -2 * K.c3e * y * z * wk[14]; gz += K.c3e * (xx - yy) * wk[14];
    gx += -K.c3a * (3 * xx - 3 * yy) * wk[15]; gy += 6 * K.c3a * x * y * wk[15];
    const T dd = gx * x + gy * y + gz * z;
    dmu0 += (gx - dd * x) * il;
    dmu1 += (gy - dd * y) * il;
    dmu2 += (gz - dd * z) * il;
  }
}

// Thread per processing index; only active rows work.  Each kept camera's
// 36-byte record of 2-D gradients is read once, as one object: pass 1 chains
// its geometry part (u, v, conic) back to mean, log-scale and quaternion,
// cameras in order, and parks its opacity and colour part in LDS; pass 2
// runs the opacity and then the colour, one channel at a time (that
// channel's 16 coefficients and 16 sums live at once; the viewing direction
// and SH basis are recomputed per channel), cameras in order.  91 VGPRs and
// 32 KB of LDS per 256 threads: five waves per SIMD, against two when the
// 48 SH sums were held together.
// With kAdam the row's gradient is not stored: each column goes straight
// into the masked Adam update of that row (the moments and the parameter,
// the step counter and bias corrections first), with the same arithmetic as
// the Adam sweep over a stored gradient, so both give the same bits.  A
// column's parameter is read before it is written and every other access
// of the row is by this thread; the means are updated last, as the colour
// pass reads them.
template <typename T>
struct AdamRows {
  T* m1;
  T* m2;
  uint32_t* step;
  AdamK<T> K;
  double lb1, lb2;
};

template <typename T, bool kAdam>
__device__ __forceinline__ void adjoint_row(T* params, const int32_t* __restrict__ order, int32_t B, int64_t n_pidx,
                                            const CamSet<T>& cs, const uint32_t* __restrict__ tt,
                                            const uint32_t* __restrict__ active, const uint32_t* __restrict__ act_idx,
                                            const T* __restrict__ g2d, T* __restrict__ grad, int64_t ld,
                                            const AdamRows<T>& ad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pidx || !active[i]) return;
  const int64_t k = i / B;
  const int32_t row = (int32_t)(i - k * B);
  const int32_t slot = order[k];
  T* const P = params + (int64_t)slot * kD * B + row;
  const int V = cs.n;
  uint32_t keepm = 0;
#pragma unroll 1
  for (int c = 0; c < V; ++c) keepm |= (tt[(int64_t)c * n_pidx + i] != 0 ? 1u : 0u) << c;
  T bcx = 0, bcy = 0;
  if constexpr (kAdam) adam_step_bias<T>(ad.step + (int64_t)slot * B + row, ad.lb1, ad.lb2, bcx, bcy);
  // Adam state (m, v) of column j; a group of columns loads its states
  // together before updating them, so the loads are in flight at once
  const int64_t so = (int64_t)slot * kD * B + row;
  auto load_mv = [&](int j, T& m, T& v) {
    if constexpr (kAdam) {
      m = __builtin_nontemporal_load(ad.m1 + so + (int64_t)j * B);
      v = __builtin_nontemporal_load(ad.m2 + so + (int64_t)j * B);
    }
  };
  // column j of the row's gradient, with the column's parameter value p and
  // its Adam state loaded by load_mv
  auto put = [&](int j, T g, T p, T m, T v) {
    if constexpr (kAdam) {
      // the update sees g and p as the sweep does, as values from memory: the
      // compiler may not fuse the update's products into the arithmetic
      // that made them
      asm volatile("" : "+v"(g), "+v"(p));
      const int64_t o = (int64_t)j * B;
      adam_col<T>(p, m, v, g, ad.K.lr[j], ad.K.b1, ad.K.b2, ad.K.eps, bcx, bcy);
      __builtin_nontemporal_store(m, ad.m1 + so + o);
      __builtin_nontemporal_store(v, ad.m2 + so + o);
      __builtin_nontemporal_store(p, P + o);
    } else {
      grad[(int64_t)act_idx[i] + (int64_t)j * ld] = g;
    }
  };

  const T mu0 = P[0], mu1 = P[B], mu2 = P[2 * (int64_t)B];
  const T ls0 = P[3 * (int64_t)B], ls1 = P[4 * (int64_t)B], ls2 = P[5 * (int64_t)B];
  const T s0 = Mth<T>::exp(ls0), s1 = Mth<T>::exp(ls1), s2 = Mth<T>::exp(ls2);
  const T qw0 = P[6 * (int64_t)B], qx0 = P[7 * (int64_t)B], qy0 = P[8 * (int64_t)B], qz0 = P[9 * (int64_t)B];
  const T qn = Mth<T>::sqrt(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
  const T iq = (T)1 / qn;
  const T qw = qw0 * iq, qx = qx0 * iq, qy = qy0 * iq, qz = qz0 * iq;
  const T Rq[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                   2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                   2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
  const T sv[3] = {s0, s1, s2};
  T M[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[3 * a + b] = Rq[3 * a + b] * sv[b];
  T Sg[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Sg[3 * a + b] = M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1] + M[3 * a + 2] * M[3 * b + 2];
  T dSig[9];
#pragma unroll
  for (int m = 0; m < 9; ++m) dSig[m] = 0;
  T dmu0 = 0, dmu1 = 0, dmu2 = 0;
  // per camera, d/dopacity and d/dcolour wait in LDS for pass 2
  __shared__ T s_q[TIDE_MAX_CAMS][4][256];
  const int tx = threadIdx.x;
#pragma unroll 1
  for (int c = 0; c < V; ++c) {
    if (!((keepm >> c) & 1u)) continue;
    const VecN<T, 9> r = *reinterpret_cast<const VecN<T, 9>*>(g2d + ((int64_t)c * n_pidx + i) * kG2);
    s_q[c][0][tx] = r.v[5]; s_q[c][1][tx] = r.v[6]; s_q[c][2][tx] = r.v[7]; s_q[c][3][tx] = r.v[8];
    adj_geom_cam<T>(cs.c[c], mu0, mu1, mu2, Sg, r.v[0], r.v[1], r.v[2], r.v[3], r.v[4], dSig, dmu0, dmu1, dmu2);
  }
  // Sigma = M M^T: dM = 2 dSig M (dSig symmetric)
  T dM[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      dM[3 * a + b] = 2 * (dSig[3 * a] * M[b] + dSig[3 * a + 1] * M[3 + b] + dSig[3 * a + 2] * M[6 + b]);
  T gls[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) gls[b] = (dM[b] * Rq[b] + dM[3 + b] * Rq[3 + b] + dM[6 + b] * Rq[6 + b]) * sv[b];
  T g9[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) g9[3 * a + b] = dM[3 * a + b] * sv[b];
  const T w = qw, x = qx, y = qy, z = qz;
  T dq[4];
  dq[0] = 2 * (-z * g9[1] + y * g9[2] + z * g9[3] - x * g9[5] - y * g9[6] + x * g9[7]);
  dq[1] = 2 * (y * g9[1] + z * g9[2] + y * g9[3] - 2 * x * g9[4] - w * g9[5] + z * g9[6] + w * g9[7] - 2 * x * g9[8]);
  dq[2] = 2 * (-2 * y * g9[0] + x * g9[1] + w * g9[2] + x * g9[3] + z * g9[5] - w * g9[6] + z * g9[7] - 2 * y * g9[8]);
  dq[3] = 2 * (-2 * z * g9[0] - w * g9[1] + x * g9[2] + w * g9[3] - 2 * z * g9[4] + y * g9[5] + x * g9[6] + y * g9[7]);
  const T dqq = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
  T mq[7], vq[7];   // columns 3..9 (scales, rotation)
#pragma unroll
  for (int j = 0; j < 7; ++j) load_mv(3 + j, mq[j], vq[j]);
  put(3, gls[0], ls0, mq[0], vq[0]); put(4, gls[1], ls1, mq[1], vq[1]); put(5, gls[2], ls2, mq[2], vq[2]);
  put(6, (dq[0] - dqq * w) * iq, qw0, mq[3], vq[3]);
  put(7, (dq[1] - dqq * x) * iq, qx0, mq[4], vq[4]);
  put(8, (dq[2] - dqq * y) * iq, qy0, mq[5], vq[5]);
  put(9, (dq[3] - dqq * z) * iq, qz0, mq[6], vq[6]);
  // opacity
  const T logit = P[10 * (int64_t)B];
  const T op = (T)1 / ((T)1 + Mth<T>::exp(-logit));
  T dlogit = 0;
#pragma unroll 1
  for (int c = 0; c < V; ++c)
    if ((keepm >> c) & 1u) dlogit += s_q[c][0][tx] * op * ((T)1 - op);
  T m10, v10;
  load_mv(10, m10, v10);
  put(10, dlogit, logit, m10, v10);
  // colour, one channel at a time
#pragma unroll 1
  for (int ch = 0; ch < 3; ++ch) {
    T sh[16], gs[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      sh[m] = P[(int64_t)(11 + 3 * m + ch) * B];
      gs[m] = 0;
    }
#pragma unroll 1
    for (int c = 0; c < V; ++c) {
      if (!((keepm >> c) & 1u)) continue;
      const T gcol = s_q[c][1 + ch][tx];
      adj_colour_cam<T>(cs.sh, cs.c[c], mu0, mu1, mu2, sh, gcol, gs, dmu0, dmu1, dmu2);
    }
#pragma unroll
    for (int h = 0; h < 16; h += kMvGroup) {
      T mc[kMvGroup], vc[kMvGroup];
#pragma unroll
      for (int m = 0; m < kMvGroup; ++m) load_mv(11 + 3 * (h + m) + ch, mc[m], vc[m]);
#pragma unroll
      for (int m = 0; m < kMvGroup; ++m) put(11 + 3 * (h + m) + ch, gs[h + m], sh[h + m], mc[m], vc[m]);
    }
  }
  T m0, v0, m1, v1, m2, v2;
  load_mv(0, m0, v0); load_mv(1, m1, v1); load_mv(2, m2, v2);
  put(0, dmu0, mu0, m0, v0); put(1, dmu1, mu1, m1, v1); put(2, dmu2, mu2, m2, v2);
}

template <typename T>
__global__ void __launch_bounds__(256) k_adjoint(T* params, const int32_t* __restrict__ order, int32_t B,
                                                 int64_t n_pidx, CamSet<T> cs, const uint32_t* __restrict__ tt,
                                                 const uint32_t* __restrict__ active,
                                                 const uint32_t* __restrict__ act_idx, const T* __restrict__ g2d,
                                                 T* __restrict__ grad, int64_t ld) {
  adjoint_row<T, false>(params, order, B, n_pidx, cs, tt, active, act_idx, g2d, grad, ld, AdamRows<T>{});
}

// The fused variant holds the Adam state of the row besides the adjoint's:
// at most 128 registers keep four waves per SIMD.
template <typename T>
__global__ void __launch_bounds__(256, 4) k_adjoint_adam(T* params, const int32_t* __restrict__ order, int32_t B,
                                                         int64_t n_pidx, CamSet<T> cs,
                                                         const uint32_t* __restrict__ tt,
                                                         const uint32_t* __restrict__ active,
                                                         const uint32_t* __restrict__ act_idx,
                                                         const T* __restrict__ g2d, AdamRows<T> ad) {
  adjoint_row<T, true>(params, order, B, n_pidx, cs, tt, active, act_idx, g2d, nullptr, 0, ad);
}

template <typename T>
static void launch_adjoint(const tide_pool* pool, const tide_proj* proj, const CamSet<T>& cs, const T* g2d,
                           T* grad, int64_t ld, hipStream_t st) {
  hipLaunchKernelGGL(k_adjoint<T>, dim3((uint32_t)ceil_div(proj->n_pidx, 256)), dim3(256), 0, st,
                     (T*)pool->params, pool->order, pool->block_rows, proj->n_pidx, cs, proj->tiles_touched,
                     proj->active, proj->act_idx, g2d, grad, ld);
}

template <typename T>
static void launch_adjoint_adam(const tide_pool* pool, const tide_proj* proj, const CamSet<T>& cs, const T* g2d,
                                const tide_adam_cfg* cfg, hipStream_t st) {
  AdamRows<T> ad;
  ad.m1 = (T*)pool->exp_avg;
  ad.m2 = (T*)pool->exp_avg_sq;
  ad.step = pool->step;
  ad.K = make_adam_k<T>(cfg);
  ad.lb1 = std::log2((double)cfg->beta1);
  ad.lb2 = std::log2((double)cfg->beta2);
  hipLaunchKernelGGL(k_adjoint_adam<T>, dim3((uint32_t)ceil_div(proj->n_pidx, 256)), dim3(256), 0, st,
                     (T*)pool->params, pool->order, pool->block_rows, proj->n_pidx, cs, proj->tiles_touched,
                     proj->active, proj->act_idx, g2d, ad);
}

template <typename T>
CamSet<T> make_camset(const tide_camera* cams, int n);

}  // namespace tide

using namespace tide;

extern "C" size_t tide_render_bwd_ws_bytes(const tide_bins* bins, int32_t dtype) {
  if (!bins) return 0;
  const size_t es = dtype == TIDE_F64 ? 8 : 4;
  return align_up((size_t)(bins->n_inst > 0 ? bins->n_inst : 1) * kG2 * es) +
         align_up((size_t)kG2 * bins->n_cams * bins->n_pidx * es) + 256;
}

// The three stages on one stream; with cfg the last one applies the masked
// Adam update instead of storing the gradient.
static tide_status render_bwd_run(const tide_pool* pool, const tide_camera* cams, int32_t n_cams,
                                  const tide_proj* proj, const tide_bins* bins, const tide_frame* fr, const float* bg,
                                  const void* d_dimage, void* grad, int64_t grad_ld, const tide_adam_cfg* cfg,
                                  void* ws, hipStream_t st) {
  const uint32_t grid = (uint32_t)(bins->n_cams * bins->tiles_x * bins->tiles_y);
  const int64_t nrec = (int64_t)n_cams * proj->n_pidx;
  Carver cv(ws);
  if (proj->dtype == TIDE_F32) {
    float* partial = cv.take<float>((size_t)(bins->n_inst > 0 ? bins->n_inst : 1) * kG2);
    float* g2d = cv.take<float>((size_t)kG2 * nrec);

    TIDE_TIMED("render_bwd", st, hipLaunchKernelGGL(k_render_bwd<float>, dim3(grid), dim3(64), 0, st, bins->tile_order, bins->ranges, bins->inst_e, bins->inst_rec,
                       (const float*)proj->rec, bins->tiles_x, bins->tiles_y, fr->width, fr->height, bg[0], bg[1],
                       bg[2], (const float*)fr->t_final, fr->last, (const float*)d_dimage, partial));
    TIDE_LAUNCH_CHECK("k_render_bwd");
    if (bins->n_vis > 0)
      TIDE_TIMED("reduce_pairs", st, hipLaunchKernelGGL(k_reduce_pairs<float>, dim3((uint32_t)ceil_div(bins->n_vis, kWave)),
                                                        dim3(kWave), 0, st, bins->vis_rec, bins->inst_off, bins->n_vis, nrec,
                                                        (const float*)partial, g2d));
    TIDE_LAUNCH_CHECK("k_reduce_pairs");
    const CamSet<float> cs = make_camset<float>(cams, n_cams);
    if (proj->n_pidx > 0) {
      if (cfg)
        TIDE_TIMED("adjoint_adam", st, launch_adjoint_adam<float>(pool, proj, cs, g2d, cfg, st));
      else
        TIDE_TIMED("adjoint", st, launch_adjoint<float>(pool, proj, cs, g2d, (float*)grad, grad_ld, st));
    }
    TIDE_LAUNCH_CHECK("k_adjoint");
  } else {
    double* partial = cv.take<double>((size_t)(bins->n_inst > 0 ? bins->n_inst : 1) * kG2);
    double* g2d = cv.take<double>((size_t)kG2 * nrec);

    TIDE_TIMED("render_bwd", st, hipLaunchKernelGGL(k_render_bwd<double>, dim3(grid), dim3(64), 0, st, bins->tile_order, bins->ranges, bins->inst_e,
                       bins->inst_rec, (const double*)proj->rec, bins->tiles_x, bins->tiles_y, fr->width,
                       fr->height, (double)bg[0], (double)bg[1], (double)bg[2], (const double*)fr->t_final,
                       fr->last, (const double*)d_dimage, partial));
    TIDE_LAUNCH_CHECK("k_render_bwd");
    if (bins->n_vis > 0)
      TIDE_TIMED("reduce_pairs", st, hipLaunchKernelGGL(k_reduce_pairs<double>, dim3((uint32_t)ceil_div(bins->n_vis, kWave)),
                                                        dim3(kWave), 0, st, bins->vis_rec, bins->inst_off, bins->n_vis, nrec,
                                                        (const double*)partial, g2d));
    TIDE_LAUNCH_CHECK("k_reduce_pairs");
    const CamSet<double> cs = make_camset<double>(cams, n_cams);
    if (proj->n_pidx > 0) {
      if (cfg)
        TIDE_TIMED("adjoint_adam", st, launch_adjoint_adam<double>(pool, proj, cs, g2d, cfg, st));
      else
        TIDE_TIMED("adjoint", st, launch_adjoint<double>(pool, proj, cs, g2d, (double*)grad, grad_ld, st));
    }
    TIDE_LAUNCH_CHECK("k_adjoint");
  }
  return TIDE_OK;
}

static tide_status render_bwd_check(const tide_pool* pool, const tide_camera* cams, int32_t n_cams,
                                    const tide_proj* proj, const tide_bins* bins, const tide_frame* fr,
                                    const float* bg, const void* d_dimage, void* ws, size_t ws_bytes) {
  TIDE_CHECK_ARG(pool && cams && proj && bins && fr && bg && d_dimage && ws, "null argument");
  TIDE_CHECK_ARG(n_cams == proj->n_cams && n_cams == bins->n_cams, "camera counts differ");
  TIDE_CHECK_ARG(proj->dtype == pool->dtype, "dtype mismatch");
  TIDE_CHECK_ARG(proj->n_pidx == (int64_t)pool->n_order * pool->block_rows, "proj does not match pool");
  const size_t need = tide_render_bwd_ws_bytes(bins, proj->dtype);
  if (ws_bytes < need) {
    set_error("render_bwd workspace too small (%zu < %zu)", ws_bytes, need);
    return TIDE_ECAPACITY;
  }
  return TIDE_OK;
}

extern "C" tide_status tide_render_bwd(const tide_pool* pool, const tide_camera* cams, int32_t n_cams,
                                       const tide_proj* proj, const tide_bins* bins, const tide_frame* fr,
                                       const float* bg, const void* d_dimage, void* grad, int64_t grad_ld, void* ws,
                                       size_t ws_bytes, void* stream) {
  TIDE_CHECK_ARG(grad, "null argument");
  const tide_status e = render_bwd_check(pool, cams, n_cams, proj, bins, fr, bg, d_dimage, ws, ws_bytes);
  if (e != TIDE_OK) return e;
  TIDE_CHECK_ARG(grad_ld >= proj->n_pidx, "grad_ld (%lld) < n_pidx (%lld)", (long long)grad_ld,
                 (long long)proj->n_pidx);
  return render_bwd_run(pool, cams, n_cams, proj, bins, fr, bg, d_dimage, grad, grad_ld, nullptr, ws,
                        (hipStream_t)stream);
}

extern "C" tide_status tide_render_bwd_adam(tide_pool* pool, const tide_camera* cams, int32_t n_cams,
                                            const tide_proj* proj, const tide_bins* bins, const tide_frame* fr,
                                            const float* bg, const void* d_dimage, const tide_adam_cfg* cfg,
                                            float* spheres, uint8_t* dirty, int64_t n_blocks, void* ws,
                                            size_t ws_bytes, void* stream) {
  TIDE_CHECK_ARG(cfg, "null argument");
  const tide_status e = render_bwd_check(pool, cams, n_cams, proj, bins, fr, bg, d_dimage, ws, ws_bytes);
  if (e != TIDE_OK) return e;
  TIDE_CHECK_ARG(pool->params && pool->exp_avg && pool->exp_avg_sq && pool->step && pool->order && pool->slot_block,
                 "pool has a null pointer");
  TIDE_CHECK_ARG(cfg->beta1 > 0 && cfg->beta1 < 1 && cfg->beta2 > 0 && cfg->beta2 < 1 && cfg->eps >= 0,
                 "bad Adam constants");
  TIDE_CHECK_ARG((!spheres && !dirty) || n_blocks > 0, "n_blocks must be given with spheres/dirty");
  hipStream_t st = (hipStream_t)stream;
  const tide_status r =
      render_bwd_run(pool, cams, n_cams, proj, bins, fr, bg, d_dimage, nullptr, 0, cfg, ws, st);
  if (r != TIDE_OK) return r;
  launch_adam_bounds(pool, proj, cfg->kappa, spheres, dirty, st);
  TIDE_LAUNCH_CHECK("k_adam_bounds");
  return TIDE_OK;
}
