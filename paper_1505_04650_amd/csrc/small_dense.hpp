// FP64 building blocks for the small (<= 128 x 128) dense steps: fixed-order
// reduction of per-block partial sums and a single-wave Cholesky whose
// products run on the MFMA.
#pragma once

#include "cnmf_internal.hpp"

namespace cnmf {

// Sum parts [0, nparts) of `count` elements laid out as in[p * stride + e]
// (TI: FP64 or FP32 parts, summed in FP64) for the elements [e0, e0 + EPB)
// handled by this block.  NT threads:
// thread (el = tid % EPB, pg = tid / EPB) sums parts pg, pg + PG, ... with
// four independent chains, then the PG groups are combined by a fixed tree in
// LDS.  The order depends only on nparts, so results are reproducible.
template <int NT, int EPB, typename TI = double>
__device__ __forceinline__ void block_sum_parts(const TI* __restrict__ in, int nparts, int64_t stride,
                                                int64_t count, int64_t e0, double* __restrict__ out,
                                                double* red /* LDS, NT doubles */) {
  constexpr int PG = NT / EPB;
  const int tid = threadIdx.x;
  const int el = tid % EPB, pg = tid / EPB;
  const int64_t e = e0 + el;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (e < count) {
    int p = pg;
    for (; p + 3 * PG < nparts; p += 4 * PG) {
      s0 += (double)in[(int64_t)p * stride + e];
      s1 += (double)in[(int64_t)(p + PG) * stride + e];
      s2 += (double)in[(int64_t)(p + 2 * PG) * stride + e];
      s3 += (double)in[(int64_t)(p + 3 * PG) * stride + e];
    }
    for (; p < nparts; p += PG) s0 += (double)in[(int64_t)p * stride + e];
  }
  red[tid] = (s0 + s1) + (s2 + s3);
  __syncthreads();
#pragma unroll
  for (int w = PG / 2; w > 0; w >>= 1) {
    if (pg < w) red[tid] += red[tid + w * EPB];
    __syncthreads();
  }
  if (pg == 0 && e < count) out[e] = red[el];
  __syncthreads();
}

// G consecutive element ranges of block_sum_parts at once: range q covers
// the elements [e0 + q EPB, e0 + (q + 1) EPB).  Each element is summed in
// exactly block_sum_parts's order (same chains, same tree), so the results
// are bit for bit those of G separate calls; the loads of the G ranges are
// issued together, so the block waits for the memory latency once per step
// rather than G times.  red: G NT doubles of LDS.
template <int NT, int EPB, int G, typename TI = double>
__device__ __forceinline__ void block_sum_parts_groups(const TI* __restrict__ in, int nparts, int64_t stride,
                                                       int64_t count, int64_t e0, double* __restrict__ out,
                                                       double* red) {
  constexpr int PG = NT / EPB;
  const int tid = threadIdx.x;
  const int el = tid % EPB, pg = tid / EPB;
  double s[G][4];
  bool ok[G];
#pragma unroll
  for (int q = 0; q < G; ++q) {
    ok[q] = e0 + q * EPB + el < count;
    s[q][0] = s[q][1] = s[q][2] = s[q][3] = 0.0;
  }
  int p = pg;
  for (; p + 3 * PG < nparts; p += 4 * PG) {
#pragma unroll
    for (int q = 0; q < G; ++q)
      if (ok[q]) {
        const int64_t e = e0 + q * EPB + el;
        s[q][0] += (double)in[(int64_t)p * stride + e];
        s[q][1] += (double)in[(int64_t)(p + PG) * stride + e];
        s[q][2] += (double)in[(int64_t)(p + 2 * PG) * stride + e];
        s[q][3] += (double)in[(int64_t)(p + 3 * PG) * stride + e];
      }
  }
  for (; p < nparts; p += PG)
#pragma unroll
    for (int q = 0; q < G; ++q)
      if (ok[q]) s[q][0] += (double)in[(int64_t)p * stride + e0 + q * EPB + el];
#pragma unroll
  for (int q = 0; q < G; ++q) red[q * NT + tid] = (s[q][0] + s[q][1]) + (s[q][2] + s[q][3]);
  __syncthreads();
#pragma unroll
  for (int w = PG / 2; w > 0; w >>= 1) {
    if (pg < w)
#pragma unroll
      for (int q = 0; q < G; ++q) red[q * NT + tid] += red[q * NT + tid + w * EPB];
    __syncthreads();
  }
  if (pg == 0)
#pragma unroll
    for (int q = 0; q < G; ++q)
      if (ok[q]) out[e0 + q * EPB + el] = red[q * NT + el];
  __syncthreads();
}

__device__ __forceinline__ double readlane_d(double x, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// 1 / sqrt(d) for d > 0 in four dependent operations: the hardware estimate
// y0 (relative error below 2^-24) and one second-order correction
// y = y0 (1 + e / 2 + 3 e^2 / 8), e = 1 - d y0^2, whose truncation error is
// of order e^3 (below 1e-21), so y is within rounding of 1 / sqrt(d).
__device__ __forceinline__ double rsqrt_fast(double d) {
  const double y0 = __builtin_amdgcn_rsq(d);
  const double e = fma(-d * y0, y0, 1.0);
  return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}

// Scalar-type traits of the single-wave factorisation and the solves built
// on it: the 16x16x4 MFMA of the type, where its result item i of lane
// group g = lane / 16 sits (row out_row(g, i) of the tile, column lane % 16:
// g + 4 i for FP64, 4 g + i for FP32, measured), and the K index a lane
// group supplies in K step s when a result tile is fed back as the right
// operand of the next product (kx(s, g), the row of item s), so chained
// products need no data movement.  Operands loaded from memory may use any
// K order as long as both operands agree.
template <typename T>
struct SD;
template <>
struct SD<double> {
  typedef doublex4 v4;
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int i) { return g + 4 * i; }
  static __device__ __forceinline__ int kx(int s, int g) { return 4 * s + g; }
  static __device__ __forceinline__ double readlane(double x, int l) { return readlane_d(x, l); }
  static __device__ __forceinline__ double rsq(double d) { return rsqrt_fast(d); }
  static __device__ __forceinline__ double fmax_(double a, double b) { return fmax(a, b); }
  static __device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }
};
template <>
struct SD<float> {
  typedef floatx4 v4;
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int i) { return 4 * g + i; }
  static __device__ __forceinline__ int kx(int s, int g) { return 4 * g + s; }
  static __device__ __forceinline__ float readlane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
  }
  // hardware reciprocal square root (about 1 ulp)
  static __device__ __forceinline__ float rsq(float d) { return __builtin_amdgcn_rsqf(d); }
  static __device__ __forceinline__ float fmax_(float a, float b) { return fmaxf(a, b); }
  static __device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
};

// Steps of one 16-column panel (see wave_chol_lower).  FULL: all 16 steps,
// no branches, so the scheduler can overlap consecutive steps; otherwise
// only the first `steps` (uniform) are taken.  The dependent chain of a step
// is: pivot by readlane, floor, 1 / sqrt, the column entry, its readlane by
// the next pivot row and that row's update.
// extra(s) is called before step s (every s < 16, taken or not): the caller
// issues independent MFMA work there, which runs while the step's dependent
// VALU chain waits.
// DEC (decoupling): a pivot <= floor_piv (or NaN) marks its column as
// dependent on the earlier ones: the column of the factor becomes the unit
// vector (1 on the diagonal, 0 below), so the column takes no part in the
// later steps; bit c0 + s of mbits records it and NaN pivots are also
// counted in nnan.  Without DEC such a pivot is replaced by floor_piv.
template <typename T, bool FULL, bool DEC, typename X>
__device__ __forceinline__ void wave_panel_steps(T (&a)[16], int c0, int steps, T* colbuf, T floor_piv, T& myinv,
                                                 int& nbad, uint64_t& mbits, int& nnan, X extra) {
  typedef SD<T> D;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    extra(s);
    if (FULL || s < steps) {
      const T d0 = D::readlane(a[s], c0 + s);
      const bool bad = !(d0 > floor_piv);   // also true for NaN
      nbad += bad ? 1 : 0;
      const bool piv = lane == c0 + s;
      T l, y;
      if constexpr (DEC) {
        nnan += (d0 != d0) ? 1 : 0;
        mbits |= bad ? (1ull << (c0 + s)) : 0ull;
        const T d = bad ? T(1) : d0;
        const T as = piv ? d : a[s];
        y = D::rsq(d);
        l = bad ? (piv ? T(1) : T(0)) : as * y;
      } else {
        const T d = D::fmax_(d0, floor_piv);
        const T as = piv ? d : a[s];
        y = D::rsq(d);
        l = as * y;   // L[lane][c0 + s]; sqrt(d) on the pivot lane
      }
      a[s] = l;
      myinv = piv ? y : myinv;
      if (s + 1 < 16) {
        a[s + 1] = D::fma_(-l, D::readlane(l, c0 + s + 1), a[s + 1]);
        if (s + 2 < 16) {
          colbuf[lane] = l;
#pragma unroll
          for (int t = s + 2; t < 16; ++t) a[t] = D::fma_(-l, colbuf[c0 + t], a[t]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// One wave, no barriers: M (N x N, N = 16 NB <= 64, LDS, row stride ld) =
// L L^T with L lower triangular and a positive diagonal, in T (FP64 or FP32,
// the products on that type's MFMA).  Read: the lower triangle and diagonal
// of M (the strict upper triangle of the diagonal 16 x 16 blocks may hold
// anything).  On return L is in M's lower triangle (the strict upper
// triangle is left undefined) and V[b] (16 x 17 each) holds the inverse of
// the diagonal block L[b][b] (lower, zeros above).  Rows and columns from n
// on must be those of the identity (no coupling), so their steps are skipped
// and L is the identity there too.  A pivot <= floor (or NaN) is replaced by
// floor (floor > 0), or with DEC its column is decoupled (see
// wave_panel_steps); the number of such pivots is added to *flag, with DEC
// the number of NaN pivots to *nanflag and the decoupled columns (bit j:
// column j) are or-ed into *mask (one wave-uniform word, N <= 64).  W: 128
// elements of LDS scratch.
//
// Right-looking by 16-column panels: lane j keeps row j of the panel in
// registers.  Step s takes the pivot of lane c0 + s by readlane; the entry
// of the next pivot row comes by readlane too, so the dependent chain of a
// step is short, and the rest of the column is broadcast through LDS.  The
// trailing lower block triangle is updated with 16x16x4 MFMA tile products,
// all operands loaded before the first product.  At the end the lanes
// 16 q + v (v < 16) invert block q, column v, by forward substitution.  A
// wave's LDS operations complete in order, so no barrier is needed between
// them.
// ---------------------------------------------------------------------------
template <typename T, int NB, bool DEC = false>
__device__ __forceinline__ void wave_chol_lower(T* M, int ld, int n, T* V, T* W, T floor_piv, int* flag,
                                                int* nanflag = nullptr, uint64_t* mask = nullptr) {
  typedef SD<T> D;
  typedef typename D::v4 v4;
  constexpr int N = 16 * NB;
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, g = lane >> 4;
  T* colbuf = W;       // the current column of L
  T* dinv = W + 64;    // 1 / L[i][i]
  int nbad = 0, nnan = 0;
  uint64_t mbits = 0;
  // The trailing tiles (ti >= tj >= 1) stay in registers in the MFMA result
  // layout (item i of lane (c, g): row 16 ti + out_row(g, i), column
  // 16 tj + c).  After panel P only column P + 1 is updated at once (the
  // next panel needs it); the updates of the tiles right of it are issued
  // between the next panel's steps.  Each tile still receives the panels'
  // updates in panel order, by the same products.
  constexpr int NT = NB > 1 ? NB * (NB - 1) / 2 : 1;
  v4 tl[NT];
#pragma unroll
  for (int ti = 1; ti < NB; ++ti)
#pragma unroll
    for (int tj = 1; tj <= ti; ++tj)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        tl[(ti - 1) * ti / 2 + tj - 1][i] = M[(16 * ti + D::out_row(g, i)) * ld + 16 * tj + c];
  constexpr int kMaxT = NB > 1 ? NB - 1 : 1;
  T lv[kMaxT][4];   // L[16 (P + 1 + u) + c][16 P + 4 s + g] of the last factored panel P
#pragma unroll
  for (int P = 0; P < NB; ++P) {
    const int c0 = 16 * P;
    const bool act = lane >= c0 && lane < N;
    if (P >= 1) {
#pragma unroll
      for (int ti = P; ti < NB; ++ti)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          M[(16 * ti + D::out_row(g, i)) * ld + c0 + c] = tl[(ti - 1) * ti / 2 + P - 1][i];
    }
    T a[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) a[t] = act ? M[lane * ld + c0 + t] : T(0);
    T myinv = T(1);
    const int steps = n - c0;   // uniform
    // panel P - 1's updates of the tiles ti >= tj >= P + 1, one product per step
    auto deferred = [&](int q) {
      if (P >= 1) {
        int idx = 0;
#pragma unroll
        for (int ti = P + 1; ti < NB; ++ti)
#pragma unroll
          for (int tj = P + 1; tj <= ti; ++tj)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              if (idx == q) {
                v4& t = tl[(ti - 1) * ti / 2 + tj - 1];
                t = D::mma(-lv[ti - P][s4], lv[tj - P][s4], t);
              }
              ++idx;
            }
      }
    };
    if (steps >= 16)
      wave_panel_steps<T, true, DEC>(a, c0, steps, colbuf, floor_piv, myinv, nbad, mbits, nnan, deferred);
    else
      wave_panel_steps<T, false, DEC>(a, c0, steps, colbuf, floor_piv, myinv, nbad, mbits, nnan, deferred);
    if (act) {
#pragma unroll
      for (int t = 0; t < 16; ++t) M[lane * ld + c0 + t] = a[t];
    }
    if (lane >= c0 && lane < c0 + 16) dinv[lane] = myinv;
    if (P + 1 < NB) {
      // column P + 1 now: M[ti][P + 1] -= L[ti][P] L[P + 1][P]^T
#pragma unroll
      for (int u = 0; u < kMaxT; ++u)
        if (P + 1 + u < NB) {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) lv[u][s4] = M[(16 * (P + 1 + u) + c) * ld + c0 + 4 * s4 + g];
        }
#pragma unroll
      for (int ti = P + 1; ti < NB; ++ti) {
        v4& t = tl[(ti - 1) * ti / 2 + P];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) t = D::mma(-lv[ti - P - 1][s4], lv[0][s4], t);
      }
    }
  }
  // V_q = L[q][q]^-1, lanes 16 q + v: column v, x = e_v, then for each i
  // x_i /= L[i][i] and x_t -= L[t][i] x_i (t > i)
  if (g < NB) {
    const int q0 = 16 * g;
    T x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = i == c ? T(1) : T(0);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      x[i] *= dinv[q0 + i];
#pragma unroll
      for (int t = i + 1; t < 16; ++t) x[t] = D::fma_(-M[(q0 + t) * ld + q0 + i], x[i], x[t]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) V[g * 272 + i * 17 + c] = x[i];
  }
  if (nbad && lane == 0 && flag) atomicAdd(flag, nbad);
  if constexpr (DEC) {
    if (nnan && lane == 0 && nanflag) atomicAdd(nanflag, nnan);
    if (lane == 0 && mask) *mask |= mbits;
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
}
}  // namespace cnmf
