// Orthonormalisation of the tall range samples (Alg. 1, QR step) by
// CholeskyQR2 in FP64, plus the small k x k products of the sketch.
//   G = Y^T Y (FP64 accumulation, deterministic partials)
//   T = chol(G) upper with positive diagonal, Tinv = T^-1
//   Q = Y Tinv; repeat once on Q (the second pass restores orthogonality
//   to working precision).
// With diag(T) > 0 this Q is the same basis as the Householder QR with a
// nonnegative diagonal for full-column-rank Y.
#include "cnmf_internal.hpp"
#include "small_dense.hpp"

namespace cnmf {

template <typename T>
__device__ __forceinline__ double to_d(T x) {
  return (double)x;
}

// ---------------------------------------------------------------------------
// Y[i][c] = sum_s P[s][i][c], s in increasing order (c < cols, ld = ld).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void reduce_splits_kernel(const T* __restrict__ P, int splits, int64_t slice, int64_t count,
                                     T* __restrict__ Y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    T acc = P[e];
    for (int s = 1; s < splits; ++s) acc += P[s * slice + e];
    Y[e] = acc;
  }
}

template <typename T>
hipError_t launch_reduce_splits(const T* P, int splits, int64_t rows, int ld, T* Y, hipStream_t st) {
  int64_t count = rows * ld;
  int blocks = (int)std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(reduce_splits_kernel<T>, dim3(blocks), dim3(256), 0, st, P, splits, count, count, Y);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_reduce_splits<float>(const float*, int, int64_t, int, float*, hipStream_t);
template hipError_t launch_reduce_splits<double>(const double*, int, int64_t, int, double*, hipStream_t);

// ---------------------------------------------------------------------------
// Cross products C_h = X[:, x0 + h*hs : + ka]^T Y[:, y0 + h*hs : + kb] over a
// slice of rows, FP64 accumulation; partial for (slice p, half h) at
// Cp[(p * nh + h) * ka * kb].  Thread (ta, tb) owns entries
// (ta + 16 i, tb + 16 j).
// ---------------------------------------------------------------------------
template <typename TX, typename TY, int KH16>
__global__ __launch_bounds__(256) void cross_kernel(const TX* __restrict__ X, int ldx, int x0,
                                                   const TY* __restrict__ Y, int ldy, int y0, int hs,
                                                   int rows, int ka, int kb, double* __restrict__ Cp,
                                                   int rows_per_part) {
  constexpr int CR = 32;
  constexpr int KW = KH16 * 16;
  __shared__ double xs[CR][KW + 1];
  __shared__ double ys[CR][KW + 1];
  const int tid = threadIdx.x;
  const int ta = tid >> 4, tb = tid & 15;
  const int p = blockIdx.x, h = blockIdx.y, nh = gridDim.y;
  const int xc = x0 + h * hs, yc = y0 + h * hs;
  const int i0 = p * rows_per_part;
  const int i1 = min(rows, i0 + rows_per_part);
  double acc[KH16][KH16];
#pragma unroll
  for (int i = 0; i < KH16; ++i)
#pragma unroll
    for (int j = 0; j < KH16; ++j) acc[i][j] = 0.0;

  for (int base = i0; base < i1; base += CR) {
    for (int e = tid; e < CR * KW; e += 256) {
      int rr = e / KW, c = e - rr * KW;
      int row = base + rr;
      bool ok = row < i1;
      xs[rr][c] = (ok && c < ka) ? to_d(X[(int64_t)row * ldx + xc + c]) : 0.0;
      ys[rr][c] = (ok && c < kb) ? to_d(Y[(int64_t)row * ldy + yc + c]) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < CR; ++rr) {
      double xa[KH16], yb[KH16];
#pragma unroll
      for (int i = 0; i < KH16; ++i) xa[i] = xs[rr][ta + 16 * i];
#pragma unroll
      for (int j = 0; j < KH16; ++j) yb[j] = ys[rr][tb + 16 * j];
#pragma unroll
      for (int i = 0; i < KH16; ++i)
#pragma unroll
        for (int j = 0; j < KH16; ++j) acc[i][j] = fma(xa[i], yb[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* out = Cp + ((int64_t)p * nh + h) * ka * kb;
#pragma unroll
  for (int i = 0; i < KH16; ++i)
#pragma unroll
    for (int j = 0; j < KH16; ++j) {
      int a = ta + 16 * i, b = tb + 16 * j;
      if (a < ka && b < kb) out[a * kb + b] = acc[i][j];
    }
}

template <typename TX, typename TY, int KH16>
static hipError_t cross_kh(const TX* X, int ldx, int x0, const TY* Y, int ldy, int y0, int hs, int nh,
                           int rows, int ka, int kb, double* Cp, int parts, hipStream_t st) {
  int rpp = (rows + parts - 1) / parts;
  hipLaunchKernelGGL((cross_kernel<TX, TY, KH16>), dim3(parts, nh), dim3(256), 0, st, X, ldx, x0, Y, ldy,
                     y0, hs, rows, ka, kb, Cp, rpp);
  CNMF_LAUNCH_CHECK();
}

template <typename TX, typename TY>
hipError_t launch_cross2(const TX* X, int ldx, int x0, const TY* Y, int ldy, int y0, int hs, int nh,
                         int rows, int ka, int kb, double* Cp, int parts, hipStream_t st) {
  int kmax = std::max(ka, kb);
  int k16 = (kmax + 15) / 16;
  switch (k16) {
    case 1: return cross_kh<TX, TY, 1>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, st);
    case 2: return cross_kh<TX, TY, 2>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, st);
    case 3: return cross_kh<TX, TY, 3>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, st);
    case 4: return cross_kh<TX, TY, 4>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, st);
    case 5: return cross_kh<TX, TY, 5>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, st);
    case 6: return cross_kh<TX, TY, 6>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, st);
    case 7: return cross_kh<TX, TY, 7>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, st);
    case 8: return cross_kh<TX, TY, 8>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, st);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_cross2<float, float>(const float*, int, int, const float*, int, int, int, int, int, int, int, double*, int, hipStream_t);
template hipError_t launch_cross2<double, double>(const double*, int, int, const double*, int, int, int, int, int, int, int, double*, int, hipStream_t);
template hipError_t launch_cross2<float, double>(const float*, int, int, const double*, int, int, int, int, int, int, int, double*, int, hipStream_t);

// ---------------------------------------------------------------------------
// out[e] = sum_p in[p * count + e], p increasing.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sum_parts_kernel(const double* __restrict__ in, int parts, int64_t count,
                                                        double* __restrict__ out) {
  __shared__ double red[256];
  block_sum_parts<256, 32>(in, parts, count, count, (int64_t)blockIdx.x * 32, out, red);
}

hipError_t launch_sum_parts(const double* in, int parts, int64_t count, double* out, hipStream_t st) {
  int blocks = (int)((count + 31) / 32);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(blocks), dim3(256), 0, st, in, parts, count, out);
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// G_h = sum of the Gram partials (fixed order; sum_parts kernel), then one
// workgroup per half: G_h = T^T T (Cholesky, T upper with positive diagonal)
// and Tinv_h = T^-1 written to global memory (upper, zero lower triangle).
// Partials: Gp[(p * nh + h) * kh * kh].  A pivot <= 1e-20 max_i G_ii (or
// not finite) counts as a breakdown in flags[h] and is replaced by that floor.
// ---------------------------------------------------------------------------
constexpr int kCholNT = 512;

// kh > 64: LDS factorisation by the whole workgroup.
__global__ __launch_bounds__(kCholNT) void chol_kernel(const double* __restrict__ G, int kh,
                                                       double* __restrict__ Tinv, int* flags) {
  constexpr int NT = kCholNT;
  const int h = blockIdx.x;
  const int64_t cnt = (int64_t)kh * kh;
  extern __shared__ double sm[];
  const int ld = kh + 1;
  double* M = sm;
  double* Td = sm + kh * ld;
  const double* Gh = G + h * cnt;
  for (int e = threadIdx.x; e < kh * kh; e += NT) {
    int i = e / kh, j = e - i * kh;
    if (j >= i) M[i * ld + j] = 0.5 * (Gh[i * kh + j] + Gh[j * kh + i]);
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = 0; i < kh; ++i) mx = fmax(mx, M[i * ld + i]);
  wg_cholesky_inverse<NT>(M, kh, ld, Td, 1e-20 * mx, flags ? flags + h : nullptr);
  double* out = Tinv + h * cnt;
  for (int e = threadIdx.x; e < kh * kh; e += NT) {
    int i = e / kh, j = e - i * kh;
    out[e] = j >= i ? M[i * ld + j] : 0.0;
  }
}

// kh <= 64: factor only (blocked, padded to 16 ceil(kh / 16) with I);
// Tf_h = T (upper, zero lower) for the substitution in apply_tri_kernel.
constexpr int kFacNT = 256;
__global__ __launch_bounds__(kFacNT) void chol_fac_kernel(const double* __restrict__ G, int kh,
                                                          double* __restrict__ Tf, int* flags) {
  const int h = blockIdx.x;
  const int64_t cnt = (int64_t)kh * kh;
  const int NB = (kh + 15) / 16, N = 16 * NB, ld = N + 1;
  extern __shared__ double sm[];
  double* M = sm;              // N x ld
  double* TI = M + N * ld;     // NB x 272
  double* PN = TI + NB * 272;  // 16 x ld
  const double* Gh = G + h * cnt;
  for (int e = threadIdx.x; e < N * N; e += kFacNT) {
    int i = e / N, j = e - i * N;
    double v;
    if (i < kh && j < kh)
      v = 0.5 * (Gh[i * kh + j] + Gh[j * kh + i]);
    else
      v = (i == j) ? 1.0 : 0.0;
    M[i * ld + j] = v;
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = 0; i < kh; ++i) mx = fmax(mx, M[i * ld + i]);
  wg_chol_blocked<kFacNT>(M, ld, NB, TI, PN, 1e-20 * mx, flags ? flags + h : nullptr);
  double* out = Tf + h * cnt;
  for (int e = threadIdx.x; e < kh * kh; e += kFacNT) {
    int i = e / kh, j = e - i * kh;
    out[e] = j >= i ? M[i * ld + j] : 0.0;
  }
}

// Q[i][h*kh + c] for one row per thread: forward substitution z T = y with
// the upper factor T (staged in LDS, read uniformly), z in registers.
template <typename TY, int KH>
__global__ __launch_bounds__(256) void apply_tri_kernel(const TY* __restrict__ Y, int rows, int ldy, int kh,
                                                        const double* __restrict__ Tf, double* __restrict__ Q,
                                                        int ldq) {
  const int h = blockIdx.y;
  const int row = blockIdx.x * 256 + threadIdx.x;
  __shared__ double T[KH * KH];
  const double* __restrict__ Tg = Tf + (int64_t)h * kh * kh;
  for (int e = threadIdx.x; e < kh * kh; e += 256) T[e] = Tg[e];
  __syncthreads();
  if (row >= rows) return;
  const TY* y = Y + (int64_t)row * ldy + h * kh;
  double z[KH];
#pragma unroll
  for (int c = 0; c < KH; ++c) z[c] = c < kh ? (double)y[c] : 0.0;
#pragma unroll
  for (int c = 0; c < KH; ++c) {
    if (c < kh) {
      double s0 = z[c], s1 = 0.0;
#pragma unroll
      for (int l = 0; l < c; l += 2) {
        s0 = fma(-z[l], T[l * kh + c], s0);
        if (l + 1 < c) s1 = fma(-z[l + 1], T[(l + 1) * kh + c], s1);
      }
      z[c] = (s0 + s1) / T[c * kh + c];
    }
  }
  double* q = Q + (int64_t)row * ldq + h * kh;
#pragma unroll
  for (int c = 0; c < KH; ++c)
    if (c < kh) q[c] = z[c];
}

template <typename TY>
hipError_t launch_apply_tri(const TY* Y, int rows, int ldy, int nh, int kh, const double* Tf, double* Q64, int ldq,
                            hipStream_t st) {
  dim3 grid((rows + 255) / 256, nh);
  if (kh <= 16)
    hipLaunchKernelGGL((apply_tri_kernel<TY, 16>), grid, dim3(256), 0, st, Y, rows, ldy, kh, Tf, Q64, ldq);
  else if (kh <= 32)
    hipLaunchKernelGGL((apply_tri_kernel<TY, 32>), grid, dim3(256), 0, st, Y, rows, ldy, kh, Tf, Q64, ldq);
  else if (kh <= 48)
    hipLaunchKernelGGL((apply_tri_kernel<TY, 48>), grid, dim3(256), 0, st, Y, rows, ldy, kh, Tf, Q64, ldq);
  else if (kh <= 64)
    hipLaunchKernelGGL((apply_tri_kernel<TY, 64>), grid, dim3(256), 0, st, Y, rows, ldy, kh, Tf, Q64, ldq);
  else
    return hipErrorInvalidValue;
  CNMF_LAUNCH_CHECK();
}

hipError_t launch_gram_chol(const double* Gp, int parts, int nh, int kh, double* G, double* Tinv, int* flags,
                            unsigned* /*counters*/, hipStream_t st) {
  hipError_t e = launch_sum_parts(Gp, parts, (int64_t)nh * kh * kh, G, st);
  if (e != hipSuccess) return e;
  if (kh <= 64) {
    const int NB = (kh + 15) / 16, N = 16 * NB, ld = N + 1;
    size_t sm = ((size_t)N * ld + (size_t)NB * 272 + 16 * (size_t)ld) * sizeof(double);
    hipFuncSetAttribute((const void*)chol_fac_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    hipLaunchKernelGGL(chol_fac_kernel, dim3(nh), dim3(kFacNT), sm, st, G, kh, Tinv, flags);
  } else {
    size_t sm = ((size_t)kh * (kh + 1) + kh) * sizeof(double);
    hipFuncSetAttribute((const void*)chol_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    hipLaunchKernelGGL(chol_kernel, dim3(nh), dim3(kCholNT), sm, st, G, kh, Tinv, flags);
  }
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Q64[i][h*kh + c] = sum_{l <= c} Y[i][h*kh + l] Tinv_h[l][c]   (FP64)
// ---------------------------------------------------------------------------
template <typename TY>
__global__ __launch_bounds__(256) void apply_tinv_kernel(const TY* __restrict__ Y, int rows, int ldy, int kh,
                                                         const double* __restrict__ Tinv,
                                                         double* __restrict__ Q, int ldq, int rows_per_block,
                                                         int rb) {
  extern __shared__ double sm[];
  double* Ti = sm;               // kh x kh (upper part used)
  double* ys = sm + kh * kh;     // rb x kh rows
  const int h = blockIdx.y;
  const int tid = threadIdx.x;
  const double* Th = Tinv + (int64_t)h * kh * kh;
  for (int e = tid; e < kh * kh; e += 256) Ti[e] = Th[e];
  const int i0 = blockIdx.x * rows_per_block;
  const int i1 = min(rows, i0 + rows_per_block);
  for (int base = i0; base < i1; base += rb) {
    const int nr = min(rb, i1 - base);
    __syncthreads();
    for (int e = tid; e < nr * kh; e += 256) {
      int rr = e / kh, c = e - rr * kh;
      ys[e] = (double)Y[(int64_t)(base + rr) * ldy + h * kh + c];
    }
    __syncthreads();
    for (int e = tid; e < nr * kh; e += 256) {
      int rr = e / kh, c = e - rr * kh;
      const double* y = ys + rr * kh;
      double s0 = 0.0, s1 = 0.0;
      int l = 0;
      for (; l + 1 <= c; l += 2) {
        s0 = fma(y[l], Ti[l * kh + c], s0);
        s1 = fma(y[l + 1], Ti[(l + 1) * kh + c], s1);
      }
      if (l <= c) s0 = fma(y[l], Ti[l * kh + c], s0);
      Q[(int64_t)(base + rr) * ldq + h * kh + c] = s0 + s1;
    }
  }
}

template <typename TY>
hipError_t launch_apply_tinv(const TY* Y, int rows, int ldy, int nh, int kh, const double* Tinv,
                             double* Q64, int ldq, hipStream_t st) {
  if (kh <= 64) return launch_apply_tri<TY>(Y, rows, ldy, nh, kh, Tinv, Q64, ldq, st);
  const size_t cap = 160 * 1024;
  int rb = (int)std::min<size_t>(64, (cap - (size_t)kh * kh * 8) / ((size_t)kh * 8));
  rb = std::max(rb, 1);
  int blocks = std::max(1, std::min(512, (rows + 2 * rb - 1) / (2 * rb)));
  int rpb = (rows + blocks - 1) / blocks;
  size_t sm = ((size_t)kh * kh + (size_t)rb * kh) * sizeof(double);
  hipFuncSetAttribute((const void*)apply_tinv_kernel<TY>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL(apply_tinv_kernel<TY>, dim3(blocks, nh), dim3(256), sm, st, Y, rows, ldy, kh, Tinv, Q64,
                     ldq, rpb, rb);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_apply_tinv<float>(const float*, int, int, int, int, const double*, double*, int, hipStream_t);
template hipError_t launch_apply_tinv<double>(const double*, int, int, int, int, const double*, double*, int, hipStream_t);

// ---------------------------------------------------------------------------
// max |G - I| (G the Gram of an orthonormalised half)
// ---------------------------------------------------------------------------
__global__ void orth_error_kernel(const double* __restrict__ G, int kh, double* out) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int e = threadIdx.x; e < kh * kh; e += 256) {
    int i = e / kh, j = e - i * kh;
    mx = fmax(mx, fabs(G[e] - (i == j ? 1.0 : 0.0)));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_orth_error(const double* G, int kh, double* out, hipStream_t st) {
  hipLaunchKernelGGL(orth_error_kernel, dim3(1), dim3(256), 0, st, G, kh, out);
  CNMF_LAUNCH_CHECK();
}

}  // namespace cnmf
