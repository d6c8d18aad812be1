// Orthonormalisation of the tall range samples (Alg. 1, QR step) by
// CholeskyQR2 in FP64, plus the small k x k products of the sketch.
//   G = Y^T Y (FP64 accumulation, deterministic partials)
//   T = chol(G) upper with positive diagonal, Tinv = T^-1
//   Q = Y Tinv; repeat once on Q (the second pass restores orthogonality
//   to working precision).
// With diag(T) > 0 this Q is the same basis as the Householder QR with a
// nonnegative diagonal for full-column-rank Y.
#include "cnmf_internal.hpp"

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
__global__ void sum_parts_kernel(const double* __restrict__ in, int parts, int64_t count,
                                 double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int p = 0; p < parts; ++p) acc += in[p * count + e];
    out[e] = acc;
  }
}

hipError_t launch_sum_parts(const double* in, int parts, int64_t count, double* out, hipStream_t st) {
  int blocks = (int)std::min<int64_t>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(blocks), dim3(256), 0, st, in, parts, count, out);
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Cholesky G = T^T T (T upper, positive diagonal) and Tinv = T^-1, one
// workgroup per half.  Upper triangles are packed in LDS:
//   idx(i, j) = i*kh - i*(i-1)/2 + (j - i), j >= i.
// A pivot <= tol * max_i G_ii (or not finite) is a breakdown: flags[h] += 1
// and the pivot is replaced by tol * max_i G_ii so the factor stays finite.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pk(int i, int j, int kh) { return i * kh - (i * (i - 1)) / 2 + (j - i); }

__global__ __launch_bounds__(256) void chol_inv_kernel(const double* __restrict__ G, int kh,
                                                       double* __restrict__ Tinv, int* flags,
                                                       double tol) {
  extern __shared__ double sm[];
  const int np = kh * (kh + 1) / 2;
  double* S = sm;        // packed T
  double* Ti = sm + np;  // packed Tinv
  __shared__ double s_piv;
  __shared__ double s_maxd;
  const int h = blockIdx.x;
  const double* Gh = G + (int64_t)h * kh * kh;
  const int tid = threadIdx.x;
  for (int e = tid; e < kh * kh; e += 256) {
    int i = e / kh, j = e - i * kh;
    if (j >= i) S[pk(i, j, kh)] = 0.5 * (Gh[i * kh + j] + Gh[j * kh + i]);
  }
  __syncthreads();
  if (tid == 0) {
    double md = 0.0;
    for (int i = 0; i < kh; ++i) md = fmax(md, S[pk(i, i, kh)]);
    s_maxd = md;
  }
  __syncthreads();
  const double floor_piv = tol * s_maxd;
  for (int j = 0; j < kh; ++j) {
    if (tid == 0) {
      double d = S[pk(j, j, kh)];
      if (!(d > floor_piv) || !isfinite(d)) {
        d = floor_piv > 0 ? floor_piv : 1.0;
        if (flags) atomicAdd(&flags[h], 1);
      }
      s_piv = sqrt(d);
      S[pk(j, j, kh)] = s_piv;
    }
    __syncthreads();
    const double t = s_piv;
    for (int c = j + 1 + tid; c < kh; c += 256) S[pk(j, c, kh)] /= t;
    __syncthreads();
    // trailing update: S[a][b] -= S[j][a] S[j][b], j < a <= b
    const int rem = kh - j - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      int a = e / rem, b = e - a * rem;
      if (b >= a) {
        a += j + 1;
        b += j + 1;
        S[pk(a, b, kh)] -= S[pk(j, a, kh)] * S[pk(j, b, kh)];
      }
    }
    __syncthreads();
  }
  // Tinv by rows from the bottom: Ti[i][i] = 1/T_ii,
  // Ti[i][j] = -(sum_{l=i+1..j} T[i][l] Ti[l][j]) / T_ii.
  for (int i = kh - 1; i >= 0; --i) {
    const double tii = S[pk(i, i, kh)];
    for (int j = i + tid; j < kh; j += 256) {
      if (j == i) {
        Ti[pk(i, i, kh)] = 1.0 / tii;
      } else {
        double s = 0.0;
        for (int l = i + 1; l <= j; ++l) s = fma(S[pk(i, l, kh)], Ti[pk(l, j, kh)], s);
        Ti[pk(i, j, kh)] = -s / tii;
      }
    }
    __syncthreads();
  }
  double* out = Tinv + (int64_t)h * kh * kh;
  for (int e = tid; e < kh * kh; e += 256) {
    int i = e / kh, j = e - i * kh;
    out[e] = (j >= i) ? Ti[pk(i, j, kh)] : 0.0;
  }
}

hipError_t launch_chol_inv(const double* G, int nh, int kh, double* Tinv, double* /*Tacc*/, int* flags,
                           hipStream_t st) {
  size_t sm = (size_t)kh * (kh + 1) * sizeof(double);  // two packed triangles
  hipFuncSetAttribute((const void*)chol_inv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL(chol_inv_kernel, dim3(nh), dim3(256), sm, st, G, kh, Tinv, flags, 1e-28);
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Q64[i][h*kh + c] = sum_{l <= c} Y[i][h*kh + l] Tinv_h[l][c]   (FP64)
// ---------------------------------------------------------------------------
template <typename TY>
__global__ __launch_bounds__(256) void apply_tinv_kernel(const TY* __restrict__ Y, int rows, int ldy,
                                                         int kh, const double* __restrict__ Tinv,
                                                         double* __restrict__ Q, int ldq,
                                                         int rows_per_block) {
  extern __shared__ double sm[];
  double* Ti = sm;               // kh x kh (full, upper part used)
  double* ys = sm + kh * kh;     // RB x kh rows
  const int h = blockIdx.y;
  const int tid = threadIdx.x;
  const double* Th = Tinv + (int64_t)h * kh * kh;
  for (int e = tid; e < kh * kh; e += 256) Ti[e] = Th[e];
  const int RBK = 256 / kh > 0 ? 256 / kh : 1;  // rows per sweep
  const int i0 = blockIdx.x * rows_per_block;
  const int i1 = min(rows, i0 + rows_per_block);
  __syncthreads();
  for (int base = i0; base < i1; base += RBK) {
    for (int e = tid; e < RBK * kh; e += 256) {
      int rr = e / kh, c = e - rr * kh;
      int row = base + rr;
      ys[e] = row < i1 ? (double)Y[(int64_t)row * ldy + h * kh + c] : 0.0;
    }
    __syncthreads();
    if (tid < RBK * kh) {
      int rr = tid / kh, c = tid - rr * kh;
      int row = base + rr;
      const double* y = ys + rr * kh;
      double s = 0.0;
      for (int l = 0; l <= c; ++l) s = fma(y[l], Ti[l * kh + c], s);
      if (row < i1) Q[(int64_t)row * ldq + h * kh + c] = s;
    }
    __syncthreads();
  }
}

template <typename TY>
hipError_t launch_apply_tinv(const TY* Y, int rows, int ldy, int nh, int kh, const double* Tinv,
                             double* Q64, int ldq, hipStream_t st) {
  int blocks = std::max(1, std::min(1024, (rows + 63) / 64));
  int rpb = (rows + blocks - 1) / blocks;
  int rbk = std::max(1, 256 / kh);
  size_t sm = ((size_t)kh * kh + (size_t)rbk * kh) * sizeof(double);
  hipFuncSetAttribute((const void*)apply_tinv_kernel<TY>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL(apply_tinv_kernel<TY>, dim3(blocks, nh), dim3(256), sm, st, Y, rows, ldy, kh, Tinv,
                     Q64, ldq, rpb);
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
