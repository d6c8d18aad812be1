// Data movement, the reported residual and SPA.
#include <algorithm>
#include <type_traits>

#include "cnmf_internal.hpp"

namespace cnmf {

// ---------------------------------------------------------------------------
// dst[i][j] = TD(scale * src[i][j])
// ---------------------------------------------------------------------------
template <typename TD>
__device__ __forceinline__ TD cvt(double x) {
  return (TD)x;
}
template <>
__device__ __forceinline__ __hip_bfloat16 cvt<__hip_bfloat16>(double x) {
  return __float2bfloat16((float)x);
}

template <typename TS, typename TD>
__global__ void copy2d_kernel(const TS* __restrict__ src, int64_t lds, TD* __restrict__ dst, int64_t ldd,
                              int rows, int cols, double scale) {
  int64_t total = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / cols, j = e - i * cols;
    dst[i * ldd + j] = cvt<TD>(scale * (double)src[i * lds + j]);
  }
}

template <typename TS, typename TD>
hipError_t launch_copy2d(const TS* src, int64_t lds, TD* dst, int64_t ldd, int rows, int cols, double scale,
                         hipStream_t st) {
  int64_t total = (int64_t)rows * cols;
  if (total == 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL((copy2d_kernel<TS, TD>), dim3(blocks), dim3(256), 0, st, src, lds, dst, ldd, rows, cols,
                     scale);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_copy2d<double, double>(const double*, int64_t, double*, int64_t, int, int, double, hipStream_t);
template hipError_t launch_copy2d<double, float>(const double*, int64_t, float*, int64_t, int, int, double, hipStream_t);
template hipError_t launch_copy2d<float, float>(const float*, int64_t, float*, int64_t, int, int, double, hipStream_t);
template hipError_t launch_copy2d<float, double>(const float*, int64_t, double*, int64_t, int, int, double, hipStream_t);
template hipError_t launch_copy2d<double, __hip_bfloat16>(const double*, int64_t, __hip_bfloat16*, int64_t, int, int, double, hipStream_t);

// dst[i][j] += src[i][j] (sums over the row blocks of a streamed A^T Z pass,
// added in block order)
template <typename T>
__global__ void add2d_kernel(const T* __restrict__ src, int64_t lds, T* __restrict__ dst, int64_t ldd, int rows,
                             int cols) {
  int64_t total = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / cols, j = e - i * cols;
    dst[i * ldd + j] += src[i * lds + j];
  }
}

template <typename T>
hipError_t launch_add2d(const T* src, int64_t lds, T* dst, int64_t ldd, int rows, int cols, hipStream_t st) {
  int64_t total = (int64_t)rows * cols;
  if (total == 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL((add2d_kernel<T>), dim3(blocks), dim3(256), 0, st, src, lds, dst, ldd, rows, cols);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_add2d<float>(const float*, int64_t, float*, int64_t, int, int, hipStream_t);
template hipError_t launch_add2d<double>(const double*, int64_t, double*, int64_t, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// dst[j][i] = src[i][j] through a 32 x 32 LDS tile
// ---------------------------------------------------------------------------
template <typename TS, typename TD>
__global__ void transpose_kernel(const TS* __restrict__ src, int64_t lds, TD* __restrict__ dst, int64_t ldd,
                                 int rows, int cols) {
  __shared__ double tile[32][33];
  int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: ty 0..7
  for (int yy = ty; yy < 32; yy += 8) {
    int i = by + yy, j = bx + tx;
    tile[yy][tx] = (i < rows && j < cols) ? (double)src[(int64_t)i * lds + j] : 0.0;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    int j = bx + yy, i = by + tx;
    if (j < cols && i < rows) dst[(int64_t)j * ldd + i] = (TD)tile[tx][yy];
  }
}

template <typename TS, typename TD>
hipError_t launch_transpose(const TS* src, int64_t lds, TD* dst, int64_t ldd, int rows, int cols,
                            hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  dim3 grid((cols + 31) / 32, (rows + 31) / 32);
  hipLaunchKernelGGL((transpose_kernel<TS, TD>), grid, dim3(256), 0, st, src, lds, dst, ldd, rows, cols);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_transpose<double, double>(const double*, int64_t, double*, int64_t, int, int, hipStream_t);
template hipError_t launch_transpose<double, float>(const double*, int64_t, float*, int64_t, int, int, hipStream_t);
template hipError_t launch_transpose<float, float>(const float*, int64_t, float*, int64_t, int, int, hipStream_t);
template hipError_t launch_transpose<float, double>(const float*, int64_t, double*, int64_t, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// zero fill (a kernel, so it can live inside captured graphs)
// ---------------------------------------------------------------------------
__global__ void fill_kernel(uint32_t* __restrict__ p, size_t words) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < words; e += (size_t)gridDim.x * blockDim.x)
    p[e] = 0u;
}
__global__ void fill_bytes_kernel(uint8_t* __restrict__ p, size_t bytes) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < bytes; e += (size_t)gridDim.x * blockDim.x)
    p[e] = 0u;
}

hipError_t launch_fill(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if ((uintptr_t)p % 4 == 0 && bytes % 4 == 0) {
    size_t words = bytes / 4;
    int blocks = (int)std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, st, (uint32_t*)p, words);
  } else {
    int blocks = (int)std::min<size_t>((bytes + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_bytes_kernel, dim3(blocks), dim3(256), 0, st, (uint8_t*)p, bytes);
  }
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Relative residual ||A - U V||_F / ||A||_F.  A block takes 64 rows (wave w:
// rows 16 w .. 16 w + 15, whose U rows are the MFMA's left operands, held in
// registers) and a range of 64-column chunks.  Each chunk's V^T rows are
// staged in LDS (double buffered; the next chunk's V^T and A values are
// loaded while the current one is used), the U V tile is formed in T on the
// 16x16x4 MFMA, and the differences and squares are accumulated in FP64.
// partial[blk] = (sum (a - uv)^2, sum a^2), blk = y * gridDim.x + x.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void residual_kernel(const T* __restrict__ A, int64_t lda, int m, int n,
                                                       const T* __restrict__ U, int ldu,
                                                       const T* __restrict__ Vt, int ldv, int r, int chunks_per_split,
                                                       double* __restrict__ partial) {
  constexpr bool F32 = std::is_same<T, float>::value;
  typedef typename std::conditional<F32, floatx4, doublex4>::type acc_t;
  constexpr int LDV = 66;   // V^T chunk row stride in LDS (conflict-free FP32 operand reads)
  __shared__ T vs[2][64 * LDV];
  __shared__ double red[2][256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int row0 = blockIdx.x * 64;
  const int nch = (n + 63) / 64;
  const int ch0 = blockIdx.y * chunks_per_split, ch1 = min(nch, ch0 + chunks_per_split);
  const int KS = (r + 3) / 4;
  auto out_row = [&](int i) { return F32 ? 4 * g + i : g + 4 * i; };
  // U rows of the wave as left operands: lane (c, g), K step s -> U[row c][4 s + g]
  T ua[16];
  {
    const int ur = row0 + 16 * w + c;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int kk = 4 * s + g;
      ua[s] = (ur < m && kk < r) ? U[(int64_t)ur * ldu + kk] : T(0);
    }
  }
  T vreg[16];
  T areg[16], anext[16];   // raw A values (converted where they are used, so the prefetch does not wait)
  auto load_v = [&](int ch) {
    const int j0 = 64 * ch;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q, col = e >> 6, kk = e & 63;
      vreg[q] = (j0 + col < n && kk < r) ? Vt[(int64_t)(j0 + col) * ldv + kk] : T(0);
    }
  };
  auto store_v = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q, col = e >> 6, kk = e & 63;
      vs[buf][col * LDV + kk] = vreg[q];
    }
  };
  auto load_a = [&](int ch, T (&dst)[16]) {
    const int j0 = 64 * ch;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = row0 + 16 * w + out_row(i), col = j0 + 16 * cb + c;
        dst[4 * cb + i] = (row < m && col < n) ? A[(int64_t)row * lda + col] : T(0);
      }
  };
  double num = 0.0, den = 0.0;
  if (ch0 < ch1) {
    load_v(ch0);
    load_a(ch0, areg);
    store_v(0);
  }
  // every load so far (U operands included) has landed: the loop's MFMAs
  // then wait only for LDS, not for the next chunk's prefetch
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  __syncthreads();
  for (int ch = ch0; ch < ch1; ++ch) {
    const int buf = (ch - ch0) & 1;
    const bool more = ch + 1 < ch1;
    if (more) {
      load_v(ch + 1);
      load_a(ch + 1, anext);
    }
    const T* vb = vs[buf];
    acc_t acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      if (s < KS) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const T bv = vb[(16 * cb + c) * LDV + 4 * s + g];
          if constexpr (F32)
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[s], bv, acc[cb], 0, 0, 0);
          else
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[s], bv, acc[cb], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double a = (double)areg[4 * cb + i];
        const double d = a - (double)acc[cb][i];
        num = fma(d, d, num);
        den = fma(a, a, den);
      }
    if (more) {
      store_v(buf ^ 1);
#pragma unroll
      for (int q = 0; q < 16; ++q) areg[q] = anext[q];
    }
    __syncthreads();
  }
  red[0][tid] = num;
  red[1][tid] = den;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (tid < s2) {
      red[0][tid] += red[0][tid + s2];
      red[1][tid] += red[1][tid + s2];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    partial[2 * blk] = red[0][0];
    partial[2 * blk + 1] = red[1][0];
  }
}

// Blocks of the residual launch (its partial count): ceil(m / 64) row blocks
// times up to 4 column splits.
int residual_blocks(int m, int n) {
  const int rb = (m + 63) / 64, nch = (n + 63) / 64;
  const int cs = std::max(1, std::min({4, nch, (1024 + rb - 1) / rb}));
  return rb * cs;
}

template <typename T>
hipError_t launch_residual(const T* A, int64_t lda, int m, int n, const T* U, int ldu, const T* Vt, int ldv,
                           int r, double* partial, int parts, hipStream_t st) {
  if (r > 64 || m < 1 || n < 1) return hipErrorInvalidValue;
  const int rb = (m + 63) / 64, nch = (n + 63) / 64;
  const int cs = std::max(1, std::min({4, nch, (1024 + rb - 1) / rb}));
  if (rb * cs != parts) return hipErrorInvalidValue;
  const int cps = (nch + cs - 1) / cs;
  hipLaunchKernelGGL(residual_kernel<T>, dim3(rb, cs), dim3(256), 0, st, A, lda, m, n, U, ldu, Vt, ldv, r, cps,
                     partial);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_residual<float>(const float*, int64_t, int, int, const float*, int, const float*, int, int, double*, int, hipStream_t);
template hipError_t launch_residual<double>(const double*, int64_t, int, int, const double*, int, const double*, int, int, double*, int, hipStream_t);

__global__ void residual_finish_kernel(const double* __restrict__ partial, int parts, double* out) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  // fixed-order: thread t sums parts t, t+256, ...; then a fixed tree
  double num = 0.0, den = 0.0;
  for (int p = tid; p < parts; p += 256) {
    num += partial[2 * p];
    den += partial[2 * p + 1];
  }
  red[0][tid] = num;
  red[1][tid] = den;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] += red[0][tid + s];
      red[1][tid] += red[1][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) *out = red[1][0] > 0 ? sqrt(red[0][0]) / sqrt(red[1][0]) : 0.0;
}

hipError_t launch_residual_finish(const double* partial, int parts, double* out, hipStream_t st) {
  hipLaunchKernelGGL(residual_finish_kernel, dim3(1), dim3(256), 0, st, partial, parts, out);
  CNMF_LAUNCH_CHECK();
}

__global__ void flags_to_stats_kernel(const int* flags, int nflags, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nflags; ++i) s += (double)flags[i];
    *out = s;
  }
}

hipError_t launch_flags_to_stats(const int* flags, int nflags, double* out, hipStream_t st) {
  hipLaunchKernelGGL(flags_to_stats_kernel, dim3(1), dim3(64), 0, st, flags, nflags, out);
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// SPA (Section 4, Alg. SNMF step 2) on Bt = B^T (n x k, FP64 working copy).
// Selection step t is two launches:
//   spa_norms (all rows): t > 0: b_j <- b_j - u (u^T b_j) with u the previous
//     step's unit pivot; s_j = ||b_j||^2; block argmax (largest s, lowest j on
//     ties) into wg_best / wg_idx;
//   spa_pick (one block): argmax over the block winners, records K[t],
//     score[t] and u = b_p / sqrt(s_p) for the next step.
// Each norms block stages 64 rows in LDS; 4 threads per row.
// ---------------------------------------------------------------------------
constexpr int kSpaRows = 64;

__device__ __forceinline__ bool spa_better(double s1, int64_t j1, double s2, int64_t j2) {
  return s1 > s2 || (s1 == s2 && j1 < j2);
}

__global__ __launch_bounds__(256) void spa_norms_kernel(double* __restrict__ Bt, int n, int k, int ldb, int t,
                                                        const double* __restrict__ u, double* __restrict__ wg_best,
                                                        int64_t* __restrict__ wg_idx) {
  extern __shared__ double sm[];
  double* bs = sm;                 // kSpaRows x (k + 1)
  double* us = bs + kSpaRows * (k + 1);
  __shared__ double part[256];
  __shared__ double rs[kSpaRows];
  __shared__ int64_t ri[kSpaRows];
  const int tid = threadIdx.x;
  const int ld = k + 1;
  const int64_t row0 = (int64_t)blockIdx.x * kSpaRows;
  for (int e = tid; e < kSpaRows * k; e += 256) {
    int rr = e / k, a = e - rr * k;
    bs[rr * ld + a] = row0 + rr < n ? Bt[(row0 + rr) * ldb + a] : 0.0;
  }
  if (t > 0)
    for (int a = tid; a < k; a += 256) us[a] = u[a];
  __syncthreads();
  const int rr = tid >> 2, q = tid & 3;
  double* b = bs + rr * ld;
  if (t > 0) {
    double d = 0.0;
    for (int a = q; a < k; a += 4) d = fma(us[a], b[a], d);
    part[tid] = d;
    __syncthreads();
    // fixed combination order within the 4-thread group
    const int g0 = tid & ~3;
    const double dot = (part[g0] + part[g0 + 1]) + (part[g0 + 2] + part[g0 + 3]);
    for (int a = q; a < k; a += 4) b[a] = fma(-us[a], dot, b[a]);
    __syncthreads();
    for (int e = tid; e < kSpaRows * k; e += 256) {
      int r2 = e / k, a = e - r2 * k;
      if (row0 + r2 < n) Bt[(row0 + r2) * ldb + a] = bs[r2 * ld + a];
    }
  }
  double s = 0.0;
  for (int a = q; a < k; a += 4) s = fma(b[a], b[a], s);
  __syncthreads();
  part[tid] = s;
  __syncthreads();
  if (q == 0) {
    double tot = (part[tid] + part[tid + 1]) + (part[tid + 2] + part[tid + 3]);
    rs[rr] = (row0 + rr < n) ? tot : -1.0;
    ri[rr] = row0 + rr;
  }
  __syncthreads();
  if (tid == 0) {
    double bv = rs[0];
    int64_t bi = ri[0];
    for (int i = 1; i < kSpaRows; ++i)
      if (spa_better(rs[i], ri[i], bv, bi)) {
        bv = rs[i];
        bi = ri[i];
      }
    wg_best[blockIdx.x] = bv;
    wg_idx[blockIdx.x] = bi;
  }
}

__global__ __launch_bounds__(256) void spa_pick_kernel(const double* __restrict__ Bt, int k, int ldb, int t,
                                                       int nblocks, int64_t* __restrict__ K,
                                                       double* __restrict__ score, double* __restrict__ u,
                                                       const double* __restrict__ wg_best,
                                                       const int64_t* __restrict__ wg_idx) {
  __shared__ double tv[256];
  __shared__ int64_t ti[256];
  const int tid = threadIdx.x;
  // block winners in block order: thread-strided, then a fixed tree
  double bv = -2.0;
  int64_t bi = INT64_MAX;
  for (int p = tid; p < nblocks; p += 256) {
    double v = wg_best[p];
    int64_t i = wg_idx[p];
    if (spa_better(v, i, bv, bi)) {
      bv = v;
      bi = i;
    }
  }
  tv[tid] = bv;
  ti[tid] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w && spa_better(tv[tid + w], ti[tid + w], tv[tid], ti[tid])) {
      tv[tid] = tv[tid + w];
      ti[tid] = ti[tid + w];
    }
    __syncthreads();
  }
  const int64_t p = ti[0];
  const double sp = tv[0];
  if (tid == 0) {
    K[t] = p;
    if (score) score[t] = sp;
  }
  const double inv = sp > 0 ? 1.0 / sqrt(sp) : 0.0;
  for (int a = tid; a < k; a += 256) u[a] = Bt[p * ldb + a] * inv;
}

hipError_t launch_spa_step(double* Bt, int n, int k, int ldb, int t, int64_t* K, double* score, double* u,
                           double* wg_best, int64_t* wg_idx, unsigned* /*counter*/, int nblocks, hipStream_t st) {
  if (nblocks != (n + kSpaRows - 1) / kSpaRows) return hipErrorInvalidValue;
  size_t sm = ((size_t)kSpaRows * (k + 1) + k) * sizeof(double);
  hipFuncSetAttribute((const void*)spa_norms_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL(spa_norms_kernel, dim3(nblocks), dim3(256), sm, st, Bt, n, k, ldb, t, u, wg_best, wg_idx);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(spa_pick_kernel, dim3(1), dim3(256), 0, st, Bt, k, ldb, t, nblocks, K, score, u, wg_best,
                     wg_idx);
  CNMF_LAUNCH_CHECK();
}

}  // namespace cnmf
