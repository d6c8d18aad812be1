// Sparse A in compressed-row form (the paper's synthetic sparse inputs,
// Section 5.1): the passes of Alg. 1 and the small sketches multiply with A
// and A^T directly, and the FP64 residual is formed from the nonzeros and
// two r x r Gram matrices.
//
// A^T is built once per call as CSR of the transpose: a stable radix sort of
// the column indices (hipCUB) keeps the rows of each column in ascending
// order, so the transpose, and every product, is the same bit for bit from
// run to run.
#include <hipcub/hipcub.hpp>

#include "cnmf_internal.hpp"

namespace cnmf {

size_t csr_sort_temp_bytes(int nnz, int n) {
  size_t a = 0, b = 0;
  hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const int32_t*)nullptr, (int32_t*)nullptr,
                                     (const int32_t*)nullptr, (int32_t*)nullptr, std::max(nnz, 1));
  hipcub::DeviceScan::InclusiveSum(nullptr, b, (const int64_t*)nullptr, (int64_t*)nullptr, std::max(n, 1));
  return std::max(a, b) + 256;
}

__global__ void iota_kernel(int32_t* __restrict__ p, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = (int32_t)e;
}

// cnt[c + 1] += 1 for every nonzero in column c (cnt zeroed, n + 1 words)
__global__ void col_count_kernel(const int32_t* __restrict__ col, int64_t nnz, int n, int64_t* __restrict__ cnt,
                                 int* __restrict__ bad) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = col[e];
    if (c >= 0 && c < n)
      atomicAdd((unsigned long long*)(cnt + c + 1), 1ull);
    else
      atomicAdd(bad, 1);
  }
}

// Row of nonzero p: the last i with rowptr[i] <= p (rowptr nondecreasing).
__device__ __forceinline__ int row_of(const int64_t* __restrict__ rowptr, int m, int64_t p) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rowptr[mid] <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__global__ void csr_t_fill_kernel(const int64_t* __restrict__ rowptr, int m, const T* __restrict__ val,
                                  const int32_t* __restrict__ perm, int64_t nnz, int32_t* __restrict__ tcol,
                                  T* __restrict__ tval) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = perm[e];
    tcol[e] = row_of(rowptr, m, p);
    tval[e] = val[p];
  }
}

template <typename T>
hipError_t launch_csr_transpose(const int64_t* rowptr, const int32_t* col, const T* val, int m, int n, int64_t nnz,
                                int64_t* trow, int32_t* tcol, T* tval, int32_t* keys, int32_t* perm,
                                int32_t* keys_out, int32_t* perm_out, void* tmp, size_t tmp_bytes, int* bad,
                                hipStream_t st) {
  hipError_t e = hipMemcpyAsync(keys, col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  const int g = (int)std::min<int64_t>((std::max<int64_t>(nnz, 1) + 255) / 256, 4096);
  e = launch_fill(trow, sizeof(int64_t) * ((size_t)n + 1), st);
  if (e != hipSuccess) return e;
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3(g), dim3(256), 0, st, perm, nnz);
  hipLaunchKernelGGL(col_count_kernel, dim3(g), dim3(256), 0, st, col, nnz, n, trow, bad);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int end_bit = 1;
  while (end_bit < 31 && (1ll << end_bit) < (int64_t)n) ++end_bit;
  size_t tb = tmp_bytes;
  e = hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys, keys_out, perm, perm_out, (int)nnz, 0, end_bit, st);
  if (e != hipSuccess) return e;
  tb = tmp_bytes;
  e = hipcub::DeviceScan::InclusiveSum(tmp, tb, trow + 1, trow + 1, n, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((csr_t_fill_kernel<T>), dim3(g), dim3(256), 0, st, rowptr, m, val, perm_out, nnz, tcol, tval);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_csr_transpose<float>(const int64_t*, const int32_t*, const float*, int, int, int64_t,
                                                int64_t*, int32_t*, float*, int32_t*, int32_t*, int32_t*, int32_t*,
                                                void*, size_t, int*, hipStream_t);
template hipError_t launch_csr_transpose<double>(const int64_t*, const int32_t*, const double*, int, int, int64_t,
                                                 int64_t*, int32_t*, double*, int32_t*, int32_t*, int32_t*, int32_t*,
                                                 void*, size_t, int*, hipStream_t);

// Y (rows x kk) = S X for a CSR S (rows x cols, nnz nonzeros) and a
// row-major X (cols x kk): one wave per row (grid-stride), lane c holding
// columns c, c + 64, ... of the row; the row's nonzeros are taken in order,
// so each sum has a fixed order.  Row offsets are clamped to [0, nnz] and a
// column index outside [0, cols) is skipped (the transpose's column count
// reports them).
template <typename T, int NC>
__global__ __launch_bounds__(256) void csr_spmm_kernel(const int64_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col, const T* __restrict__ val,
                                                       int rows, int cols, int64_t nnz, const T* __restrict__ X,
                                                       int kk, T* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  for (int i = w; i < rows; i += gridDim.x * 4) {
    T acc[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] = (T)0;
    const int64_t p0 = max((int64_t)0, rowptr[i]), p1 = min(nnz, rowptr[i + 1]);
    // eight nonzeros at a time: their indices and values first, then the
    // operand rows, so that the gathers of a group are in flight together
    // (the order of the additions is still p0, p0 + 1, ...)
    constexpr int G = 8;
    for (int64_t q = p0; q < p1; q += G) {
      int cg[G];
      T ag[G];
      bool okg[G];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const bool in = q + u < p1;
        const int c = in ? col[q + u] : -1;
        okg[u] = c >= 0 && c < cols;
        cg[u] = okg[u] ? c : 0;
        ag[u] = okg[u] ? val[q + u] : (T)0;
      }
      T xg[G][NC];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const T* x = X + (int64_t)cg[u] * kk;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const int cc = lane + 64 * j;
          xg[u][j] = cc < kk ? x[cc] : (T)0;
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u)
        if (okg[u])   // the same for every lane: col and the bounds are wave-uniform
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[j] = fma(ag[u], xg[u][j], acc[j]);
    }
    T* y = Y + (int64_t)i * kk;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int cc = lane + 64 * j;
      if (cc < kk) y[cc] = acc[j];
    }
  }
}

template <typename T>
hipError_t launch_csr_spmm(const int64_t* rowptr, const int32_t* col, const T* val, int rows, int cols, int64_t nnz,
                           const T* X, int kk, T* Y, hipStream_t st) {
  if (kk < 1 || kk > 256) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>(((int64_t)rows + 3) / 4, 8192);
  if (kk <= 64)
    hipLaunchKernelGGL((csr_spmm_kernel<T, 1>), dim3(grid), dim3(256), 0, st, rowptr, col, val, rows, cols, nnz, X,
                       kk, Y);
  else if (kk <= 128)
    hipLaunchKernelGGL((csr_spmm_kernel<T, 2>), dim3(grid), dim3(256), 0, st, rowptr, col, val, rows, cols, nnz, X,
                       kk, Y);
  else
    hipLaunchKernelGGL((csr_spmm_kernel<T, 4>), dim3(grid), dim3(256), 0, st, rowptr, col, val, rows, cols, nnz, X,
                       kk, Y);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_csr_spmm<float>(const int64_t*, const int32_t*, const float*, int, int, int64_t,
                                           const float*, int, float*, hipStream_t);
template hipError_t launch_csr_spmm<double>(const int64_t*, const int32_t*, const double*, int, int, int64_t,
                                            const double*, int, double*, hipStream_t);

// Residual terms over the nonzeros, FP64: per workgroup, sum a_ij^2 and
// sum a_ij (U_i . V_j) (U m x r, Vt n x r, ld r).  One wave per row; lane l
// takes the row's nonzeros l, l + 64, ...  Partials [block][2].
template <typename T>
__global__ __launch_bounds__(256) void csr_resid_kernel(const int64_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col, const T* __restrict__ val,
                                                        int rows, int cols, int64_t nnz, const T* __restrict__ U,
                                                        const T* __restrict__ Vt, int r, double* __restrict__ part) {
  __shared__ double red[2][256];
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  double asq = 0.0, cross = 0.0;
  for (int i = w; i < rows; i += gridDim.x * 4) {
    const int64_t p0 = max((int64_t)0, rowptr[i]), p1 = min(nnz, rowptr[i + 1]);
    const T* u = U + (int64_t)i * r;
    for (int64_t p = p0 + lane; p < p1; p += 64) {
      const int c = col[p];
      if (c < 0 || c >= cols) continue;
      const double a = (double)val[p];
      const T* v = Vt + (int64_t)c * r;
      double d = 0.0;
      for (int l = 0; l < r; ++l) d = fma((double)u[l], (double)v[l], d);
      asq = fma(a, a, asq);
      cross = fma(a, d, cross);
    }
  }
  red[0][threadIdx.x] = asq;
  red[1][threadIdx.x] = cross;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

// ||A - U V||_F^2 = sum a^2 - 2 sum a (U V)_ij + sum (U^T U) o (V V^T), all
// in FP64; out = sqrt(max(that, 0)) / sqrt(sum a^2).
__global__ void csr_resid_finish_kernel(const double* __restrict__ part, int parts, const double* __restrict__ GU,
                                        const double* __restrict__ GV, int r, double* out) {
  __shared__ double red[3][256];
  const int tid = threadIdx.x;
  double a = 0.0, c = 0.0, g = 0.0;
  for (int p = tid; p < parts; p += 256) {
    a += part[2 * p];
    c += part[2 * p + 1];
  }
  for (int e = tid; e < r * r; e += 256) g = fma(GU[e], GV[e], g);
  red[0][tid] = a;
  red[1][tid] = c;
  red[2][tid] = g;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s)
      for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    const double asq = red[0][0];
    const double num = asq - 2.0 * red[1][0] + red[2][0];
    *out = asq > 0.0 ? sqrt(num > 0.0 ? num : 0.0) / sqrt(asq) : 0.0;
  }
}

int csr_resid_blocks(int rows) { return (int)std::min<int64_t>(((int64_t)rows + 3) / 4, 1024); }

template <typename T>
hipError_t launch_csr_resid(const int64_t* rowptr, const int32_t* col, const T* val, int rows, int cols, int64_t nnz,
                            const T* U, const T* Vt, int r, double* part, hipStream_t st) {
  hipLaunchKernelGGL((csr_resid_kernel<T>), dim3(csr_resid_blocks(rows)), dim3(256), 0, st, rowptr, col, val, rows,
                     cols, nnz, U, Vt, r, part);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_csr_resid<float>(const int64_t*, const int32_t*, const float*, int, int, int64_t,
                                            const float*, const float*, int, double*, hipStream_t);
template hipError_t launch_csr_resid<double>(const int64_t*, const int32_t*, const double*, int, int, int64_t,
                                             const double*, const double*, int, double*, hipStream_t);

hipError_t launch_csr_resid_finish(const double* part, int parts, const double* GU, const double* GV, int r,
                                   double* out, hipStream_t st) {
  hipLaunchKernelGGL(csr_resid_finish_kernel, dim3(1), dim3(256), 0, st, part, parts, GU, GV, r, out);
  CNMF_LAUNCH_CHECK();
}

}  // namespace cnmf
