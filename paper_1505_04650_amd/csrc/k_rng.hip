// Test matrices on the device, from the counter-based generator in rng.hpp:
// Gaussian (Alg. 1: "draw a Gaussian random matrix") and the subsampled
// randomized Hadamard transform that Section 2 names as an alternative
// (remark after Thm. 3).
#include "cnmf_internal.hpp"
#include "rng.hpp"

namespace cnmf {

// One thread per entry pair (row i, columns 2p and 2p + 1): consecutive
// threads write consecutive pairs of a row.
__global__ __launch_bounds__(256) void gaussian_fill_kernel(double* __restrict__ out, int64_t ld, int rows, int cols,
                                                            uint64_t seed, uint32_t id) {
  const int pairs = (cols + 1) >> 1;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)rows * pairs) return;
  const int i = (int)(t / pairs), p = (int)(t - (int64_t)i * pairs);
  double z0, z1;
  gauss_pair(seed, id, (uint32_t)i, (uint32_t)p, z0, z1);
  double* o = out + (int64_t)i * ld + 2 * p;
  o[0] = z0;
  if (2 * p + 1 < cols) o[1] = z1;
}

hipError_t launch_gaussian_fill(double* out, int64_t ld, int rows, int cols, uint64_t seed, uint32_t id,
                                hipStream_t st) {
  if (rows < 0 || cols < 0 || ld < cols) return hipErrorInvalidValue;
  const int64_t work = (int64_t)rows * ((cols + 1) / 2);
  if (work == 0) return hipSuccess;
  hipLaunchKernelGGL(gaussian_fill_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, out, ld, rows,
                     cols, seed, id);
  CNMF_LAUNCH_CHECK();
}

// SRHT: for `rows` rows padded to p = 2^ceil(log2 rows), Omega = D H S /
// sqrt(k) with D random signs, H the p x p Walsh-Hadamard (Sylvester)
// matrix, entries (-1)^popcount(i & j), and S k distinct sampled columns;
// entry (i, c) = d_i (-1)^popcount(i & s_c) / sqrt(k).  d_i = -1 when bit 0
// of word x0 of the counter (0, i, id, 1) is set; s_c for c = 0, 1, ... is
// the first of the words x0 of the counters (c, t, id, 2), t = 0, 1, ...,
// masked to [0, p), not taken by s_0..s_{c-1}; after 64 taken draws, the
// first free index at or after the last draw (cyclically).
__device__ __forceinline__ uint32_t philox_word0(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  return c0;
}

// One wave: s_0..s_{k-1} in order (the lanes test a candidate against the
// taken indices together).
__global__ void srht_sample_kernel(int32_t* __restrict__ S, uint32_t p, int k, uint64_t seed, uint32_t id) {
  __shared__ int32_t taken[128];
  const int lane = threadIdx.x;
  for (int c = 0; c < k; ++c) {
    uint32_t v = 0;
    bool found = false;
    for (int t = 0; t < 64 && !found; ++t) {
      v = philox_word0(seed, (uint32_t)c, (uint32_t)t, id, 2u) & (p - 1);
      bool clash = false;
      for (int j = lane; j < c; j += 64) clash |= taken[j] == (int32_t)v;
      found = __ballot(clash) == 0;
    }
    while (!found) {   // at most c further probes: c < k <= p indices are taken
      v = (v + 1) & (p - 1);
      bool clash = false;
      for (int j = lane; j < c; j += 64) clash |= taken[j] == (int32_t)v;
      found = __ballot(clash) == 0;
    }
    if (lane == 0) taken[c] = (int32_t)v;
    __syncthreads();
  }
  for (int j = lane; j < k; j += 64) S[j] = taken[j];
}

__global__ __launch_bounds__(256) void srht_fill_kernel(double* __restrict__ out, int64_t ld, int rows, int cols,
                                                        const int32_t* __restrict__ S, uint64_t seed, uint32_t id) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)rows * cols) return;
  const int i = (int)(t / cols), c = (int)(t - (int64_t)i * cols);
  const bool neg_d = philox_word0(seed, 0u, (uint32_t)i, id, 1u) & 1u;
  const bool neg_h = __popc((uint32_t)i & (uint32_t)S[c]) & 1;
  const double a = 1.0 / sqrt((double)cols);
  out[(int64_t)i * ld + c] = (neg_d != neg_h) ? -a : a;
}

hipError_t launch_srht_fill(double* out, int64_t ld, int rows, int cols, uint64_t seed, uint32_t id, int32_t* S,
                            hipStream_t st) {
  if (rows < 1 || cols < 1 || cols > 128 || ld < cols) return hipErrorInvalidValue;
  uint32_t p = 1;
  while (p < (uint32_t)rows) p <<= 1;
  if ((uint32_t)cols > p) return hipErrorInvalidValue;
  hipLaunchKernelGGL(srht_sample_kernel, dim3(1), dim3(64), 0, st, S, p, cols, seed, id);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t work = (int64_t)rows * cols;
  hipLaunchKernelGGL(srht_fill_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, out, ld, rows, cols, S,
                     seed, id);
  CNMF_LAUNCH_CHECK();
}

}  // namespace cnmf
