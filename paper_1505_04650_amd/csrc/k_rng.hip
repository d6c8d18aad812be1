// Gaussian test matrices on the device (Alg. 1: "draw a Gaussian random
// matrix"), from the counter-based generator in rng.hpp.
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

}  // namespace cnmf
