// Right factor of compressed separable NMF (Section 4, Alg. SNMF, last
// step; Eq. snmf_right_factor_col): for every column j of the compressed
// matrix B (k x n) and the selected columns K (r of them),
//   H[:, j] = argmin_{h >= 0} || B[:, j] - B[:, K] h ||_2,
// n independent nonnegative least-squares problems with the same matrix
// C = B[:, K].  They are solved on the normal equations, G h = c_j with
// G = C^T C (shared) and c_j = C^T B[:, j], by the Lawson-Hanson
// active-set method, one wave per column, FP64.
#include "cnmf_internal.hpp"
#include "small_dense.hpp"

namespace cnmf {

// c_j = C^T b_j for every column: Cr[j * r + i] = sum_a Bt[K_i][a] Bt[j][a],
// one thread per (j, i); Bt is B^T (n x k, ld ldbt).  An index K_i outside
// [0, n) is reported in info[2] and its row of Cr is zero.
__global__ __launch_bounds__(256) void nnls_rhs_kernel(const double* __restrict__ Bt, int64_t ldbt, int n, int k,
                                                       int r, const int64_t* __restrict__ K, double* __restrict__ Cr,
                                                       int* info) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n * r) return;
  const int j = (int)(t / r), i = (int)(t - (int64_t)j * r);
  const int64_t ki = K[i];
  double s = 0.0;
  if (ki >= 0 && ki < n) {
    const double* a = Bt + ki * ldbt;
    const double* b = Bt + (int64_t)j * ldbt;
    for (int e = 0; e < k; ++e) s = fma(a[e], b[e], s);
  } else if (j == 0) {
    atomicAdd(info + 2, 1);
  }
  Cr[t] = s;
}

// Masked solve on one wave (lane i: variable i, RM = rows padded): z with
// G_PP z_P = c_P and z_i = 0 off P, P given as the wave-uniform bit mask pm.
// Gauss-Jordan on the rows held in registers (row i of [M | rhs] by lane i,
// M = G on P x P, the identity elsewhere); only the passive pivots are
// eliminated (the other columns are already unit columns).  G is SPD, so
// no pivoting is needed.
template <int RM>
__device__ __forceinline__ double nnls_masked_solve(const double* Gs, int r, uint64_t pm, double c) {
  const int lane = threadIdx.x & 63;
  const int row = min(lane, RM - 1);   // lanes past RM hold identity rows; keep their reads inside G
  const bool pi = (pm >> lane) & 1ull;
  double aug[RM + 1];
#pragma unroll
  for (int l = 0; l < RM; ++l) {
    const bool pl = (pm >> l) & 1ull;
    const double gv = Gs[row * RM + l];
    aug[l] = (pi && pl) ? gv : (lane == l ? 1.0 : 0.0);
  }
  aug[RM] = pi ? c : 0.0;
  double mydiag = 1.0;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    if (j < r && ((pm >> j) & 1ull)) {
      const double piv = readlane_d(aug[j], j);
      mydiag = lane == j ? piv : mydiag;
      const double f = lane == j ? 0.0 : aug[j] / piv;
#pragma unroll
      for (int l = j; l <= RM; ++l) aug[l] = fma(-f, readlane_d(aug[l], j), aug[l]);
    }
  }
  return pi ? aug[RM] / mydiag : 0.0;
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

// One wave per column (grid-stride over the columns).  Lawson-Hanson:
// start from h = 0 with every variable at its bound; repeatedly free the
// bound variable whose dual w_i = (c - G h)_i is largest (lowest index on
// ties) while it exceeds tol = 1e-13 max|c|; solve the free system; if a
// free variable comes out <= 0, move from h towards the solution until the
// first one reaches 0, bind every variable at 0 and solve again (a variable
// bound again within its own step is not freed again).  At most
// 3 r outer steps; a column that needs more is counted in info[0] (its last
// feasible h is kept).  info[1]: largest number of outer steps.
template <int RM>
__global__ __launch_bounds__(256) void nnls_kernel(const double* __restrict__ Bt, int64_t ldbt, int n, int k, int r,
                                                   const int64_t* __restrict__ K, const double* __restrict__ Cr,
                                                   double* __restrict__ H, int64_t ldh, int* info) {
  __shared__ double Gs[RM * RM];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // G = C^T C on this workgroup (padded with zeros)
  for (int e = threadIdx.x; e < RM * RM; e += 256) {
    const int i = e / RM, l = e - i * RM;
    double s = 0.0;
    if (i < r && l < r) {
      const int64_t ki = K[i], kl = K[l];
      if (ki >= 0 && ki < n && kl >= 0 && kl < n) {
        const double* a = Bt + ki * ldbt;
        const double* b = Bt + kl * ldbt;
        for (int t = 0; t < k; ++t) s = fma(a[t], b[t], s);
      }
    }
    Gs[e] = s;
  }
  __syncthreads();
  const bool real = lane < r;
  int worst = 0, failed = 0;
  for (int j = blockIdx.x * 4 + w; j < n; j += gridDim.x * 4) {
    const double c = real ? Cr[(int64_t)j * r + lane] : 0.0;
    const double tol = 1e-13 * wave_max_d(fabs(c));
    double h = 0.0;
    uint64_t pm = 0;
    int outer = 0;
    bool ok = true;
    double wdual = c;
    uint64_t excl = 0;   // variables that came straight back to their bound (anti-cycling)
    while (true) {
      // the bound variable with the largest dual above tol (lowest index on ties)
      const double cand =
          (real && !(((pm | excl) >> lane) & 1ull) && wdual > tol) ? wdual : -1.0;
      const double best = wave_max_d(cand);
      if (!(best > 0.0)) break;
      const uint64_t at = __ballot(cand == best);
      const int p = __builtin_ctzll(at);
      if (++outer > 3 * r) {
        ok = false;
        break;
      }
      pm |= 1ull << p;
      for (int inner = 0; inner <= r; ++inner) {
        const double z = nnls_masked_solve<RM>(Gs, r, pm, c);
        const bool pi = (pm >> lane) & 1ull;
        const bool bad = pi && !(z > 0.0);
        if (__ballot(bad) == 0) {
          h = z;
          break;
        }
        // step from h towards z until the first free variable reaches 0
        const double ratio = bad ? (h - z > 0.0 ? h / (h - z) : 0.0) : 2.0;
        const double alpha = wave_min_d(ratio);
        const double hn = h + alpha * (z - h);
        const bool drop = pi && (bad ? ratio <= alpha : false);
        const bool keep = pi && !drop && hn > 0.0;
        pm = __ballot(keep);
        h = keep ? hn : 0.0;
      }
      // a variable freed and bound again at once (its dual was positive only
      // by rounding) is not freed again for this column
      if (!((pm >> p) & 1ull)) excl |= 1ull << p;
      // dual w = c - G h over the free variables
      double gh = 0.0;
      uint64_t rest = pm;
      while (rest) {
        const int l = __builtin_ctzll(rest);
        rest &= rest - 1;
        gh = fma(Gs[min(lane, RM - 1) * RM + l], readlane_d(h, l), gh);
      }
      wdual = c - gh;
    }
    worst = max(worst, outer);
    failed += ok ? 0 : 1;
    if (real) H[(int64_t)lane * ldh + j] = h;
  }
  if (lane == 0) {
    if (failed) atomicAdd(info, failed);
    atomicMax(info + 1, worst);
  }
}

hipError_t launch_snmf_nnls(const double* Bt, int64_t ldbt, int n, int k, int r, const int64_t* K, double* Cr,
                            double* H, int64_t ldh, int* info, hipStream_t st) {
  if (r < 1 || r > 64 || k < 1 || n < 1) return hipErrorInvalidValue;
  const int64_t nr = (int64_t)n * r;
  hipLaunchKernelGGL(nnls_rhs_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, Bt, ldbt, n, k, r, K, Cr,
                     info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int grid = (int)std::min<int64_t>(((int64_t)n + 3) / 4, 2048);
  if (r <= 8)
    hipLaunchKernelGGL(nnls_kernel<8>, dim3(grid), dim3(256), 0, st, Bt, ldbt, n, k, r, K, Cr, H, ldh, info);
  else if (r <= 16)
    hipLaunchKernelGGL(nnls_kernel<16>, dim3(grid), dim3(256), 0, st, Bt, ldbt, n, k, r, K, Cr, H, ldh, info);
  else if (r <= 24)
    hipLaunchKernelGGL(nnls_kernel<24>, dim3(grid), dim3(256), 0, st, Bt, ldbt, n, k, r, K, Cr, H, ldh, info);
  else if (r <= 32)
    hipLaunchKernelGGL(nnls_kernel<32>, dim3(grid), dim3(256), 0, st, Bt, ldbt, n, k, r, K, Cr, H, ldh, info);
  else if (r <= 48)
    hipLaunchKernelGGL(nnls_kernel<48>, dim3(grid), dim3(256), 0, st, Bt, ldbt, n, k, r, K, Cr, H, ldh, info);
  else
    hipLaunchKernelGGL(nnls_kernel<64>, dim3(grid), dim3(256), 0, st, Bt, ldbt, n, k, r, K, Cr, H, ldh, info);
  CNMF_LAUNCH_CHECK();
}

}  // namespace cnmf
