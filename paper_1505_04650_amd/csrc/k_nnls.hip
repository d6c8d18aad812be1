// Batched nonnegative least squares on one wave per problem, FP64, for
//  * the right factor of compressed separable NMF (Section 4, Alg. SNMF,
//    last step; Eq. snmf_right_factor_col): for every column j of the
//    compressed matrix B (k x n) and the selected columns K (r of them),
//      H[:, j] = argmin_{h >= 0} || B[:, j] - B[:, K] h ||_2;
//  * the half-steps of compressed alternating NNLS (Section 3,
//    Eq. alternateLS_nmf_compressed): every row of X against (Y R^T)^T and
//    every column of Y against L^T X (and their uncompressed forms).
// Every problem of a launch shares its matrix C (k x r), so the problems are
// solved on the normal equations, G h = c with G = C^T C shared (in LDS) and
// c = C^T b per problem, by the Lawson-Hanson active-set method.
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
// eliminated, and a pivot row is applied only to the columns still needed:
// the later passive ones and the right-hand side (the other entries of the
// pivot row are zero, and eliminated columns are not read again).  G is SPD,
// so no pivoting is needed.
template <int RM>
__device__ __noinline__ double nnls_masked_solve(const double* Gs, int r, uint64_t pm, double c) {
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
      for (int l = j + 1; l < RM; ++l)
        if ((pm >> l) & 1ull) aug[l] = fma(-f, readlane_d(aug[l], j), aug[l]);
      aug[RM] = fma(-f, readlane_d(aug[RM], j), aug[RM]);
    }
  }
  return pi ? aug[RM] / mydiag : 0.0;
}

// The same solution through H = G^-1 when few variables are bound: with the
// bound set B (live, off P), G_PP^-1 = H_PP - H_PB H_BB^-1 H_BP (the Schur
// complement identity), so z_P is the right-hand side of rows P of
// [H | H c~] (c~ = c on P, 0 on B) after eliminating the pivots B.  Only the
// columns of B and the right-hand side are updated.
template <int RM>
__device__ __noinline__ double nnls_masked_solve_h(const double* Hs, int r, uint64_t pm, uint64_t bm, double c) {
  const int lane = threadIdx.x & 63;
  const int row = min(lane, RM - 1);
  const bool pi = (pm >> lane) & 1ull;
  double y = 0.0;
  uint64_t rest = pm;
  while (rest) {
    const int l = __builtin_ctzll(rest);
    rest &= rest - 1;
    y = fma(Hs[row * RM + l], readlane_d(c, l), y);
  }
  double aug[RM + 1];
#pragma unroll
  for (int l = 0; l < RM; ++l) aug[l] = ((bm >> l) & 1ull) ? Hs[row * RM + l] : 0.0;
  aug[RM] = y;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    if (j < r && ((bm >> j) & 1ull)) {
      const double piv = readlane_d(aug[j], j);
      const double f = lane == j ? 0.0 : aug[j] / piv;
#pragma unroll
      for (int l = j + 1; l < RM; ++l)
        if ((bm >> l) & 1ull) aug[l] = fma(-f, readlane_d(aug[l], j), aug[l]);
      aug[RM] = fma(-f, readlane_d(aug[RM], j), aug[RM]);
    }
  }
  return pi ? aug[RM] : 0.0;
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

// Lawson-Hanson on one wave (lane i: variable i, lanes >= r idle):
// minimise 1/2 h^T G h - c^T h over h >= 0.  h0 is a feasible start (>= 0;
// its support is the first passive set, 0 for a cold start): the free
// system is solved on it and, where a free variable comes out <= 0, the
// iterate moves from h towards the solution until the first one reaches 0,
// which is bound again (repeatedly).  Then the bound variable whose dual
// w_i = (c - G h)_i is largest (lowest index on ties) is freed while it
// exceeds tol = 1e-13 max|c|, and the free system is solved again (a
// variable bound again within its own step is not freed again).  The
// minimiser is unique for positive definite G, so the start changes the
// number of steps, not the result.  At most 3 r freeing steps; *ok = false
// when a problem needs more (its last feasible h is returned).
template <int RM>
__device__ double lh_wave(const double* Gs, int r, double c, double h0, int* outer_out, bool* ok) {
  const int lane = threadIdx.x & 63;
  const bool real = lane < r;
  const double tol = 1e-13 * wave_max_d(fabs(c));
  double h = (real && h0 > 0.0) ? h0 : 0.0;
  uint64_t pm = __ballot(h > 0.0);
  uint64_t excl = 0;   // variables that came straight back to their bound (anti-cycling)
  int outer = 0, p = -1;
  bool solve = pm != 0;
  *ok = true;
  while (true) {
    if (solve) {
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
      // by rounding) is not freed again for this problem
      if (p >= 0 && !((pm >> p) & 1ull)) excl |= 1ull << p;
    }
    // dual w = c - G h over the free variables
    double gh = 0.0;
    uint64_t rest = pm;
    while (rest) {
      const int l = __builtin_ctzll(rest);
      rest &= rest - 1;
      gh = fma(Gs[min(lane, RM - 1) * RM + l], readlane_d(h, l), gh);
    }
    const double wdual = c - gh;
    // the bound variable with the largest dual above tol (lowest index on ties)
    const double cand = (real && !(((pm | excl) >> lane) & 1ull) && wdual > tol) ? wdual : -1.0;
    const double best = wave_max_d(cand);
    if (!(best > 0.0)) break;
    const uint64_t at = __ballot(cand == best);
    p = __builtin_ctzll(at);
    if (++outer > 3 * r) {
      *ok = false;
      break;
    }
    pm |= 1ull << p;
    solve = true;
  }
  *outer_out = outer;
  return h;
}

// Block principal pivoting (Kim and Park, "Fast nonnegative matrix
// factorization: an active-set-like method and comparisons", SIAM J. Sci.
// Comput. 2011) on one wave, for the same problem as lh_wave: with a free set
// F (the rest bound at 0), solve G_FF z_F = c_F and form the dual
// y = G z - c; the variables with z_i < 0 in F or y_i < 0 off F are
// infeasible.  All of them change sides at once while their number keeps
// falling (at most three tries without a decrease); otherwise only the one of
// largest index does (the finite backup rule).  It stops when none is
// infeasible, which is the optimality condition, so the minimiser is the same
// as Lawson-Hanson's; a good first F (the support of h0) usually needs one or
// two solves.  Tolerances: z_i < -1e-13 max|z_F|, y_i < -1e-13 max|c|.  A
// variable with G_ii = 0 (its column of C is zero) stays at 0.  With Hs =
// G^-1 (checked), a free system with fewer bound than free variables is
// solved through H (nnls_masked_solve_h), which eliminates only the bound
// pivots.  At most 5 r exchanges; *ok = false when a problem needs more or a
// solve breaks down (the last iterate, clamped at 0, is returned).
template <int RM>
__device__ double bpp_wave(const double* Gs, const double* Hs, int r, double c, double h0, int* steps_out,
                           bool* ok) {
  const int lane = threadIdx.x & 63;
  const int row = min(lane, RM - 1);
  const bool real = lane < r;
  const bool live = real && Gs[row * RM + row] > 0.0;
  const uint64_t lm = __ballot(live);
  const double tol_y = 1e-13 * wave_max_d(fabs(c));
  uint64_t F = __ballot(live && h0 > 0.0);
  int alpha = 3, beta = r + 1, steps = 0;
  double z = 0.0;
  bool good = true;
  while (true) {
    const uint64_t Bm = lm & ~F;
    if (Hs && __popcll(Bm) < __popcll(F))
      z = nnls_masked_solve_h<RM>(Hs, r, F, Bm, c);
    else
      z = nnls_masked_solve<RM>(Gs, r, F, c);
    double gz = 0.0;
    uint64_t rest = F;
    while (rest) {
      const int l = __builtin_ctzll(rest);
      rest &= rest - 1;
      gz = fma(Gs[row * RM + l], readlane_d(z, l), gz);
    }
    const double y = gz - c;
    const bool inF = (F >> lane) & 1ull;
    if (__ballot(inF && !(z == z)) != 0) {   // a NaN: the free system broke down
      good = false;
      break;
    }
    const double zmax = wave_max_d(inF ? fabs(z) : 0.0);
    const bool bad = live && (inF ? (z < -1e-13 * zmax) : (y < -tol_y));
    const uint64_t V = __ballot(bad);
    if (V == 0) break;
    if (++steps > 5 * r) {
      good = false;
      break;
    }
    const int nv = __popcll(V);
    uint64_t X;
    if (nv < beta) {
      beta = nv;
      alpha = 3;
      X = V;
    } else if (alpha >= 1) {
      alpha -= 1;
      X = V;
    } else {
      X = 1ull << (63 - __clzll(V));
    }
    F ^= X;   // infeasible free variables are bound, infeasible bound ones freed
  }
  *steps_out = steps;
  *ok = good;
  const bool inF = (F >> lane) & 1ull;
  return (inF && z > 0.0) ? z : 0.0;
}

// G (r x r, row-major, FP64) into LDS, padded to RM x RM with zeros.
template <int RM>
__device__ __forceinline__ void stage_gram(double* Gs, const double* __restrict__ G, int r) {
  staged_copy<8>(
      RM * RM, threadIdx.x, blockDim.x,
      [&](int e) {
        const int i = e / RM, l = e - i * RM;
        return (i < r && l < r) ? G[i * r + l] : 0.0;
      },
      [&](int e, double v) { Gs[e] = v; });
}

// Right factor: one wave per column (grid-stride over the columns), cold
// start.  info[0]: columns that needed more than 3 r steps; info[1]:
// largest number of freeing steps.
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
    int outer;
    bool ok;
    const double h = lh_wave<RM>(Gs, r, c, 0.0, &outer, &ok);
    worst = max(worst, outer);
    failed += ok ? 0 : 1;
    if (real) H[(int64_t)lane * ldh + j] = h;
  }
  if (lane == 0) {
    if (failed) atomicAdd(info, failed);
    atomicMax(info + 1, worst);
  }
}

// One half-step of alternating NNLS: one wave per row of F (grid-stride),
// the right-hand side c = C^T b of row i formed in the wave, solved by block
// principal pivoting from the row's current support.
template <typename T, int RM>
__global__ __launch_bounds__(256) void anls_rows_kernel(AnlsArgs a) {
  __shared__ double Gs[RM * RM];
  __shared__ double Hs[RM * RM];
  stage_gram<RM>(Gs, a.G, a.r);
  const bool use_h = a.H && a.hok && *a.hok;
  if (use_h) stage_gram<RM>(Hs, a.H, a.r);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = a.r;
  const bool real = lane < r;
  const int col = min(lane, r - 1);
  const T* __restrict__ B1 = (const T*)a.B1;
  T* __restrict__ F = (T*)a.F;
  T* __restrict__ Op = (T*)a.Op;
  int worst = 0, failed = 0;
  for (int i = blockIdx.x * 4 + w; i < a.rows; i += gridDim.x * 4) {
    const T* b = B1 + (int64_t)i * a.ldb1;
    double c = 0.0;
    if (a.C) {
      // c_l = sum_t b_t C[t][l] (C^T b with C stored k1 x r)
      double s0 = 0.0, s1 = 0.0;
      int t = 0;
      for (; t + 1 < a.k1; t += 2) {
        s0 = fma((double)b[t], a.C[t * r + col], s0);
        s1 = fma((double)b[t + 1], a.C[(t + 1) * r + col], s1);
      }
      if (t < a.k1) s0 = fma((double)b[t], a.C[t * r + col], s0);
      c = s0 + s1;
    } else {
      c = (double)b[col];
    }
    c = real ? c : 0.0;
    const double h0 = real ? (double)F[(int64_t)i * a.ldf + col] : 0.0;
    int steps;
    bool ok;
    const double h = bpp_wave<RM>(Gs, use_h ? Hs : nullptr, r, c, h0, &steps, &ok);
    worst = max(worst, steps);
    failed += ok ? 0 : 1;
    if (real) {
      F[(int64_t)i * a.ldf + lane] = (T)h;
      if (Op) Op[(int64_t)i * a.ldop + lane] = (T)h;
    }
  }
  if (lane == 0 && a.info) {
    if (failed) atomicAdd(a.info, failed);
    atomicMax(a.info + 1, worst);
  }
}

template <typename T>
hipError_t launch_anls_rows(const AnlsArgs& a, hipStream_t st) {
  if (a.r < 1 || a.r > 64 || a.rows < 0 || (a.C && a.k1 < 1)) return hipErrorInvalidValue;
  if (a.rows == 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(((int64_t)a.rows + 3) / 4, 4096);
  if (a.r <= 8)
    hipLaunchKernelGGL((anls_rows_kernel<T, 8>), dim3(grid), dim3(256), 0, st, a);
  else if (a.r <= 16)
    hipLaunchKernelGGL((anls_rows_kernel<T, 16>), dim3(grid), dim3(256), 0, st, a);
  else if (a.r <= 24)
    hipLaunchKernelGGL((anls_rows_kernel<T, 24>), dim3(grid), dim3(256), 0, st, a);
  else if (a.r <= 32)
    hipLaunchKernelGGL((anls_rows_kernel<T, 32>), dim3(grid), dim3(256), 0, st, a);
  else if (a.r <= 48)
    hipLaunchKernelGGL((anls_rows_kernel<T, 48>), dim3(grid), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((anls_rows_kernel<T, 64>), dim3(grid), dim3(256), 0, st, a);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_anls_rows<float>(const AnlsArgs&, hipStream_t);
template hipError_t launch_anls_rows<double>(const AnlsArgs&, hipStream_t);

// *dst += *src (one thread): folds a launch's failure count into a running total.
__global__ void add_count_kernel(const int* __restrict__ src, int* __restrict__ dst) {
  if (threadIdx.x == 0 && *src) atomicAdd(dst, *src);
}
hipError_t launch_add_count(const int* src, int* dst, hipStream_t st) {
  hipLaunchKernelGGL(add_count_kernel, dim3(1), dim3(64), 0, st, src, dst);
  CNMF_LAUNCH_CHECK();
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
