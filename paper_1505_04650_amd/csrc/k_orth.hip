// Orthonormalisation of the tall range samples (Alg. 1, QR step) by
// CholeskyQR2 in FP64, plus the small k x k products of the sketch.
//   G = Y^T Y (FP64 accumulation, deterministic partials)
//   T = chol(G) upper with positive diagonal, Tinv = T^-1
//   Q = Y Tinv; repeat once on Q (the second pass restores orthogonality
//   to working precision).
// With diag(T) > 0 this Q is the same basis as the Householder QR with a
// nonnegative diagonal for full-column-rank Y.
#include "cnmf_internal.hpp"
#include "rng.hpp"
#include "small_dense.hpp"

namespace cnmf {

typedef double doublex2 __attribute__((ext_vector_type(2)));

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
// (ta + 16 i, tb + 16 j).  SYM (a Gram matrix, X == Y): only the blocks
// i >= j are formed and the strictly lower ones are mirrored.
// ---------------------------------------------------------------------------
template <typename TX, typename TY, int KH16, bool SYM>
__global__ __launch_bounds__(256) void cross_kernel(const TX* __restrict__ X, int ldx, int x0,
                                                   const TY* __restrict__ Y, int ldy, int y0, int hs,
                                                   int rows, int ka, int kb, double* __restrict__ Cp,
                                                   int rows_per_part, const int* __restrict__ run_if) {
  if (run_if && run_if[blockIdx.y] == 0) return;
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
    staged_copy<4>(
        CR * KW, tid, 256,
        [&](int e) {
          const int rr = e / KW, c = e - rr * KW, row = base + rr;
          const bool ok = row < i1;
          return doublex2{(ok && c < ka) ? to_d(X[(int64_t)row * ldx + xc + c]) : 0.0,
                          (ok && c < kb) ? to_d(Y[(int64_t)row * ldy + yc + c]) : 0.0};
        },
        [&](int e, doublex2 v) {
          const int rr = e / KW, c = e - rr * KW;
          xs[rr][c] = v.x;
          ys[rr][c] = v.y;
        });
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
        for (int j = 0; j < KH16; ++j)
          if (!SYM || i >= j) acc[i][j] = fma(xa[i], yb[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* out = Cp + ((int64_t)p * nh + h) * ka * kb;
#pragma unroll
  for (int i = 0; i < KH16; ++i)
#pragma unroll
    for (int j = 0; j < KH16; ++j) {
      if (SYM && i < j) continue;
      int a = ta + 16 * i, b = tb + 16 * j;
      if (a < ka && b < kb) {
        out[a * kb + b] = acc[i][j];
        if (SYM && i > j) out[b * kb + a] = acc[i][j];
      }
    }
}

// Gram partials on the FP64 MFMA (X == Y, k <= 16 KB16): the rows of a
// part are staged in LDS as FP64, 32 at a time (the next 32 are loaded into
// registers while the current ones are used); the lower 16 x 16 tiles
// (ti >= tj) are dealt round robin to the waves, each tile an FP64 16x16x4
// MFMA chain over the rows, and the strictly lower ones are mirrored.
// Same partial layout as cross_kernel.  FP32 inputs give exact products in
// FP64, as there.
template <typename TY, int KB16>
__global__ __launch_bounds__(256) void gram_mfma_kernel(const TY* __restrict__ Y, int ldy, int y0, int hs, int rows,
                                                        int k, double* __restrict__ Cp, int rows_per_part,
                                                        const int* __restrict__ run_if) {
  if (run_if && run_if[blockIdx.y] == 0) return;
  constexpr int CR = 32, KW = 16 * KB16, LDC = KW + 1;
  constexpr int NT = KB16 * (KB16 + 1) / 2, NQ = (NT + 3) / 4;
  constexpr int PER = CR * KW / 256;   // staged values per thread and chunk
  __shared__ double ys[2][CR * LDC];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int p = blockIdx.x, h = blockIdx.y, nh = gridDim.y;
  const int yc = y0 + h * hs;
  const int i0 = p * rows_per_part, i1 = min(rows, i0 + rows_per_part);
  int ti[NQ], tj[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = w + 4 * q;
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= e) ++a;
    ti[q] = a;
    tj[q] = e - a * (a + 1) / 2;
  }
  doublex4 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = doublex4{0.0, 0.0, 0.0, 0.0};
  TY v[PER];
  auto load = [&](int base) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = tid + 256 * e, rr = idx / KW, cc = idx - rr * KW;
      const int row = base + rr;
      v[e] = (row < i1 && cc < k) ? Y[(int64_t)row * ldy + yc + cc] : TY(0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = tid + 256 * e, rr = idx / KW, cc = idx - rr * KW;
      ys[buf][rr * LDC + cc] = (double)v[e];
    }
  };
  const int nch = i1 > i0 ? (i1 - i0 + CR - 1) / CR : 0;
  if (nch > 0) {
    load(i0);
    store(0);
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
    if (more) load(i0 + CR * (ch + 1));
    const double* yb = ys[buf];
#pragma unroll
    for (int s = 0; s < CR / 4; ++s) {
      const double* yr = yb + (4 * s + g) * LDC + c;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (w + 4 * q < NT) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(yr[16 * ti[q]], yr[16 * tj[q]], acc[q], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
  }
  double* out = Cp + ((int64_t)p * nh + h) * k * k;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (w + 4 * q >= NT) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int a = 16 * ti[q] + g + 4 * i, b = 16 * tj[q] + c;
      if (a < k && b < k) {
        out[a * k + b] = acc[q][i];
        if (ti[q] > tj[q]) out[b * k + a] = acc[q][i];
      }
    }
  }
}

template <typename TX, typename TY, int KH16>
static hipError_t cross_kh(const TX* X, int ldx, int x0, const TY* Y, int ldy, int y0, int hs, int nh,
                           int rows, int ka, int kb, double* Cp, int parts, const int* run_if, hipStream_t st) {
  int rpp = (rows + parts - 1) / parts;
  const bool sym = (const void*)X == (const void*)Y && ldx == ldy && x0 == y0 && ka == kb;
  if (sym)
    hipLaunchKernelGGL((gram_mfma_kernel<TY, KH16>), dim3(parts, nh), dim3(256), 0, st, Y, ldy, y0, hs, rows, ka, Cp,
                       rpp, run_if);
  else
    hipLaunchKernelGGL((cross_kernel<TX, TY, KH16, false>), dim3(parts, nh), dim3(256), 0, st, X, ldx, x0, Y, ldy,
                       y0, hs, rows, ka, kb, Cp, rpp, run_if);
  CNMF_LAUNCH_CHECK();
}

template <typename TX, typename TY>
hipError_t launch_cross2(const TX* X, int ldx, int x0, const TY* Y, int ldy, int y0, int hs, int nh,
                         int rows, int ka, int kb, double* Cp, int parts, hipStream_t st, const int* run_if) {
  int kmax = std::max(ka, kb);
  int k16 = (kmax + 15) / 16;
  switch (k16) {
    case 1: return cross_kh<TX, TY, 1>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, run_if, st);
    case 2: return cross_kh<TX, TY, 2>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, run_if, st);
    case 3: return cross_kh<TX, TY, 3>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, run_if, st);
    case 4: return cross_kh<TX, TY, 4>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, run_if, st);
    case 5: return cross_kh<TX, TY, 5>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, run_if, st);
    case 6: return cross_kh<TX, TY, 6>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, run_if, st);
    case 7: return cross_kh<TX, TY, 7>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, run_if, st);
    case 8: return cross_kh<TX, TY, 8>(X, ldx, x0, Y, ldy, y0, hs, nh, rows, ka, kb, Cp, parts, run_if, st);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_cross2<float, float>(const float*, int, int, const float*, int, int, int, int, int, int, int, double*, int, hipStream_t, const int*);
template hipError_t launch_cross2<double, double>(const double*, int, int, const double*, int, int, int, int, int, int, int, double*, int, hipStream_t, const int*);
template hipError_t launch_cross2<float, double>(const float*, int, int, const double*, int, int, int, int, int, int, int, double*, int, hipStream_t, const int*);

// ---------------------------------------------------------------------------
// out[e] = sum_p in[p * count + e], p increasing.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sum_parts_kernel(const double* __restrict__ in, int parts, int64_t count,
                                                        double* __restrict__ out, const int* __restrict__ run_if,
                                                        int nrun) {
  if (run_if) {
    int any = 0;
    for (int i = 0; i < nrun; ++i) any |= run_if[i];
    if (!any) return;
  }
  __shared__ double red[256];
  block_sum_parts<256, 32>(in, parts, count, count, (int64_t)blockIdx.x * 32, out, red);
}

hipError_t launch_sum_parts(const double* in, int parts, int64_t count, double* out, hipStream_t st,
                            const int* run_if, int nrun) {
  int blocks = (int)((count + 31) / 32);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(blocks), dim3(256), 0, st, in, parts, count, out, run_if, nrun);
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// G_h = sum of the Gram partials (fixed order; sum_parts kernel), then one
// workgroup per half: G_h (padded to N = 16 ceil(kh / 16) with an identity
// block) = T^T T (T upper, positive diagonal) and Tinv_h = T^-1 written to
// global memory (kh x kh, zero below the diagonal).
// Breakdown (see CholOpts): with o.mask a pivot <= o.tau max_i G_ii marks
// its column as dependent on the earlier ones; the column is decoupled (its
// factor column is the unit vector), counted in o.repaired[h] and marked in
// o.mask[2 h + (column / 64)] for the apply step to replace by a fresh
// Gaussian column, and o.need[h] tells whether any was.  Without o.mask
// such a pivot is floored and counted as unresolved.  NaN pivots are always
// unresolved.  With o.run_if, half h runs only if o.run_if[h] != 0.
// ---------------------------------------------------------------------------
constexpr int kFacNT = 256;

// M (N x N, ld) = (G + G^T) / 2 for the kh x kh Gram G in global memory,
// identity outside it.  Eight elements per thread are loaded before any is
// stored: G was just written and comes from L2, and a load-store pair per
// element would leave the workgroup waiting on the L2 latency N^2 / 256 times.
template <int N>
__device__ __forceinline__ void load_sym_gram(const double* __restrict__ Gh, int kh, double* M, int ld) {
  constexpr int U = 8;
  for (int e0 = threadIdx.x; e0 < N * N; e0 += kFacNT * U) {
    double a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + kFacNT * u, i = e / N, j = e - i * N;
      const bool ok = e < N * N && i < kh && j < kh;
      a[u] = ok ? Gh[i * kh + j] : 0.0;
      b[u] = ok ? Gh[j * kh + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + kFacNT * u, i = e / N, j = e - i * N;
      if (e < N * N) M[i * ld + j] = (i < kh && j < kh) ? 0.5 * (a[u] + b[u]) : (i == j ? 1.0 : 0.0);
    }
  }
}

// kh <= 64, with the products on the FP64 MFMA: wave 0
// factors G_h = L L^T (wave_chol_lower: 16-column register panels, MFMA
// trailing updates, inverses V_b of the diagonal blocks); then wave j forms
// column strip j of Z = L^-1 by block forward substitution,
//   Z_jj = V_j,  Z_bj = -V_b sum_{j <= a < b} L[b][a] Z_aj   (b > j),
// with the strip's tiles in registers (a 16x16x4 FP64 MFMA result is the
// right operand of the next product as it stands), and writes Tinv_h =
// T^-1 = Z^T, since T = L^T.
template <int NB, bool DEC>
__device__ __forceinline__ void chol_tinv_wave_body(const double* __restrict__ Gh, int kh, double* __restrict__ out,
                                                    double tau, int* flag, int* nanflag, uint64_t* mask, double* sm) {
  constexpr int N = 16 * NB, ld = N + 2;
  double* M = sm;                 // N x ld
  double* V = M + N * ld;         // NB x 272
  double* W = V + NB * 272;       // 128
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  load_sym_gram<N>(Gh, kh, M, ld);
  __syncthreads();
  if (w == 0) {
    double dg = lane < kh ? M[lane * ld + lane] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dg = fmax(dg, __shfl_xor(dg, o));
    wave_chol_lower<double, NB, DEC>(M, ld, kh, V, W, dg > 0.0 ? tau * dg : 1.0, flag, nanflag, mask);
  }
  __syncthreads();
  if (w < NB) {
    const int j = w;
    doublex4 z[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b < j) {
        z[b] = doublex4{0.0, 0.0, 0.0, 0.0};
      } else if (b == j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) z[b][i] = V[b * 272 + (g + 4 * i) * 17 + c];
      } else {
        doublex4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < b; ++a) {
          if (a < j) continue;
#pragma unroll
          for (int s = 0; s < 4; ++s)
            t = __builtin_amdgcn_mfma_f64_16x16x4f64(M[(16 * b + c) * ld + 16 * a + 4 * s + g], z[a][s], t, 0, 0, 0);
        }
        doublex4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s)
          y = __builtin_amdgcn_mfma_f64_16x16x4f64(-V[b * 272 + c * 17 + 4 * s + g], t[s], y, 0, 0, 0);
        z[b] = y;
      }
    }
    // Tinv[16 j + c][16 b + g + 4 i] = Z[16 b + g + 4 i][16 j + c] = item i of tile b
    const int trow = 16 * j + c;
    if (trow < kh) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int tcol = 16 * b + g + 4 * i;
          if (tcol < kh) out[trow * kh + tcol] = z[b][i];
        }
    }
  }
}

// 64 < kh <= 128 (N = 128, identity padding), from the same pieces in 2 x 2
// blocks of 64:  L11 = chol(G11) (wave 0);  L21 from L21 L11^T = G21, each
// wave solving its 16 rows by block substitution in registers;
// S22 = G22 - L21 L21^T on the MFMA (wave w: block row w);  L22 = chol(S22)
// (wave 0);  then Z = L^-1 over all 8 block rows, two column strips per
// wave, and Tinv = Z^T.
template <bool DEC>
__device__ __forceinline__ void chol_tinv_wave128_body(const double* __restrict__ Gh, int kh, double* __restrict__ out,
                                                       double tau, int* flag, int* nanflag, uint64_t* mask,
                                                       double* sm) {
  constexpr int N = 128, ld = N + 2;
  double* M = sm;                 // N x ld
  double* V = M + N * ld;         // 8 x 272: V[b], b < 4 from L11, b >= 4 from L22
  double* W = V + 8 * 272;        // 128
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  load_sym_gram<N>(Gh, kh, M, ld);
  __syncthreads();
  double fl = 1.0;
  {
    double dg = 0.0;
    for (int i = lane; i < kh; i += 64) dg = fmax(dg, M[i * ld + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dg = fmax(dg, __shfl_xor(dg, o));
    if (dg > 0.0) fl = tau * dg;
  }
  if (w == 0) wave_chol_lower<double, 4, DEC>(M, ld, 64, V, W, fl, flag, nanflag, mask);
  __syncthreads();
  // L21: wave w solves rows 64 + 16 w .. + 15 of X L11^T = G21 as L11 X^T = G21^T
  {
    double* R = M + (64 + 16 * w) * ld;   // the wave's rows of G21 (columns 0..63)
    doublex4 z[4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) z[b][i] = R[c * ld + 16 * b + g + 4 * i];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      doublex4 t = z[b];
#pragma unroll
      for (int a = 0; a < b; ++a)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          t = __builtin_amdgcn_mfma_f64_16x16x4f64(-M[(16 * b + c) * ld + 16 * a + 4 * s + g], z[a][s], t, 0, 0, 0);
      doublex4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s)
        y = __builtin_amdgcn_mfma_f64_16x16x4f64(V[b * 272 + c * 17 + 4 * s + g], t[s], y, 0, 0, 0);
      z[b] = y;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) R[c * ld + 16 * b + g + 4 * i] = z[b][i];
  }
  __syncthreads();
  // S22 = G22 - L21 L21^T, block row w (all four column tiles)
  {
    doublex4 acc[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[jb][i] = M[(64 + 16 * w + g + 4 * i) * ld + 64 + 16 * jb + c];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const double a = -M[(64 + 16 * w + c) * ld + 4 * s + g];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
        acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, M[(64 + 16 * jb + c) * ld + 4 * s + g], acc[jb], 0, 0, 0);
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int i = 0; i < 4; ++i) M[(64 + 16 * w + g + 4 * i) * ld + 64 + 16 * jb + c] = acc[jb][i];
  }
  __syncthreads();
  if (w == 0) wave_chol_lower<double, 4, DEC>(M + 64 * ld + 64, ld, kh - 64, V + 4 * 272, W, fl, flag, nanflag, mask + 1);
  __syncthreads();
  // Z = L^-1, column strips j = w and w + 4
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int j = w + 4 * q;
    doublex4 z[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (b < j) {
        z[b] = doublex4{0.0, 0.0, 0.0, 0.0};
      } else if (b == j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) z[b][i] = V[b * 272 + (g + 4 * i) * 17 + c];
      } else {
        doublex4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < b; ++a) {
          if (a < j) continue;
#pragma unroll
          for (int s = 0; s < 4; ++s)
            t = __builtin_amdgcn_mfma_f64_16x16x4f64(M[(16 * b + c) * ld + 16 * a + 4 * s + g], z[a][s], t, 0, 0, 0);
        }
        doublex4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s)
          y = __builtin_amdgcn_mfma_f64_16x16x4f64(-V[b * 272 + c * 17 + 4 * s + g], t[s], y, 0, 0, 0);
        z[b] = y;
      }
    }
    const int trow = 16 * j + c;
    if (trow < kh) {
#pragma unroll
      for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int tcol = 16 * b + g + 4 * i;
          if (tcol < kh) out[trow * kh + tcol] = z[b][i];
        }
    }
  }
}

template <bool DEC>
__device__ __forceinline__ void chol_tinv_dispatch(const double* Gh, int kh, double* out, double tau, int* flag,
                                                   int* nanflag, uint64_t* mask, double* sm) {
  switch ((kh + 15) / 16) {
    case 1: chol_tinv_wave_body<1, DEC>(Gh, kh, out, tau, flag, nanflag, mask, sm); break;
    case 2: chol_tinv_wave_body<2, DEC>(Gh, kh, out, tau, flag, nanflag, mask, sm); break;
    case 3: chol_tinv_wave_body<3, DEC>(Gh, kh, out, tau, flag, nanflag, mask, sm); break;
    case 4: chol_tinv_wave_body<4, DEC>(Gh, kh, out, tau, flag, nanflag, mask, sm); break;
    default: chol_tinv_wave128_body<DEC>(Gh, kh, out, tau, flag, nanflag, mask, sm); break;
  }
}

__global__ __launch_bounds__(kFacNT) void chol_tinv_wave_kernel(const double* __restrict__ G, int kh,
                                                                double* __restrict__ Tinv, CholOpts o) {
  const int h = blockIdx.x;
  if (o.run_if && o.run_if[h] == 0) return;
  extern __shared__ double sm[];
  __shared__ int cnt_s[2];        // [0] pivots below the threshold, [1] NaN pivots
  __shared__ uint64_t mask_s[2];
  const int64_t cnt = (int64_t)kh * kh;
  if (threadIdx.x < 2) {
    cnt_s[threadIdx.x] = 0;
    mask_s[threadIdx.x] = 0;
  }
  __syncthreads();
  if (o.mask)
    chol_tinv_dispatch<true>(G + h * cnt, kh, Tinv + h * cnt, o.tau, &cnt_s[0], &cnt_s[1], mask_s, sm);
  else
    chol_tinv_dispatch<false>(G + h * cnt, kh, Tinv + h * cnt, o.tau, &cnt_s[0], nullptr, nullptr, sm);
  __syncthreads();
  if (threadIdx.x == 0) {
    // decoupling: low pivots are repaired, NaN ones are not; otherwise every
    // low (or NaN) pivot is unresolved
    const int unres = o.mask ? cnt_s[1] : cnt_s[0];
    if (o.mask) {
      const int fixed = cnt_s[0] - cnt_s[1];
      o.mask[2 * h] = mask_s[0];
      o.mask[2 * h + 1] = mask_s[1];
      if (o.repaired && fixed > 0) atomicAdd(o.repaired + h, fixed);
      if (o.need) o.need[h] = cnt_s[0] > 0 ? 1 : 0;
    }
    if (unres) {
      if (o.unresolved) atomicAdd(o.unresolved, unres);
      if (o.unresolved_total) atomicAdd(o.unresolved_total, unres);
    }
  }
}

hipError_t launch_gram_chol(const double* Gp, int parts, int nh, int kh, double* G, double* Tinv, const CholOpts& o,
                            hipStream_t st) {
  if (kh > 128) return hipErrorInvalidValue;
  hipError_t e = launch_sum_parts(Gp, parts, (int64_t)nh * kh * kh, G, st, o.run_if, nh);
  if (e != hipSuccess) return e;
  return launch_chol_tinv(G, nh, kh, Tinv, o, st);
}

hipError_t launch_chol_tinv(const double* G, int nh, int kh, double* Tinv, const CholOpts& o, hipStream_t st) {
  if (kh > 128 || kh < 1) return hipErrorInvalidValue;
  const int NB = (kh + 15) / 16, N = 16 * NB;
  // kh <= 64: N x (N + 2) + NB x 272 + 128 doubles; kh > 64: 128 x 130 + 8 x 272 + 128
  const size_t smw = kh <= 64 ? ((size_t)N * (N + 2) + (size_t)NB * 272 + 128) * sizeof(double)
                              : ((size_t)128 * 130 + 8 * 272 + 128) * sizeof(double);
  hipFuncSetAttribute((const void*)chol_tinv_wave_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smw);
  hipLaunchKernelGGL(chol_tinv_wave_kernel, dim3(nh), dim3(kFacNT), smw, st, G, kh, Tinv, o);
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Q64[i][h*kh + c] = sum_{l <= c} Y[i][h*kh + l] Tinv_h[l][c] on the FP64
// MFMA (16x16x4).  Workgroup: 64 rows (wave w: rows 16 w .. 16 w + 15) of
// one half; each lane first loads its K values of Y (lane (r, g) supplies
// Y[row r][4 s + g]), then the 64-column slabs of Tinv_h are staged in LDS
// one after the other.  All reads of a row precede the writes of that row,
// so Q64 == Y (in place) is allowed.  Columns marked in mask (2 words per
// half, see launch_gram_chol) receive entries of the Gaussian test matrix
// id0 + h (seed `seed`) divided by sqrt(rows) instead, a unit-scale column
// that the second CholeskyQR pass orthonormalises against the others.
// ---------------------------------------------------------------------------
template <typename TY>
__global__ __launch_bounds__(256, 2) void apply_mfma_kernel(const TY* __restrict__ Y, int rows, int ldy, int kh,
                                                            const double* __restrict__ Tinv, double* Q, int ldq,
                                                            const uint64_t* __restrict__ mask, uint64_t seed,
                                                            uint32_t id0, const int* __restrict__ run_if) {
  constexpr int SL = 64, LDT = SL + 4, KS = 32;   // kh <= 128: at most 32 K steps of 4
  __shared__ double Ts[4 * KS * LDT];
  const int h = blockIdx.y;
  if (run_if && run_if[h] == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int row0 = blockIdx.x * 64 + w * 16;
  const int row = row0 + r;
  const int nsteps = (kh + 3) >> 2;
  const double* Th = Tinv + (int64_t)h * kh * kh;
  const uint64_t mk0 = mask ? mask[2 * h] : 0ull, mk1 = mask ? mask[2 * h + 1] : 0ull;
  const double inv_sqrt_rows = 1.0 / sqrt((double)rows);
  double yv[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int l = 4 * s + g;
    yv[s] = (s < nsteps && row < rows && l < kh) ? (double)Y[(int64_t)row * ldy + h * kh + l] : 0.0;
  }
  const int nslab = (kh + SL - 1) / SL;
  for (int sl = 0; sl < nslab; ++sl) {
    const int c0 = sl * SL;
    __syncthreads();
    // eight loads in flight per thread before their stores (the slab comes
    // from L2; one load and store at a time left each workgroup waiting on
    // the L2 latency once per element row)
    const int lim = 4 * nsteps * SL;
    for (int e0 = tid; e0 < lim; e0 += 256 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u, l = e / SL, c = e - l * SL;
        v[u] = (e < lim && l < kh && c0 + c < kh) ? Th[l * kh + c0 + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u, l = e / SL, c = e - l * SL;
        if (e < lim) Ts[l * LDT + c] = v[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < SL / 16; ++cb) {
      const int cbase = c0 + 16 * cb;
      if (cbase >= kh) break;
      // Tinv is upper triangular: rows l <= cbase + 15 contribute
      const int smax = min(nsteps, (cbase + 16 + 3) >> 2);
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s)
        if (s < smax) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(yv[s], Ts[(4 * s + g) * LDT + 16 * cb + r], acc, 0, 0, 0);
      const int col = cbase + r;
      const bool fresh = (mk0 | mk1) && col < kh && (((col < 64 ? mk0 >> col : mk1 >> (col - 64)) & 1ull) != 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int orow = row0 + g + 4 * i;
        double v = acc[i];
        if (fresh && orow < rows) v = gauss_entry(seed, id0 + h, (uint32_t)orow, (uint32_t)col) * inv_sqrt_rows;
        if (orow < rows && col < kh) Q[(int64_t)orow * ldq + h * kh + col] = v;
      }
    }
  }
}

template <typename TY>
hipError_t launch_apply_tinv(const TY* Y, int rows, int ldy, int nh, int kh, const double* Tinv, double* Q64,
                             int ldq, const uint64_t* mask, uint64_t seed, uint32_t id0, hipStream_t st,
                             const int* run_if) {
  if (kh > 128) return hipErrorInvalidValue;
  dim3 grid((rows + 63) / 64, nh);
  hipLaunchKernelGGL(apply_mfma_kernel<TY>, grid, dim3(256), 0, st, Y, rows, ldy, kh, Tinv, Q64, ldq, mask, seed,
                     id0, run_if);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_apply_tinv<float>(const float*, int, int, int, int, const double*, double*, int,
                                             const uint64_t*, uint64_t, uint32_t, hipStream_t, const int*);
template hipError_t launch_apply_tinv<double>(const double*, int, int, int, int, const double*, double*, int,
                                              const uint64_t*, uint64_t, uint32_t, hipStream_t, const int*);

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
