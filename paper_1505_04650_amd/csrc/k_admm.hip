// ADMM for NMF on the two-sided compressed problem (Appendix B, Alg. 3).
//
// One iteration of the box, with Xt (k x r) and Yt^T (k x r) kept in FP64:
//   Xt   <- (At Yt^T + P_U) (Yt Yt^T + lam I)^-1,   P_U = L^T (lam U - Lam)
//   Yt^T <- (At^T Xt + P_V) (Xt^T Xt + phi I)^-1,   P_V = R (phi V^T - Phi^T)
//   U   <- max(L Xt + Lam/lam, 0);  Lam <- Lam + xi lam (L Xt - U)
//   V^T <- max(R^T Yt^T + Phi^T/phi, 0);  Phi^T <- Phi^T + xi phi (R^T Yt^T - V^T)
// The row updates (U, Lam over the m rows of L; V^T, Phi^T over the n rows of
// R^T) are the same operation on two "sides" and run in one launch
// (admm_uv_kernel).  That launch also forms the partial sums of
// basis^T (pen * F - M) for the next iteration's P_U / P_V, so the big
// matrices are read once per iteration.  admm_solve_kernel reduces those
// partials in a fixed order and does the r x r solves by Cholesky in FP64.
#include "cnmf_internal.hpp"
#include "small_dense.hpp"

namespace cnmf {

// MFMA helpers (16x16x4; see k_gemm.hip for the measured result layout).
template <typename T>
struct Mf;
template <>
struct Mf<float> {
  typedef floatx4 acc_t;
  static __device__ __forceinline__ void mma(float a, float b, floatx4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int i) { return 4 * g + i; }
};
template <>
struct Mf<double> {
  typedef doublex4 acc_t;
  static __device__ __forceinline__ void mma(double a, double b, doublex4& c) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int i) { return g + 4 * i; }
};

// mode 0: only partials of basis^T (pen F - M)  (initialisation)
// mode 1: update F, M, then partials
// Per sweep of CH rows: the basis rows go to LDS; LX = basis * C on the
// MFMA (wave w owns rows 16w..16w+15); the row update is applied in the
// MFMA's result layout; then the k x r partial basis^T (pen F - M) is
// accumulated on the MFMA in registers across sweeps (wave w owns M-blocks
// w and w + 4).  KP, RP: k, r padded to 16.
template <typename T, int CH>
__device__ __forceinline__ void admm_uv_body(const AdmmSide& s0, const AdmmSide& s1, int nblk0, int bid,
                                             const double* __restrict__ XY, int k, int r, double xi, int mode,
                                             double* __restrict__ Pp, int rows_per_blk0, int rows_per_blk1,
                                             char* smraw) {
  typedef typename Mf<T>::acc_t acc_t;
  const bool side1 = bid >= nblk0;
  const AdmmSide S = side1 ? s1 : s0;
  const int blk = side1 ? bid - nblk0 : bid;
  const int rpb = side1 ? rows_per_blk1 : rows_per_blk0;
  const double* C = XY + (side1 ? (int64_t)k * r : 0);
  double* out = Pp + (int64_t)bid * k * r;   // partial slot = block index within the request
  const T* __restrict__ Bm = (const T*)S.Bm;
  T* __restrict__ F = (T*)S.F;
  T* __restrict__ M = (T*)S.M;
  const T pen = (T)S.pen;
  const T inv_pen = (T)(1.0 / S.pen);
  const T xpen = (T)(xi * S.pen);
  const int KP16 = (k + 15) >> 4, RP16 = (r + 15) >> 4;
  const int KP = KP16 * 16, RP = RP16 * 16;
  const int ldb = KP + 1, ldc = RP + 1;

  T* cs = reinterpret_cast<T*>(smraw);   // KP x ldc
  T* bs = cs + KP * ldc;                 // CH x ldb
  T* ws = bs + CH * ldb;                 // CH x ldc
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, g = lane >> 4;
  for (int e = tid; e < KP * RP; e += 256) {
    int a = e / RP, c = e - a * RP;
    cs[a * ldc + c] = (a < k && c < r) ? (T)C[a * r + c] : T(0);
  }
  acc_t pacc[2][4];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) pacc[u][v] = acc_t{0, 0, 0, 0};

  const int i0 = blk * rpb;
  const int i1 = min(S.rows, i0 + rpb);
  for (int base = i0; base < i1; base += CH) {
    const int nr = min(CH, i1 - base);
    // prefetch this lane's F / M entries of the sweep (MFMA result layout)
    T fv[CH / 64 > 0 ? CH / 64 : 1][4][4], mv[CH / 64 > 0 ? CH / 64 : 1][4][4];
#pragma unroll
    for (int q = 0; q < (CH / 64 > 0 ? CH / 64 : 1); ++q) {
      const int rg = w + 4 * q;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * rg + Mf<T>::out_row(g, i), col = 16 * cb + lr;
          const bool ok = rg < CH / 16 && cb < RP16 && row < nr && col < r;
          const int64_t off = (int64_t)(base + row) * S.ldf + col;
          fv[q][cb][i] = ok ? F[off] : T(0);
          mv[q][cb][i] = ok ? M[off] : T(0);
        }
    }
    __syncthreads();
    for (int e = tid; e < CH * KP; e += 256) {
      int rr = e / KP, a = e - rr * KP;
      bs[rr * ldb + a] = (rr < nr && a < k) ? Bm[(int64_t)(base + rr) * S.ldb + a] : T(0);
    }
    __syncthreads();
    // ---- LX and the row update (waves own 16-row groups) ----
#pragma unroll
    for (int q = 0; q < (CH / 64 > 0 ? CH / 64 : 1); ++q) {
      const int rg = w + 4 * q;
      if (rg >= CH / 16) continue;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        if (cb >= RP16) continue;
        acc_t acc = acc_t{0, 0, 0, 0};
        if (mode == 1) {
          const T* ap = bs + (16 * rg + lr) * ldb + g;
          const T* bp = cs + g * ldc + 16 * cb + lr;
          for (int ks = 0; ks < KP / 4; ++ks) Mf<T>::mma(ap[4 * ks], bp[4 * ks * ldc], acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * rg + Mf<T>::out_row(g, i), col = 16 * cb + lr;
          const bool ok = row < nr && col < r;
          T f = fv[q][cb][i], mu = mv[q][cb][i];
          if (ok && mode == 1) {
            const T lx = acc[i];
            const T t = lx + mu * inv_pen;
            f = t > T(0) ? t : T(0);
            mu = mu + xpen * (lx - f);
            const int64_t off = (int64_t)(base + row) * S.ldf + col;
            F[off] = f;
            M[off] = mu;
          }
          ws[row * ldc + col] = ok ? pen * f - mu : T(0);
        }
      }
    }
    __syncthreads();
    // ---- partial: P (KP x RP) += bs^T (KP x CH) * ws (CH x RP) ----
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int mb = w + 4 * u;
      if (mb < KP16) {
        for (int ks = 0; ks < CH / 4; ++ks) {
          const T a = bs[(4 * ks + g) * ldb + 16 * mb + lr];
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (v < RP16) Mf<T>::mma(a, ws[(4 * ks + g) * ldc + 16 * v + lr], pacc[u][v]);
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int mb = w + 4 * u;
    if (mb < KP16) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int a = 16 * mb + Mf<T>::out_row(g, i), c = 16 * v + lr;
          if (v < RP16 && a < k && c < r) out[a * r + c] = (double)pacc[u][v][i];
        }
    }
  }
}

template <typename T, int CH>
__global__ __launch_bounds__(256) void admm_uv_kernel(AdmmSide s0, AdmmSide s1, int nblk0,
                                                      const double* __restrict__ XY, int k, int r,
                                                      double xi, int mode, double* __restrict__ Pp,
                                                      int rows_per_blk0, int rows_per_blk1) {
  extern __shared__ char smraw[];
  admm_uv_body<T, CH>(s0, s1, nblk0, blockIdx.x, XY, k, r, xi, mode, Pp, rows_per_blk0, rows_per_blk1, smraw);
}

// Job of global block b in a batched launch: the last job whose first
// block is <= b (first blocks ascending, jobs[0].first == 0).
__device__ __forceinline__ int batch_job(const int* __restrict__ first, int njobs, int b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One ADMM row update (mode 1) for every job of a batch: the blocks of job j
// are [uv_first[j], uv_first[j + 1]).
template <typename T, int CH>
__global__ __launch_bounds__(256) void admm_uv_batch_kernel(const AdmmJob* __restrict__ jobs,
                                                            const int* __restrict__ uv_first, int njobs) {
  extern __shared__ char smraw[];
  const int j = batch_job(uv_first, njobs, blockIdx.x);
  const AdmmJob& J = jobs[j];
  admm_uv_body<T, CH>(J.s0, J.s1, J.parts0, (int)blockIdx.x - uv_first[j], J.XY, J.k, J.r, J.xi, 1, J.Pp,
                      J.rpb0, J.rpb1, smraw);
}

template <typename T>
hipError_t launch_admm_uv(AdmmSide s0, AdmmSide s1, int nsides, const double* XY, int k, int r, double xi,
                          int mode, double* Pp, int parts0, int parts1, hipStream_t st) {
  if (k > 128 || r > 64) return hipErrorInvalidValue;
  const int KP = (k + 15) / 16 * 16, RP = (r + 15) / 16 * 16;
  int rpb0 = (s0.rows + parts0 - 1) / parts0;
  int rpb1 = nsides > 1 ? (s1.rows + parts1 - 1) / parts1 : 1;
  int nb = parts0 + (nsides > 1 ? parts1 : 0);
  auto lds = [&](int ch) { return ((size_t)KP * (RP + 1) + (size_t)ch * (KP + 1) + (size_t)ch * (RP + 1)) * sizeof(T); };
  if (lds(64) <= 160 * 1024) {
    hipFuncSetAttribute((const void*)admm_uv_kernel<T, 64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds(64));
    hipLaunchKernelGGL((admm_uv_kernel<T, 64>), dim3(nb), dim3(256), lds(64), st, s0, s1, parts0, XY, k, r, xi, mode,
                       Pp, rpb0, rpb1);
  } else {
    hipFuncSetAttribute((const void*)admm_uv_kernel<T, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds(32));
    hipLaunchKernelGGL((admm_uv_kernel<T, 32>), dim3(nb), dim3(256), lds(32), st, s0, s1, parts0, XY, k, r, xi, mode,
                       Pp, rpb0, rpb1);
  }
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_admm_uv<float>(AdmmSide, AdmmSide, int, const double*, int, int, double, int, double*, int, int, hipStream_t);
template hipError_t launch_admm_uv<double>(AdmmSide, AdmmSide, int, const double*, int, int, double, int, double*, int, int, hipStream_t);

// Fixed-order sums of the partials: P_U over the parts0 blocks of the U
// side and P_V over the parts1 blocks of the V side, into Pred[0], Pred[1].
// Blocks [0, nbh) reduce P_U, blocks [nbh, 2 nbh) reduce P_V.
constexpr int kRedNT = 256;
constexpr int kRedEPB = 32;

__device__ __forceinline__ void admm_reduce_body(const double* __restrict__ Pp, int parts0, int parts1, int64_t kr,
                                                 double* __restrict__ Pred, int nbh, int bid, double* red) {
  const bool vside = bid >= nbh;
  const int64_t e0 = (int64_t)(vside ? bid - nbh : bid) * kRedEPB;
  if (!vside)
    block_sum_parts<kRedNT, kRedEPB>(Pp, parts0, kr, kr, e0, Pred, red);
  else
    block_sum_parts<kRedNT, kRedEPB>(Pp + (int64_t)parts0 * kr, parts1, kr, kr, e0, Pred + kr, red);
}

__global__ __launch_bounds__(kRedNT) void admm_reduce_kernel(const double* __restrict__ Pp, int parts0,
                                                             int parts1, int64_t kr, double* __restrict__ Pred) {
  __shared__ double red[kRedNT];
  admm_reduce_body(Pp, parts0, parts1, kr, Pred, gridDim.x / 2, blockIdx.x, red);
}

int admm_reduce_blocks(int k, int r) { return 2 * (int)(((int64_t)k * r + kRedEPB - 1) / kRedEPB); }

__global__ __launch_bounds__(kRedNT) void admm_reduce_batch_kernel(const AdmmJob* __restrict__ jobs,
                                                                   const int* __restrict__ red_first, int njobs) {
  __shared__ double red[kRedNT];
  const int j = batch_job(red_first, njobs, blockIdx.x);
  const AdmmJob& J = jobs[j];
  const int64_t kr = (int64_t)J.k * J.r;
  const int nbh = (int)((kr + kRedEPB - 1) / kRedEPB);
  admm_reduce_body(J.Pp, J.parts0, J.parts1, kr, J.Pred, nbh, (int)blockIdx.x - red_first[j], red);
}

// The two r x r solves of one iteration in one workgroup.  XY: [0] Xt
// (k x r), [1] Yt^T (k x r), FP64.  first != 0: Yt^T = P_V / phi before the
// Xt solve (Alg. 3 initialisation Yt = V R^T, the partial having been
// formed as R (phi V^T)).  The systems are padded to N = 16 ceil(r / 16)
// with an identity block and solved by the blocked Cholesky in LDS.
constexpr int kSolveNT = 256;

__device__ __forceinline__ void admm_solve_body(const double* __restrict__ Pred, const double* __restrict__ At,
                                                int k, int r, double lam, double phi, int first,
                                                double* __restrict__ XY, int* flags, int at_in_lds, double* sm) {
  constexpr int NT = kSolveNT;
  const int tid = threadIdx.x;
  const int64_t kr = (int64_t)k * r;
  const int NB = (r + 15) / 16, N = 16 * NB, ld = N + 1;
  double* Y = sm;                  // Yt^T, k x ld
  double* X = Y + k * ld;          // Xt / RHS, k x ld
  double* Mm = X + k * ld;         // N x ld: system matrix, then its factor
  double* TI = Mm + N * ld;        // NB x 16 x 17
  double* PN = TI + NB * 272;      // 16 x ld
  double* Rs = PN + 16 * ld;       // k x 17
  double* Ats = Rs + k * 17;       // k x k when at_in_lds
  const double* Aa = at_in_lds ? Ats : At;
  const double* PU = Pred;
  const double* PV = Pred + kr;
  for (int e = tid; e < k * N; e += NT) {
    int i = e / N, c = e - i * N;
    Y[i * ld + c] = c < r ? (first ? PV[i * r + c] / phi : XY[kr + i * r + c]) : 0.0;
  }
  if (at_in_lds)
    for (int e = tid; e < k * k; e += NT) Ats[e] = At[e];
  __syncthreads();
  // pass 0: Xt from (At, Yt, P_U, lam); pass 1: Yt^T from (At^T, Xt, P_V, phi)
  for (int pass = 0; pass < 2; ++pass) {
    const double* S = pass ? X : Y;     // k x ld (the other factor)
    double* D = pass ? Y : X;           // RHS, then the solution
    const double* P = pass ? PV : PU;
    const double pen = pass ? phi : lam;
    // system matrix S^T S + pen I (padded with I), 4 x 4 tiles of the upper
    // block triangle
    const int NQ = N / 4;
    for (int e = tid; e < NQ * NQ; e += NT) {
      const int ta = e / NQ, tb = e - ta * NQ;
      if (tb < ta) continue;
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll 4
      for (int l = 0; l < k; ++l) {
        const double* sl = S + l * ld;
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          x[u] = sl[4 * ta + u];
          y[u] = sl[4 * tb + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(x[u], y[v], acc[u][v]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 4 * ta + u, b = 4 * tb + v;
          if (b < a) continue;
          const double val = acc[u][v] + (a == b ? (a < r ? pen : 1.0) : 0.0);
          Mm[a * ld + b] = val;
          Mm[b * ld + a] = val;
        }
    }
    // RHS = At S + P (pass 0) or At^T S + P (pass 1), zero padding; 4 x 4 tiles
    const int KQ = (k + 3) / 4;
    for (int e = tid; e < KQ * NQ; e += NT) {
      const int ta = e / NQ, tc = e - ta * NQ;
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll 4
      for (int l = 0; l < k; ++l) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int a = min(4 * ta + u, k - 1);
          x[u] = pass == 0 ? Aa[a * k + l] : Aa[l * k + a];
          y[u] = S[l * ld + 4 * tc + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(x[u], y[v], acc[u][v]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 4 * ta + u, c = 4 * tc + v;
          if (a < k) D[a * ld + c] = c < r ? acc[u][v] + P[a * r + c] : 0.0;
        }
    }
    __syncthreads();
    double mx = 0.0;
    for (int i = 0; i < r; ++i) mx = fmax(mx, Mm[i * ld + i]);
    wg_chol_blocked<NT>(Mm, ld, NB, TI, PN, 1e-300 * mx, flags);
    wg_right_solve_blocked<NT>(D, k, ld, NB, Mm, ld, TI, Rs);
    double* out = XY + (pass ? kr : 0);
    for (int e = tid; e < kr; e += NT) {
      int i = e / r, c = e - i * r;
      out[e] = D[i * ld + c];
    }
  }
}

// ---------------------------------------------------------------------------
// The same two solves with an explicit inverse kept from one iteration to the
// next (k <= 80, r <= 64).  For each side the system matrix M = S^T S + pen I
// (padded to N = 16 ceil(r / 16) with an identity block) is inverted by
// Newton-Schulz steps Z <- Z + Z (I - M Z), warm-started from the previous
// iteration's inverse, until ||I - M Z||_F <= tol (8 N eps for FP64
// factors; 1e-10 for FP32 factors, far below their rounding) or it stops
// shrinking by half; the first iteration, a warm start with ||I - M Z||_F > 1/2 and a
// non-converging start use the blocked Cholesky and solve for Z = M^-1
// instead.  Then X = RHS Z.  Every product is a 16x16x4 FP64 MFMA tile
// product in LDS; Z is stored for the next iteration.
// ---------------------------------------------------------------------------
constexpr int kNsMaxK = 80;

struct NsLayout {
  int NB, N, ld, kp, KB16;
  size_t s_off, m_off, z_off, e_off, red_off, total;  // in doubles
};
__host__ __device__ inline NsLayout ns_layout(int k, int r) {
  NsLayout L;
  L.NB = (r + 15) / 16;
  L.N = 16 * L.NB;
  L.ld = L.N + 2;
  L.KB16 = (k + 15) / 16;
  L.kp = 16 * L.KB16;
  const size_t rowsE = (size_t)(L.kp > L.N ? L.kp : L.N);
  size_t eb = rowsE * L.ld;
  const size_t fb = (size_t)L.NB * 272 + 16 * (size_t)L.ld + (size_t)L.N * 17;  // fallback scratch
  if (fb > eb) eb = fb;
  L.s_off = 0;
  L.m_off = L.s_off + (size_t)L.kp * L.ld;
  L.z_off = L.m_off + (size_t)L.N * L.ld;
  L.e_off = L.z_off + (size_t)L.N * L.ld;
  L.red_off = L.e_off + eb;
  L.total = L.red_off + 8;
  return L;
}

// acc[cb] = rows 16 rb + g + 4 i, cols 16 cb + c of A B for cb < ncb, where
// lane (c, g) supplies A(16 rb + c, kk) and B(kk, 16 cb + c) for kk = 4 s + g.
template <int NCB, typename FA, typename FB>
__device__ __forceinline__ void ns_tile_rows(FA fa, FB fb, int K, int rb, int c, int g, doublex4 (&acc)[4]) {
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int nsteps = K / 4;
#pragma unroll 4
  for (int s = 0; s < nsteps; ++s) {
    const int kk = 4 * s + g;
    const double a = fa(16 * rb + c, kk);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, fb(kk, 16 * cb + c), acc[cb], 0, 0, 0);
  }
}

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Z = M^-1 by the blocked Cholesky of M (in place) and a solve of Z M = I;
// kept out of line so that the register budget of the Newton-Schulz path is
// not set by it.
__device__ __attribute__((noinline)) void ns_chol_inverse(double* Mb, double* Zb, double* Eb, int ld, int NB, int N,
                                                          int r, int* flags) {
  constexpr int NT = kSolveNT;
  const int tid = threadIdx.x;
  double* TI = Eb;
  double* PN = TI + NB * 272;
  double* Rs = PN + 16 * ld;
  double mx = 0.0;
  for (int i = 0; i < r; ++i) mx = fmax(mx, Mb[i * ld + i]);
  wg_chol_blocked<NT>(Mb, ld, NB, TI, PN, 1e-300 * mx, flags);
  for (int e = tid; e < N * N; e += NT) {
    const int i = e / N, j = e - i * N;
    Zb[i * ld + j] = i == j ? 1.0 : 0.0;
  }
  wg_right_solve_blocked<NT>(Zb, N, ld, NB, Mb, ld, TI, Rs);
  __syncthreads();
}

template <int NB>
__device__ __forceinline__ void admm_solve_ns_nb(const double* __restrict__ Pred, const double* __restrict__ At, int k,
                                                 int r, double lam, double phi, int first, double* __restrict__ XY,
                                                 double* __restrict__ Zg, int* flags, double tol_in, double* sm) {
  constexpr int NT = kSolveNT;
  constexpr int N = 16 * NB;
  const NsLayout Ly = ns_layout(k, r);
  const int ld = Ly.ld, kp = Ly.kp, KB16 = Ly.KB16;
  double* S = sm + Ly.s_off;
  double* Mb = sm + Ly.m_off;
  double* Zb = sm + Ly.z_off;
  double* Eb = sm + Ly.e_off;
  double* red = sm + Ly.red_off;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int64_t kr = (int64_t)k * r;
  const double tol = tol_in > 0.0 ? tol_in : 8.0 * N * 2.220446049250313e-16;
  // S = Yt^T (k x r, zero padded to kp x N)
  for (int e = tid; e < kp * N; e += NT) {
    const int i = e / N, j = e - i * N;
    S[i * ld + j] = (i < k && j < r) ? (first ? Pred[kr + i * r + j] / phi : XY[kr + i * r + j]) : 0.0;
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    const double pen = pass ? phi : lam;
    const double* P = Pred + (pass ? kr : 0);
    double* Zh = Zg + (size_t)pass * 64 * 64;
    doublex4 acc[4];
    // (a) M = S^T S + pen I_r, identity on the padding
    if (w < NB) {
      ns_tile_rows<NB>([&](int i, int kk) { return S[kk * ld + i]; }, [&](int kk, int j) { return S[kk * ld + j]; }, kp,
                   w, c, g, acc);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (cb >= NB) continue;
          const int row = 16 * w + g + 4 * i, col = 16 * cb + c;
          Mb[row * ld + col] = acc[cb][i] + (row == col ? (row < r ? pen : 1.0) : 0.0);
        }
    }
    // warm start
    if (!first)
      for (int e = tid; e < N * N; e += NT) Zb[(e / N) * ld + (e % N)] = Zh[e];
    __syncthreads();
    bool need_chol = first != 0;
    if (!need_chol) {
      double e_prev = 0.0;
      int it = 0;
      const int kMaxIt = 8;
      for (;; ++it) {
        // E = I - M Z
        double ss = 0.0;
        if (w < NB) {
          ns_tile_rows<NB>([&](int i, int kk) { return Mb[i * ld + kk]; }, [&](int kk, int j) { return Zb[kk * ld + j]; },
                       N, w, c, g, acc);
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              if (cb >= NB) continue;
              const int row = 16 * w + g + 4 * i, col = 16 * cb + c;
              const double ev = (row == col ? 1.0 : 0.0) - acc[cb][i];
              Eb[row * ld + col] = ev;
              ss = fma(ev, ev, ss);
            }
        }
        ss = wave_sum_d(ss);
        if (lane == 0) red[w] = ss;
        __syncthreads();
        const double en = sqrt((red[0] + red[1]) + (red[2] + red[3]));
        if (!isfinite(en) || (it == 0 && en > 0.5)) {
          need_chol = true;
          break;
        }
        if (en <= tol || (it > 0 && en > 0.5 * e_prev)) break;
        if (it == kMaxIt) {
          need_chol = true;
          break;
        }
        // Z <- Z + Z E
        if (w < NB) {
          ns_tile_rows<NB>([&](int i, int kk) { return Zb[i * ld + kk]; }, [&](int kk, int j) { return Eb[kk * ld + j]; },
                       N, w, c, g, acc);
        }
        __syncthreads();
        if (w < NB) {
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              if (cb >= NB) continue;
              const int row = 16 * w + g + 4 * i, col = 16 * cb + c;
              Zb[row * ld + col] += acc[cb][i];
            }
        }
        __syncthreads();
        e_prev = en;
      }
    }
    if (need_chol) ns_chol_inverse(Mb, Zb, Eb, ld, NB, N, r, flags);
    // (d) RHS = At S + P (pass 0) or At^T S + P (pass 1) into Eb (kp x N).
    // The lane's At values for all K steps are loaded from global memory up
    // front, so their latency is paid once.
    for (int rb = w; rb < KB16; rb += 4) {
      const int i = 16 * rb + c;
      double av[kNsMaxK / 4];
#pragma unroll
      for (int s = 0; s < kNsMaxK / 4; ++s) {
        const int kk = 4 * s + g;
        double v = 0.0;
        if (i < k && kk < k) v = pass == 0 ? At[i * k + kk] : At[kk * k + i];
        av[s] = v;
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < kNsMaxK / 4; ++s) {
        if (4 * s < kp) {
          const int kk = 4 * s + g;
#pragma unroll
          for (int cb = 0; cb < NB; ++cb)
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], S[kk * ld + 16 * cb + c], acc[cb], 0, 0, 0);
        }
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          if (cb >= NB) continue;
          const int row = 16 * rb + g + 4 * ii, col = 16 * cb + c;
          Eb[row * ld + col] = (row < k && col < r) ? acc[cb][ii] + P[row * r + col] : 0.0;
        }
    }
    __syncthreads();
    // (e) X = RHS Z, written to XY and, for pass 0, into S for the other side
    double* out = XY + (pass ? kr : 0);
    for (int rb = w; rb < KB16; rb += 4) {
      ns_tile_rows<NB>([&](int i, int kk) { return Eb[i * ld + kk]; }, [&](int kk, int j) { return Zb[kk * ld + j]; }, N,
                   rb, c, g, acc);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (cb >= NB) continue;
          const int row = 16 * rb + g + 4 * i, col = 16 * cb + c;
          const double v = (row < k && col < r) ? acc[cb][i] : 0.0;
          if (row < k && col < r) out[row * r + col] = v;
          if (pass == 0) S[row * ld + col] = v;
        }
    }
    // (f) keep Z for the next iteration
    for (int e = tid; e < N * N; e += NT) Zh[e] = Zb[(e / N) * ld + (e % N)];
    __syncthreads();
  }
}

__device__ __forceinline__ void admm_solve_ns_body(const double* __restrict__ Pred, const double* __restrict__ At,
                                                   int k, int r, double lam, double phi, int first,
                                                   double* __restrict__ XY, double* __restrict__ Zg, int* flags,
                                                   double tol, double* sm) {
  switch ((r + 15) / 16) {
    case 1: admm_solve_ns_nb<1>(Pred, At, k, r, lam, phi, first, XY, Zg, flags, tol, sm); break;
    case 2: admm_solve_ns_nb<2>(Pred, At, k, r, lam, phi, first, XY, Zg, flags, tol, sm); break;
    case 3: admm_solve_ns_nb<3>(Pred, At, k, r, lam, phi, first, XY, Zg, flags, tol, sm); break;
    default: admm_solve_ns_nb<4>(Pred, At, k, r, lam, phi, first, XY, Zg, flags, tol, sm); break;
  }
}

__global__ __launch_bounds__(kSolveNT) void admm_solve_ns_kernel(const double* __restrict__ Pred,
                                                                 const double* __restrict__ At, int k, int r,
                                                                 double lam, double phi, int first,
                                                                 double* __restrict__ XY, double* __restrict__ Z,
                                                                 int* flags, double tol) {
  extern __shared__ double sm[];
  admm_solve_ns_body(Pred, At, k, r, lam, phi, first, XY, Z, flags, tol, sm);
}

__global__ __launch_bounds__(kSolveNT) void admm_solve_kernel(const double* __restrict__ Pred,
                                                              const double* __restrict__ At, int k, int r,
                                                              double lam, double phi, int first,
                                                              double* __restrict__ XY, int* flags, int at_in_lds) {
  extern __shared__ double sm[];
  admm_solve_body(Pred, At, k, r, lam, phi, first, XY, flags, at_in_lds, sm);
}

// One workgroup per job.
__global__ __launch_bounds__(kSolveNT) void admm_solve_batch_kernel(const AdmmJob* __restrict__ jobs) {
  extern __shared__ double sm[];
  const AdmmJob& J = jobs[blockIdx.x];
  if (J.Z && J.k <= kNsMaxK)
    admm_solve_ns_body(J.Pred, J.At, J.k, J.r, J.lam, J.phi, J.first, J.XY, J.Z, J.flags, 1e-10, sm);
  else
    admm_solve_body(J.Pred, J.At, J.k, J.r, J.lam, J.phi, J.first, J.XY, J.flags, J.at_in_lds, sm);
}

static size_t admm_solve_lds(int k, int r, bool with_at) {
  const int NB = (r + 15) / 16, N = 16 * NB, ld = N + 1;
  size_t d = 2 * (size_t)k * ld + (size_t)N * ld + (size_t)NB * 272 + 16 * (size_t)ld + (size_t)k * 17;
  if (with_at) d += (size_t)k * k;
  return d * sizeof(double);
}

template <typename T>
hipError_t launch_admm_solve(const double* Pp, int parts0, int parts1, const double* At, int k, int r,
                             double lam, double phi, int first, double* XY, double* Pred, double* Z,
                             int* flags, hipStream_t st) {
  if (r > 64 || k > 128) return hipErrorInvalidValue;
  const size_t cap = 160 * 1024;
  if (Z && k <= kNsMaxK) {
    int64_t kr = (int64_t)k * r;
    int nbh = (int)((kr + kRedEPB - 1) / kRedEPB);
    hipLaunchKernelGGL(admm_reduce_kernel, dim3(2 * nbh), dim3(kRedNT), 0, st, Pp, parts0, parts1, kr, Pred);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t sm = ns_layout(k, r).total * sizeof(double);
    hipFuncSetAttribute((const void*)admm_solve_ns_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    const double tol = sizeof(T) == 4 ? 1e-10 : 0.0;   // 0: 8 N eps
    hipLaunchKernelGGL(admm_solve_ns_kernel, dim3(1), dim3(kSolveNT), sm, st, Pred, At, k, r, lam, phi, first, XY, Z,
                       flags, tol);
    CNMF_LAUNCH_CHECK();
  }
  int at_in_lds = admm_solve_lds(k, r, true) <= cap;
  size_t sm = admm_solve_lds(k, r, at_in_lds);
  if (sm > cap) return hipErrorInvalidValue;
  int64_t kr = (int64_t)k * r;
  int nbh = (int)((kr + kRedEPB - 1) / kRedEPB);
  hipLaunchKernelGGL(admm_reduce_kernel, dim3(2 * nbh), dim3(kRedNT), 0, st, Pp, parts0, parts1, kr, Pred);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipFuncSetAttribute((const void*)admm_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL(admm_solve_kernel, dim3(1), dim3(kSolveNT), sm, st, Pred, At, k, r, lam, phi, first, XY, flags,
                     at_in_lds);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_admm_solve<float>(const double*, int, int, const double*, int, int, double, double, int, double*, double*, double*, int*, hipStream_t);
template hipError_t launch_admm_solve<double>(const double*, int, int, const double*, int, int, double, double, int, double*, double*, double*, int*, hipStream_t);

// ---------------------------------------------------------------------------
// Batched ADMM step (serving): for every job, the fixed-order partial sums,
// the two r x r solves and the mode-1 row update, as three launches over all
// jobs.  Each job runs exactly the per-request code above, so its result does
// not depend on which other jobs share the launch.
// ---------------------------------------------------------------------------
void admm_job_prepare(AdmmJob& J) {
  J.rpb0 = (J.s0.rows + J.parts0 - 1) / J.parts0;
  J.rpb1 = (J.s1.rows + J.parts1 - 1) / J.parts1;
  J.at_in_lds = admm_solve_lds(J.k, J.r, true) <= 160 * 1024;
}

int admm_job_uv_blocks(const AdmmJob& J) { return J.parts0 + J.parts1; }
int admm_job_red_blocks(const AdmmJob& J) { return admm_reduce_blocks(J.k, J.r); }

hipError_t launch_admm_step_batch(const AdmmJob* jobs_dev, const int* uv_first_dev, const int* red_first_dev,
                                  int njobs, int uv_blocks, int red_blocks, int max_k, int max_r, size_t solve_lds,
                                  hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  if (max_r > 64 || max_k > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(admm_reduce_batch_kernel, dim3(red_blocks), dim3(kRedNT), 0, st, jobs_dev, red_first_dev, njobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (solve_lds > 160 * 1024) return hipErrorInvalidValue;
  hipFuncSetAttribute((const void*)admm_solve_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)solve_lds);
  hipLaunchKernelGGL(admm_solve_batch_kernel, dim3(njobs), dim3(kSolveNT), solve_lds, st, jobs_dev);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int KP = (max_k + 15) / 16 * 16, RP = (max_r + 15) / 16 * 16;
  const size_t lds = ((size_t)KP * (RP + 1) + 64 * (size_t)(KP + 1) + 64 * (size_t)(RP + 1)) * sizeof(float);
  hipFuncSetAttribute((const void*)admm_uv_batch_kernel<float, 64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  hipLaunchKernelGGL((admm_uv_batch_kernel<float, 64>), dim3(uv_blocks), dim3(256), lds, st, jobs_dev, uv_first_dev,
                     njobs);
  CNMF_LAUNCH_CHECK();
}

size_t admm_job_solve_lds(const AdmmJob& J) {
  if (J.Z && J.k <= kNsMaxK) return ns_layout(J.k, J.r).total * sizeof(double);
  return admm_solve_lds(J.k, J.r, J.at_in_lds != 0);
}

}  // namespace cnmf
