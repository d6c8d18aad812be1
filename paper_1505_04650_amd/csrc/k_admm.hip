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

namespace cnmf {

constexpr int kUvRows = 32;   // rows staged per sweep
constexpr int kMaxK16 = 8;    // k <= 128
constexpr int kMaxR16 = 4;    // r <= 64

// mode 0: only partials of basis^T (pen F - M)  (initialisation)
// mode 1: update F, M, then partials
template <typename T>
__global__ __launch_bounds__(256) void admm_uv_kernel(AdmmSide s0, AdmmSide s1, int nblk0,
                                                      const double* __restrict__ XY, int k, int r,
                                                      double xi, int mode, double* __restrict__ Pp,
                                                      int rows_per_blk0, int rows_per_blk1) {
  const bool side1 = (int)blockIdx.x >= nblk0;
  const AdmmSide S = side1 ? s1 : s0;
  const int blk = side1 ? blockIdx.x - nblk0 : blockIdx.x;
  const int rpb = side1 ? rows_per_blk1 : rows_per_blk0;
  const double* C = XY + (side1 ? (int64_t)k * r : 0);
  double* out = Pp + (int64_t)blockIdx.x * k * r;   // partial slot = global block index
  const T* Bm = (const T*)S.Bm;
  T* F = (T*)S.F;
  T* M = (T*)S.M;
  const T pen = (T)S.pen;
  const T inv_pen = (T)(1.0 / S.pen);
  const T xpen = (T)(xi * S.pen);

  __shared__ T cs[128 * 64];             // C: k x r
  __shared__ T bs[kUvRows][129];         // basis rows
  __shared__ T ws[kUvRows][65];          // pen F - M for the staged rows
  const int tid = threadIdx.x;
  for (int e = tid; e < k * r; e += 256) cs[e] = (T)C[e];
  const int ta = tid >> 4, tb = tid & 15;
  double acc[kMaxK16][kMaxR16];
#pragma unroll
  for (int i = 0; i < kMaxK16; ++i)
#pragma unroll
    for (int j = 0; j < kMaxR16; ++j) acc[i][j] = 0.0;

  const int i0 = blk * rpb;
  const int i1 = min(S.rows, i0 + rpb);
  __syncthreads();
  for (int base = i0; base < i1; base += kUvRows) {
    const int nr = min(kUvRows, i1 - base);
    for (int e = tid; e < kUvRows * k; e += 256) {
      int rr = e / k, a = e - rr * k;
      bs[rr][a] = rr < nr ? Bm[(int64_t)(base + rr) * S.ldb + a] : T(0);
    }
    __syncthreads();
    for (int e = tid; e < nr * r; e += 256) {
      int rr = e / r, c = e - rr * r;
      int64_t off = (int64_t)(base + rr) * S.ldf + c;
      T f = F[off];
      T mu = M[off];
      if (mode == 1) {
        T lx = 0;
        for (int a = 0; a < k; ++a) lx = fma(bs[rr][a], cs[a * r + c], lx);
        T t = lx + mu * inv_pen;
        f = t > T(0) ? t : T(0);
        mu = mu + xpen * (lx - f);
        F[off] = f;
        M[off] = mu;
      }
      ws[rr][c] = pen * f - mu;
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
#pragma unroll
      for (int i = 0; i < kMaxK16; ++i) {
        int a = ta + 16 * i;
        double b = a < k ? (double)bs[rr][a] : 0.0;
#pragma unroll
        for (int j = 0; j < kMaxR16; ++j) {
          int c = tb + 16 * j;
          double w = c < r ? (double)ws[rr][c] : 0.0;
          acc[i][j] = fma(b, w, acc[i][j]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < kMaxK16; ++i)
#pragma unroll
    for (int j = 0; j < kMaxR16; ++j) {
      int a = ta + 16 * i, c = tb + 16 * j;
      if (a < k && c < r) out[a * r + c] = acc[i][j];
    }
}

template <typename T>
hipError_t launch_admm_uv(AdmmSide s0, AdmmSide s1, int nsides, const double* XY, int k, int r, double xi,
                          int mode, double* Pp, int parts0, int parts1, hipStream_t st) {
  if (k > 128 || r > 64) return hipErrorInvalidValue;
  int rpb0 = (s0.rows + parts0 - 1) / parts0;
  int rpb1 = nsides > 1 ? (s1.rows + parts1 - 1) / parts1 : 1;
  int nb = parts0 + (nsides > 1 ? parts1 : 0);
  hipLaunchKernelGGL(admm_uv_kernel<T>, dim3(nb), dim3(256), 0, st, s0, s1, parts0, XY, k, r, xi, mode, Pp,
                     rpb0, rpb1);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_admm_uv<float>(AdmmSide, AdmmSide, int, const double*, int, int, double, int, double*, int, int, hipStream_t);
template hipError_t launch_admm_uv<double>(AdmmSide, AdmmSide, int, const double*, int, int, double, int, double*, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Small dense helpers for one workgroup (NT threads), FP64 in LDS.
// ---------------------------------------------------------------------------
template <int NT>
__device__ void wg_chol_inv(double* Mm, int r, double* Ci, int* flag) {
  // Mm (r x r, row-major, SPD) -> upper Cholesky factor in place (Mm = C^T C),
  // then Ci = C^-1 (upper).
  const int tid = threadIdx.x;
  for (int j = 0; j < r; ++j) {
    __syncthreads();
    double d = Mm[j * r + j];
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0 && flag) atomicAdd(flag, 1);
      d = 1e-300;
    }
    const double t = sqrt(d);
    __syncthreads();
    if (tid == 0) Mm[j * r + j] = t;
    for (int c = j + 1 + tid; c < r; c += NT) Mm[j * r + c] /= t;
    __syncthreads();
    const int rem = r - j - 1;
    for (int e = tid; e < rem * rem; e += NT) {
      int a = e / rem, b = e - a * rem;
      if (b >= a) Mm[(j + 1 + a) * r + (j + 1 + b)] -= Mm[j * r + j + 1 + a] * Mm[j * r + j + 1 + b];
    }
  }
  __syncthreads();
  for (int i = r - 1; i >= 0; --i) {
    const double tii = Mm[i * r + i];
    for (int j = i + tid; j < r; j += NT) {
      if (j == i) {
        Ci[i * r + i] = 1.0 / tii;
      } else {
        double s = 0.0;
        for (int l = i + 1; l <= j; ++l) s = fma(Mm[i * r + l], Ci[l * r + j], s);
        Ci[i * r + j] = -s / tii;
      }
    }
    for (int j = tid; j < i; j += NT) Ci[i * r + j] = 0.0;
    __syncthreads();
  }
}

// X (rows x r) <- X C^-1 C^-T  (solve X M = RHS for M = C^T C), in place,
// using tmp (rows x r).
template <int NT>
__device__ void wg_right_solve(double* X, int rows, int r, const double* Ci, double* tmp) {
  const int tid = threadIdx.x;
  // tmp = X Ci   (Ci upper: tmp[i][c] = sum_{l <= c} X[i][l] Ci[l][c])
  for (int e = tid; e < rows * r; e += NT) {
    int i = e / r, c = e - i * r;
    double s = 0.0;
    for (int l = 0; l <= c; ++l) s = fma(X[i * r + l], Ci[l * r + c], s);
    tmp[e] = s;
  }
  __syncthreads();
  // X = tmp Ci^T  (X[i][c] = sum_{l >= c} tmp[i][l] Ci[c][l])
  for (int e = tid; e < rows * r; e += NT) {
    int i = e / r, c = e - i * r;
    double s = 0.0;
    for (int l = c; l < r; ++l) s = fma(tmp[i * r + l], Ci[c * r + l], s);
    X[e] = s;
  }
  __syncthreads();
}

// Reduce the partials (blocks of the first phase), then one workgroup does
// the two solves.  Pp: [parts0] k x r for P_U then [parts1] k x r for P_V.
// XY: [0] Xt (k x r), [1] Yt^T (k x r), FP64.  first != 0: Yt^T = P_V / phi
// before the Xt solve (Alg. 3 initialisation Yt = V R^T, with the partial
// computed as R (phi V^T)).
template <int NT>
__global__ __launch_bounds__(NT) void admm_solve_kernel(const double* __restrict__ Pp, int parts0,
                                                        int parts1, const double* __restrict__ At, int k,
                                                        int r, double lam, double phi, int first,
                                                        double* __restrict__ XY, double* __restrict__ Pred,
                                                        unsigned* counter, int* flags) {
  const int tid = threadIdx.x;
  const int64_t kr = (int64_t)k * r;
  // phase 1: Pred[0] = sum P_U partials, Pred[1] = sum P_V partials
  for (int64_t e = blockIdx.x * (int64_t)NT + tid; e < 2 * kr; e += (int64_t)gridDim.x * NT) {
    const bool v = e >= kr;
    const int64_t ee = v ? e - kr : e;
    const int p0 = v ? parts0 : 0;
    const int np = v ? parts1 : parts0;
    double s = 0.0;
    for (int p = 0; p < np; ++p) s += Pp[(int64_t)(p0 + p) * kr + ee];
    Pred[e] = s;
  }
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  extern __shared__ double sm[];
  double* Y = sm;                // Yt^T, k x r
  double* X = Y + kr;            // Xt / RHS, k x r
  double* Mm = X + kr;           // r x r
  double* Ci = Mm + r * r;       // r x r
  const double* PU = Pred;
  const double* PV = Pred + kr;
  for (int e = tid; e < kr; e += NT) Y[e] = first ? PV[e] / phi : XY[kr + e];
  __syncthreads();
  // M1 = Yt Yt^T + lam I = Y^T Y + lam I (r x r)
  for (int e = tid; e < r * r; e += NT) {
    int a = e / r, b = e - a * r;
    double s = 0.0;
    for (int l = 0; l < k; ++l) s = fma(Y[l * r + a], Y[l * r + b], s);
    Mm[e] = s + (a == b ? lam : 0.0);
  }
  // RHS1 = At Y + P_U (k x r)
  for (int e = tid; e < kr; e += NT) {
    int a = e / r, c = e - a * r;
    double s = 0.0;
    for (int l = 0; l < k; ++l) s = fma(At[a * k + l], Y[l * r + c], s);
    X[e] = s + PU[e];
  }
  __syncthreads();
  wg_chol_inv<NT>(Mm, r, Ci, flags);
  wg_right_solve<NT>(X, k, r, Ci, Y);     // X = Xt (Y is scratch here)
  // M2 = Xt^T Xt + phi I
  for (int e = tid; e < r * r; e += NT) {
    int a = e / r, b = e - a * r;
    double s = 0.0;
    for (int l = 0; l < k; ++l) s = fma(X[l * r + a], X[l * r + b], s);
    Mm[e] = s + (a == b ? phi : 0.0);
  }
  // RHS2 = At^T Xt + P_V (k x r)
  for (int e = tid; e < kr; e += NT) {
    int a = e / r, c = e - a * r;
    double s = 0.0;
    for (int l = 0; l < k; ++l) s = fma(At[l * k + a], X[l * r + c], s);
    Y[e] = s + PV[e];
  }
  __syncthreads();
  for (int e = tid; e < kr; e += NT) XY[e] = X[e];
  wg_chol_inv<NT>(Mm, r, Ci, flags);
  wg_right_solve<NT>(Y, k, r, Ci, X);     // Y = Yt^T (X is scratch here)
  for (int e = tid; e < kr; e += NT) XY[kr + e] = Y[e];
  if (tid == 0) *counter = 0u;
}

template <typename T>
hipError_t launch_admm_solve(const double* Pp, int parts0, int parts1, const double* At, int k, int r,
                             double lam, double phi, int first, double* XY, double* Pred, unsigned* counter,
                             int* flags, hipStream_t st) {
  constexpr int NT = 512;
  size_t sm = (2 * (size_t)k * r + 2 * (size_t)r * r) * sizeof(double);
  if (sm > 160 * 1024) return hipErrorInvalidValue;
  int64_t kr2 = 2LL * k * r;
  int nb = (int)std::max<int64_t>(1, std::min<int64_t>(64, (kr2 + NT - 1) / NT));
  hipFuncSetAttribute((const void*)admm_solve_kernel<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL(admm_solve_kernel<NT>, dim3(nb), dim3(NT), sm, st, Pp, parts0, parts1, At, k, r, lam, phi,
                     first, XY, Pred, counter, flags);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_admm_solve<float>(const double*, int, int, const double*, int, int, double, double, int, double*, double*, unsigned*, int*, hipStream_t);
template hipError_t launch_admm_solve<double>(const double*, int, int, const double*, int, int, double, double, int, double*, double*, unsigned*, int*, hipStream_t);

}  // namespace cnmf
