// ADMM for NMF on the two-sided compressed problem (Appendix B, Alg. 3).
//
// One iteration of the box, with Xt (k x r) and Yt^T (k x r) kept in FP64:
//   Xt   <- (At Yt^T + P_U) (Yt Yt^T + lam I)^-1,   P_U = L^T (lam U - Lam)
//   Yt^T <- (At^T Xt + P_V) (Xt^T Xt + phi I)^-1,   P_V = R (phi V^T - Phi^T)
//   U   <- max(L Xt + Lam/lam, 0);  Lam <- Lam + xi lam (L Xt - U)
//   V^T <- max(R^T Yt^T + Phi^T/phi, 0);  Phi^T <- Phi^T + xi phi (R^T Yt^T - V^T)
// The row updates (U, Lam over the m rows of L; V^T, Phi^T over the n rows of
// R^T) are the same operation on two "sides" (admm_uv_body).  It also forms
// the partial sums of basis^T (pen * F - M) for the next iteration's P_U /
// P_V, so the big matrices are read once per iteration; admm_reduce_body
// sums those partials in a fixed order, and the r x r solves are Cholesky
// factorisations in FP64 in one workgroup.  For one request the iteration
// runs as two launches (admm_half_kernel): the Yt^T solve beside the U-side
// row update, then the next Xt solve beside the V-side row update, each
// launch also summing its solve's partials in workgroups of its own that
// the solve waits for (where they fit beside it and finish in time; else
// the sums are separate launches after each half); serving runs both solves
// and both sides per launch over a batch of requests, with the sums in a
// launch before the solves.
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
// mode 1: update M, then partials; F (U or V^T) is not read: Alg. 3 sets it
//         from L Xt and the previous multipliers only, so within the
//         iterations it is needed only in registers
// mode 2: mode 1 and F stored (the last iteration)
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
  T* out = reinterpret_cast<T*>(Pp) + (int64_t)bid * k * r;   // partial slot = block index within the request
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
  // C of this side into LDS.  T = float: from the zero-padded FP32 copy
  // (KP x RP) the solve leaves after XY, 16-byte loads; T = double: from XY.
  // The loads are issued here and stored with the first sweep's, so the
  // block pays one memory latency for both.
  constexpr int NCV = std::is_same<T, float>::value ? 8 : 32;
  T cv[NCV][std::is_same<T, float>::value ? 4 : 1];
  {
    if constexpr (std::is_same<T, float>::value) {
      const float* Cf = reinterpret_cast<const float*>(XY + 2 * (int64_t)k * r) + (side1 ? KP * RP : 0);
#pragma unroll
      for (int j = 0; j < NCV; ++j) {
        const int v4 = tid + 256 * j;
        if (4 * v4 < KP * RP) {
          const float4 q = *reinterpret_cast<const float4*>(Cf + 4 * v4);
          cv[j][0] = q.x; cv[j][1] = q.y; cv[j][2] = q.z; cv[j][3] = q.w;
        }
      }
    } else {
      const int cc = tid & 63, rg0 = tid >> 6;
#pragma unroll
      for (int j = 0; j < NCV; ++j) {
        const int a = rg0 + 4 * j;
        cv[j][0] = (a < k && cc < r) ? (T)C[a * r + cc] : T(0);
      }
    }
  }
  auto store_c = [&]() {
    if constexpr (std::is_same<T, float>::value) {
#pragma unroll
      for (int j = 0; j < NCV; ++j) {
        const int v4 = tid + 256 * j;
        if (4 * v4 < KP * RP) {
          const int a = (4 * v4) / RP, c = 4 * v4 - a * RP;
#pragma unroll
          for (int u = 0; u < 4; ++u) cs[a * ldc + c + u] = cv[j][u];
        }
      }
    } else {
      const int cc = tid & 63, rg0 = tid >> 6;
#pragma unroll
      for (int j = 0; j < NCV; ++j) {
        const int a = rg0 + 4 * j;
        if (a < KP && cc < RP) cs[a * ldc + cc] = cv[j][0];
      }
    }
  };
  for (int e = tid; e < CH * ldb; e += 256) bs[e] = T(0);
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
          fv[q][cb][i] = (ok && mode == 0) ? F[off] : T(0);
          mv[q][cb][i] = ok ? M[off] : T(0);
        }
    }
    __syncthreads();
    if (base == i0) store_c();
    // basis rows of the sweep straight into LDS (global_load_lds: lane l of
    // a wave writes dword l after the row's LDS base), one row per wave
    // instruction and 64-dword chunk; lanes past the row's k entries are
    // masked off, so bs keeps the zeros written at the start there (and in
    // rows from nr on, which only meet zero rows of ws)
    {
      constexpr int DW = sizeof(T) / 4;   // dwords per element
      const int rowdw = k * DW;
      for (int rr = w; rr < nr; rr += 4) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(Bm + (int64_t)(base + rr) * S.ldb);
        for (int d0 = 0; d0 < rowdw; d0 += 64) {
          if (d0 + lane < rowdw)
            __builtin_amdgcn_global_load_lds(src + d0 + lane, reinterpret_cast<uint32_t*>(bs + rr * ldb) + d0, 4, 0,
                                             0);
        }
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
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
        if (mode != 0) {
          const T* ap = bs + (16 * rg + lr) * ldb + g;
          const T* bp = cs + g * ldc + 16 * cb + lr;
          for (int ks = 0; ks < KP / 4; ++ks) Mf<T>::mma(ap[4 * ks], bp[4 * ks * ldc], acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * rg + Mf<T>::out_row(g, i), col = 16 * cb + lr;
          const bool ok = row < nr && col < r;
          T f = fv[q][cb][i], mu = mv[q][cb][i];
          if (ok && mode != 0) {
            const T lx = acc[i];
            const T t = lx + mu * inv_pen;
            f = t > T(0) ? t : T(0);
            mu = mu + xpen * (lx - f);
            const int64_t off = (int64_t)(base + row) * S.ldf + col;
            if (mode == 2) F[off] = f;
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
          if (v < RP16 && a < k && c < r) out[a * r + c] = (T)pacc[u][v][i];
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
  admm_uv_body<T, CH>(J.s0, J.s1, J.parts0, (int)blockIdx.x - uv_first[j], J.XY, J.k, J.r, J.xi, J.last ? 2 : 1,
                      J.Pp, J.rpb0, J.rpb1, smraw);
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
constexpr int kRedEPB = 16;

// The partials are stored in the factors' precision T (the row updates
// accumulate them in T on the MFMA) and summed in FP64.
template <typename T>
__device__ __forceinline__ void admm_reduce_body(const double* __restrict__ Pp, int parts0, int parts1, int64_t kr,
                                                 double* __restrict__ Pred, int nbh, int bid, double* red) {
  const bool vside = bid >= nbh;
  const int64_t e0 = (int64_t)(vside ? bid - nbh : bid) * kRedEPB;
  const T* P = reinterpret_cast<const T*>(Pp);
  if (!vside)
    block_sum_parts<kRedNT, kRedEPB, T>(P, parts0, kr, kr, e0, Pred, red);
  else
    block_sum_parts<kRedNT, kRedEPB, T>(P + (int64_t)parts0 * kr, parts1, kr, kr, e0, Pred + kr, red);
}

int admm_reduce_blocks(int k, int r) { return 2 * (int)(((int64_t)k * r + kRedEPB - 1) / kRedEPB); }

__global__ __launch_bounds__(kRedNT) void admm_reduce_batch_kernel(const AdmmJob* __restrict__ jobs,
                                                                   const int* __restrict__ red_first, int njobs) {
  __shared__ double red[kRedNT];
  const int j = batch_job(red_first, njobs, blockIdx.x);
  const AdmmJob& J = jobs[j];
  const int64_t kr = (int64_t)J.k * J.r;
  const int nbh = (int)((kr + kRedEPB - 1) / kRedEPB);
  admm_reduce_body<float>(J.Pp, J.parts0, J.parts1, kr, J.Pred, nbh, (int)blockIdx.x - red_first[j], red);
}

// The two r x r solves of one iteration run in one workgroup.  XY: [0] Xt
// (k x r), [1] Yt^T (k x r), FP64, followed by both again in FP32, zero
// padded to KP x RP (k, r rounded up to 16) for the row updates.  first != 0: Yt^T = P_V / phi before the
// Xt solve (Alg. 3 initialisation Yt = V R^T, the partial having been
// formed as R (phi V^T)).
constexpr int kSolveNT = 256;

// ---------------------------------------------------------------------------
// The solves by a direct Cholesky factorisation, every product on the FP64
// MFMA (r <= 64, k <= 128 within the LDS budget).  Per side, with the system
// padded to N = 16 ceil(r / 16) by an identity block, X M = RHS is solved as
// M X^T = RHS^T:
//   (a) all waves: M = S^T S + pen I (wave w: block row w);
//   (b) wave 0: M = L L^T (wave_chol_lower: 16-column panels in registers,
//       MFMA trailing updates, inverses V_b of the diagonal blocks); waves
//       1-3 meanwhile form the 16-row strips of RHS = At S + P (pass 0) or
//       At^T S + P (pass 1) into E;
//   (c) each wave, on its strips (one 16-row block of X, as X^T tiles in
//       registers):
//         W_b = V_b (RHS^T_b - sum_{a<b} L[b][a] W_a),        b ascending,
//         X^T_b = V_b^T (W_b - sum_{a>b} L[a][b]^T X^T_a),    b descending.
// A 16x16x4 FP64 MFMA leaves item i of lane (c, g) at row g + 4 i, column c
// of its tile, which is where the next product takes its right operand for
// K step i, so a strip stays in registers through both substitutions; L and
// V come from LDS.
// ---------------------------------------------------------------------------
constexpr int kCholMaxK = 128;

struct CholLayout {
  int NB, N, ld, kp, KB16;
  size_t s_off, e_off, m_off, v_off, w_off, total;  // in doubles
};
__host__ __device__ inline CholLayout chol_layout(int k, int r) {
  CholLayout L;
  L.NB = (r + 15) / 16;
  L.N = 16 * L.NB;
  L.ld = L.N + 2;
  L.KB16 = (k + 15) / 16;
  L.kp = 16 * L.KB16;
  L.s_off = 0;
  L.e_off = L.s_off + (size_t)L.kp * L.ld;
  L.m_off = L.e_off + (size_t)L.kp * L.ld;
  L.v_off = L.m_off + (size_t)L.N * L.ld;
  L.w_off = L.v_off + (size_t)L.NB * 272;
  L.total = L.w_off + 128;
  return L;
}

size_t admm_solve_lds_bytes(int k, int r) { return chol_layout(k, r).total * sizeof(double); }

// K loop over the kp rows of S (LDS, row stride ld) in chunks of 16 rows;
// the next chunk's operands are loaded (row clamped into S) before this
// chunk's products, so their LDS latency overlaps the MFMA work.  For K step
// s (rows 4 s + g of lane (c, g)) f(s, sv, sx) gets sv[b] = S[4 s + g][16 b + c]
// (b < NB) and sx = fx(4 s + g).
template <int NB, typename FX, typename F>
__device__ __forceinline__ void s_chunks(const double* S, int ld, int kp, int c, int g, FX fx, F f) {
  constexpr int KS = kCholMaxK / 4;
  double cur[4][NB + 1], nxt[4][NB + 1];
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
#pragma unroll
    for (int b = 0; b < NB; ++b) cur[s4][b] = S[(4 * s4 + g) * ld + 16 * b + c];
    cur[s4][NB] = fx(4 * s4 + g);
  }
#pragma unroll
  for (int ch = 0; ch < KS / 4; ++ch) {
    if (16 * ch < kp) {
      if (ch + 1 < KS / 4) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int row = min(16 * (ch + 1) + 4 * s4 + g, kp - 1);
#pragma unroll
          for (int b = 0; b < NB; ++b) nxt[s4][b] = S[row * ld + 16 * b + c];
          nxt[s4][NB] = fx(row);
        }
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) f(4 * ch + s4, cur[s4], cur[s4][NB]);
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int b = 0; b <= NB; ++b) cur[s4][b] = nxt[s4][b];
    }
  }
}

// Waits (every lane of the calling wave) until *ready has reached target
// (modulo 2^32), then acquires at agent scope, so that what the signalling
// workgroups stored before their release is visible to the wave's loads.
// The wait is bounded (about two seconds of the constant 100 MHz clock):
// past that, *wait_fail is incremented and the wave goes on.
__device__ __forceinline__ void wait_ready(const unsigned* ready, unsigned target, int* wait_fail) {
  const uint64_t t0 = wall_clock64();
  bool late = false;
  while ((int)(__hip_atomic_load(ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
    if (wall_clock64() - t0 > 200000000ull) {
      late = true;
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  if (late && (threadIdx.x & 63) == 0) atomicAdd(wait_fail, 1);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// One side of the iteration: PASS 0 solves for Xt (S = Yt^T, At), PASS 1
// for Yt^T (S = Xt, At^T).  Starts after a barrier, ends with one.  With
// ready != nullptr the reduced partials P are produced by other workgroups
// of the same launch: the waves that read P (the right-hand sides) first
// wait for *ready to reach target.
template <int NB, int PASS>
__device__ __forceinline__ void chol_side(const double* __restrict__ At, const double* __restrict__ P, int k, int r,
                                          double pen, double* __restrict__ out, float* __restrict__ outf,
                                          int* flags, const CholLayout& Ly, double* sm,
                                          const unsigned* ready = nullptr, unsigned target = 0,
                                          int* wait_fail = nullptr) {
  constexpr int KS = kCholMaxK / 4;
  constexpr int N = 16 * NB;
  const int ld = Ly.ld, kp = Ly.kp, KB16 = Ly.KB16;
  double* S = sm + Ly.s_off;
  double* E = sm + Ly.e_off;
  double* Mb = sm + Ly.m_off;
  double* V = sm + Ly.v_off;
  double* W = sm + Ly.w_off;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  // (a) block row w of M = S^T S + pen I_r (identity on the padding)
  if (w < NB) {
    doublex4 am[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) am[b] = doublex4{0.0, 0.0, 0.0, 0.0};
    s_chunks<NB>(S, ld, kp, c, g, [&](int kk) { return S[kk * ld + 16 * w + c]; },
                 [&](int, const double* sv, double sx) {
#pragma unroll
                   for (int b = 0; b < NB; ++b) am[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(sx, sv[b], am[b], 0, 0, 0);
                 });
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * w + g + 4 * i, col = 16 * b + c;
        Mb[row * ld + col] = am[b][i] + (row == col ? (row < r ? pen : 1.0) : 0.0);
      }
  }
  __syncthreads();
  if (w == 0) {
    // (b) the factor; pivots below 1e-300 max diag(M) are floored
    double dg = lane < r ? Mb[lane * ld + lane] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dg = fmax(dg, __shfl_xor(dg, o));
    wave_chol_lower<double, NB>(Mb, ld, r, V, W, 1e-300 * dg, flags);
  } else {
    // (b) strips of RHS into E (kp x ld, row xr = 16 rb + c): the lane's At
    // and P values are loaded up front, then RHS^T tiles = S^T At^T (+ P^T)
    if (ready) wait_ready(ready, target, wait_fail);
    for (int rb = w - 1; rb < KB16; rb += 3) {
      const int xr = 16 * rb + c;
      double at[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int kk = 4 * s + g;
        at[s] = (xr < k && kk < k) ? (PASS == 0 ? At[xr * k + kk] : At[kk * k + xr]) : 0.0;
      }
      double pv[NB][4];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pr = 16 * b + g + 4 * i;
          pv[b][i] = (xr < k && pr < r) ? P[xr * r + pr] : 0.0;
        }
      doublex4 acc[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = doublex4{0.0, 0.0, 0.0, 0.0};
      s_chunks<NB>(S, ld, kp, c, g, [](int) { return 0.0; }, [&](int s, const double* sv, double) {
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(sv[b], at[s], acc[b], 0, 0, 0);
      });
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) E[xr * ld + 16 * b + g + 4 * i] = acc[b][i] + pv[b][i];
    }
  }
  __syncthreads();
  // (c) substitutions; strip rb belongs to wave 3 - (rb % 4)
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int rb = 4 * q + 3 - w;
    if (rb < KB16) {
      const int xr = 16 * rb + c;
      doublex4 z[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) z[b][i] = E[xr * ld + 16 * b + g + 4 * i];
      // The LDS operands of block b + 1 (b - 1 going back) are loaded before
      // block b's products, and sched_barrier keeps that order, so their
      // latency overlaps the dependent MFMA chain.  ol[a][s]: -L entries of
      // the tiles that meet block b, ov[s]: V_b (transposed going back).
      double ol[2][NB][4], ov[2][4];
      auto load_fwd = [&](int b, double (&l)[NB][4], double (&v)[4]) {
#pragma unroll
        for (int a = 0; a < NB; ++a)
          if (a < b)
#pragma unroll
            for (int s = 0; s < 4; ++s) l[a][s] = -Mb[(16 * b + c) * ld + 16 * a + 4 * s + g];
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = V[b * 272 + c * 17 + 4 * s + g];
      };
      auto load_bwd = [&](int b, double (&l)[NB][4], double (&v)[4]) {
#pragma unroll
        for (int a = 0; a < NB; ++a)
          if (a > b)
#pragma unroll
            for (int s = 0; s < 4; ++s) l[a][s] = -Mb[(16 * a + 4 * s + g) * ld + 16 * b + c];
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = V[b * 272 + (4 * s + g) * 17 + c];
      };
      load_fwd(0, ol[0], ov[0]);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b + 1 < NB)
          load_fwd(b + 1, ol[(b + 1) & 1], ov[(b + 1) & 1]);
        else
          load_bwd(NB - 1, ol[(b + 1) & 1], ov[(b + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        doublex4 t = z[b];
#pragma unroll
        for (int a = 0; a < b; ++a)
#pragma unroll
          for (int s = 0; s < 4; ++s)
            t = __builtin_amdgcn_mfma_f64_16x16x4f64(ol[b & 1][a][s], z[a][s], t, 0, 0, 0);
        doublex4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s)
          y = __builtin_amdgcn_mfma_f64_16x16x4f64(ov[b & 1][s], t[s], y, 0, 0, 0);
        z[b] = y;
        __builtin_amdgcn_sched_barrier(0);
      }
      // back: buffer (NB + u) & 1 holds block NB - 1 - u
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = NB - 1 - u, cur = (NB + u) & 1;
        if (b > 0) load_bwd(b - 1, ol[cur ^ 1], ov[cur ^ 1]);
        __builtin_amdgcn_sched_barrier(0);
        doublex4 t = z[b];
#pragma unroll
        for (int a = 0; a < NB; ++a)
          if (a > b)
#pragma unroll
            for (int s = 0; s < 4; ++s)
              t = __builtin_amdgcn_mfma_f64_16x16x4f64(ol[cur][a][s], z[a][s], t, 0, 0, 0);
        doublex4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s)
          x = __builtin_amdgcn_mfma_f64_16x16x4f64(ov[cur][s], t[s], x, 0, 0, 0);
        z[b] = x;
        __builtin_amdgcn_sched_barrier(0);
      }
      // X[xr][16 b + g + 4 i] = item i of tile b: back into this wave's rows
      // of E (and, for pass 0, into S for the other side; no wave reads S in
      // this phase); then the strip's rows of out (k x r) and outf (kp x N),
      // one contiguous range each, in coalesced stores
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int col = 16 * b + g + 4 * i;
          E[xr * ld + col] = z[b][i];
          if (PASS == 0) S[xr * ld + col] = z[b][i];
        }
      const int r0 = 16 * rb;
      const int nrow = min(16, k - r0);
      for (int row = 0; row < nrow; ++row)
        if (lane < r) out[(r0 + row) * r + lane] = E[(r0 + row) * ld + lane];
      for (int e4 = lane; e4 < 4 * N; e4 += 64) {
        const int row = e4 / (N / 4), col = 4 * e4 - row * N;
        const double* src = E + (r0 + row) * ld + col;
        *reinterpret_cast<float4*>(outf + (r0 + row) * N + col) =
            make_float4((float)src[0], (float)src[1], (float)src[2], (float)src[3]);
      }
    }
  }
  __syncthreads();
}

template <int NB>
__device__ __forceinline__ void admm_solve_chol_nb(const double* __restrict__ Pred, const double* __restrict__ At,
                                                   int k, int r, double lam, double phi, int first,
                                                   double* __restrict__ XY, int* flags, double* sm) {
  constexpr int NT = kSolveNT;
  constexpr int N = 16 * NB;
  const CholLayout Ly = chol_layout(k, r);
  double* S = sm + Ly.s_off;
  const int64_t kr = (int64_t)k * r;
  // S = Yt^T (k x r, zero padded to kp x N); eight loads in flight per
  // thread before their stores (one load-store pair at a time waits on the
  // L2 latency per element row)
  for (int e0 = threadIdx.x; e0 < Ly.kp * N; e0 += NT * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + NT * u, i = e / N, j = e - i * N;
      v[u] = (e < Ly.kp * N && i < k && j < r) ? (first ? Pred[kr + i * r + j] / phi : XY[kr + i * r + j]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + NT * u, i = e / N, j = e - i * N;
      if (e < Ly.kp * N) S[i * Ly.ld + j] = v[u];
    }
  }
  __syncthreads();
  // the zero-padded FP32 copies (kp x N per side) after XY feed the row updates
  float* XYf = reinterpret_cast<float*>(XY + 2 * kr);
  chol_side<NB, 0>(At, Pred, k, r, lam, XY, XYf, flags, Ly, sm);
  chol_side<NB, 1>(At, Pred + kr, k, r, phi, XY + kr, XYf + Ly.kp * N, flags, Ly, sm);
}

__device__ __forceinline__ void admm_solve_chol_body(const double* __restrict__ Pred, const double* __restrict__ At,
                                                     int k, int r, double lam, double phi, int first,
                                                     double* __restrict__ XY, int* flags, double* sm) {
  switch ((r + 15) / 16) {
    case 1: admm_solve_chol_nb<1>(Pred, At, k, r, lam, phi, first, XY, flags, sm); break;
    case 2: admm_solve_chol_nb<2>(Pred, At, k, r, lam, phi, first, XY, flags, sm); break;
    case 3: admm_solve_chol_nb<3>(Pred, At, k, r, lam, phi, first, XY, flags, sm); break;
    default: admm_solve_chol_nb<4>(Pred, At, k, r, lam, phi, first, XY, flags, sm); break;
  }
}

// One workgroup per job.
__global__ __launch_bounds__(kSolveNT) void admm_solve_batch_kernel(const AdmmJob* __restrict__ jobs) {
  extern __shared__ double sm[];
  const AdmmJob& J = jobs[blockIdx.x];
  admm_solve_chol_body(J.Pred, J.At, J.k, J.r, J.lam, J.phi, J.first, J.XY, J.flags, sm);
}

// ---------------------------------------------------------------------------
// Split schedule for one request.  In Alg. 3 the U-side row update of an
// iteration reads Xt but not Yt^T, and only the next iteration's Xt solve
// needs its partial P_U; likewise the V side with Yt^T and the next Yt^T
// solve.  So the U-side row update shares a launch with the Yt^T solve, and
// the V-side row update one with the next iteration's Xt solve: block 0 is
// the solve of one side, the other blocks are the row update.  Each value is
// computed by the same code as in the serving batch, where both solves share
// a workgroup.
// ---------------------------------------------------------------------------
template <int NB, int PASS>
__device__ __forceinline__ void admm_solve_side_nb(const AdmmHalf& a, double* sm) {
  constexpr int NT = kSolveNT;
  constexpr int N = 16 * NB;
  const int k = a.k, r = a.r;
  const CholLayout Ly = chol_layout(k, r);
  double* S = sm + Ly.s_off;
  const int64_t kr = (int64_t)k * r;
  const double* XY = a.XY;
  // S = Yt^T for pass 0 (P_V / phi on the first iteration, Alg. 3's
  // initialisation), Xt for pass 1; zero padded to kp x N
  // (sixteen loads in flight per thread before their stores: one memory
  // round trip for k, r <= 64, where S is 64 x 64 after padding)
  for (int e0 = threadIdx.x; e0 < Ly.kp * N; e0 += NT * 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + NT * u, i = e / N, j = e - i * N;
      v[u] = 0.0;
      if (e < Ly.kp * N && i < k && j < r)
        v[u] = PASS == 1 ? XY[i * r + j] : (a.first ? a.Pred[kr + i * r + j] / a.phi : XY[kr + i * r + j]);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + NT * u, i = e / N, j = e - i * N;
      if (e < Ly.kp * N) S[i * Ly.ld + j] = v[u];
    }
  }
  __syncthreads();
  float* XYf = reinterpret_cast<float*>(a.XY + 2 * kr);
  const unsigned* ready = a.nred > 0 ? a.ready : nullptr;
  if constexpr (PASS == 0)
    chol_side<NB, 0>(a.At, a.Pred, k, r, a.lam, a.XY, XYf, a.flags, Ly, sm, ready, a.ready_target, a.wait_fail);
  else
    chol_side<NB, 1>(a.At, a.Pred + kr, k, r, a.phi, a.XY + kr, XYf + Ly.kp * N, a.flags, Ly, sm, ready,
                     a.ready_target, a.wait_fail);
}

template <int PASS>
__device__ __forceinline__ void admm_solve_side(const AdmmHalf& a, double* sm) {
  switch ((a.r + 15) / 16) {
    case 1: admm_solve_side_nb<1, PASS>(a, sm); break;
    case 2: admm_solve_side_nb<2, PASS>(a, sm); break;
    case 3: admm_solve_side_nb<3, PASS>(a, sm); break;
    default: admm_solve_side_nb<4, PASS>(a, sm); break;
  }
}

static_assert(kSolveNT == kRedNT, "the half kernel's reduction blocks run the reduction with its block size");

// Reduction workgroup b of a fused launch: the element groups
// [b G, b G + G) of the solve's side (P_V for pass 1, P_U for pass 0), each
// element summed exactly as by admm_reduce_body.
template <int G, typename T>
__device__ __forceinline__ void fused_reduce(const AdmmHalf& a, int b, double* sm) {
  const int64_t kr = (int64_t)a.k * a.r;
  const bool vside = a.pass == 1;
  const T* P = reinterpret_cast<const T*>(a.Pp) + (vside ? (int64_t)a.parts0 * kr : 0);
  block_sum_parts_groups<kRedNT, kRedEPB, G, T>(P, vside ? a.parts1 : a.parts0, kr, kr,
                                                (int64_t)b * G * kRedEPB, a.Pred + (vside ? kr : 0), sm);
}

template <typename T, int CH>
__global__ __launch_bounds__(kSolveNT) void admm_half_kernel(AdmmHalf a) {
  extern __shared__ double sm[];
  if (a.solve && blockIdx.x == 0) {
    if (a.pass == 0)
      admm_solve_side<0>(a, sm);
    else
      admm_solve_side<1>(a, sm);
    return;
  }
  int b = (int)blockIdx.x - (a.solve ? 1 : 0);
  if (b < a.nred) {
    // the fixed-order sums of the solve's partials (P_V for the Yt^T
    // solve, P_U for Xt), rgroups groups of 16 elements, then a release and
    // one count on *ready
    switch (a.rgroups) {
      case 1: fused_reduce<1, T>(a, b, sm); break;
      case 2: fused_reduce<2, T>(a, b, sm); break;
      default: fused_reduce<4, T>(a, b, sm); break;
    }
    if (threadIdx.x == 0) __hip_atomic_fetch_add(a.ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  b -= a.nred;
  admm_uv_body<T, CH>(a.s0, a.s1, a.parts0, a.side ? a.parts0 + b : b, a.XY, a.k, a.r, a.xi, a.mode, a.Pp,
                      a.rpb0, a.rpb1, reinterpret_cast<char*>(sm));
}

template <typename T>
hipError_t launch_admm_half(const AdmmHalf& a, hipStream_t st) {
  const int k = a.k, r = a.r;
  if (r > 64 || k > kCholMaxK || a.parts0 < 1 || a.parts1 < 1 || (!a.solve && !a.uv)) return hipErrorInvalidValue;
  // fused reductions: exactly the solve side's blocks, a counter and a
  // failure word, and only beside a solve (which is what waits for them)
  const int nbh_ = (int)(((int64_t)k * r + kRedEPB - 1) / kRedEPB);
  const bool pow2 = a.rgroups == 1 || a.rgroups == 2 || a.rgroups == 4;
  if (a.nred != 0 && (!pow2 || a.nred != (nbh_ + a.rgroups - 1) / a.rgroups || !a.solve || a.first || !a.ready ||
                      !a.wait_fail))
    return hipErrorInvalidValue;
  const size_t red_lds = a.nred ? (size_t)a.rgroups * kRedNT * sizeof(double) : 0;
  const size_t solve_lds = a.solve ? chol_layout(k, r).total * sizeof(double) : 0;
  if (solve_lds > 160 * 1024) return hipErrorInvalidValue;
  const int nuv = a.side ? a.parts1 : a.parts0;
  const int KP = (k + 15) / 16 * 16, RP = (r + 15) / 16 * 16;
  auto lds = [&](int ch) { return ((size_t)KP * (RP + 1) + (size_t)ch * (KP + 1) + (size_t)ch * (RP + 1)) * sizeof(T); };
  const dim3 grid((a.uv ? nuv : 0) + (a.solve ? 1 : 0) + a.nred);
  if (lds(64) <= 160 * 1024) {
    const size_t sm = std::max({solve_lds, lds(64), red_lds});
    hipFuncSetAttribute((const void*)admm_half_kernel<T, 64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    hipLaunchKernelGGL((admm_half_kernel<T, 64>), grid, dim3(kSolveNT), sm, st, a);
  } else {
    const size_t sm = std::max({solve_lds, lds(32), red_lds});
    hipFuncSetAttribute((const void*)admm_half_kernel<T, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    hipLaunchKernelGGL((admm_half_kernel<T, 32>), grid, dim3(kSolveNT), sm, st, a);
  }
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_admm_half<float>(const AdmmHalf&, hipStream_t);
template hipError_t launch_admm_half<double>(const AdmmHalf&, hipStream_t);

int admm_fused_reduce_groups(int k, int r, int nuv) {
  // compute units of the device current at the first call (queried once,
  // thread-safe; 256 if the query fails); only the group count depends on it
  static const int cus = [] {
    int dev = 0;
    hipDeviceProp_t p;
    return hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess &&
                   p.multiProcessorCount > 0
               ? p.multiProcessorCount
               : 256;
  }();
  const int nbh = (int)(((int64_t)k * r + kRedEPB - 1) / kRedEPB);
  int g = 1;
  while (g < 4 && 1 + (nbh + g - 1) / g + nuv > cus) g *= 2;
  if (1 + (nbh + g - 1) / g + nuv > cus) return 0;
  // a sum workgroup that loads more than about 640 partial rows (groups x
  // parts) finishes after the solve needs its sums: separate launches then
  // cost less (20000 x 5000: 2 x 157 and 4 x 157 faster fused, 8 x 157
  // slower; 40000 x 30000 with 235 parts: 8 groups slower)
  if (g * nuv > 640) return 0;
  return g;
}

// The fixed-order sums of one side's partials (side 0: P_U, 1: P_V, 2: both).
template <typename T>
__global__ __launch_bounds__(kRedNT) void admm_reduce_side_kernel(const double* __restrict__ Pp, int parts0,
                                                                  int parts1, int64_t kr, double* __restrict__ Pred,
                                                                  int nbh, int b0) {
  __shared__ double red[kRedNT];
  admm_reduce_body<T>(Pp, parts0, parts1, kr, Pred, nbh, b0 + (int)blockIdx.x, red);
}

template <typename T>
hipError_t launch_admm_reduce(const double* Pp, int parts0, int parts1, int k, int r, int side, double* Pred,
                              hipStream_t st) {
  if (side < 0 || side > 2) return hipErrorInvalidValue;
  const int64_t kr = (int64_t)k * r;
  const int nbh = (int)((kr + kRedEPB - 1) / kRedEPB);
  hipLaunchKernelGGL(admm_reduce_side_kernel<T>, dim3(side == 2 ? 2 * nbh : nbh), dim3(kRedNT), 0, st, Pp, parts0,
                     parts1, kr, Pred, nbh, side == 1 ? nbh : 0);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_admm_reduce<float>(const double*, int, int, int, int, int, double*, hipStream_t);
template hipError_t launch_admm_reduce<double>(const double*, int, int, int, int, int, double*, hipStream_t);

// ---------------------------------------------------------------------------
// Batched ADMM step (serving): for every job, the fixed-order partial sums,
// the two r x r solves and the mode-1 row update, as three launches over all
// jobs.  Each job runs exactly the per-request code above, so its result does
// not depend on which other jobs share the launch.
// ---------------------------------------------------------------------------
void admm_job_prepare(AdmmJob& J) {
  J.rpb0 = (J.s0.rows + J.parts0 - 1) / J.parts0;
  J.rpb1 = (J.s1.rows + J.parts1 - 1) / J.parts1;
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

// ---------------------------------------------------------------------------
// The same batched step with fixed grids, for replay as a captured graph:
// the counts come from the descriptor's header in device memory (written by
// the copy that precedes the launches), so the launch configuration does not
// depend on the batch.  The workgroups of the reduce and row-update launches
// take the step's block indices one at a time from a counter in the header
// and run, for index b, exactly the code of block b of
// launch_admm_step_batch, so the results do not depend on which workgroup
// takes which index.
// ---------------------------------------------------------------------------
// Next block index of a work loop for the whole workgroup.
__device__ __forceinline__ int take_index(int* counter, int* slot) {
  __syncthreads();   // every wave is done with the previous index (and its LDS)
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
  __syncthreads();
  return *slot;
}

__global__ __launch_bounds__(kRedNT) void admm_reduce_fixed_kernel(char* __restrict__ desc, size_t off_jobs,
                                                                   size_t off_red) {
  __shared__ double red[kRedNT];
  __shared__ int bslot;
  BatchHeader* hp = reinterpret_cast<BatchHeader*>(desc);
  const int njobs = hp->njobs, total = hp->red_total;
  const AdmmJob* jobs = reinterpret_cast<const AdmmJob*>(desc + off_jobs);
  const int* red_first = reinterpret_cast<const int*>(desc + off_red);
  for (;;) {
    const int b = take_index(&hp->red_next, &bslot);
    if (b >= total) break;
    const int j = batch_job(red_first, njobs, b);
    const AdmmJob& J = jobs[j];
    const int64_t kr = (int64_t)J.k * J.r;
    const int nbh = (int)((kr + kRedEPB - 1) / kRedEPB);
    admm_reduce_body<float>(J.Pp, J.parts0, J.parts1, kr, J.Pred, nbh, b - red_first[j], red);
  }
}

__global__ __launch_bounds__(kSolveNT) void admm_solve_fixed_kernel(const char* __restrict__ desc, size_t off_jobs) {
  extern __shared__ double sm[];
  const int njobs = reinterpret_cast<const BatchHeader*>(desc)->njobs;
  const AdmmJob* jobs = reinterpret_cast<const AdmmJob*>(desc + off_jobs);
  for (int j = blockIdx.x; j < njobs; j += gridDim.x) {
    __syncthreads();
    const AdmmJob& J = jobs[j];
    admm_solve_chol_body(J.Pred, J.At, J.k, J.r, J.lam, J.phi, J.first, J.XY, J.flags, sm);
  }
}

template <typename T, int CH>
__global__ __launch_bounds__(256) void admm_uv_fixed_kernel(char* __restrict__ desc, size_t off_jobs,
                                                            size_t off_uv) {
  extern __shared__ char smraw[];
  __shared__ int bslot;
  BatchHeader* hp = reinterpret_cast<BatchHeader*>(desc);
  const int njobs = hp->njobs, total = hp->uv_total;
  const AdmmJob* jobs = reinterpret_cast<const AdmmJob*>(desc + off_jobs);
  const int* uv_first = reinterpret_cast<const int*>(desc + off_uv);
  for (;;) {
    const int b = take_index(&hp->uv_next, &bslot);
    if (b >= total) break;
    const int j = batch_job(uv_first, njobs, b);
    const AdmmJob& J = jobs[j];
    admm_uv_body<T, CH>(J.s0, J.s1, J.parts0, b - uv_first[j], J.XY, J.k, J.r, J.xi, J.last ? 2 : 1, J.Pp, J.rpb0,
                        J.rpb1, smraw);
  }
}

constexpr size_t kUvFixedLdsMax = 128 * 1024;

size_t admm_batch_uv_lds(int max_k, int max_r) {
  const int KP = (max_k + 15) / 16 * 16, RP = (max_r + 15) / 16 * 16;
  return ((size_t)KP * (RP + 1) + 64 * (size_t)(KP + 1) + 64 * (size_t)(RP + 1)) * sizeof(float);
}

hipError_t admm_step_fixed_init() {
  hipError_t e = hipFuncSetAttribute((const void*)admm_solve_fixed_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  // the row update needs at most admm_batch_uv_lds(128, 64) = 83 KB (its
  // static LDS is not part of this limit)
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)admm_uv_fixed_kernel<float, 64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kUvFixedLdsMax);
  return e;
}

hipError_t launch_admm_step_fixed(char* desc_dev, size_t off_jobs, size_t off_uv, size_t off_red,
                                  int grid_solve, int grid_red, int grid_uv, size_t uv_lds, size_t solve_lds,
                                  hipStream_t st) {
  if (solve_lds > 160 * 1024 || uv_lds > kUvFixedLdsMax || grid_solve < 1 || grid_red < 1 || grid_uv < 1)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(admm_reduce_fixed_kernel, dim3(grid_red), dim3(kRedNT), 0, st, desc_dev, off_jobs, off_red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(admm_solve_fixed_kernel, dim3(grid_solve), dim3(kSolveNT), solve_lds, st, desc_dev, off_jobs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((admm_uv_fixed_kernel<float, 64>), dim3(grid_uv), dim3(256), uv_lds, st, desc_dev, off_jobs,
                     off_uv);
  CNMF_LAUNCH_CHECK();
}

size_t admm_job_solve_lds(const AdmmJob& J) {
  return chol_layout(J.k, J.r).total * sizeof(double);
}

}  // namespace cnmf
