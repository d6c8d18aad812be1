// Reduced-precision range-finder passes (BF16, FP8 E4M3 with per-tile
// scales) on the gfx950 16x16x32 MFMAs with FP32 accumulation.
//
// Layout: the FP32 input A is converted once into a copy of A and a copy of
// A^T in the pass precision, so every pass is the same "rows of a matrix
// times a tall operand" kernel reading contiguous rows.  The operand is
// stored transposed (kk x cols), so each lane's eight K-consecutive operand
// values are one 16-byte (BF16) or 8-byte (FP8) LDS read.
// FP8: each 128 x 128 tile of A has its own scale s = max|tile| / 448; the
// same tile grid serves A^T.  A pass accumulates each 128-column chunk
// separately and adds s_tile times the chunk product to the accumulator.
#include "cnmf_internal.hpp"

namespace cnmf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint8_t to_fp8(float x) {
  // round to nearest even, OCP E4M3 (gfx950 conversion)
  int packed = __builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false);
  return (uint8_t)(packed & 0xff);
}

// ---------------------------------------------------------------------------
// FP32 A -> reduced-precision copies of A (ld ldo) and A^T (ld ldt), one
// workgroup per 128 x 128 tile of A.  BF16: round to nearest even.  FP8:
// s = max|tile| / 448 (1 for an all-zero tile), element = e4m3(a * (1/s)),
// s stored in scale[ti * ntj + tj].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void convert_lowp_kernel(const float* __restrict__ A, int64_t lda, int m, int n,
                                                           __hip_bfloat16* __restrict__ A16,
                                                           __hip_bfloat16* __restrict__ At16,
                                                           uint8_t* __restrict__ A8, uint8_t* __restrict__ At8,
                                                           int64_t ldo, int64_t ldt, float* __restrict__ scale,
                                                           int ntj) {
  constexpr int TS = kFp8Tile;
  __shared__ __hip_bfloat16 t16[TS][TS + 2];
  __shared__ uint8_t t8[TS][TS + 4];
  __shared__ float red[256];
  const int ti = blockIdx.y, tj = blockIdx.x;
  const int i0 = ti * TS, j0 = tj * TS;
  const int tx = threadIdx.x & 127, ty = threadIdx.x >> 7;  // two rows per sweep
  const bool want16 = A16 || At16, want8 = A8 || At8;
  float v[TS / 2];
  float mx = 0.0f;
#pragma unroll
  for (int s = 0; s < TS / 2; ++s) {
    const int i = i0 + ty + 2 * s, j = j0 + tx;
    v[s] = (i < m && j < n) ? A[(int64_t)i * lda + j] : 0.0f;
    mx = fmaxf(mx, fabsf(v[s]));
  }
  if (want16) {
#pragma unroll
    for (int s = 0; s < TS / 2; ++s) {
      const int ii = ty + 2 * s, i = i0 + ii, j = j0 + tx;
      const __hip_bfloat16 q = __float2bfloat16(v[s]);
      t16[ii][tx] = q;
      if (A16 && i < m && j < n) A16[(int64_t)i * ldo + j] = q;
    }
  }
  if (want8) {
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    const float tmax = red[0];
    const float sc = tmax > 0.0f ? tmax / 448.0f : 1.0f;
    const float inv = 1.0f / sc;
    if (threadIdx.x == 0) scale[ti * ntj + tj] = sc;
#pragma unroll
    for (int s = 0; s < TS / 2; ++s) {
      const int ii = ty + 2 * s, i = i0 + ii, j = j0 + tx;
      const uint8_t q = to_fp8(v[s] * inv);
      t8[ii][tx] = q;
      if (A8 && i < m && j < n) A8[(int64_t)i * ldo + j] = q;
    }
  }
  __syncthreads();
  if (At16) {
#pragma unroll 8
    for (int s = 0; s < TS / 2; ++s) {
      const int jj = ty + 2 * s, j = j0 + jj, i = i0 + tx;
      if (j < n && i < m) At16[(int64_t)j * ldt + i] = t16[tx][jj];
    }
  }
  if (At8) {
#pragma unroll 8
    for (int s = 0; s < TS / 2; ++s) {
      const int jj = ty + 2 * s, j = j0 + jj, i = i0 + tx;
      if (j < n && i < m) At8[(int64_t)j * ldt + i] = t8[tx][jj];
    }
  }
}

hipError_t launch_convert_lowp(const float* A, int64_t lda, int m, int n, __hip_bfloat16* A16, __hip_bfloat16* At16,
                               uint8_t* A8, uint8_t* At8, int64_t ldo, int64_t ldt, float* scale, hipStream_t st) {
  const int ntj = (n + kFp8Tile - 1) / kFp8Tile, nti = (m + kFp8Tile - 1) / kFp8Tile;
  hipLaunchKernelGGL(convert_lowp_kernel, dim3(ntj, nti), dim3(256), 0, st, A, lda, m, n, A16, At16, A8, At8, ldo,
                     ldt, scale, ntj);
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Y (partials [split][rows][kk], FP32) = M (rows x cols, TA, ld ldm) times
// the operand given transposed as Xt (kk x cols, TA, ld ldx), kk <= 256.
// Workgroup: 4 waves x RB row blocks of 16; chunks of KC columns (128, or
// 64 for kk > 128 to bound LDS); lane group g takes columns
// [g KC/4, (g + 1) KC/4) of the chunk, 8 per MFMA step.
// FP8: each chunk lies in one 128-column scale tile and each wave's rows in
// one 128-row tile; the chunk's product is accumulated separately and added
// to the FP32 accumulator times the tile scale.
// ---------------------------------------------------------------------------
template <int ES>
struct Lowp;
template <>
struct Lowp<2> {  // BF16
  typedef __hip_bfloat16 T;
  typedef bf16x8 opnd;
  static __device__ __forceinline__ void mma(const opnd& a, const opnd& b, floatx4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  // eight K-consecutive elements s of a lane's column run (16 bytes each)
  template <int NV>
  static __device__ __forceinline__ opnd part(const uint4 (&v)[NV], int s) {
    return __builtin_bit_cast(opnd, v[s]);
  }
};
template <>
struct Lowp<1> {  // FP8 E4M3
  typedef uint8_t T;
  typedef long opnd;
  static __device__ __forceinline__ void mma(const opnd& a, const opnd& b, floatx4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
  }
  template <int NV>
  static __device__ __forceinline__ opnd part(const uint4 (&v)[NV], int s) {
    const uint4 q = v[s >> 1];
    const uint2 h = (s & 1) ? uint2{q.z, q.w} : uint2{q.x, q.y};
    return __builtin_bit_cast(opnd, h);
  }
};

template <int ES, int KB, int RB, int KC>
__global__ __launch_bounds__(256, 2) void gemm_lowp_kernel(const void* __restrict__ Mv, int64_t ldm, int rows,
                                                           int cols, const void* __restrict__ Xv, int64_t ldx,
                                                           float* __restrict__ P, int cols_per_split,
                                                           const float* __restrict__ scale, int scale_ld,
                                                           int scale_transposed) {
  typedef typename Lowp<ES>::opnd opnd;
  typedef uint4 v16;
  constexpr bool SCALED = ES == 1;
  constexpr int KK = 16 * KB;
  constexpr int CPG = KC / 4;           // columns per lane group and chunk
  constexpr int STEPS = CPG / 8;        // MFMA steps per chunk
  constexpr int LDX = KC * ES + 16;     // bytes per operand row in LDS (padded)
  constexpr int NV = CPG * ES / 16;     // 16-byte A vectors per lane and row block
  constexpr int VPR = KC * ES / 16;     // 16-byte vectors per operand row of a chunk
  constexpr int TOTV = KK * VPR;        // operand vectors per chunk
  constexpr int XV = (TOTV + 255) / 256;
  static_assert(16 * RB <= kFp8Tile && kFp8Tile % (16 * RB) == 0, "wave rows must stay in one scale tile");
  static_assert(kFp8Tile % KC == 0 && NV >= 1, "chunks must stay in one scale tile");
  __shared__ __attribute__((aligned(16))) uint8_t Xs[2][KK * LDX];
  const uint8_t* __restrict__ M = (const uint8_t*)Mv;
  const uint8_t* __restrict__ X = (const uint8_t*)Xv;

  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, g = lane >> 4;
  const int split = blockIdx.y;
  const int kbeg = split * cols_per_split;
  const int kend = min(cols, kbeg + cols_per_split);
  const int nchunk = kend > kbeg ? (kend - kbeg + KC - 1) / KC : 0;
  const int row_base = blockIdx.x * (64 * RB) + w * 16 * RB;
  const bool vec_a = ((uintptr_t)M % 16 == 0) && ((ldm * ES) % 16 == 0);
  const bool vec_x = ((uintptr_t)X % 16 == 0) && ((ldx * ES) % 16 == 0);

  floatx4 acc[RB][KB];
  floatx4 cacc[SCALED ? RB : 1][SCALED ? KB : 1];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int jb = 0; jb < KB; ++jb) acc[rb][jb] = floatx4{0, 0, 0, 0};

  v16 a_cur[RB][NV], a_nxt[RB][NV];
  v16 xr[XV];

  auto load_a = [&](int chunk, v16(&dst)[RB][NV]) {
    const int c0 = kbeg + chunk * KC + CPG * g;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int row = row_base + rb * 16 + lr;
      const bool rok = row < rows;
      const uint8_t* p = M + ((int64_t)(rok ? row : 0) * ldm + c0) * ES;
      if (vec_a && rok && c0 + CPG <= kend) {
#pragma unroll
        for (int v = 0; v < NV; ++v) dst[rb][v] = *reinterpret_cast<const v16*>(p + 16 * v);
      } else {
        // ragged tail: assemble the bytes in range into dwords, zeros beyond
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          uint32_t wd[4];
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            uint32_t val = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const int byte = 16 * v + 4 * d + b;
              if (rok && c0 + byte / ES < kend) val |= (uint32_t)p[byte] << (8 * b);
            }
            wd[d] = val;
          }
          dst[rb][v] = v16{wd[0], wd[1], wd[2], wd[3]};
        }
      }
    }
  };
  // operand chunk: the KK rows of Xt over columns [k0, k0 + KC)
  auto load_x = [&](int chunk) {
    const int k0 = kbeg + chunk * KC;
#pragma unroll
    for (int e = 0; e < XV; ++e) {
      const int idx = e * 256 + tid;
      if (TOTV % 256 == 0 || idx < TOTV) {
        const int c = idx / VPR, v = idx - c * VPR;
        const int col = k0 + v * (16 / ES);
        const uint8_t* p = X + ((int64_t)c * ldx + col) * ES;
        if (vec_x && col + 16 / ES <= kend) {
          xr[e] = *reinterpret_cast<const v16*>(p);
        } else {
          uint32_t wd[4];
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            uint32_t val = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b)
              if (col + (4 * d + b) / ES < kend) val |= (uint32_t)p[4 * d + b] << (8 * b);
            wd[d] = val;
          }
          xr[e] = v16{wd[0], wd[1], wd[2], wd[3]};
        }
      }
    }
  };
  auto store_x = [&](int buf) {
#pragma unroll
    for (int e = 0; e < XV; ++e) {
      const int idx = e * 256 + tid;
      if (TOTV % 256 == 0 || idx < TOTV) {
        const int c = idx / VPR, v = idx - c * VPR;
        *reinterpret_cast<v16*>(&Xs[buf][c * LDX + 16 * v]) = xr[e];
      }
    }
  };

  if (nchunk > 0) {
    load_a(0, a_cur);
    load_x(0);
    store_x(0);
  }
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunk;
    if (more) {
      load_a(ch + 1, a_nxt);
      load_x(ch + 1);
    }
    if (SCALED) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int jb = 0; jb < KB; ++jb) cacc[SCALED ? rb : 0][SCALED ? jb : 0] = floatx4{0, 0, 0, 0};
    }
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
#pragma unroll
      for (int jb = 0; jb < KB; ++jb) {
        const opnd b = *reinterpret_cast<const opnd*>(&Xs[buf][(jb * 16 + lr) * LDX + (CPG * g + 8 * s) * ES]);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const opnd a = Lowp<ES>::template part<NV>(a_cur[rb], s);
          if (SCALED)
            Lowp<ES>::mma(a, b, cacc[SCALED ? rb : 0][SCALED ? jb : 0]);
          else
            Lowp<ES>::mma(a, b, acc[rb][jb]);
        }
      }
    }
    if (SCALED) {
      const int tr = row_base / kFp8Tile, tc = (kbeg + ch * KC) / kFp8Tile;
      const float sc = scale_transposed ? scale[(int64_t)tc * scale_ld + tr] : scale[(int64_t)tr * scale_ld + tc];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int jb = 0; jb < KB; ++jb)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            acc[rb][jb][i] = fmaf(sc, cacc[SCALED ? rb : 0][SCALED ? jb : 0][i], acc[rb][jb][i]);
    }
    if (more) store_x(buf ^ 1);
    __syncthreads();
    if (more) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < NV; ++v) a_cur[rb][v] = a_nxt[rb][v];
    }
  }
  float* out = P + (int64_t)split * rows * KK;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = row_base + rb * 16 + 4 * g + i;
      if (row < rows) {
#pragma unroll
        for (int jb = 0; jb < KB; ++jb) out[(int64_t)row * KK + jb * 16 + lr] = acc[rb][jb][i];
      }
    }
}

int choose_splits_lowp(int rows, int cols, int kk) {
  // tiles of 128 rows; same occupancy heuristic as the FP32 passes
  int tiles = (rows + 127) / 128;
  int slots = 512;
  int best = 1;
  double best_eff = -1.0;
  int max_s = std::max(1, std::min(64, cols / 1024));
  for (int s = 1; s <= max_s; ++s) {
    long long wgs = (long long)tiles * s;
    long long rounds = (wgs + slots - 1) / slots;
    double eff = (double)wgs / (double)(rounds * slots) - 0.004 * s;
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = s;
    }
    if (wgs >= 4LL * slots) break;
  }
  return best;
}

template <int ES, int KB>
static hipError_t gemm_lowp_kb(const void* M, int64_t ldm, int rows, int cols, const void* Xt, int64_t ldx,
                               float* P, int splits, const float* scale, int scale_ld, int scale_t, hipStream_t st) {
  constexpr int RB = KB > 8 ? 1 : 2;
  constexpr int KC = KB > 8 ? 64 : 128;
  int per = (cols + splits - 1) / splits;
  per = (per + 127) / 128 * 128;
  dim3 grid((rows + 64 * RB - 1) / (64 * RB), splits);
  hipLaunchKernelGGL((gemm_lowp_kernel<ES, KB, RB, KC>), grid, dim3(256), 0, st, M, ldm, rows, cols, Xt, ldx, P, per,
                     scale, scale_ld, scale_t);
  CNMF_LAUNCH_CHECK();
}

template <int ES>
static hipError_t gemm_lowp_es(const void* M, int64_t ldm, int rows, int cols, const void* Xt, int64_t ldx, int kk,
                               float* P, int splits, const float* scale, int scale_ld, int scale_t, hipStream_t st) {
#define CNMF_LOWP_CASE(KB) \
  case 16 * KB: return gemm_lowp_kb<ES, KB>(M, ldm, rows, cols, Xt, ldx, P, splits, scale, scale_ld, scale_t, st);
  switch (kk) {
    CNMF_LOWP_CASE(1)
    CNMF_LOWP_CASE(2)
    CNMF_LOWP_CASE(3)
    CNMF_LOWP_CASE(4)
    CNMF_LOWP_CASE(5)
    CNMF_LOWP_CASE(6)
    CNMF_LOWP_CASE(7)
    CNMF_LOWP_CASE(8)
    CNMF_LOWP_CASE(9)
    CNMF_LOWP_CASE(10)
    CNMF_LOWP_CASE(11)
    CNMF_LOWP_CASE(12)
    CNMF_LOWP_CASE(13)
    CNMF_LOWP_CASE(14)
    CNMF_LOWP_CASE(15)
    CNMF_LOWP_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef CNMF_LOWP_CASE
}

hipError_t launch_gemm_lowp(int es, const void* M, int64_t ldm, int rows, int cols, const void* Xt, int64_t ldx,
                            int kk, float* P, int splits, const float* scale, int scale_ld, int scale_t,
                            hipStream_t st) {
  if (es == 2) return gemm_lowp_es<2>(M, ldm, rows, cols, Xt, ldx, kk, P, splits, nullptr, 0, 0, st);
  if (es == 1) return gemm_lowp_es<1>(M, ldm, rows, cols, Xt, ldx, kk, P, splits, scale, scale_ld, scale_t, st);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Operands: columns [c0, c0 + k) of Q64 (rows x ldq, FP64) -> rows
// [dr0, dr0 + k) of the transposed operand Xt (kk x rows, ld ldx) in BF16 or
// FP8.  FP8: column c is multiplied by colscale[c] (a power of two chosen
// from the column's max magnitude) before rounding; scaling a column of the
// range-finder operand does not change the orthonormalised result.
// ---------------------------------------------------------------------------
__global__ void colmax_kernel(const double* __restrict__ Q, int rows, int ldq, int c0, int k,
                              float* __restrict__ colscale, int scol0) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double mx = 0.0;
  for (int i = threadIdx.x; i < rows; i += 256) mx = fmax(mx, fabs(Q[(int64_t)i * ldq + c0 + c]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // largest power of two s with max * s <= 256 (headroom below 448):
    // 256 / max = f 2^e with f in [0.5, 1) gives s = 2^(e - 1)
    const double mxv = red[0];
    float s = 1.0f;
    if (mxv > 0.0) {
      int e = 0;
      frexp(256.0 / mxv, &e);
      s = (float)ldexp(1.0, e - 1);
    }
    colscale[scol0 + c] = s;
  }
}

template <int ES>
__global__ void store_lowp_kernel(const double* __restrict__ Q, int rows, int ldq, int c0, int k,
                                  uint8_t* __restrict__ Xt, int64_t ldx, int dr0, const float* __restrict__ colscale,
                                  int scol0) {
  __shared__ double tile[32][33];
  const int i0 = blockIdx.x * 32, cb = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    const int i = i0 + yy, c = cb + tx;
    tile[yy][tx] = (i < rows && c < k) ? Q[(int64_t)i * ldq + c0 + c] : 0.0;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int c = cb + yy, i = i0 + tx;
    if (c < k && i < rows) {
      const double v = tile[tx][yy];
      uint8_t* dst = Xt + ((int64_t)(dr0 + c) * ldx + i) * ES;
      if (ES == 2) {
        *reinterpret_cast<__hip_bfloat16*>(dst) = __float2bfloat16((float)v);
      } else {
        *dst = to_fp8((float)(v * colscale[scol0 + c]));
      }
    }
  }
}

hipError_t launch_store_lowp(int es, const double* Q, int rows, int ldq, int c0, int k, void* Xt, int64_t ldx, int dr0,
                             float* colscale, int scol0, hipStream_t st) {
  if (es == 1) {
    hipLaunchKernelGGL(colmax_kernel, dim3(k), dim3(256), 0, st, Q, rows, ldq, c0, k, colscale, scol0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  dim3 grid((rows + 31) / 32, (k + 31) / 32);
  if (es == 2)
    hipLaunchKernelGGL(store_lowp_kernel<2>, grid, dim3(256), 0, st, Q, rows, ldq, c0, k, (uint8_t*)Xt, ldx, dr0,
                       colscale, scol0);
  else
    hipLaunchKernelGGL(store_lowp_kernel<1>, grid, dim3(256), 0, st, Q, rows, ldq, c0, k, (uint8_t*)Xt, ldx, dr0,
                       colscale, scol0);
  CNMF_LAUNCH_CHECK();
}

// Y[:, c] /= colscale[c] for c < k (Y rows x ld, FP32); undoes the FP8
// operand column scaling where a product is used directly.
__global__ void unscale_cols_kernel(float* __restrict__ Y, int rows, int ld, int k, const float* __restrict__ cs) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)rows * k) return;
  const int i = (int)(idx / k), c = (int)(idx - (int64_t)i * k);
  Y[(int64_t)i * ld + c] /= cs[c];
}

hipError_t launch_unscale_cols(float* Y, int rows, int ld, int k, const float* colscale, hipStream_t st) {
  const int64_t tot = (int64_t)rows * k;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(unscale_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Y, rows, ld, k,
                     colscale);
  CNMF_LAUNCH_CHECK();
}

}  // namespace cnmf
