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
// Y (partials [split][rows][kk], FP32) = M (rows x cols, element size ES,
// ld ldm) times the operand given transposed as Xt (kk x cols, ld ldx),
// kk <= 256.
// Workgroup: 16 RB rows of M (RB row blocks of 16: 128 rows for BF16, 64
// for FP8, whose per-chunk accumulators double the registers) and all kk
// output columns;
// wave w owns output column blocks [w KBW, (w + 1) KBW).  Per chunk of KC
// columns of M (128 bytes per row): the 64 x KC tile of M is staged in LDS
// (double buffered) and read by all four waves; each wave loads its own
// operand rows for the chunk straight into registers (prefetched one chunk
// ahead).  Operand traffic from L2 per byte of M is kk / (16 RB), LDS reads
// per byte of M staged are 4.  Lane group g covers K [g KC/4, (g + 1) KC/4) of the chunk, eight
// K values per MFMA step, the same mapping on both operands.
// FP8: a chunk is one 128-column scale tile and the workgroup's rows lie in
// one 128-row tile; the chunk's product is accumulated separately and added
// to the FP32 accumulator times the tile scale.
// ---------------------------------------------------------------------------
template <int ES>
struct Lowp;
template <>
struct Lowp<2> {  // BF16
  typedef bf16x8 opnd;
  static __device__ __forceinline__ void mma(const opnd& a, const opnd& b, floatx4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  // eight K-consecutive elements s of a lane's 32-byte run
  static __device__ __forceinline__ opnd part(const uint4 (&v)[2], int s) { return __builtin_bit_cast(opnd, v[s]); }
};
template <>
struct Lowp<1> {  // FP8 E4M3
  typedef long opnd;
  static __device__ __forceinline__ void mma(const opnd& a, const opnd& b, floatx4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ opnd part(const uint4 (&v)[2], int s) {
    const uint4 q = v[s >> 1];
    const uint2 h = (s & 1) ? uint2{q.z, q.w} : uint2{q.x, q.y};
    return __builtin_bit_cast(opnd, h);
  }
};

typedef uint4 v16;

// 32 bytes at p (16-byte aligned when vec), bytes at or beyond `lim` (a
// byte count from p) read as zero.
__device__ __forceinline__ void load32(const uint8_t* p, int lim, bool vec, v16 (&d)[2]) {
  if (vec && lim >= 32) {
    d[0] = *reinterpret_cast<const v16*>(p);
    d[1] = *reinterpret_cast<const v16*>(p + 16);
    return;
  }
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    uint32_t wd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t val = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int byte = 16 * v + 4 * q + b;
        if (byte < lim) val |= (uint32_t)p[byte] << (8 * b);
      }
      wd[q] = val;
    }
    d[v] = v16{wd[0], wd[1], wd[2], wd[3]};
  }
}

template <int ES, int KB, int RB>
__global__ __launch_bounds__(256, 2) void gemm_lowp_kernel(const void* __restrict__ Mv, int64_t ldm, int rows,
                                                           int cols, const void* __restrict__ Xv, int64_t ldx,
                                                           float* __restrict__ P, int cols_per_split,
                                                           const float* __restrict__ scale, int scale_ld,
                                                           int scale_transposed) {
  typedef typename Lowp<ES>::opnd opnd;
  constexpr bool SCALED = ES == 1;
  constexpr int KC = 128 / ES;      // chunk columns (128 bytes per row)
  constexpr int STEPS = KC / 32;    // MFMA steps per chunk
  constexpr int KK = 16 * KB;
  constexpr int KBW = (KB + 3) / 4;  // column blocks per wave
  constexpr int LDA = 128 + 16;      // LDS bytes per staged row
  static_assert(kFp8Tile % KC == 0 && kFp8Tile % (16 * RB) == 0, "chunks and rows must stay in one scale tile");
  __shared__ __attribute__((aligned(16))) uint8_t As[2][16 * RB * LDA];
  const uint8_t* __restrict__ M = (const uint8_t*)Mv;
  const uint8_t* __restrict__ X = (const uint8_t*)Xv;

  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, g = lane >> 4;
  const int split = blockIdx.y;
  const int kbeg = split * cols_per_split;
  const int kend = min(cols, kbeg + cols_per_split);
  const int nchunk = kend > kbeg ? (kend - kbeg + KC - 1) / KC : 0;
  const int row_blk = blockIdx.x * (16 * RB);
  const int jb0 = w * KBW;
  const bool vec_a = ((uintptr_t)M % 16 == 0) && ((ldm * ES) % 16 == 0);
  const bool vec_x = ((uintptr_t)X % 16 == 0) && ((ldx * ES) % 16 == 0);

  floatx4 acc[RB][KBW];
  floatx4 cacc[SCALED ? RB : 1][SCALED ? KBW : 1];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int jj = 0; jj < KBW; ++jj) acc[rb][jj] = floatx4{0, 0, 0, 0};

  // staging of the M tile: thread t moves 32 bytes of rows t / 4 + 64 q
  constexpr int SR = RB / 4;
  const int srow = tid >> 2, sseg = tid & 3;
  v16 ast[SR][2];
  auto load_a = [&](int chunk) {
    const int c0 = kbeg + chunk * KC + sseg * (KC / 4);
#pragma unroll
    for (int q = 0; q < SR; ++q) {
      const int rr = row_blk + srow + 64 * q;
      const bool ok = rr < rows;
      const int lim = ok ? (kend - c0) * ES : 0;
      load32(M + ((int64_t)(ok ? rr : 0) * ldm + c0) * ES, lim, vec_a, ast[q]);
    }
  };
  auto store_a = [&](int buf) {
#pragma unroll
    for (int q = 0; q < SR; ++q) {
      uint8_t* p = &As[buf][(srow + 64 * q) * LDA + sseg * 32];
      *reinterpret_cast<v16*>(p) = ast[q][0];
      *reinterpret_cast<v16*>(p + 16) = ast[q][1];
    }
  };
  // this wave's operand fragments: lane (lr, g) of column block jj holds
  // Xt[(jb0 + jj) 16 + lr][chunk cols g KC/4 .. + KC/4)
  v16 bcur[KBW][2], bnxt[KBW][2];
  auto load_b = [&](int chunk, v16 (&d)[KBW][2]) {
    const int c0 = kbeg + chunk * KC + g * (KC / 4);
    const int lim = (kend - c0) * ES;
#pragma unroll
    for (int jj = 0; jj < KBW; ++jj) {
      if (jb0 + jj < KB) {
        const uint8_t* p = X + ((int64_t)((jb0 + jj) * 16 + lr) * ldx + c0) * ES;
        load32(p, lim, vec_x, d[jj]);
      } else {
        d[jj][0] = v16{0, 0, 0, 0};
        d[jj][1] = v16{0, 0, 0, 0};
      }
    }
  };

  if (nchunk > 0) {
    load_a(0);
    load_b(0, bcur);
    store_a(0);
  }
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunk;
    if (more) {
      load_a(ch + 1);
      load_b(ch + 1, bnxt);
    }
    if (SCALED) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int jj = 0; jj < KBW; ++jj) cacc[SCALED ? rb : 0][SCALED ? jj : 0] = floatx4{0, 0, 0, 0};
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      v16 af[2];
      const uint8_t* ap = &As[buf][(rb * 16 + lr) * LDA + g * 32];
      af[0] = *reinterpret_cast<const v16*>(ap);
      af[1] = *reinterpret_cast<const v16*>(ap + 16);
#pragma unroll
      for (int s = 0; s < STEPS; ++s) {
        const opnd a = Lowp<ES>::part(af, s);
#pragma unroll
        for (int jj = 0; jj < KBW; ++jj) {
          if (jb0 + jj < KB) {
            const opnd b = Lowp<ES>::part(bcur[jj], s);
            if (SCALED)
              Lowp<ES>::mma(a, b, cacc[SCALED ? rb : 0][SCALED ? jj : 0]);
            else
              Lowp<ES>::mma(a, b, acc[rb][jj]);
          }
        }
      }
    }
    if (SCALED) {
      const int tr = row_blk / kFp8Tile, tc = (kbeg + ch * KC) / kFp8Tile;
      const float sc = scale_transposed ? scale[(int64_t)tc * scale_ld + tr] : scale[(int64_t)tr * scale_ld + tc];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int jj = 0; jj < KBW; ++jj)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            acc[rb][jj][i] = fmaf(sc, cacc[SCALED ? rb : 0][SCALED ? jj : 0][i], acc[rb][jj][i]);
    }
    if (more) {
      store_a(buf ^ 1);
#pragma unroll
      for (int jj = 0; jj < KBW; ++jj) {
        bcur[jj][0] = bnxt[jj][0];
        bcur[jj][1] = bnxt[jj][1];
      }
    }
    __syncthreads();
  }
  float* out = P + (int64_t)split * rows * KK;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = row_blk + rb * 16 + 4 * g + i;
      if (row < rows) {
#pragma unroll
        for (int jj = 0; jj < KBW; ++jj)
          if (jb0 + jj < KB) out[(int64_t)row * KK + (jb0 + jj) * 16 + lr] = acc[rb][jj][i];
      }
    }
}

int choose_splits_lowp(int rows, int cols, int kk, int es) {
  // about 3000 workgroups (six rounds of two per CU) for latency hiding, while
  // the FP32 partials stay below a tenth of the bytes of M read
  const int tile_rows = es == 2 ? 128 : 64;
  const int tiles = (rows + tile_rows - 1) / tile_rows;
  int s = (3072 + tiles - 1) / tiles;
  const int cap_bytes = (int)std::max<int64_t>(1, (int64_t)cols * es / (10LL * kk * 4));
  s = std::min(s, cap_bytes);
  s = std::min(s, std::max(1, cols / 256));
  return std::max(1, std::min(s, 64));
}

template <int ES, int KB>
static hipError_t gemm_lowp_kb(const void* M, int64_t ldm, int rows, int cols, const void* Xt, int64_t ldx,
                               float* P, int splits, const float* scale, int scale_ld, int scale_t, hipStream_t st) {
  constexpr int RB = ES == 2 ? 8 : 4;
  int per = (cols + splits - 1) / splits;
  per = (per + 127) / 128 * 128;
  dim3 grid((rows + 16 * RB - 1) / (16 * RB), splits);
  hipLaunchKernelGGL((gemm_lowp_kernel<ES, KB, RB>), grid, dim3(256), 0, st, M, ldm, rows, cols, Xt, ldx, P, per,
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
// Column maxima of |Q[:, c0 + c]| for c < k <= 128, rows in blocks of 256:
// thread (c, rs) scans every other row of its block, then one exact atomic
// max per column and block on the bit patterns (nonnegative doubles order
// like their bits, so the result does not depend on the order).
__global__ __launch_bounds__(256) void colmax_kernel(const double* __restrict__ Q, int rows, int ldq, int c0, int k,
                                                     unsigned long long* __restrict__ cmax) {
  __shared__ double red[256];
  const int c = threadIdx.x & 127, rs = threadIdx.x >> 7;
  const int i0 = blockIdx.x * 256, i1 = min(rows, i0 + 256);
  double mx = 0.0;
  if (c < k)
    for (int i = i0 + rs; i < i1; i += 2) mx = fmax(mx, fabs(Q[(int64_t)i * ldq + c0 + c]));
  red[threadIdx.x] = mx;
  __syncthreads();
  if (rs == 0 && c < k) {
    mx = fmax(red[threadIdx.x], red[threadIdx.x + 128]);
    atomicMax(&cmax[c], (unsigned long long)__double_as_longlong(mx));
  }
}

// colscale[scol0 + c]: the largest power of two s with max * s <= 256
// (headroom below 448); 256 / max = f 2^e with f in [0.5, 1) gives 2^(e - 1).
__global__ void colscale_kernel(const unsigned long long* __restrict__ cmax, int k, float* __restrict__ colscale,
                                int scol0) {
  const int c = threadIdx.x;
  if (c >= k) return;
  const double mxv = __longlong_as_double((long long)cmax[c]);
  float s = 1.0f;
  if (mxv > 0.0) {
    int e = 0;
    frexp(256.0 / mxv, &e);
    s = (float)ldexp(1.0, e - 1);
  }
  colscale[scol0 + c] = s;
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
                             float* colscale, int scol0, unsigned long long* cmax, hipStream_t st) {
  if (k > 128) return hipErrorInvalidValue;
  if (es == 1) {
    hipError_t e = launch_fill(cmax, (size_t)k * sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colmax_kernel, dim3((rows + 255) / 256), dim3(256), 0, st, Q, rows, ldq, c0, k, cmax);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colscale_kernel, dim3(1), dim3(128), 0, st, cmax, k, colscale, scol0);
    e = hipGetLastError();
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
