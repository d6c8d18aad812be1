// Reduced-precision range-finder passes (BF16, FP8 E4M3 with per-tile
// power-of-two scales) on the gfx950 MFMAs with FP32 accumulation: BF16 on
// the 16x16x32 instruction, FP8 on the scaled 16x16x128 one (twice the FP8
// rate of the 16x16x32 FP8 instruction), the tile's scale given to the
// instruction as its block exponent.
//
// Layout: the FP32 input A is converted once into a copy of A and a copy of
// A^T in the pass precision, so every pass is the same "rows of a matrix
// times a tall operand" kernel reading contiguous rows.  Both copies are
// padded to whole 128 x 128 tiles (rows and leading dimension), and the
// padding holds zeros, so a pass reads whole 128-byte row chunks without
// bounds checks.  The operand is stored transposed (kk x cols, zero beyond
// the columns), so each lane's K-consecutive operand values are one or two
// 16-byte loads.
// FP8: each 128 x 128 tile of A has its own scale s = 2^e, the smallest
// power of two with max|tile| / s <= 448; the same tile grid serves A^T.
#include "cnmf_internal.hpp"
#include "lds_dma.hpp"

namespace cnmf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint8_t to_fp8(float x) {
  // round to nearest even, OCP E4M3 (gfx950 conversion)
  int packed = __builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false);
  return (uint8_t)(packed & 0xff);
}

// Exponent e of the FP8 tile scale 2^e for a tile maximum tmax > 0: with
// tmax = f 2^t, f in [0.5, 1), tmax / 2^e <= 448 = 0.875 2^9 holds for
// e = t - 9 when f <= 0.875 and needs e = t - 8 otherwise.  Clamped to
// [-126, 127] so that the scale is a normal FP32 number (a tile whose
// maximum is below 448 2^-126 loses its smallest values to FP8 underflow).
__device__ __forceinline__ int fp8_tile_exponent(float tmax) {
  int t = 0;
  const float f = frexpf(tmax, &t);
  const int e = f <= 0.875f ? t - 9 : t - 8;
  return min(127, max(-126, e));
}

// ---------------------------------------------------------------------------
// FP32 A -> reduced-precision copies of A (ld ldo) and A^T (ld ldt), one
// workgroup per 128 x 128 tile of A.  The grid covers the padded matrix:
// ceil(m / 128) 128 rows of A (ld ldo >= 128 ceil(n / 128)) and
// ceil(n / 128) 128 rows of A^T (ld ldt >= 128 ceil(m / 128)); entries
// outside m x n are written as zeros.  BF16: round to nearest even.  FP8:
// s = 2^e as above (1 for an all-zero tile), element = e4m3(a * 2^-e), s
// stored in scale[ti * ntj + tj].
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
      if (A16) A16[(int64_t)i * ldo + j] = q;
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
    const int e = tmax > 0.0f ? fp8_tile_exponent(tmax) : 0;
    const float sc = ldexpf(1.0f, e), inv = ldexpf(1.0f, -e);
    if (threadIdx.x == 0) scale[ti * ntj + tj] = sc;
#pragma unroll
    for (int s = 0; s < TS / 2; ++s) {
      const int ii = ty + 2 * s, i = i0 + ii, j = j0 + tx;
      const uint8_t q = to_fp8(v[s] * inv);
      t8[ii][tx] = q;
      if (A8) A8[(int64_t)i * ldo + j] = q;
    }
  }
  __syncthreads();
  if (At16) {
#pragma unroll 8
    for (int s = 0; s < TS / 2; ++s) {
      const int jj = ty + 2 * s, j = j0 + jj, i = i0 + tx;
      At16[(int64_t)j * ldt + i] = t16[tx][jj];
    }
  }
  if (At8) {
#pragma unroll 8
    for (int s = 0; s < TS / 2; ++s) {
      const int jj = ty + 2 * s, j = j0 + jj, i = i0 + tx;
      At8[(int64_t)j * ldt + i] = t8[tx][jj];
    }
  }
}

hipError_t launch_convert_lowp(const float* A, int64_t lda, int m, int n, __hip_bfloat16* A16, __hip_bfloat16* At16,
                               uint8_t* A8, uint8_t* At8, int64_t ldo, int64_t ldt, float* scale, hipStream_t st) {
  const int ntj = (n + kFp8Tile - 1) / kFp8Tile, nti = (m + kFp8Tile - 1) / kFp8Tile;
  if (m < 1 || n < 1 || ldo < (int64_t)ntj * kFp8Tile || ldt < (int64_t)nti * kFp8Tile) return hipErrorInvalidValue;
  hipLaunchKernelGGL(convert_lowp_kernel, dim3(ntj, nti), dim3(256), 0, st, A, lda, m, n, A16, At16, A8, At8, ldo,
                     ldt, scale, ntj);
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Y (partials [split][rows][kk], FP32) = M (rows x cols, element size ES,
// ldm elements per row) times the operand given transposed as Xt (kk x cols,
// ld ldx), kk <= 256.
// Requirements (checked by the launcher where it can): M has m_rows >=
// 128 ceil(rows / 128) rows, ldm and ldx hold whole 128-byte chunks and at
// least 128 ceil(cols / 128) columns, the padding of M and of Xt is zero,
// M, Xt 16-byte aligned.
//
// Workgroup: 512 threads, 256 rows of M and all kk output columns, one
// workgroup per CU.  Wave w owns rows [128 (w / 4), + 128) and output column
// blocks [(w % 4) KBW, + KBW).  M and Xt are read in chunks of 128 bytes per
// row (KC = 128 / ES columns).  Every chunk of M (32 KB) and of Xt (kk x 128
// bytes) goes straight from global memory into LDS (global_load_lds, 16
// bytes per lane): M through a three-stage ring, issued two chunks ahead,
// Xt through a two-stage ring, issued one chunk ahead (it comes from L2).
// Nothing passes through registers on the way, so the only waits for the
// loads are the explicit ones at the top of each step.  Within a row the
// 16-byte segment j of a chunk sits in slot j ^ h(row), h(row) = (row & 7)
// ^ ((row >> 3) & 1), so the fragment reads of 8 consecutive rows use 8
// distinct slots, and those of 16 consecutive rows 16 distinct 16-byte bank
// groups of a 256-byte bank line.  Lane group g covers
// bytes [32 g, 32 g + 32) of a chunk row, the same mapping on both operands
// (the MFMA's K order is the same for its two inputs, so any common
// assignment sums the full dot product).
// FP8: a chunk lies in one 128-column scale tile and a wave's rows in one
// 128-row tile, so the tile's exponent is the instruction's block scale for
// A (the operand's scale is 1) and products are accumulated in FP32
// directly (the instruction adds C at FP32 precision).
// ---------------------------------------------------------------------------
typedef uint4 v16;

template <int ES>
struct Lowp;
template <>
struct Lowp<2> {  // BF16: two 16x16x32 steps per 32-byte lane run
  static __device__ __forceinline__ void mma(const v16 (&a)[2], const v16 (&b)[2], int, floatx4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[0]), __builtin_bit_cast(bf16x8, b[0]),
                                                c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[1]), __builtin_bit_cast(bf16x8, b[1]),
                                                c, 0, 0, 0);
  }
};
template <>
struct Lowp<1> {  // FP8 E4M3: one scaled 16x16x128 step per 32-byte lane run
  static __device__ __forceinline__ intx8 cat(const v16 (&v)[2]) {
    return intx8{(int)v[0].x, (int)v[0].y, (int)v[0].z, (int)v[0].w,
                 (int)v[1].x, (int)v[1].y, (int)v[1].z, (int)v[1].w};
  }
  static __device__ __forceinline__ void mma(const v16 (&a)[2], const v16 (&b)[2], int e8a, floatx4& c) {
    // formats 0 / 0: E4M3 for both inputs; block exponents e8a for A, 127 (2^0) for the operand
    c = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(cat(a), cat(b), c, 0, 0, 0, e8a, 0, 127);
  }
};

constexpr int kLowpRows = 256;      // rows of M per workgroup
constexpr int kLowpThreads = 512;
constexpr int kLowpStagesA = 3;     // LDS ring depths (chunks)
constexpr int kLowpStagesB = 2;

template <int ES, int KB>
__global__ __launch_bounds__(512, 1) void gemm_lowp_kernel(const uint8_t* M, int64_t ldmb, int64_t m_rows, int rows,
                                                           int cols, const uint8_t* X, int64_t ldxb,
                                                           float* __restrict__ P, int cols_per_split,
                                                           const float* __restrict__ scale, int scale_ld,
                                                           int scale_transposed) {
  constexpr int KC = 128 / ES;        // chunk columns (128 bytes per row)
  constexpr int KK = 16 * KB;
  constexpr int KBW = (KB + 3) / 4;   // column blocks per wave
  constexpr int SA = kLowpRows * 128; // bytes per ring stage
  constexpr int SB = KK * 128;
  constexpr int BI = KK / 8;          // 1 KB DMA instructions per operand chunk
  static_assert(kFp8Tile % KC == 0 && kFp8Tile == 128, "chunks and wave rows must stay in one scale tile");
  static_assert(kLowpStagesA * SA + kLowpStagesB * SB <= 160 * 1024, "LDS");
  __shared__ __attribute__((aligned(16))) uint8_t As[kLowpStagesA * SA];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[kLowpStagesB * SB];

  const int tid = threadIdx.x;
  const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, g = lane >> 4;
  const int half = w >> 2, jb0 = (w & 3) * KBW;
  const int split = blockIdx.y;
  const int kbeg = split * cols_per_split;
  const int kend = min(cols, kbeg + cols_per_split);
  const int nchunk = kend > kbeg ? (kend - kbeg + KC - 1) / KC : 0;
  const int row_blk = blockIdx.x * kLowpRows;

  floatx4 acc[8][KBW];
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int jj = 0; jj < KBW; ++jj) acc[rb][jj] = floatx4{0, 0, 0, 0};

  if (nchunk > 0) {
    // DMA lane mapping: an instruction moves 8 rows of 128 bytes (1 KB);
    // lane l writes LDS bytes [16 l, 16 l + 16) of it, i.e. row 8 b + l / 8
    // (b the instruction's row group), slot l % 8, which holds segment
    // (l % 8) ^ h(row) = (l % 8) ^ (l / 8) ^ (b & 1)
    const int drow = lane >> 3, dseg = (lane & 7) ^ drow;
    // M: wave w moves rows [32 w, 32 w + 32) of a chunk, four instructions;
    // rows past the allocation (the last tile) re-read its last row, whose
    // results are not stored
    const uint8_t* asrc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = min<int64_t>(row_blk + 32 * w + 8 * i + drow, m_rows - 1);
      asrc[i] = M + r * ldmb + (int64_t)kbeg * ES + (dseg ^ (i & 1)) * 16;  // row group 4 w + i
    }
    // Xt: instruction i (rows 8 i .. 8 i + 7) is issued by wave i % 8
    const uint8_t* bsrc = X + (int64_t)(8 * w + drow) * ldxb + (int64_t)kbeg * ES + (dseg ^ (w & 1)) * 16;
    // the destination slot is always one that every wave has finished
    // reading; past the last chunk the source is clamped to it and the slot
    // is never read
    const uint32_t as0 = lds_addr(As), bs0 = lds_addr(Bs);
    auto issue_a = [&](int chunk) {
      const int64_t off = (int64_t)min(chunk, nchunk - 1) * 128;
      const uint32_t dst = as0 + (chunk % kLowpStagesA) * SA + 32 * w * 128;
#pragma unroll
      for (int i = 0; i < 4; ++i) dma16(asrc[i] + off, __builtin_amdgcn_readfirstlane(dst + 8 * i * 128));
    };
    auto issue_b = [&](int chunk) {
      const int64_t off = (int64_t)min(chunk, nchunk - 1) * 128;
      const uint32_t dst = bs0 + (chunk % kLowpStagesB) * SB + 8 * w * 128;
#pragma unroll
      for (int i = 0; i < (BI + 7) / 8; ++i)
        if (w + 8 * i < BI)
          dma16(bsrc + (int64_t)(64 * i) * ldxb + off, __builtin_amdgcn_readfirstlane(dst + 64 * i * 128));
    };
    const int tr = (row_blk + 128 * half) / kFp8Tile;
    // the loop for a wave owning NB column blocks (KBW, KB % KBW or none:
    // a wave without columns still moves its share of every chunk)
    auto run = [&](auto nb_const) {
      constexpr int NB = decltype(nb_const)::value;
      constexpr int NBA = NB > 0 ? NB : 1;
      // order of issue: A(0), B(0), A(1) before the loop; step ch issues
      // B(ch + 1), then A(ch + 2) (asm statements keep their order).  So at
      // the top of step ch all but the last four DMAs of this wave (A(ch + 1))
      // have landed, A(ch) and B(ch) among them; the barrier then covers
      // every wave's share.
      issue_a(0);
      issue_b(0);
      issue_a(1);
      for (int ch = 0; ch < nchunk; ++ch) {
        // (a plain barrier: the workgroup fence of __syncthreads would wait
        // for every DMA in flight)
        asm volatile("s_waitcnt vmcnt(4)\n\ts_barrier" ::: "memory");
        issue_b(ch + 1);
        issue_a(ch + 2);
        if (NB > 0) {
          int e8a = 127;
          if (ES == 1) {
            const int tc = (kbeg + ch * KC) / kFp8Tile;
            const float sc =
                scale_transposed ? scale[(int64_t)tc * scale_ld + tr] : scale[(int64_t)tr * scale_ld + tc];
            e8a = (int)((__float_as_uint(sc) >> 23) & 0xffu);
          }
          // fragment reads: lane (lr, g) reads segments 2g and 2g + 1 of
          // its row (h(16 i + lr) == (lr & 7) ^ (lr >> 3))
          const int hl = (lr & 7) ^ (lr >> 3);
          const uint32_t o0 = ((2 * g) ^ hl) << 4, o1 = ((2 * g + 1) ^ hl) << 4;
          const uint8_t* bst = Bs + (ch % kLowpStagesB) * SB + (jb0 * 16 + lr) * 128;
          v16 bf[NBA][2];
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) {
            bf[jj][0] = *reinterpret_cast<const v16*>(bst + jj * 2048 + o0);
            bf[jj][1] = *reinterpret_cast<const v16*>(bst + jj * 2048 + o1);
          }
          const uint8_t* ast = As + (ch % kLowpStagesA) * SA + (128 * half + lr) * 128;
#pragma unroll
          for (int rb = 0; rb < 8; ++rb) {
            v16 af[2];
            af[0] = *reinterpret_cast<const v16*>(ast + rb * 2048 + o0);
            af[1] = *reinterpret_cast<const v16*>(ast + rb * 2048 + o1);
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) Lowp<ES>::mma(af, bf[jj], e8a, acc[rb][jj]);
          }
        }
      }
    };
    const int nb = min(KBW, max(0, KB - jb0));
    if (nb == KBW)
      run(std::integral_constant<int, KBW>());
    else if (KB % KBW != 0 && nb == KB % KBW)
      run(std::integral_constant<int, (KB % KBW)>());
    else
      run(std::integral_constant<int, 0>());
    // drain the clamped DMAs issued past the last chunk before the wave ends
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  float* out = P + (int64_t)split * rows * KK;
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = row_blk + 128 * half + rb * 16 + 4 * g + i;
      if (row < rows) {
#pragma unroll
        for (int jj = 0; jj < KBW; ++jj)
          if (jb0 + jj < KB) out[(int64_t)row * KK + (jb0 + jj) * 16 + lr] = acc[rb][jj][i];
      }
    }
}

int choose_splits_lowp(int rows, int cols, int kk, int es) {
  // One workgroup per CU: the launch runs in ceil(W / CUs) rounds for W =
  // tiles * splits workgroups, each reading 1 / W of M and writing one FP32
  // partial per row.  Choose the split count (at most 16, at least 256
  // columns per split) minimising rounds * (bytes per workgroup, partials
  // included).
  constexpr int kCUs = 256;
  const int64_t tiles = (rows + kLowpRows - 1) / kLowpRows;
  const double mbytes = (double)rows * cols * es, pbytes = (double)rows * kk * 4;
  int best = 1;
  double best_t = 0.0;
  for (int s = 1; s <= 16 && (s == 1 || cols / s >= 256); ++s) {
    const int64_t wgs = tiles * s;
    const double t = (double)((wgs + kCUs - 1) / kCUs) * (mbytes + s * pbytes) / (double)wgs;
    if (s == 1 || t < best_t * 0.999) {
      best = s;
      best_t = t;
    }
  }
  return best;
}

template <int ES, int KB>
static hipError_t gemm_lowp_kb(const void* M, int64_t ldm, int64_t m_rows, int rows, int cols, const void* Xt, int64_t ldx,
                               float* P, int splits, const float* scale, int scale_ld, int scale_t, hipStream_t st) {
  int per = (cols + splits - 1) / splits;
  per = (per + 127) / 128 * 128;
  dim3 grid((rows + kLowpRows - 1) / kLowpRows, splits);
  hipLaunchKernelGGL((gemm_lowp_kernel<ES, KB>), grid, dim3(kLowpThreads), 0, st, (const uint8_t*)M, ldm * ES, m_rows,
                     rows, cols, (const uint8_t*)Xt, ldx * ES, P, per, scale, scale_ld, scale_t);
  CNMF_LAUNCH_CHECK();
}

template <int ES>
static hipError_t gemm_lowp_es(const void* M, int64_t ldm, int64_t m_rows, int rows, int cols, const void* Xt, int64_t ldx, int kk,
                               float* P, int splits, const float* scale, int scale_ld, int scale_t, hipStream_t st) {
#define CNMF_LOWP_CASE(KB) \
  case 16 * KB: return gemm_lowp_kb<ES, KB>(M, ldm, m_rows, rows, cols, Xt, ldx, P, splits, scale, scale_ld, scale_t, st);
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

hipError_t launch_gemm_lowp(int es, const void* M, int64_t ldm, int64_t m_rows, int rows, int cols, const void* Xt,
                            int64_t ldx, int kk, float* P, int splits, const float* scale, int scale_ld, int scale_t,
                            hipStream_t st) {
  if (es != 1 && es != 2) return hipErrorInvalidValue;
  const int64_t cpad = ((int64_t)cols + 127) / 128 * 128;
  if (rows < 1 || cols < 1 || splits < 1 || m_rows < lowp_pad(rows) ||
      ldm < cpad || ldx < cpad || (ldm * es) % 128 != 0 || (ldx * es) % 16 != 0 || (uintptr_t)M % 16 != 0 ||
      (uintptr_t)Xt % 16 != 0)
    return hipErrorInvalidValue;
  if (es == 2) return gemm_lowp_es<2>(M, ldm, m_rows, rows, cols, Xt, ldx, kk, P, splits, nullptr, 0, 0, st);
  if (!scale) return hipErrorInvalidValue;
  return gemm_lowp_es<1>(M, ldm, m_rows, rows, cols, Xt, ldx, kk, P, splits, scale, scale_ld, scale_t, st);
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
