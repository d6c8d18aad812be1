// Streaming passes over A for the structured random compression (Alg. 1,
// Section 2): Y = A X and W = A^T Z with tall-skinny X, Z (kk <= 128
// columns).  Each pass reads A exactly once; the operand chunk is staged in
// LDS and shared by the four waves of a workgroup; A goes straight from HBM
// into registers in 16-byte loads.  Products run on the 16x16x4 FP32 / FP64
// MFMA.  The reduction dimension can be split over `splits` workgroup
// columns; each slice writes its own partial (no atomics), and the partials
// are summed later in a fixed order, so results are bit-reproducible.
#include "cnmf_internal.hpp"
#include "lds_dma.hpp"

namespace cnmf {

template <typename T>
struct Mfma;
// Operand layout shared by both 16x16x4 MFMAs: lane (r = lane % 16,
// g = lane / 16) supplies A[r][g] and B[g][r].  Result element i of lane
// (c, g) is D[out_row(g, i)][c]: row 4g + i for FP32, but g + 4i for FP64
// (measured on gfx950).
template <>
struct Mfma<float> {
  typedef floatx4 acc_t;
  static __device__ __forceinline__ void mma(float a, float b, floatx4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int i) { return 4 * g + i; }
};
template <>
struct Mfma<double> {
  typedef doublex4 acc_t;
  static __device__ __forceinline__ void mma(double a, double b, doublex4& c) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int i) { return g + 4 * i; }
};

template <typename T, int N>
struct alignas(16) Vec {
  T v[N];
};

// Load `cnt` consecutive elements of one row of A starting at column col
// (cnt elements, all guarded against [.., kend)).  With FULL the whole run
// is in range and 16-byte aligned.
template <typename T, int CNT, bool VEC>
__device__ __forceinline__ void load_run(const T* __restrict__ p, int col, int kend, bool row_ok,
                                         T* out) {
  constexpr int VW = 16 / sizeof(T);
  if (VEC && row_ok && col + CNT <= kend) {
#pragma unroll
    for (int v = 0; v < CNT / VW; ++v) {
      Vec<T, VW> x = *reinterpret_cast<const Vec<T, VW>*>(p + col + v * VW);
#pragma unroll
      for (int e = 0; e < VW; ++e) out[v * VW + e] = x.v[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < CNT; ++e) out[e] = (row_ok && col + e < kend) ? p[col + e] : T(0);
  }
}

// ---------------------------------------------------------------------------
// Y = A X.  Workgroup: 256 threads = 4 waves; wave w owns RB blocks of 16
// rows.  Per K chunk of KC columns, lane (r = lane % 16, g = lane / 16)
// holds columns [g*G, g*G + G) of its rows (a permutation of the MFMA K
// index that both operands share, so the contraction is unchanged).
// ---------------------------------------------------------------------------
// Tile and split of this workgroup (1-D grid of ntiles * nsplits).  The
// hardware hands workgroups to the 8 XCDs round-robin by id, so consecutive
// ids run on different XCDs, each with its own L2.  The ids are renumbered so
// that every XCD takes one contiguous run of (tile, split) pairs, tiles
// fastest: the workgroups that read the same split's slice of the operand
// then run on the same XCD and share it in that L2.  Any numbering computes
// the same tiles; only the cache reuse changes.
__device__ __forceinline__ void xcd_tile(int ntiles, int nsplits, int& tile, int& split) {
  const int nb = ntiles * nsplits, b = blockIdx.x;
  const int q = nb / 8, rem = nb % 8, x = b % 8, slot = b / 8;
  const int lid = x * q + min(x, rem) + slot;
  tile = lid % ntiles;
  split = lid / ntiles;
}

template <typename T, int KB, int RB, bool VEC>
__global__ __launch_bounds__(256, 2) void gemm_n_kernel(const T* __restrict__ A, int64_t lda, int m,
                                                        int n, const T* __restrict__ X,
                                                        T* __restrict__ P, int cols_per_split, int ntiles,
                                                        int nsplits) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int KC = sizeof(T) == 4 ? 64 : 32;
  constexpr int G = KC / 4;
  constexpr int KK = 16 * KB;
  constexpr int LDX = KK + 1;
  constexpr int XPER = KC * KK / 256;  // operand elements staged per thread
  __shared__ T Xs[2][KC * LDX];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int r = lane & 15;
  const int g = lane >> 4;
  int tile, split;
  xcd_tile(ntiles, nsplits, tile, split);
  const int kbeg = split * cols_per_split;
  const int kend = min(n, kbeg + cols_per_split);
  const int nchunk = kend > kbeg ? (kend - kbeg + KC - 1) / KC : 0;
  const int row_base = tile * (64 * RB) + w * 16 * RB;

  const T* arow[RB];
  bool rok[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    int row = row_base + rb * 16 + r;
    rok[rb] = row < m;
    arow[rb] = A + (int64_t)(rok[rb] ? row : 0) * lda;
  }

  acc_t acc[RB][KB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int jb = 0; jb < KB; ++jb) acc[rb][jb] = acc_t{0, 0, 0, 0};

  T a_cur[RB][G], a_nxt[RB][G];
  T xr[XPER];

  auto load_a = [&](int chunk, T (&dst)[RB][G]) {
    int col = kbeg + chunk * KC + g * G;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) load_run<T, G, VEC>(arow[rb], col, kend, rok[rb], dst[rb]);
  };
  // operand chunk: rows [k0, k0 + KC) of X, all KK columns (contiguous)
  auto load_x = [&](int chunk) {
    int k0 = kbeg + chunk * KC;
#pragma unroll
    for (int e = 0; e < XPER; ++e) {
      int idx = e * 256 + tid;
      int kr = idx / KK, c = idx - kr * KK;
      xr[e] = (k0 + kr < kend) ? X[(int64_t)(k0 + kr) * KK + c] : T(0);
    }
  };
  auto store_x = [&](int buf) {
#pragma unroll
    for (int e = 0; e < XPER; ++e) {
      int idx = e * 256 + tid;
      int kr = idx / KK, c = idx - kr * KK;
      Xs[buf][kr * LDX + c] = xr[e];
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
    // operand values of step s + 1 are read from LDS while step s's
    // products issue (the scheduling barrier keeps the reads ahead)
    const T* xs = Xs[buf] + (g * G) * LDX + r;
    T bb[2][KB];
#pragma unroll
    for (int jb = 0; jb < KB; ++jb) bb[0][jb] = xs[jb * 16];
#pragma unroll
    for (int s = 0; s < G; ++s) {
      if (s + 1 < G) {
#pragma unroll
        for (int jb = 0; jb < KB; ++jb) bb[(s + 1) & 1][jb] = xs[(s + 1) * LDX + jb * 16];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int jb = 0; jb < KB; ++jb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) Mfma<T>::mma(a_cur[rb][s], bb[s & 1][jb], acc[rb][jb]);
    }
    if (more) store_x(buf ^ 1);
    __syncthreads();
    if (more) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int s = 0; s < G; ++s) a_cur[rb][s] = a_nxt[rb][s];
    }
  }

  // epilogue: acc[rb][jb][i] = Y[row_base + rb*16 + out_row(g, i)][jb*16 + r]
  T* out = P + (int64_t)split * m * KK;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int row = row_base + rb * 16 + Mfma<T>::out_row(g, i);
      if (row < m) {
#pragma unroll
        for (int jb = 0; jb < KB; ++jb) out[(int64_t)row * KK + jb * 16 + r] = acc[rb][jb][i];
      }
    }
}

// ---------------------------------------------------------------------------
// Y = A X for FP32 A whose rows are 16-byte aligned with n % 4 == 0: both
// operands stream from global memory into LDS rings (global_load_lds, 16
// bytes per lane), so the only waits for the loads are the explicit counts
// at the top of each step and the waves spend their issue slots on the MFMA.
// Workgroup: 512 threads, 256 rows of A and all KK operand columns, one
// workgroup per CU; wave w owns rows [128 (w / 4), + 128) and column blocks
// [(w % 4) KBW, + KBW).  A chunk: 32 columns (128 bytes per row) through a
// three-stage ring issued two chunks ahead, the 16-byte segment j of a row
// in slot j ^ h(row), h(row) = (row & 7) ^ ((row >> 3) & 1); X chunk: its 32
// operand rows (KK floats each) through a two-stage ring, for KK = 64 or 128
// the segment j of row k in slot j ^ (4 ((k >> 3) & 3)), so that the four
// lane groups read distinct banks.  Lane (r, g) holds the chunk columns
// 8 g .. 8 g + 7 of its rows and multiplies them with operand rows 8 g + t in
// step t (a K permutation both operands share).  Segments of A past the end
// of the split re-read an in-range segment, and the matching operand rows are
// zeroed in LDS after they land, so the last chunk needs no other guard.
// ---------------------------------------------------------------------------
constexpr int kDmaRows = 256;

template <int KB, bool DW16>
__global__ __launch_bounds__(512, 1) void gemm_n_dma_kernel(const float* A, int64_t lda, int m, int n,
                                                            const float* X, float* __restrict__ P,
                                                            int cols_per_split, int ntiles, int nsplits) {
  constexpr int KK = 16 * KB, KBW = (KB + 3) / 4;
  constexpr int SA = kDmaRows * 128;   // bytes per A stage
  constexpr int SB = 32 * KK * 4;      // bytes per X stage
  constexpr int RSEG = KK / 4;         // 16-byte segments per operand row
  constexpr int BI = 32 * RSEG / 64;   // 1 KB DMA instructions per operand chunk
  constexpr bool SWB = RSEG % 16 == 0;
  __shared__ __attribute__((aligned(16))) uint8_t As[3 * SA];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2 * SB];

  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, g = lane >> 4;
  const int half = w >> 2, jb0 = (w & 3) * KBW;
  int tile, split;
  xcd_tile(ntiles, nsplits, tile, split);
  const int kbeg = split * cols_per_split;
  const int kend = min(n, kbeg + cols_per_split);
  const int nchunk = kend > kbeg ? (kend - kbeg + 31) / 32 : 0;
  const int row_blk = tile * kDmaRows;

  floatx4 acc[8][KBW];
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int jj = 0; jj < KBW; ++jj) acc[rb][jj] = floatx4{0, 0, 0, 0};

  if (nchunk > 0) {
    const uint32_t as0 = lds_addr(As), bs0 = lds_addr(Bs);
    // A: wave w moves rows [32 w, 32 w + 32) of a chunk, eight per
    // instruction; lane l: row 8 b + l / 8 (b = 4 w + i), slot l % 8, which
    // holds segment (l % 8) ^ (l / 8) ^ (b & 1); rows past m re-read row m - 1
    const int drow = lane >> 3;
    const float* abase[4];
    int aseg[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = min(row_blk + 32 * w + 8 * i + drow, m - 1);
      abase[i] = A + (int64_t)r * lda + kbeg;
      aseg[i] = (lane & 7) ^ drow ^ (i & 1);
    }
    // without 16-byte aligned rows the same LDS image is written 4 bytes per
    // lane: instruction j moves chunk rows 32 w + 2 j, + 1 (256 bytes), lane
    // l row 32 w + 2 j + l / 32, slot (l % 32) / 4, float l % 4 of it, which
    // holds float l % 4 of segment slot ^ h(row); columns past the end re-read
    // the chunk's first column
    const int dhi = lane >> 5, dslot = (lane & 31) >> 2, ddw = lane & 3;
    auto issue_a = [&](int chunk) {
      const int c0 = 32 * min(chunk, nchunk - 1);
      const uint32_t dst = as0 + (chunk % 3) * SA + 32 * w * 128;
      if constexpr (DW16) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int sg = (kbeg + c0 + 4 * aseg[i] < kend) ? aseg[i] : 0;
          dma16(abase[i] + c0 + 4 * sg, __builtin_amdgcn_readfirstlane(dst + 8 * i * 128));
        }
      } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int x = 2 * j + dhi;                     // row within the wave's 32
          const int hrow = (x & 7) ^ ((x >> 3) & 1);     // h of the chunk row (32 w adds no low bits)
          const int col = 4 * (dslot ^ hrow) + ddw;
          const int r = min(row_blk + 32 * w + x, m - 1);
          const int cc = (kbeg + c0 + col < kend) ? col : 0;
          dma4(A + (int64_t)r * lda + kbeg + c0 + cc, __builtin_amdgcn_readfirstlane(dst + j * 256));
        }
      }
    };
    // X: instruction i covers LDS segments [64 i, 64 i + 64) of the stage
    // and is issued by wave i % 8; operand rows past the end re-read the
    // chunk's first row (zeroed after landing)
    auto issue_b = [&](int chunk) {
      const int c0 = 32 * min(chunk, nchunk - 1);
      const uint32_t dst0 = bs0 + (chunk % 2) * SB;
      for (int i = w; i < BI; i += 8) {
        const int p = 64 * i + lane;
        const int row = p / RSEG, slot = p - row * RSEG;
        const int seg = SWB ? (slot ^ (((row >> 3) & 3) << 2)) : slot;
        const int krow = kbeg + c0 + (kbeg + c0 + row < kend ? row : 0);
        dma16(X + (int64_t)krow * KK + 4 * seg, __builtin_amdgcn_readfirstlane(dst0 + 64 * i * 16));
      }
    };
    const int hl = (lr & 7) ^ (lr >> 3);
    const uint32_t o0 = ((2 * g) ^ hl) << 4, o1 = ((2 * g + 1) ^ hl) << 4;
    auto run = [&](auto nb_const) {
      constexpr int NB = decltype(nb_const)::value;
      constexpr int NBA = NB > 0 ? NB : 1;
      // order of issue: A(0), B(0), A(1); step ch issues B(ch + 1), then
      // A(ch + 2): at the top of step ch all but this wave's last DMAs of
      // A(ch + 1) (four, or sixteen 4-byte ones) have landed
      issue_a(0);
      issue_b(0);
      issue_a(1);
      for (int ch = 0; ch < nchunk; ++ch) {
        // (a plain barrier: the fence of __syncthreads would wait for every DMA)
        if constexpr (DW16)
          asm volatile("s_waitcnt vmcnt(4)\n\ts_barrier" ::: "memory");
        else
          asm volatile("s_waitcnt vmcnt(16)\n\ts_barrier" ::: "memory");
        const int valid = min(32, kend - kbeg - 32 * ch);
        if (valid < 32) {
          float* bz = reinterpret_cast<float*>(Bs + (ch % 2) * SB);
          for (int e = tid; e < (32 - valid) * KK; e += 512) bz[valid * KK + e] = 0.0f;
          __syncthreads();
        }
        issue_b(ch + 1);
        issue_a(ch + 2);
        if (NB > 0) {
          const float* bst = reinterpret_cast<const float*>(Bs + (ch % 2) * SB);
          float bf[NBA][8];
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) {
            const int col = (jb0 + jj) * 16 + lr;
            const int slot = SWB ? ((col >> 2) ^ (g << 2)) : (col >> 2);
#pragma unroll
            for (int t = 0; t < 8; ++t) bf[jj][t] = bst[(8 * g + t) * KK + 4 * slot + (col & 3)];
          }
          const uint8_t* ast = As + (ch % 3) * SA + (128 * half + lr) * 128;
          float af[8][8];
#pragma unroll
          for (int rb = 0; rb < 8; ++rb) {
            const float4 x0 = *reinterpret_cast<const float4*>(ast + rb * 2048 + o0);
            const float4 x1 = *reinterpret_cast<const float4*>(ast + rb * 2048 + o1);
            af[rb][0] = x0.x; af[rb][1] = x0.y; af[rb][2] = x0.z; af[rb][3] = x0.w;
            af[rb][4] = x1.x; af[rb][5] = x1.y; af[rb][6] = x1.z; af[rb][7] = x1.w;
          }
#pragma unroll
          for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int rb = 0; rb < 8; ++rb)
#pragma unroll
              for (int jj = 0; jj < NB; ++jj) Mfma<float>::mma(af[rb][t], bf[jj][t], acc[rb][jj]);
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
  float* out = P + (int64_t)split * m * KK;
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = row_blk + 128 * half + rb * 16 + 4 * g + i;
      if (row < m) {
#pragma unroll
        for (int jj = 0; jj < KBW; ++jj)
          if (jb0 + jj < KB) out[(int64_t)row * KK + (jb0 + jj) * 16 + lr] = acc[rb][jj][i];
      }
    }
}

// ---------------------------------------------------------------------------
// W = A^T Z for FP32 A with 16-byte aligned rows (n % 4 == 0), the same LDS
// rings as gemm_n_dma_kernel with the roles of A's dimensions swapped: a
// workgroup owns 256 columns of A (MFMA M index) and a slice of its rows
// (K); a chunk is 32 rows of A restricted to the workgroup's columns (1 KB
// per row, one DMA instruction) and the same 32 rows of Z.  In both stages
// the 16-byte segment j of chunk row k sits in slot j ^ (4 ((k >> 3) & 3)),
// so that lane groups g (rows 8 g + t in step t) read distinct banks; lane
// (r, g) reads one A value per step (column r of its block).  Columns past
// n re-read the tile's first segment (their results are not stored); rows
// past the slice re-read its first row and meet zeroed rows of Z.
// ---------------------------------------------------------------------------
template <int KB, bool DW16>
__global__ __launch_bounds__(512, 1) void gemm_t_dma_kernel(const float* A, int64_t lda, int m, int n,
                                                            const float* Z, float* __restrict__ P,
                                                            int rows_per_split, int ntiles, int nsplits) {
  constexpr int KK = 16 * KB, KBW = (KB + 3) / 4;
  constexpr int SA = 32 * kDmaRows * 4;   // bytes per A stage: 32 rows x 256 columns
  constexpr int SB = 32 * KK * 4;         // bytes per Z stage
  constexpr int RSEG = KK / 4;
  constexpr int BI = 32 * RSEG / 64;
  constexpr bool SWB = RSEG % 16 == 0;
  __shared__ __attribute__((aligned(16))) uint8_t As[3 * SA];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2 * SB];

  const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, g = lane >> 4;
  const int half = w >> 2, jb0 = (w & 3) * KBW;
  int tile, split;
  xcd_tile(ntiles, nsplits, tile, split);
  const int ibeg = split * rows_per_split;
  const int iend = min(m, ibeg + rows_per_split);
  const int nchunk = iend > ibeg ? (iend - ibeg + 31) / 32 : 0;
  const int col_blk = tile * kDmaRows;

  floatx4 acc[8][KBW];
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int jj = 0; jj < KBW; ++jj) acc[rb][jj] = floatx4{0, 0, 0, 0};

  if (nchunk > 0) {
    const uint32_t as0 = lds_addr(As), bs0 = lds_addr(Bs);
    // A: wave w moves chunk rows 4 w .. 4 w + 3, one 1 KB instruction each;
    // lane l writes slot l, which holds segment l ^ (4 ((row >> 3) & 3)) of
    // the row's 256 columns (row >> 3 == w >> 1)
    const int aseg = lane ^ (((w >> 1) & 3) << 2);
    const int acol = (col_blk + 4 * aseg + 4 <= n) ? col_blk + 4 * aseg : col_blk;
    // without 16-byte aligned rows, 4 bytes per lane: instruction j moves a
    // quarter (64 columns, 256 bytes) of chunk row 4 w + j / 4; lane l writes
    // slot 16 (j % 4) + l / 4, float l % 4, which holds float l % 4 of
    // segment slot ^ (4 ((row >> 3) & 3)); columns past n re-read the tile's
    // first column
    const int asw = ((w >> 1) & 3) << 2;
    auto issue_a = [&](int chunk) {
      const int c0 = 32 * min(chunk, nchunk - 1);
      const uint32_t dst = as0 + (chunk % 3) * SA + 4 * w * 1024;
      if constexpr (DW16) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = ibeg + c0 + 4 * w + i;
          const int srow = row < iend ? row : ibeg + c0;
          dma16(A + (int64_t)srow * lda + acol, __builtin_amdgcn_readfirstlane(dst + i * 1024));
        }
      } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int i = j >> 2, q = j & 3;
          const int row = ibeg + c0 + 4 * w + i;
          const int srow = row < iend ? row : ibeg + c0;
          const int slot = 16 * q + (lane >> 2);
          const int col = col_blk + 4 * (slot ^ asw) + (lane & 3);
          dma4(A + (int64_t)srow * lda + (col < n ? col : col_blk),
               __builtin_amdgcn_readfirstlane(dst + i * 1024 + q * 256));
        }
      }
    };
    auto issue_b = [&](int chunk) {
      const int c0 = 32 * min(chunk, nchunk - 1);
      const uint32_t dst0 = bs0 + (chunk % 2) * SB;
      for (int i = w; i < BI; i += 8) {
        const int p = 64 * i + lane;
        const int row = p / RSEG, slot = p - row * RSEG;
        const int seg = SWB ? (slot ^ (((row >> 3) & 3) << 2)) : slot;
        const int krow = ibeg + c0 + (ibeg + c0 + row < iend ? row : 0);
        dma16(Z + (int64_t)krow * KK + 4 * seg, __builtin_amdgcn_readfirstlane(dst0 + 64 * i * 16));
      }
    };
    auto run = [&](auto nb_const) {
      constexpr int NB = decltype(nb_const)::value;
      constexpr int NBA = NB > 0 ? NB : 1;
      // order of issue as in gemm_n_dma_kernel: the last DMAs of a wave at
      // the top of step ch are A(ch + 1)'s (four, or sixteen 4-byte ones)
      issue_a(0);
      issue_b(0);
      issue_a(1);
      for (int ch = 0; ch < nchunk; ++ch) {
        if constexpr (DW16)
          asm volatile("s_waitcnt vmcnt(4)\n\ts_barrier" ::: "memory");
        else
          asm volatile("s_waitcnt vmcnt(16)\n\ts_barrier" ::: "memory");
        const int valid = min(32, iend - ibeg - 32 * ch);
        if (valid < 32) {
          float* bz = reinterpret_cast<float*>(Bs + (ch % 2) * SB);
          for (int e = tid; e < (32 - valid) * KK; e += 512) bz[valid * KK + e] = 0.0f;
          __syncthreads();
        }
        issue_b(ch + 1);
        issue_a(ch + 2);
        if (NB > 0) {
          const float* bst = reinterpret_cast<const float*>(Bs + (ch % 2) * SB);
          float bf[NBA][8];
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) {
            const int col = (jb0 + jj) * 16 + lr;
            const int slot = SWB ? ((col >> 2) ^ (g << 2)) : (col >> 2);
#pragma unroll
            for (int t = 0; t < 8; ++t) bf[jj][t] = bst[(8 * g + t) * KK + 4 * slot + (col & 3)];
          }
          // lane (lr, g), block rb: column 128 half + 16 rb + lr of the tile
          const float* ast = reinterpret_cast<const float*>(As + (ch % 3) * SA);
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            float af[8];
#pragma unroll
            for (int rb = 0; rb < 8; ++rb) {
              const int c = 128 * half + 16 * rb + lr;
              af[rb] = ast[(8 * g + t) * kDmaRows + 4 * ((c >> 2) ^ (g << 2)) + (c & 3)];
            }
#pragma unroll
            for (int rb = 0; rb < 8; ++rb)
#pragma unroll
              for (int jj = 0; jj < NB; ++jj) Mfma<float>::mma(af[rb], bf[jj][t], acc[rb][jj]);
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
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  float* out = P + (int64_t)split * n * KK;
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int col = col_blk + 128 * half + rb * 16 + 4 * g + i;
      if (col < n) {
#pragma unroll
        for (int jj = 0; jj < KBW; ++jj)
          if (jb0 + jj < KB) out[(int64_t)col * KK + (jb0 + jj) * 16 + lr] = acc[rb][jj][i];
      }
    }
}

// ---------------------------------------------------------------------------
// W = A^T Z.  MFMA M index = column of A, N = operand column, K = row of A.
// Lane (r, g) loads VW consecutive columns [4.. of its 16-lane group] of a
// row: column col_w + VW*r + e belongs to MFMA block e at M index r.  Per K
// chunk of KC rows, group g takes rows [g*G, g*G + G).
// ---------------------------------------------------------------------------
template <typename T, int KB, int VW, bool VEC>
__global__ __launch_bounds__(256, 2) void gemm_t_kernel(const T* __restrict__ A, int64_t lda, int m,
                                                        int n, const T* __restrict__ Z,
                                                        T* __restrict__ P, int rows_per_split, int ntiles,
                                                        int nsplits) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int KC = 32;
  constexpr int G = KC / 4;
  constexpr int KK = 16 * KB;
  constexpr int LDZ = KK + 2;   // group g reads rows g G + s: 8 LDZ = 16 mod 64 words keeps the four groups on distinct banks
  constexpr int ZPER = KC * KK / 256;
  constexpr int CW = 16 * VW;  // columns per wave
  __shared__ T Zs[2][KC * LDZ];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int r = lane & 15;
  const int g = lane >> 4;
  int tile, split;
  xcd_tile(ntiles, nsplits, tile, split);
  const int ibeg = split * rows_per_split;
  const int iend = min(m, ibeg + rows_per_split);
  const int nchunk = iend > ibeg ? (iend - ibeg + KC - 1) / KC : 0;
  const int colw = tile * (4 * CW) + w * CW;
  const int mycol = colw + VW * r;
  const bool vec_ok = VEC && (mycol + VW <= n);

  acc_t acc[VW][KB];
#pragma unroll
  for (int e = 0; e < VW; ++e)
#pragma unroll
    for (int jb = 0; jb < KB; ++jb) acc[e][jb] = acc_t{0, 0, 0, 0};

  T a_cur[G][VW], a_nxt[G][VW];
  T zr[ZPER];

  auto load_a = [&](int chunk, T (&dst)[G][VW]) {
    int i0 = ibeg + chunk * KC + g * G;
#pragma unroll
    for (int s = 0; s < G; ++s) {
      int row = i0 + s;
      bool rok = row < iend;
      const T* p = A + (int64_t)(rok ? row : ibeg) * lda;
      if (vec_ok && rok) {
        Vec<T, VW> x = *reinterpret_cast<const Vec<T, VW>*>(p + mycol);
#pragma unroll
        for (int e = 0; e < VW; ++e) dst[s][e] = x.v[e];
      } else {
#pragma unroll
        for (int e = 0; e < VW; ++e) dst[s][e] = (rok && mycol + e < n) ? p[mycol + e] : T(0);
      }
    }
  };
  auto load_z = [&](int chunk) {
    int i0 = ibeg + chunk * KC;
#pragma unroll
    for (int e = 0; e < ZPER; ++e) {
      int idx = e * 256 + tid;
      int kr = idx / KK, c = idx - kr * KK;
      zr[e] = (i0 + kr < iend) ? Z[(int64_t)(i0 + kr) * KK + c] : T(0);
    }
  };
  auto store_z = [&](int buf) {
#pragma unroll
    for (int e = 0; e < ZPER; ++e) {
      int idx = e * 256 + tid;
      int kr = idx / KK, c = idx - kr * KK;
      Zs[buf][kr * LDZ + c] = zr[e];
    }
  };

  if (nchunk > 0) {
    load_a(0, a_cur);
    load_z(0);
    store_z(0);
  }
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunk;
    if (more) {
      load_a(ch + 1, a_nxt);
      load_z(ch + 1);
    }
    // operand values of step s + 1 are read from LDS while step s's
    // products issue (the scheduling barrier keeps the reads ahead)
    const T* zs = Zs[buf] + (g * G) * LDZ + r;
    T bb[2][KB];
#pragma unroll
    for (int jb = 0; jb < KB; ++jb) bb[0][jb] = zs[jb * 16];
#pragma unroll
    for (int s = 0; s < G; ++s) {
      if (s + 1 < G) {
#pragma unroll
        for (int jb = 0; jb < KB; ++jb) bb[(s + 1) & 1][jb] = zs[(s + 1) * LDZ + jb * 16];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int jb = 0; jb < KB; ++jb)
#pragma unroll
        for (int e = 0; e < VW; ++e) Mfma<T>::mma(a_cur[s][e], bb[s & 1][jb], acc[e][jb]);
    }
    if (more) store_z(buf ^ 1);
    __syncthreads();
    if (more) {
#pragma unroll
      for (int s = 0; s < G; ++s)
#pragma unroll
        for (int e = 0; e < VW; ++e) a_cur[s][e] = a_nxt[s][e];
    }
  }

  // epilogue: acc[e][jb][i] = W[colw + VW*out_row(g, i) + e][jb*16 + r]
  T* out = P + (int64_t)split * n * KK;
#pragma unroll
  for (int e = 0; e < VW; ++e)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int col = colw + VW * Mfma<T>::out_row(g, i) + e;
      if (col < n) {
#pragma unroll
        for (int jb = 0; jb < KB; ++jb) out[(int64_t)col * KK + jb * 16 + r] = acc[e][jb][i];
      }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static int g_num_cu = 0;
static int num_cu() {
  if (g_num_cu == 0) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess && p.multiProcessorCount > 0)
      g_num_cu = p.multiProcessorCount;
    else
      g_num_cu = 256;
  }
  return g_num_cu;
}

// Pick the number of reduction slices so that tiles * splits fills the
// resident workgroup slots (wg_per_cu per CU, from the variant's register
// use) with a small tail, without cutting a slice below a few chunks.
// Depends only on the shape and the CU count.
static int choose_splits(int tiles, int klen, int min_per_split, int wg_per_cu = 2) {
  const int slots = wg_per_cu * num_cu();
  int max_s = std::max(1, klen / min_per_split);
  max_s = std::min(max_s, 64);
  int best = 1;
  double best_eff = -1.0;
  for (int s = 1; s <= max_s; ++s) {
    long long wgs = (long long)tiles * s;
    long long rounds = (wgs + slots - 1) / slots;
    double eff = (double)wgs / (double)(rounds * slots);
    // penalise extra partial traffic slightly
    eff -= 0.004 * s;
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = s;
    }
    if (wgs >= 4LL * slots) break;
  }
  return best;
}

// Row blocks of 16 per wave in the A X kernel: two for FP32 except where the
// operand width makes the register budget spill.
static constexpr int rb_for(int kb, int elem_bytes) { return (elem_bytes == 4 && kb != 6 && kb != 7) ? 2 : 1; }

// FP32 A X runs the LDS-ring kernel (one 256-row workgroup per CU) when the
// rows allow it; the split count is chosen for that kernel (any count is
// valid for the other one, used when A's rows are not 16-byte aligned):
// minimise rounds * (bytes per workgroup, partials included).
// The 4-byte DMA variants (rows that are not 16-byte aligned) move four
// times as many DMA instructions and hold a whole CU per workgroup; small
// unaligned matrices (most of the serving mix, where several requests'
// passes share the GPU) keep the register-staged kernels, which leave room
// for other workgroups on a CU.
static bool dw4_worth(int m, int n) { return (int64_t)m * n >= (int64_t)4 << 20; }

static int choose_splits_dma(int m, int n, int kk) {
  const int cus = num_cu();
  const int64_t tiles = (m + kDmaRows - 1) / kDmaRows;
  const double abytes = 4.0 * m * n, pbytes = 4.0 * m * kk;
  int best = 1;
  double best_t = 0.0;
  for (int s = 1; s <= 64 && (s == 1 || n / s >= 128); ++s) {
    const int64_t wgs = tiles * s;
    const double t = (double)((wgs + cus - 1) / cus) * (abytes + s * pbytes) / (double)wgs;
    if (s == 1 || t < best_t * 0.999) {
      best = s;
      best_t = t;
    }
  }
  return best;
}

int choose_splits_n(int m, int n, int kk, int elem_bytes) {
  if (elem_bytes == 4 && kk <= 128 && (n % 4 == 0 || dw4_worth(m, n))) return choose_splits_dma(m, n, kk);
  int rb = rb_for(kk / 16, elem_bytes);
  int tiles = (m + 64 * rb - 1) / (64 * rb);
  return choose_splits(tiles, n, 512);
}

// Columns of A per lane in the A^T Z kernel: one for wide operands (the
// kernel then needs few registers and four workgroups fit on a CU, which
// measured faster than two columns at 20000 x 5000 and 100000 x 20000).
static constexpr int t_vw(int kb, int elem_bytes) { return kb > 4 ? 1 : (elem_bytes == 4 ? 4 : 2); }

int choose_splits_t(int m, int n, int kk, int elem_bytes) {
  if (elem_bytes == 4 && kk <= 128 && (n % 4 == 0 || dw4_worth(m, n))) return choose_splits_dma(n, m, kk);
  const int kb = kk / 16;
  const int cw = 4 * 16 * t_vw(kb, elem_bytes);
  const int tiles = (n + cw - 1) / cw;
  return choose_splits(tiles, m, 512, (elem_bytes == 4 && kb > 4) ? 4 : 2);
}

template <typename T, int KB>
static hipError_t gemm_n_kb(const T* A, int64_t lda, int m, int n, const T* X, T* P, int splits,
                            hipStream_t st) {
  constexpr int RB = rb_for(KB, sizeof(T));
  constexpr int KC = sizeof(T) == 4 ? 64 : 32;
  int per = (n + splits - 1) / splits;
  per = (per + KC - 1) / KC * KC;
  bool vec = ((uintptr_t)A % 16 == 0) && ((lda * (int64_t)sizeof(T)) % 16 == 0);
  if constexpr (sizeof(T) == 4) {
    if ((uintptr_t)X % 16 == 0 && (uintptr_t)A % 4 == 0) {
      int per32 = (n + splits - 1) / splits;
      per32 = (per32 + 31) / 32 * 32;
      const int nt = (m + kDmaRows - 1) / kDmaRows;
      if (vec && n % 4 == 0) {
        hipLaunchKernelGGL((gemm_n_dma_kernel<KB, true>), dim3(nt * splits), dim3(512), 0, st, (const float*)A, lda,
                           m, n, (const float*)X, (float*)P, per32, nt, splits);
        CNMF_LAUNCH_CHECK();
      }
      if (dw4_worth(m, n)) {
        hipLaunchKernelGGL((gemm_n_dma_kernel<KB, false>), dim3(nt * splits), dim3(512), 0, st, (const float*)A, lda,
                           m, n, (const float*)X, (float*)P, per32, nt, splits);
        CNMF_LAUNCH_CHECK();
      }
    }
  }
  const int ntiles = (m + 64 * RB - 1) / (64 * RB);
  dim3 grid(ntiles * splits);
  if (vec)
    hipLaunchKernelGGL((gemm_n_kernel<T, KB, RB, true>), grid, dim3(256), 0, st, A, lda, m, n, X, P, per, ntiles,
                       splits);
  else
    hipLaunchKernelGGL((gemm_n_kernel<T, KB, RB, false>), grid, dim3(256), 0, st, A, lda, m, n, X, P, per, ntiles,
                       splits);
  CNMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t launch_gemm_n(const T* A, int64_t lda, int m, int n, const T* X, int kk, T* P, int splits,
                         hipStream_t st) {
  switch (kk) {
    case 16: return gemm_n_kb<T, 1>(A, lda, m, n, X, P, splits, st);
    case 32: return gemm_n_kb<T, 2>(A, lda, m, n, X, P, splits, st);
    case 48: return gemm_n_kb<T, 3>(A, lda, m, n, X, P, splits, st);
    case 64: return gemm_n_kb<T, 4>(A, lda, m, n, X, P, splits, st);
    case 80: return gemm_n_kb<T, 5>(A, lda, m, n, X, P, splits, st);
    case 96: return gemm_n_kb<T, 6>(A, lda, m, n, X, P, splits, st);
    case 112: return gemm_n_kb<T, 7>(A, lda, m, n, X, P, splits, st);
    case 128: return gemm_n_kb<T, 8>(A, lda, m, n, X, P, splits, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int KB>
static hipError_t gemm_t_kb(const T* A, int64_t lda, int m, int n, const T* Z, T* P, int splits,
                            hipStream_t st) {
  constexpr int VW = t_vw(KB, sizeof(T));
  constexpr int KC = 32;
  int per = (m + splits - 1) / splits;
  per = (per + KC - 1) / KC * KC;
  bool vec = ((uintptr_t)A % 16 == 0) && ((lda * (int64_t)sizeof(T)) % 16 == 0);
  if constexpr (sizeof(T) == 4) {
    if ((uintptr_t)Z % 16 == 0 && (uintptr_t)A % 4 == 0) {
      const int nt = (n + kDmaRows - 1) / kDmaRows;
      if (vec && n % 4 == 0) {
        hipLaunchKernelGGL((gemm_t_dma_kernel<KB, true>), dim3(nt * splits), dim3(512), 0, st, (const float*)A, lda,
                           m, n, (const float*)Z, (float*)P, per, nt, splits);
        CNMF_LAUNCH_CHECK();
      }
      if (dw4_worth(m, n)) {
        hipLaunchKernelGGL((gemm_t_dma_kernel<KB, false>), dim3(nt * splits), dim3(512), 0, st, (const float*)A, lda,
                           m, n, (const float*)Z, (float*)P, per, nt, splits);
        CNMF_LAUNCH_CHECK();
      }
    }
  }
  const int ntiles = (n + 64 * VW - 1) / (64 * VW);
  dim3 grid(ntiles * splits);
  if (vec)
    hipLaunchKernelGGL((gemm_t_kernel<T, KB, VW, true>), grid, dim3(256), 0, st, A, lda, m, n, Z, P, per, ntiles,
                       splits);
  else
    hipLaunchKernelGGL((gemm_t_kernel<T, KB, VW, false>), grid, dim3(256), 0, st, A, lda, m, n, Z, P, per, ntiles,
                       splits);
  CNMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t launch_gemm_t(const T* A, int64_t lda, int m, int n, const T* Z, int kk, T* P, int splits,
                         hipStream_t st) {
  switch (kk) {
    case 16: return gemm_t_kb<T, 1>(A, lda, m, n, Z, P, splits, st);
    case 32: return gemm_t_kb<T, 2>(A, lda, m, n, Z, P, splits, st);
    case 48: return gemm_t_kb<T, 3>(A, lda, m, n, Z, P, splits, st);
    case 64: return gemm_t_kb<T, 4>(A, lda, m, n, Z, P, splits, st);
    case 80: return gemm_t_kb<T, 5>(A, lda, m, n, Z, P, splits, st);
    case 96: return gemm_t_kb<T, 6>(A, lda, m, n, Z, P, splits, st);
    case 112: return gemm_t_kb<T, 7>(A, lda, m, n, Z, P, splits, st);
    case 128: return gemm_t_kb<T, 8>(A, lda, m, n, Z, P, splits, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_gemm_n<float>(const float*, int64_t, int, int, const float*, int, float*, int, hipStream_t);
template hipError_t launch_gemm_n<double>(const double*, int64_t, int, int, const double*, int, double*, int, hipStream_t);
template hipError_t launch_gemm_t<float>(const float*, int64_t, int, int, const float*, int, float*, int, hipStream_t);
template hipError_t launch_gemm_t<double>(const double*, int64_t, int, int, const double*, int, double*, int, hipStream_t);

}  // namespace cnmf
