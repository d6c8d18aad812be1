// Internal declarations shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <stddef.h>

namespace cnmf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Error bookkeeping for kernel launchers: every launcher returns the HIP
// status of its launch so the runtime can map it to CNMF_EDEVICE.
#define CNMF_LAUNCH_CHECK() return hipGetLastError()

// Block-cooperative staging with up to U loads in flight per thread: for e =
// first, first + stride, ... < count, load(e) for U elements, then
// store(e, value) for them.  Staging loops that load and store one element
// at a time leave every thread waiting on the memory latency once per
// element it moves.
template <int U, typename Load, typename Store>
__device__ __forceinline__ void staged_copy(int count, int first, int stride, Load&& load, Store&& store) {
  for (int e0 = first; e0 < count; e0 += stride * U) {
    decltype(load(0)) v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + stride * u;
      if (e < count) v[u] = load(e);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + stride * u;
      if (e < count) store(e, v[u]);
    }
  }
}

// ---------------------------------------------------------------------------
// Pass GEMMs (range-finder passes over A)
// ---------------------------------------------------------------------------
// Y = A X (A m x n row-major, X n x kk, kk = 16*kb): partial products over
// `splits` slices of the n range land in P[s][m][kk]; with splits == 1 the
// result is final.  T is double or float.
template <typename T>
hipError_t launch_gemm_n(const T* A, int64_t lda, int m, int n, const T* X, int kk, T* P,
                         int splits, hipStream_t st);
// W = A^T Z (Z m x kk): partials over slices of the m range in P[s][n][kk].
template <typename T>
hipError_t launch_gemm_t(const T* A, int64_t lda, int m, int n, const T* Z, int kk, T* P,
                         int splits, hipStream_t st);
// Split count heuristic shared by the runtime (deterministic in the shape).
int choose_splits_n(int m, int n, int kk, int elem_bytes);
int choose_splits_t(int m, int n, int kk, int elem_bytes);

// Reduced-precision passes (k_lowp.hip).  A copy of A (m x n) and of A^T
// (n x m) in BF16 or FP8 E4M3, each padded with zeros to whole
// kFp8Tile x kFp8Tile tiles (A: lowp_pad(m) rows, ldo >= lowp_pad(n);
// A^T: lowp_pad(n) rows, ldt >= lowp_pad(m)); FP8 copies carry one FP32
// power-of-two scale per tile of A (scale[ti * ntj + tj], ntj column
// tiles), shared by the A^T copy.  Either output pointer may be NULL.
constexpr int kFp8Tile = 128;
inline int64_t lowp_pad(int64_t x) { return (x + kFp8Tile - 1) / kFp8Tile * kFp8Tile; }
hipError_t launch_convert_lowp(const float* A, int64_t lda, int m, int n, __hip_bfloat16* A16, __hip_bfloat16* At16,
                               uint8_t* A8, uint8_t* At8, int64_t ldo, int64_t ldt, float* scale, hipStream_t st);
// P[s][rows][kk] (FP32) = M (rows x cols, element size es: 2 BF16, 1 FP8,
// ld ldm, m_rows >= lowp_pad(rows) rows allocated) times Xt^T (Xt kk x
// cols, same type, ld ldx), partial sums over `splits` slices of the column
// range.  ldm, ldx >= lowp_pad(cols); the padding of M and Xt must be zero.
// FP8: scale as above; scale_t = 1 when M is the A^T copy.
hipError_t launch_gemm_lowp(int es, const void* M, int64_t ldm, int64_t m_rows, int rows, int cols, const void* Xt,
                            int64_t ldx, int kk, float* P, int splits, const float* scale, int scale_ld, int scale_t,
                            hipStream_t st);
int choose_splits_lowp(int rows, int cols, int kk, int es);
// Columns [c0, c0 + k) of Q (rows x ldq, FP64) -> rows [dr0, dr0 + k) of the
// transposed operand Xt (ld ldx) in BF16 (es 2) or FP8 (es 1); FP8 columns
// are scaled by a power of two (colscale[scol0 + c]) chosen from the column
// maximum so that they use the E4M3 range (cmax: k words of scratch).
hipError_t launch_store_lowp(int es, const double* Q, int rows, int ldq, int c0, int k, void* Xt, int64_t ldx,
                             int dr0, float* colscale, int scol0, unsigned long long* cmax, hipStream_t st);
// Y[:, c] /= colscale[c], c < k (FP32, rows x ld).
hipError_t launch_unscale_cols(float* Y, int rows, int ld, int k, const float* colscale, hipStream_t st);

// ---------------------------------------------------------------------------
// Orthonormalisation (CholeskyQR2 in FP64) and small products
// ---------------------------------------------------------------------------
// Y = sum_s P[s] (fixed order), rows x ld.
template <typename T>
hipError_t launch_reduce_splits(const T* P, int splits, int64_t rows, int ld, T* Y, hipStream_t st);
// Partials of X[:, x0 + h*hs : +ka]^T Y[:, y0 + h*hs : +kb] (FP64) over `parts`
// row slices, for h < nh: Cp[(p * nh + h) * ka * kb].
// With run_if, half h is skipped unless run_if[h] != 0.
template <typename TX, typename TY>
hipError_t launch_cross2(const TX* X, int ldx, int x0, const TY* Y, int ldy, int y0, int hs, int nh, int rows,
                         int ka, int kb, double* Cp, int parts, hipStream_t st, const int* run_if = nullptr);
// out[e] = sum_p in[p * count + e] in the order p = 0, 1, ...  With run_if,
// nothing is done unless one of run_if[0 .. nrun) is nonzero.
hipError_t launch_sum_parts(const double* in, int parts, int64_t count, double* out, hipStream_t st,
                            const int* run_if = nullptr, int nrun = 0);
// For each half h: G_h = fixed-order sum of the Gram partials, then
// G_h = T^T T (Cholesky, T upper with positive diagonal) and Tinv_h = T^-1
// (kh x kh).  Breakdown handling, for a pivot <= tau max diag(G_h):
//   mask != NULL (decoupling): the column is taken as dependent on the
//     earlier ones, decoupled, counted in repaired[h] and marked in mask[2 h],
//     mask[2 h + 1] (bit c of word c / 64) for launch_apply_tinv to replace;
//     need[h] (if given) is set to whether any column of half h was;
//   mask == NULL: the pivot is floored and counted as unresolved.
// NaN pivots are unresolved.  Unresolved counts are added to unresolved[0]
// and unresolved_total[0] (each may be NULL).  run_if (may be NULL): half h
// runs only if run_if[h] != 0.
struct CholOpts {
  double tau;
  int* repaired;
  int* unresolved;
  int* unresolved_total;
  uint64_t* mask;
  int* need;
  const int* run_if;
};
hipError_t launch_gram_chol(const double* Gp, int parts, int nh, int kh, double* G, double* Tinv, const CholOpts& o,
                            hipStream_t st);
// The factor-and-invert step alone on nh summed Grams G (kh x kh each).
hipError_t launch_chol_tinv(const double* G, int nh, int kh, double* Tinv, const CholOpts& o, hipStream_t st);
// (S + pen I)^-1 for a symmetric r x r S (r <= 64), FP64: G = sym(S) +
// pen I, the one-wave Cholesky G = T^T T with T^-1 (launch_chol_tinv; pivots
// below 1e-300 max diag floored and counted in *floored, which is zeroed
// first), Minv = T^-1 T^-T.  ok != nullptr: *ok = 1 when max |G Minv - I|
// <= 1e-8 and nothing was floored, else 0.  G and Tinv: r x r scratch.
hipError_t launch_spd_inverse(const double* S, int r, double pen, double* G, double* Tinv, double* Minv, int* floored,
                              int* ok, hipStream_t st);
// Q64[:, h*kh + c] = sum_{l <= c} Y[:, h*kh + l] Tinv_h[l][c] (FP64), h < nh;
// columns marked in mask (NULL: none) get entries of Gaussian test matrix
// id0 + h under `seed`, divided by sqrt(rows).  In place (Q64 == Y) is
// allowed.  run_if as for launch_gram_chol.
template <typename TY>
hipError_t launch_apply_tinv(const TY* Y, int rows, int ldy, int nh, int kh, const double* Tinv, double* Q64,
                             int ldq, const uint64_t* mask, uint64_t seed, uint32_t id0, hipStream_t st,
                             const int* run_if = nullptr);
// Ids of the Gaussian test matrices (rng.hpp): Omega_L, Omega_R, and the
// completion columns of the orthonormalisation after pass p (half h: first
// CholeskyQR pass kCompletionId0 + 4 p + h, second kCompletionId0 + 4 p + 2 + h).
constexpr uint32_t kOmegaLeftId = 0;
constexpr uint32_t kOmegaRightId = 1;
constexpr uint32_t kCompletionId0 = 16;
// out (rows x cols, ld) = Gaussian test matrix `id` under `seed` (rng.hpp).
hipError_t launch_gaussian_fill(double* out, int64_t ld, int rows, int cols, uint64_t seed, uint32_t id,
                                hipStream_t st);
// SRHT test matrix (k_rng.hip): rows x cols (cols <= 128) into out (ld);
// S receives the cols sampled Hadamard column indices (device, 128 ints).
hipError_t launch_srht_fill(double* out, int64_t ld, int rows, int cols, uint64_t seed, uint32_t id, int32_t* S,
                            hipStream_t st);
// max |Q^T Q - I| for an FP64 Gram (for stats)
hipError_t launch_orth_error(const double* G, int kh, double* out, hipStream_t st);

// ---------------------------------------------------------------------------
// Compressed / uncompressed NMF iterations
// ---------------------------------------------------------------------------
struct AdmmSide {
  const void* Bm;   // basis rows (L: m x kp, or R^T: n x kp), TA
  int ldb;
  void* F;          // factor rows (U: m x r, or V^T: n x r), ld = ldf
  void* M;          // multiplier rows (Lam or Phi^T), ld = ldf
  int ldf;
  int rows;
  double pen;       // lambda or phi
};
template <typename T>
hipError_t launch_admm_uv(AdmmSide s0, AdmmSide s1, int nsides, const double* XY, int k, int r,
                          double xi, int mode, double* Pp, int parts0, int parts1, hipStream_t st);
// The solves run in one workgroup whose LDS holds admm_solve_lds_bytes(k, r)
// (<= 160 KiB required).
size_t admm_solve_lds_bytes(int k, int r);
// Split schedule of one request (Alg. 3 order kept): with solve != 0, block
// 0 solves one side (pass 0: Xt, with S = Yt^T, or P_V / phi when first;
// pass 1: Yt^T, with S = Xt) and the other blocks run the row update of side
// `side` (0: U / Lam, parts0 blocks; 1: V^T / Phi^T, parts1 blocks) writing
// its partial slots as launch_admm_uv does, when uv != 0.
struct AdmmHalf {
  AdmmSide s0, s1;
  const double* At;
  double* Pred;
  double* XY;
  double* Pp;
  int* flags;
  double lam, phi, xi;
  int k, r, parts0, parts1, rpb0, rpb1;
  int solve, pass, first, uv, side, mode;
  // nred > 0: the launch also forms the solve's reduced partials (P_V for
  // pass 1, P_U for pass 0) in nred workgroups placed
  // between the solve's block and the row-update blocks; each adds one to
  // *ready after its release, and the solve waits until *ready reaches
  // ready_target (a count that only grows, cleared before the iterations).
  // A wait that times out adds one to *wait_fail.
  unsigned* ready;
  unsigned ready_target;
  int nred;
  int rgroups;   // 16-element groups per reduction workgroup: 1, 2 or 4 (nred = ceil(ceil(k r / 16) / rgroups))
  int* wait_fail;
};
// Groups per reduction workgroup for fused launches beside nuv row-update
// workgroups: the smallest of 1, 2, 4 that keeps the launch within one
// workgroup per CU, or 0 (sum in separate launches) if none does or the
// sum workgroups would be too slow to finish before the solve needs them.
int admm_fused_reduce_groups(int k, int r, int nuv);
template <typename T>
hipError_t launch_admm_half(const AdmmHalf& a, hipStream_t st);
// Fixed-order FP64 sums of the partials of one side (0: P_U into Pred, 1:
// P_V into Pred + k r) or of both (2).
template <typename T>
hipError_t launch_admm_reduce(const double* Pp, int parts0, int parts1, int k, int r, int side, double* Pred,
                              hipStream_t st);

// One request of a batched ADMM step (FP32 factors): its two sides, the
// FP64 solve state and its partial buffers, all in its own workspace.
struct AdmmJob {
  AdmmSide s0, s1;        // U / Lam with L, and V^T / Phi^T with R^T
  const double* At;       // k x k
  double* XY;             // Xt, Yt^T (k x r each), then FP32 copies (KP x RP each)
  double* Pp;             // (parts0 + parts1) k x r partials
  double* Pred;           // 2 k x r reduced partials
  int* flags;             // breakdown flag word
  double lam, phi, xi;
  int k, r, parts0, parts1;
  int rpb0, rpb1;         // rows per uv block (filled by admm_job_prepare)
  int first;              // 1 for the request's first iteration
  int last;               // 1 for its last iteration (U, V^T are stored)
};
void admm_job_prepare(AdmmJob& J);
int admm_job_uv_blocks(const AdmmJob& J);
int admm_job_red_blocks(const AdmmJob& J);
size_t admm_job_solve_lds(const AdmmJob& J);
// jobs_dev: njobs descriptors; uv_first_dev / red_first_dev: first block of
// each job in the uv / reduce launch (ascending, from 0), uv_blocks /
// red_blocks the totals; solve_lds = max admm_job_solve_lds over the jobs.
hipError_t launch_admm_step_batch(const AdmmJob* jobs_dev, const int* uv_first_dev, const int* red_first_dev,
                                  int njobs, int uv_blocks, int red_blocks, int max_k, int max_r, size_t solve_lds,
                                  hipStream_t st);

// The batched step with fixed grids (for capture in a graph and replay): one
// device buffer holds a BatchHeader at offset 0, the job table at off_jobs
// and the first-block tables at off_uv / off_red; the kernels read the
// counts from the header.  uv_lds = admm_batch_uv_lds(max k, max r) and
// solve_lds >= every job's admm_job_solve_lds (both <= 160 KiB); grid_solve
// >= 1 workgroups loop over the jobs, grid_red / grid_uv workgroups take the
// step's reduce / row-update blocks one at a time from the header's counters
// (which the copy of the header sets to 0).  admm_step_fixed_init() raises the kernels'
// dynamic-LDS limit (once, outside any capture).
struct BatchHeader {
  int njobs, uv_total, red_total;
  int red_next, uv_next;   // work counters of the two block loops (0 when copied in)
  int reserved[3];
};
size_t admm_batch_uv_lds(int max_k, int max_r);
hipError_t admm_step_fixed_init();
hipError_t launch_admm_step_fixed(char* desc_dev, size_t off_jobs, size_t off_uv, size_t off_red,
                                  int grid_solve, int grid_red, int grid_uv, size_t uv_lds, size_t solve_lds,
                                  hipStream_t st);

// Generic row update for MU and the uncompressed comparators (k_nmf.hip).
struct RowArgs {
  int rows, k1, r, k2;
  const void* B1;
  int ldb1;
  const double* C;
  void* F;
  int ldf;
  void* Mu;
  const double* Gp;
  const double* Gm;
  const double* Minv;
  double pen, xi, eps;
  int method;  // 0 MU, 1 ADMM (uncompressed), 2 partials only
  const void* B2;
  int ldb2;
  void* Op;
  int ldop;
  double* Pp;
  int rows_per_block;
};
template <typename T>
hipError_t launch_nmf_row(const RowArgs& a, int blocks, hipStream_t st);
// mode 0: G = C^T C (C = S, k x r) -> G+, G-; mode 1: G = S (r x r) -> G+, G-;
// mode 3: Gp = S^T S (C = S, k x r).
hipError_t launch_nmf_small(const double* S, int k, int r, int mode, double pen, double* Gp, double* Gm, int* flags,
                            hipStream_t st);

// ---------------------------------------------------------------------------
// Misc
// ---------------------------------------------------------------------------
template <typename TS, typename TD>
hipError_t launch_copy2d(const TS* src, int64_t lds, TD* dst, int64_t ldd, int rows, int cols,
                         double scale, hipStream_t st);
template <typename TS, typename TD>
hipError_t launch_transpose(const TS* src, int64_t lds, TD* dst, int64_t ldd, int rows, int cols,
                            hipStream_t st);
hipError_t launch_fill(void* p, size_t bytes, hipStream_t st);
// Sparse A in CSR form (k_sparse.hip).  Transpose: trow (n + 1), tcol / tval
// (nnz) from rowptr / col / val, with scratch keys, perm, keys_out, perm_out
// (nnz each) and tmp (csr_sort_temp_bytes); column indices outside [0, n)
// are counted in *bad (and skipped everywhere).  spmm: Y (rows x kk) = S X,
// kk <= 256, row offsets clamped to [0, nnz].  resid: per
// workgroup (csr_resid_blocks(rows) of them) the FP64 sums of a^2 and
// a (U V)_ij over the nonzeros; finish: the relative residual from those and
// the Grams GU = U^T U, GV = V V^T (r x r).
size_t csr_sort_temp_bytes(int nnz, int n);
template <typename T>
hipError_t launch_csr_transpose(const int64_t* rowptr, const int32_t* col, const T* val, int m, int n, int64_t nnz,
                                int64_t* trow, int32_t* tcol, T* tval, int32_t* keys, int32_t* perm,
                                int32_t* keys_out, int32_t* perm_out, void* tmp, size_t tmp_bytes, int* bad,
                                hipStream_t st);
template <typename T>
hipError_t launch_csr_spmm(const int64_t* rowptr, const int32_t* col, const T* val, int rows, int cols, int64_t nnz,
                           const T* X, int kk, T* Y, hipStream_t st);
int csr_resid_blocks(int rows);
template <typename T>
hipError_t launch_csr_resid(const int64_t* rowptr, const int32_t* col, const T* val, int rows, int cols, int64_t nnz,
                            const T* U, const T* Vt, int r, double* part, hipStream_t st);
hipError_t launch_csr_resid_finish(const double* part, int parts, const double* GU, const double* GV, int r,
                                   double* out, hipStream_t st);
// dst += src (rows x cols, leading dimensions lds / ldd)
template <typename T>
hipError_t launch_add2d(const T* src, int64_t lds, T* dst, int64_t ldd, int rows, int cols, hipStream_t st);
template <typename T>
hipError_t launch_residual(const T* A, int64_t lda, int m, int n, const T* U, int ldu, const T* Vt,
                           int ldv, int r, double* partial, int parts, hipStream_t st);
hipError_t launch_residual_finish(const double* partial, int parts, double* out, hipStream_t st);
// Partial count of the residual launch for an m x n A.
int residual_blocks(int m, int n);
hipError_t launch_flags_to_stats(const int* flags, int nflags, double* out, hipStream_t st);
// SNMF right factor (k_nnls.hip): Bt = B^T (n x k FP64, ld ldbt), K (r
// column indices), H (r x n, ld ldh) = per-column NNLS solutions; Cr: n x r
// workspace; info: 3 zeroed words (columns not converged, most outer steps,
// invalid indices).
// One half-step of alternating NNLS (k_nnls.hip): for every row i of F
// (rows x r, ld ldf, the current values are the warm start),
//   F[i] = argmin_{h >= 0} 1/2 h^T G h - c^T h,
//   c = C^T B1[i] (C k1 x r, FP64) or c = B1[i] (C == nullptr; ld ldb1),
// G (r x r, FP64) shared; the new rows are also copied to Op (ld ldop) when
// it is set.  With H = G^-1 (checked, *hok), a free system with fewer bound
// than free variables is solved through H (the Schur complement of the
// bound block) instead of G.  Block principal pivoting from the support of
// the current row;
// info[0] += rows that needed more than 5 r exchanges (or broke down),
// info[1] = max(info[1], exchanges).
struct AnlsArgs {
  int rows, r, k1;
  const void* B1;
  int64_t ldb1;
  const double* C;
  const double* G;
  const double* H;     // G^-1 (r x r) or nullptr; used when *hok != 0
  const int* hok;
  void* F;
  int64_t ldf;
  void* Op;
  int64_t ldop;
  int* info;
};
template <typename T>
hipError_t launch_anls_rows(const AnlsArgs& a, hipStream_t st);
hipError_t launch_add_count(const int* src, int* dst, hipStream_t st);
hipError_t launch_snmf_nnls(const double* Bt, int64_t ldbt, int n, int k, int r, const int64_t* K, double* Cr,
                            double* H, int64_t ldh, int* info, hipStream_t st);
// Fixed per-device scratch of cnmf_spa_noalloc (k_scratch.hip): bytes, the
// address lookup (once per device, with that device current) and the
// device address found (NULL before the lookup).
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch(int device);
hipError_t launch_spa_step(double* Bt, int n, int k, int ldb, int t, int64_t* K, double* score,
                           double* u, double* wg_best, int64_t* wg_idx, unsigned* counter,
                           int nblocks, hipStream_t st);

}  // namespace cnmf
