/*
 * cnmf.h -- C ABI of the MI355X (gfx950) compressed-NMF library.
 *
 * Method: Tepper & Sapiro, "Compressed Nonnegative Matrix Factorization is
 * Fast and Accurate" (arXiv:1505.04650).
 *   - Structured random compression (Section 2, Alg. 1): a Gaussian range
 *     finder orth((A A^T)^q A Omega), computed as re-orthonormalised
 *     subspace iteration, orthonormalised by CholeskyQR2 in FP64.
 *   - Two-sided compression and the small sketches (Section 3): L (m x k),
 *     R (k x n), B = L^T A (k x n), At = L^T A R^T (k x k), Ac = A R^T (m x k).
 *   - Compressed NMF: ADMM (Appendix B, Alg. 3) and alternating
 *     multiplicative updates (Section 3, Alg. 2 with the semi-NMF rule of
 *     Ding et al. 2010, Eq. 8); the same solvers with L = I, R = I are the
 *     uncompressed comparators.
 *   - Compressed separable NMF (Section 4, Alg. SNMF): SPA column
 *     selection on B = Q^T A.
 *
 * Conventions shared by every entry point
 *   - Every matrix is ROW-MAJOR with an explicit leading dimension (in
 *     elements).  Pointers named *_dev are DEVICE pointers (memory the
 *     caller allocated on the handle's device); all others are host.
 *   - The caller owns A and every output buffer; the library never frees or
 *     writes caller memory other than the declared outputs.  A is read-only.
 *   - Work is enqueued on the HIP stream given to cnmf_create.  Calls do not
 *     synchronise the stream; outputs (including device scalars) are valid
 *     once that stream has completed the call's work.
 *   - Errors: invalid shapes / parameters return CNMF_EINVAL before anything
 *     is enqueued, with outputs untouched.  A HIP launch or allocation error
 *     returns CNMF_EDEVICE / CNMF_ENOMEM.  cnmf_last_error gives a message
 *     for the last failing call on a handle.  A handle is not thread safe.
 *   - Random numbers: the Gaussian test matrices of Alg. 1 are either
 *     INPUTS (omega_*) or drawn on the device from `seed` by the
 *     counter-based generator of cnmf_gaussian, so results are a pure
 *     function of (A, Omega or seed, initial factors, params).
 */
#ifndef CNMF_H_
#define CNMF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CNMF_OK = 0,
  CNMF_EINVAL = -1,      /* invalid argument (detected before any launch)     */
  CNMF_ENOMEM = -2,      /* device workspace could not be allocated           */
  CNMF_EDEVICE = -3,     /* HIP runtime / launch error                        */
  CNMF_EBREAKDOWN = -4,  /* orthonormalisation breakdown the fallback did not
                            resolve, or an NNLS problem of CNMF_ANLS that did
                            not finish (reported by cnmf_synchronize)        */
  CNMF_ENOTSUP = -5,     /* valid but unsupported size / precision combination */
  CNMF_EBUSY = -6
} cnmf_status;

typedef enum {
  CNMF_F64 = 0,
  CNMF_F32 = 1,
  CNMF_BF16 = 2,
  CNMF_FP8_E4M3 = 3
} cnmf_dtype;

enum { CNMF_LEFT = 1, CNMF_RIGHT = 2, CNMF_BOTH = 3 };

enum {
  CNMF_ADMM = 0,       /* compressed ADMM, Appendix B Alg. 3                    */
  CNMF_MU = 1,         /* compressed alternating MU, Section 3 Alg. 2           */
  CNMF_ADMM_FULL = 2,  /* Alg. 3 with L = I_m, R = I_n (uncompressed ADMM)      */
  CNMF_MU_FULL = 3,    /* Alg. 2 with L = I_m, R = I_n (uncompressed MU)        */
  CNMF_ANLS = 4,       /* compressed alternating NNLS, Section 3
                          Eq. alternateLS_nmf_compressed (active set)         */
  CNMF_ANLS_FULL = 5   /* the same with L = I_m, R = I_n (Eq. alternateLS_nmf) */
};

typedef struct cnmf_handle cnmf_handle;

/* Create a handle bound to HIP device `device` and the HIP stream
 * `hip_stream` (a hipStream_t; NULL = the null stream).  `workspace_limit`
 * caps the device workspace the handle may allocate (0 = no cap).  The
 * workspace is allocated lazily on the first call that needs it, grown as
 * needed, and freed by cnmf_destroy. */
cnmf_status cnmf_create(int device, void* hip_stream, size_t workspace_limit, cnmf_handle** out);
cnmf_status cnmf_destroy(cnmf_handle* h);
/* Message for the last failing call on `h` (never NULL; "" if none).
 * With h == NULL: the message of the last failing call without a handle. */
const char* cnmf_last_error(const cnmf_handle* h);
const char* cnmf_status_string(cnmf_status s);
/* Library version string, e.g. "cnmf-mi355x 0.1". */
const char* cnmf_version(void);
/* Wait for the work enqueued on the handle's stream.  Returns CNMF_EDEVICE
 * for an asynchronous HIP fault, or if a compressed-ADMM solve of a
 * cnmf_factorize enqueued since the previous cnmf_synchronize gave up (after
 * about two seconds) waiting for the partial sums formed by other
 * workgroups of its own launch (its factors are then not valid; the count
 * is cleared), CNMF_EBREAKDOWN if a call enqueued since
 * the previous cnmf_synchronize hit an orthonormalisation breakdown that the
 * fallback could not resolve (see cnmf_sketch_desc) or an alternating-NNLS
 * problem that did not finish (see cnmf_factorize_desc; the count is then
 * cleared), CNMF_OK otherwise. */
cnmf_status cnmf_synchronize(cnmf_handle* h);

/* Gaussian test matrix of Alg. 1 (Section 2: "draw a Gaussian random
 * matrix"), as the sketches draw it: out_dev (device, rows x cols FP64,
 * row-major, leading dimension ld >= cols) receives iid N(0, 1) entries.
 * Generator: Philox4x32-10 (Salmon et al., SC'11) with the counter
 * (col / 2, row, matrix_id, 0) and the key (seed mod 2^32, seed / 2^32);
 * the output words x0..x3 give u1 = ((x1:x0 >> 11) + 1) 2^-53 and
 * u2 = (x3:x2 >> 11) 2^-53, and the Box-Muller pair
 * sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) fills columns (even, odd).
 * Entry (i, j) depends only on (seed, matrix_id, i, j).  Errors:
 * CNMF_EINVAL for a NULL pointer, negative sizes or ld < cols; rows above
 * 2^30: CNMF_ENOTSUP. */
cnmf_status cnmf_gaussian(cnmf_handle* h, uint64_t seed, int32_t matrix_id, int64_t rows, int32_t cols,
                          double* out_dev, int64_t ld);

/* SRHT test matrix (Section 2, remark after Thm. 3: subsampled randomized
 * Hadamard transform; Halko, Martinsson and Tropp 2011, Sec. 4.6), as the
 * sketches draw it for test_matrix = CNMF_TEST_SRHT: out_dev (device,
 * rows x cols FP64, ld >= cols) = D H S / sqrt(cols) with p =
 * 2^ceil(log2 rows), D = diag(d_i) random signs, H the p x p Walsh-Hadamard
 * (Sylvester) matrix with entries (-1)^popcount(i & j), S the selection of
 * cols distinct columns s_c; entry (i, c) = d_i (-1)^popcount(i & s_c) /
 * sqrt(cols).  Randomness from the same Philox4x32-10 as cnmf_gaussian:
 * d_i = -1 when bit 0 of output word 0 of the counter (0, i, matrix_id, 1)
 * is set; s_c (c = 0, 1, ...) is the first of the words 0 of the counters
 * (c, t, matrix_id, 2), t = 0, 1, ..., masked to [0, p), not taken by an
 * earlier column, and after 64 taken draws the first free index at or
 * after the last draw (cyclically).  Errors: CNMF_EINVAL for a NULL
 * pointer, rows < 1, cols outside [1, min(128, p)] or ld < cols. */
cnmf_status cnmf_srht(cnmf_handle* h, uint64_t seed, int32_t matrix_id, int64_t rows, int32_t cols, double* out_dev,
                      int64_t ld);

/* ---------------------------------------------------------------------------
 * Input matrix A (Section 1, problem (nmf)): m x n, dtype CNMF_F64 or
 * CNMF_F32, in one of three formats:
 *   CNMF_DENSE (0): row-major on the device, lda >= n, at data_dev.
 *   CNMF_DENSE_HOST (1): row-major in host memory, lda >= n, at data_dev
 *     (a host pointer; pinned memory, hipHostMalloc, lets the copies
 *     overlap the passes).  For matrices larger than device memory (Section
 *     2.1, algorithmic solutions for big data): every pass streams A through
 *     the device in blocks of block_rows rows (0 = about 64 MiB per block),
 *     two blocks in flight; only the k-column sketches live on the device.
 *     The host buffer must stay unchanged until the call's work has run.
 *     Passes in F32 / F64 only (no reduced-precision copies of A).
 *   CNMF_CSR (2): sparse on the device, compressed rows: rowptr_dev (m + 1
 *     int64 offsets, rowptr[0] = 0, nondecreasing, rowptr[m] = nnz),
 *     colind_dev (nnz int32 column indices in [0, n), ascending within each
 *     row) and the nnz values at data_dev (both may be NULL when nnz = 0);
 *     lda is ignored.  The passes
 *     multiply with A and A^T directly (the transpose is formed once per
 *     call in the workspace); passes in F32 / F64 only.
 * A is never written.
 * ------------------------------------------------------------------------- */
enum { CNMF_DENSE = 0, CNMF_DENSE_HOST = 1, CNMF_CSR = 2 };
typedef struct {
  const void* data_dev;
  cnmf_dtype dtype;
  int64_t m, n, lda;
  int32_t format;
  int32_t reserved;
  const int64_t* rowptr_dev;
  const int32_t* colind_dev;
  int64_t nnz;
  int64_t block_rows;
} cnmf_input;

/* Sketch parameters (Alg. 1 inputs: target rank r, oversampling r_ov with
 * k = r + r_ov, exponent w = q).  Valid: 1 <= r < k <= min(m, n), k <= 128,
 * q >= 0.  `sides` selects L (CNMF_LEFT), R (CNMF_RIGHT) or both.
 * pass_dtype: precision of the GEMM operands of the power-iteration passes
 *   (the 2q passes before the last range product of each chain):
 *   CNMF_F64 (needs F64 input: everything in FP64), CNMF_F32, CNMF_BF16 or
 *   CNMF_FP8_E4M3 (FP32 input; accumulation is FP32).  For BF16 / FP8, A
 *   is converted once per call into workspace copies of A and A^T (round
 *   to nearest even; FP8 E4M3 with one FP32 scale max|tile| / 448 per
 *   128 x 128 tile of A, each tile's partial product rescaled in FP32), and
 *   each pass operand column is rounded to the pass type (FP8: after
 *   scaling by a power of two, which the orthonormalisation absorbs).
 * final_dtype: precision of the last range pass of each chain and of the
 *   B / Ac pass (CNMF_F64 with F64 input; CNMF_F32 or CNMF_BF16 otherwise;
 *   CNMF_FP8_E4M3 returns CNMF_ENOTSUP: B and Ac are used unscaled).
 *   The workspace grows by 4 m n bytes for BF16 copies and 2 m n bytes
 *   for FP8 copies.
 * Orthonormalisation (CholeskyQR2) always runs in FP64.
 * Orthonormalisation breakdown (k > rank A makes Y rank deficient, the
 *   case Section 2's bound covers with sigma_{r+1} = 0, and plain
 *   CholeskyQR then fails): the first CholeskyQR pass treats a column whose
 *   pivot is <= 1e-14 max diag(Y^T Y) as dependent on the earlier ones, the
 *   second pass does the same for pivots <= 1e-8 max diag(Q1^T Q1) (a
 *   dependent column that the first pass's Gram could not tell apart);
 *   each such column is replaced by a fresh Gaussian column (test matrix
 *   16 + 4 p + side, or 16 + 4 p + 2 + side in the second pass, for the
 *   product of pass p, drawn from `seed`), and a third CholeskyQR pass runs
 *   when the second one replaced a column.  range(Q) then contains range(Y)
 *   and Q^T Q = I.  Replaced columns are counted in stats[2]; a breakdown
 *   the fallback cannot resolve (a NaN pivot, or a rank-deficient third
 *   pass) is counted in stats[3] and makes the next cnmf_synchronize
 *   return CNMF_EBREAKDOWN.
 * seed: key of the counter-based generator (cnmf_gaussian) for the test
 *   matrices drawn on the device and for completion columns.
 * omega_left_dev:  n x k FP64, row-major (ld = k): test matrix for A, or
 *   NULL to draw it on the device (cnmf_gaussian matrix id 0 under seed).
 * omega_right_dev: m x k FP64, row-major (ld = k): test matrix for A^T
 *   (used when CNMF_RIGHT is set), or NULL to draw it (matrix id 1).
 * test_matrix: the kind drawn for a NULL omega: CNMF_TEST_GAUSSIAN (0,
 *   cnmf_gaussian) or CNMF_TEST_SRHT (1, cnmf_srht: the subsampled
 *   randomized Hadamard transform Section 2 names as an alternative). */
enum { CNMF_TEST_GAUSSIAN = 0, CNMF_TEST_SRHT = 1 };
typedef struct {
  int32_t r, k, q, sides;
  cnmf_dtype pass_dtype;
  cnmf_dtype final_dtype;
  uint64_t seed;
  const double* omega_left_dev;
  const double* omega_right_dev;
  int32_t test_matrix;
  int32_t reserved;
} cnmf_sketch_desc;

/* Sketch outputs.  Every pointer may be NULL (= not wanted).  Element type
 * is FP64 when pass_dtype is CNMF_F64, FP32 otherwise; all row-major with
 * tight leading dimensions:
 *   L_dev  m x k   (orthonormal columns)     -- needs CNMF_LEFT
 *   R_dev  k x n   (orthonormal rows)        -- needs CNMF_RIGHT
 *   B_dev  k x n   B = L^T A                 -- needs CNMF_LEFT
 *   At_dev k x k   At = L^T A R^T            -- needs both sides
 *   Ac_dev m x k   Ac = A R^T                -- needs CNMF_RIGHT (one extra pass)
 *   stats_dev FP64[4]: max|L^T L - I|, max|R R^T - I|, number of
 *     CholeskyQR breakdowns repaired by the fallback, number left
 *     unresolved. */
typedef struct {
  void* L_dev;
  void* R_dev;
  void* B_dev;
  void* At_dev;
  void* Ac_dev;
  double* stats_dev;
} cnmf_sketch_out;

cnmf_status cnmf_sketch(cnmf_handle* h, const cnmf_input* A, const cnmf_sketch_desc* d,
                        cnmf_sketch_out* out);

/* Factorisation parameters.  method: CNMF_ADMM / CNMF_MU / CNMF_ANLS use
 * the two-sided sketch `sk` (sides must be CNMF_BOTH); the *_FULL methods
 * ignore `sk` except for sk.r and run on A itself.  iters: fixed number of
 * iterations (no early stop).  lambda, phi > 0: ADMM penalties; xi > 0:
 * ADMM step (1 in the paper).  mu_eps >= 0: added to every MU denominator.
 * U0_dev (m x r) and V0_dev (r x n): FP64 initial factors (Alg. 2 / Alg. 3
 * "Initialize"), row-major, required.  CNMF_ANLS / CNMF_ANLS_FULL minimise
 * every half-step to the end (each row of U against (V R^T)^T, each column
 * of V against L^T U, as nonnegative least-squares problems solved on their
 * normal equations in FP64 by block principal pivoting, an active-set
 * method); the iterates depend on V0 only (U0 gives the first half-step's
 * starting active sets).  A problem that needs more than 5 r exchanges, or
 * whose free system breaks down, keeps its last iterate clamped at 0 and is
 * counted: cnmf_synchronize then returns CNMF_EBREAKDOWN.
 * Limits: r <= 64 (CNMF_ENOTSUP
 * otherwise); CNMF_ADMM solves its two r x r systems per iteration in one
 * workgroup whose LDS must hold three k x r FP64 blocks and the r x r
 * system, so it also needs k <= 112 when r > 48 (CNMF_ENOTSUP). */
typedef struct {
  cnmf_sketch_desc sk;
  int32_t method;
  int32_t iters;
  double lambda, phi, xi;
  double mu_eps;
  const double* U0_dev;
  const double* V0_dev;
} cnmf_factorize_desc;

/* Outputs (NULL = not wanted): U_dev m x r, V_dev r x n in the handle's
 * accumulation precision (FP64 for F64 passes, FP32 otherwise);
 * rel_residual_dev: FP64 scalar ||A - U V||_F / ||A||_F (one more pass over
 * A, accumulated in FP64).  `sk_out` optionally receives the sketches. */
typedef struct {
  void* U_dev;
  void* V_dev;
  double* rel_residual_dev;
  cnmf_sketch_out sk_out;
} cnmf_factorize_out;

cnmf_status cnmf_factorize(cnmf_handle* h, const cnmf_input* A, const cnmf_factorize_desc* d,
                           cnmf_factorize_out* out);

/* The same factorisation captured once as a HIP graph and replayed: every
 * launch of one cnmf_factorize call (with these arguments) is recorded on
 * the handle's stream, with a workspace owned by the graph; each
 * cnmf_graph_launch then reruns the whole factorisation on the handle's
 * stream, reading the buffers named at capture (A, U0, V0, the test
 * matrices) as they are at replay time and writing the same outputs.  For
 * factorisations short enough that launch latency matters (the iterations
 * are many small launches).  The buffers must stay allocated while the graph
 * exists; replays on one handle are ordered like any other call.  Errors:
 * as cnmf_factorize; CNMF_EINVAL for a handle on the null stream (capture
 * needs a created stream); CNMF_ENOTSUP for inputs in host memory (they use
 * a second stream); CNMF_EDEVICE when the runtime refuses the capture. */
typedef struct cnmf_graph cnmf_graph;
cnmf_status cnmf_factorize_capture(cnmf_handle* h, const cnmf_input* A, const cnmf_factorize_desc* d,
                                   const cnmf_factorize_out* out, cnmf_graph** graph);
cnmf_status cnmf_graph_launch(cnmf_graph* graph);
/* Waits for the handle's stream, then frees the graph and its workspace. */
cnmf_status cnmf_graph_destroy(cnmf_graph* graph);

/* Separable NMF column selection (Section 4, Alg. SNMF, steps 1-2): left
 * sketch Q of A (or both sides when d->sides == CNMF_BOTH), B = Q^T A, then
 * SPA on the columns of B in FP64: r times pick the column of largest
 * squared norm (lowest index on ties) and project it out.
 * K_dev: int64[r] device, 0-based column indices in selection order.
 * score_dev: optional FP64[r] device, the selected squared norms.
 * B_dev: optional k x n output of B (FP32, or FP64 for F64 passes). */
cnmf_status snmf_select(cnmf_handle* h, const cnmf_input* A, const cnmf_sketch_desc* d,
                        int64_t* K_dev, double* score_dev, void* B_dev);

/* SPA alone on a given B (k x n, row-major, ld >= n, FP64 or FP32 device
 * matrix), writing r indices to K_dev (int64) and optionally the scores. */
cnmf_status cnmf_spa(cnmf_handle* h, const void* B_dev, cnmf_dtype dtype, int64_t k, int64_t n,
                     int64_t ldb, int32_t r, int64_t* K_dev, double* score_dev);

/* Right factor of compressed separable NMF (Section 4, Alg. SNMF, last
 * step, Eq. snmf_right_factor_col): for every column j of B (k x n,
 * row-major, ld ldb >= n, FP64 or FP32 device matrix; B = Q^T A from
 * snmf_select) and the r selected columns K_dev (int64 device, 0-based),
 *   H[:, j] = argmin_{h >= 0} ||B[:, j] - B[:, K] h||_2,
 * written to H_dev (r x n FP64 device, row-major, ld ldh >= n).  Each
 * column is solved exactly (to rounding) by the Lawson-Hanson active-set
 * method on the normal equations G h = B[:, K]^T B[:, j], G = B[:, K]^T
 * B[:, K], in FP64, one wave per column; a variable is freed while its dual
 * exceeds 1e-13 max_i |(B[:, K]^T B[:, j])_i|.  info_dev (optional device
 * int32[3]): columns that needed more than 3 r active-set steps (their last
 * feasible iterate is returned), the most steps any column took, and the
 * number of entries of K outside [0, n) (treated as zero columns).
 * B[:, K] must have full column rank (SPA's selection does).  Limits:
 * k <= 128, r <= 64 (CNMF_ENOTSUP); 1 <= r <= min(k, n) (CNMF_EINVAL). */
cnmf_status snmf_nnls(cnmf_handle* h, const void* B_dev, cnmf_dtype dtype, int64_t k, int64_t n, int64_t ldb,
                      int32_t r, const int64_t* K_dev, double* H_dev, int64_t ldh, int32_t* info_dev);

/* cnmf_spa for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and results as cnmf_spa, with its working storage (B^T
 * in FP64, the unit pivot, per-block winners: about (k + 2) n doubles) in a
 * fixed 32 MiB device array that the library holds on every GPU it runs on
 * until the process ends; no call allocates or frees anything.  The array's
 * address is looked up when a handle is created on a device.  Inputs and
 * outputs as for cnmf_spa.  Errors: as cnmf_spa; CNMF_ENOTSUP when the
 * working storage would exceed the 32 MiB (use cnmf_spa).  Every call on a
 * GPU shares that GPU's array (it keeps the last call's contents; nothing in
 * it needs clearing): calls that may overlap on one GPU (other streams or
 * host threads) race and must be serialised by the caller. */
cnmf_status cnmf_spa_noalloc(cnmf_handle* h, const void* B_dev, cnmf_dtype dtype, int64_t k, int64_t n,
                             int64_t ldb, int32_t r, int64_t* K_dev, double* score_dev);

/* One streaming pass of the range finder (Alg. 1, the product step):
 *   trans == 0: Y = A X    X is n x kx, Y is m x kx
 *   trans == 1: Y = A^T X  X is m x kx, Y is n x kx
 * X and Y are device matrices of A's dtype, row-major with ld = kx;
 * 1 <= kx <= 128.  The product reads A once; it is the kernel every pass of
 * cnmf_sketch runs. */
cnmf_status cnmf_range_product(cnmf_handle* h, const cnmf_input* A, int trans, const void* X_dev, int32_t kx,
                               void* Y_dev);

/* The same pass with reduced-precision operands (Alg. 1 product step in the
 * precision form of the passes): A (F32 input) is converted to BF16 or FP8
 * E4M3 exactly as cnmf_sketch converts it, X_dev (FP64, cols x kx, ld = kx,
 * cols = n for trans == 0, m for trans == 1) is rounded per column as a pass
 * operand (FP8: scaled by the largest power of two s_c with
 * max|X[:, c]| s_c <= 256, then rounded), the product is accumulated in
 * FP32 and Y_dev (FP32, rows_out x kx, ld = kx) is returned with the FP8
 * column scales divided out.  pass_dtype must be CNMF_BF16 or
 * CNMF_FP8_E4M3. */
cnmf_status cnmf_range_product_lowp(cnmf_handle* h, const cnmf_input* A, int trans, cnmf_dtype pass_dtype,
                                    const double* X_dev, int32_t kx, float* Y_dev);

/* Device workspace (bytes) that cnmf_factorize (or, with iters = 0 and
 * method CNMF_ADMM, cnmf_sketch) needs for an m x n input.  Host only; no
 * handle or GPU required. */
cnmf_status cnmf_workspace_bytes(int64_t m, int64_t n, const cnmf_factorize_desc* d, size_t* bytes);

/* Per-stage accounting of the last call on `h`.  Stages:
 *   0 precision conversion of A, 1 A X range passes, 2 A^T Z range passes,
 *   3 orthonormalisation and small sketches, 4 NMF iterations, 5 residual,
 *   6 SPA.
 * cnmf_stage_ms: device time in milliseconds from HIP events recorded on the
 *   handle's stream around each span (only while timing is enabled with
 *   cnmf_set_timing; NaN otherwise or if the stage did not run).  Reading it
 *   waits for the events of the last call.
 * cnmf_stage_flops: algorithmic flop count of the stage (for the range passes
 *   2 m n k per chain block, padding excluded).
 * cnmf_stage_launches: number of spans (for the range passes: kernel
 *   launches). */
cnmf_status cnmf_set_timing(cnmf_handle* h, int enable);
double cnmf_stage_ms(cnmf_handle* h, int stage);
double cnmf_stage_flops(cnmf_handle* h, int stage);
int cnmf_stage_launches(cnmf_handle* h, int stage);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of factorisation requests on one GPU.
 *
 * cnmf_server_start creates a server with a device arena of
 * hbm_budget_bytes (allocated once) from which every admitted request gets
 * its workspace block, `workers` worker streams (1..3) for the per-request
 * phases and one stream for the batched iterations, and a dispatcher thread
 * that owns all of the server's launches.
 *
 * A request is what cnmf_factorize takes.  Lifecycle: queued (arrival
 * order) -> admitted when its workspace footprint fits in the arena and one
 * of max_batch + 2 workers in-flight slots is free (a waiting head of the
 * queue may be passed by smaller requests only while the free bytes left
 * still cover it, at most 64 times) -> prologue on a worker stream (Alg. 1
 * sketch, small sketches, initial state) -> for FP32 compressed ADMM
 * (CNMF_ADMM, F32 input, iters > 0): member of the batch, where one step
 * advances every member by one iteration of Appendix B Alg. 3 (a copy of
 * the step's descriptor table and three descriptor-driven launches covering
 * all members, at most max_batch; optionally a replayed graph, see
 * CNMF_SERVER_GRAPHS) -> epilogue (U, V, FP64
 * residual, sketch outputs) on a worker stream -> done.  Other requests
 * (MU, uncompressed, FP64) run whole on a worker stream.  Each member runs
 * the same per-request code as cnmf_factorize, so its results equal those of
 * cnmf_factorize on the same inputs, whatever else is in the batch.
 *
 * Ownership: A and every output buffer belong to the caller and must stay
 * valid until the ticket is done.  The inputs may be produced on
 * `producer_stream` (a hipStream_t, NULL = null stream): the request's work
 * is ordered after the work enqueued there before the submit call.
 * Errors: cnmf_server_submit validates like cnmf_factorize (CNMF_EINVAL
 * before anything is enqueued) and returns CNMF_ENOMEM for a footprint
 * above the whole budget; a failure later in the request is reported by
 * cnmf_server_poll (status, message).  cnmf_server_last_error gives the text
 * of the calling thread's last failing server call.  All calls are thread
 * safe; cnmf_server_stop drains every queued and in-flight request, then
 * frees the server (tickets are invalid afterwards).
 * ------------------------------------------------------------------------- */
typedef struct cnmf_server cnmf_server;

typedef struct {
  int32_t device;
  int32_t max_batch;          /* members of a batched step, 1..4096          */
  int32_t workers;            /* worker streams, 1..3                        */
  int32_t flags;              /* CNMF_SERVER_* bits, 0 = defaults            */
  uint64_t hbm_budget_bytes;  /* device arena for request workspaces         */
} cnmf_server_config;
/* CNMF_SERVER_GRAPHS: issue every batched step as the replay of a captured
 * graph (the descriptor copy and three fixed-grid kernels whose workgroups
 * take the step's blocks from counters in the descriptor; one graph per
 * descriptor slot and shape class) instead of direct launches whose grids
 * are sized to the batch.  Both run the same per-block code, so the results
 * are the same bit for bit; which is faster depends on the mix (direct
 * launches are the default).
 * CNMF_SERVER_ONE_STEP: at most one batched step in flight instead of two
 * (the next step is built when the previous one has ended, so it gathers
 * the requests whose prologues finished meanwhile). */
enum { CNMF_SERVER_GRAPHS = 1, CNMF_SERVER_ONE_STEP = 2 };

typedef struct {
  int32_t state;              /* 0 queued, 1 prologue, 2 ready, 3 in batch,
                                 4 epilogue, 5 done                          */
  int32_t done;               /* state == 5                                  */
  cnmf_status status;         /* result once done                            */
  int32_t reserved;
  double queue_ms;            /* submit -> admission (so far if queued)      */
  double total_ms;            /* submit -> done (so far if not done)         */
  char message[192];          /* error text when status != CNMF_OK           */
} cnmf_ticket_info;

typedef struct {
  int64_t submitted, completed, failed;
  int64_t batch_steps;        /* batched launches of the iteration step      */
  int64_t batched_iterations; /* request-iterations they advanced            */
  int64_t max_batch_seen;     /* largest batch                               */
  int64_t graph_replays;      /* steps issued as a replay of a captured graph */
  int64_t graphs_built;       /* graphs captured (per descriptor slot and
                                 shape class: k, r rounded up to 16)         */
  int64_t queued, in_flight;
  uint64_t arena_bytes, arena_free_bytes, peak_arena_bytes;
} cnmf_server_stats;

cnmf_status cnmf_server_start(const cnmf_server_config* cfg, cnmf_server** out);
cnmf_status cnmf_server_submit(cnmf_server* s, const cnmf_input* A, const cnmf_factorize_desc* d,
                               const cnmf_factorize_out* out, void* producer_stream, uint64_t* ticket);
cnmf_status cnmf_server_poll(cnmf_server* s, uint64_t ticket, cnmf_ticket_info* info);
/* Forget a done ticket (CNMF_EBUSY if it is not done). */
cnmf_status cnmf_server_release(cnmf_server* s, uint64_t ticket);
cnmf_status cnmf_server_get_stats(cnmf_server* s, cnmf_server_stats* out);
cnmf_status cnmf_server_stop(cnmf_server* s);
const char* cnmf_server_last_error(void);

/* Host-only replay of the server's admission policy (no GPU needed):
 * request i arrives at arrival_ms[i] (sorted), needs bytes[i] of the arena
 * and, once admitted, holds its slot and block for service_ms[i].  Writes
 * admit_ms[i] and done_ms[i] (-1 for a request above the budget) and the
 * peak arena use.  For testing and capacity planning. */
cnmf_status cnmf_server_simulate(int32_t nreq, const double* arrival_ms, const uint64_t* bytes,
                                 const double* service_ms, uint64_t budget, int32_t max_inflight,
                                 double* admit_ms, double* done_ms, uint64_t* peak_bytes);

#ifdef __cplusplus
}
#endif

#endif /* CNMF_H_ */
