// Host runtime of the compressed-NMF library: handle, argument checks,
// workspace planning and the launch sequences of the hot path.
//
// Range finder schedule (Alg. 1 on A and on A^T, Section 3).  Each chain
// alternates products with A and A^T, with an orthonormalisation after every
// product (re-orthonormalised subspace iteration):
//   left chain L:  A Omega_L, A^T Q, A Q, ..., A Q      (2q + 1 products)
//   right chain R: A^T Omega_R, A Q, A^T Q, ..., A^T Q  (2q + 1 products)
// The right chain starts one pass later than the left one, so in every pass
// both chains multiply by the SAME operator (A or A^T) and their operands
// sit side by side: one streaming read of A serves both.  The pass after
// L's last product multiplies A^T by [L | Q_R]: its left block is
// A^T L = B^T (the small sketch B = L^T A), its right block is R's last
// range sample.  Passes: 2q + 2 for two-sided or left-only sketches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/cnmf.h"
#include "cnmf_internal.hpp"

using namespace cnmf;

static thread_local std::string g_noh_err;

constexpr int kStages = 8;

struct cnmf_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t limit = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ext_ws = false;  // ws belongs to the caller (serving arena): never freed or grown
  // device word: CholeskyQR2 breakdowns the fallback could not resolve since
  // the last cnmf_synchronize (allocated at creation; serving handles: none)
  int* unresolved_dev = nullptr;
  // inputs in host memory: a copy stream and the staging events (created on
  // first use)
  hipStream_t copy_stream = nullptr;
  hipEvent_t stage_ready[2] = {nullptr, nullptr};
  hipEvent_t stage_free[2] = {nullptr, nullptr};
  std::string err;
  // per-stage timing of the last call (HIP events on the handle's stream)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_next = 0;
  struct Span {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Span> spans;
  bool resolved = true;
  double stage_ms[kStages];
  double stage_flops[kStages];
  int stage_count[kStages];
};

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline int ru16(int x) { return (x + 15) / 16 * 16; }

cnmf_status fail(cnmf_handle* h, cnmf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h)
    h->err = buf;
  else
    g_noh_err = buf;
  return s;
}

#define HIPCHK(h, expr)                                                                          \
  do {                                                                                           \
    hipError_t _e = (expr);                                                                      \
    if (_e != hipSuccess)                                                                        \
      return fail(h, CNMF_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                  __LINE__);                                                                     \
  } while (0)

// Bump allocator over the handle's workspace (or a dry run for sizing).
struct Arena {
  char* base;
  size_t off = 0;
  explicit Arena(char* b) : base(b) {}
  template <typename T>
  T* take(size_t count) {
    size_t bytes = align_up(count * sizeof(T));
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

size_t elem_size(cnmf_dtype d) {
  switch (d) {
    case CNMF_F64: return 8;
    case CNMF_F32: return 4;
    case CNMF_BF16: return 2;
    case CNMF_FP8_E4M3: return 1;
  }
  return 0;
}

// -------------------------------------------------------------------------
// Pass plan
// -------------------------------------------------------------------------
enum BlockKind { L_RANGE = 0, R_RANGE = 1, L_B = 2, R_AC = 3 };
struct Block {
  BlockKind kind;
  int step;  // chain step (RANGE)
  int col0;
};
struct Pass {
  bool dirN;  // true: A X ; false: A^T Z
  int kk;
  std::vector<Block> blocks;
  bool final_prec;
  cnmf_dtype prec;  // precision of the pass GEMM inputs
};

inline bool is_lowp(cnmf_dtype d) { return d == CNMF_BF16 || d == CNMF_FP8_E4M3; }
inline int lowp_es(cnmf_dtype d) { return d == CNMF_BF16 ? 2 : 1; }

// Passes before 2q are power-iteration passes and run in pass_dtype; the last
// range product of each chain, B = L^T A and Ac = A R^T run in final_dtype.
std::vector<Pass> plan_passes(int k, int q, int sides, bool want_ac, cnmf_dtype pass_dtype,
                              cnmf_dtype final_dtype) {
  const bool L = sides & CNMF_LEFT, R = sides & CNMF_RIGHT;
  const int nsteps = 2 * q + 1;
  const int rstart = L ? 1 : 0;
  std::vector<Pass> out;
  int p = 0;
  for (;; ++p) {
    Pass ps;
    ps.final_prec = p >= 2 * q;
    int col = 0;
    bool any = false;
    bool dirset = false;
    if (L) {
      if (p < nsteps) {
        ps.blocks.push_back({L_RANGE, p, col});
        col += k;
        ps.dirN = (p % 2 == 0);
        dirset = any = true;
      } else if (p == nsteps) {
        ps.blocks.push_back({L_B, 0, col});
        col += k;
        ps.dirN = false;
        dirset = any = true;
      }
    }
    if (R) {
      int s = p - rstart;
      if (s >= 0 && s < nsteps) {
        ps.blocks.push_back({R_RANGE, s, col});
        col += k;
        bool d = (s % 2 == 1);
        if (dirset && d != ps.dirN) return {};  // schedule invariant
        ps.dirN = d;
        dirset = any = true;
      } else if (s == nsteps && want_ac) {
        // Ac = A R^T after R's last product (an A pass)
        if (dirset && !ps.dirN) {
          // cannot share with an A^T block; emit separately below
        } else {
          ps.blocks.push_back({R_AC, 0, col});
          col += k;
          ps.dirN = true;
          dirset = any = true;
        }
      }
    }
    if (!any) break;
    ps.kk = ru16(col);
    ps.prec = ps.final_prec ? final_dtype : pass_dtype;
    out.push_back(ps);
  }
  return out;
}

// -------------------------------------------------------------------------
// Argument checks
// -------------------------------------------------------------------------
cnmf_status check_input(cnmf_handle* h, const cnmf_input* A) {
  if (!A) return fail(h, CNMF_EINVAL, "A is NULL");
  if (A->format != CNMF_DENSE && A->format != CNMF_DENSE_HOST && A->format != CNMF_CSR)
    return fail(h, CNMF_EINVAL, "unknown A->format %d", A->format);
  if (A->dtype != CNMF_F64 && A->dtype != CNMF_F32)
    return fail(h, CNMF_EINVAL, "A->dtype must be CNMF_F64 or CNMF_F32");
  if (A->m < 1 || A->n < 1) return fail(h, CNMF_EINVAL, "A must be non-empty (m=%lld n=%lld)", (long long)A->m, (long long)A->n);
  if (A->m > INT32_MAX / 2 || A->n > INT32_MAX / 2)
    return fail(h, CNMF_ENOTSUP, "dimensions above 2^30 are not supported");
  if (A->format == CNMF_CSR) {
    if (A->nnz < 0 || A->nnz > INT32_MAX) return fail(h, CNMF_EINVAL, "nnz must be in [0, 2^31)");
    if (!A->rowptr_dev || (A->nnz > 0 && !A->colind_dev))
      return fail(h, CNMF_EINVAL, "CSR input needs rowptr_dev and colind_dev");
    if (A->nnz > 0 && !A->data_dev) return fail(h, CNMF_EINVAL, "A->data_dev (the values) is NULL");
    return CNMF_OK;
  }
  if (!A->data_dev) return fail(h, CNMF_EINVAL, "A->data_dev is NULL");
  if (A->lda < A->n) return fail(h, CNMF_EINVAL, "lda (%lld) < n (%lld)", (long long)A->lda, (long long)A->n);
  if (A->block_rows < 0) return fail(h, CNMF_EINVAL, "block_rows must be >= 0");
  return CNMF_OK;
}

cnmf_status check_sketch(cnmf_handle* h, const cnmf_input* A, const cnmf_sketch_desc* d) {
  if (!d) return fail(h, CNMF_EINVAL, "sketch descriptor is NULL");
  const int64_t mn = std::min(A->m, A->n);
  if (d->r < 1) return fail(h, CNMF_EINVAL, "r must be >= 1 (got %d)", d->r);
  if (d->k <= d->r) return fail(h, CNMF_EINVAL, "k must exceed r (r_ov >= 1): r=%d k=%d", d->r, d->k);
  if (d->k > mn) return fail(h, CNMF_EINVAL, "k=%d exceeds min(m, n)=%lld", d->k, (long long)mn);
  if (d->k > 128) return fail(h, CNMF_ENOTSUP, "k=%d > 128 is not supported", d->k);
  if (d->q < 0) return fail(h, CNMF_EINVAL, "q must be >= 0");
  if (d->q > 64) return fail(h, CNMF_EINVAL, "q=%d is unreasonably large (max 64)", d->q);
  if (d->sides < 1 || d->sides > 3) return fail(h, CNMF_EINVAL, "sides must be CNMF_LEFT, CNMF_RIGHT or CNMF_BOTH");
  if (d->test_matrix != CNMF_TEST_GAUSSIAN && d->test_matrix != CNMF_TEST_SRHT)
    return fail(h, CNMF_EINVAL, "unknown test_matrix %d", d->test_matrix);
  if (A->dtype == CNMF_F64) {
    if (d->pass_dtype != CNMF_F64 || d->final_dtype != CNMF_F64)
      return fail(h, CNMF_EINVAL, "an F64 input runs with pass_dtype = final_dtype = CNMF_F64");
  } else {
    if (d->pass_dtype == CNMF_F64 || d->final_dtype == CNMF_F64)
      return fail(h, CNMF_EINVAL, "F64 passes need an F64 input");
    if (d->pass_dtype != CNMF_F32 && d->pass_dtype != CNMF_BF16 && d->pass_dtype != CNMF_FP8_E4M3)
      return fail(h, CNMF_EINVAL, "unknown pass_dtype %d", (int)d->pass_dtype);
    if (d->final_dtype == CNMF_FP8_E4M3)
      return fail(h, CNMF_ENOTSUP, "the last range pass and B = L^T A need at least BF16 (final_dtype)");
    if (d->final_dtype != CNMF_F32 && d->final_dtype != CNMF_BF16)
      return fail(h, CNMF_EINVAL, "unknown final_dtype %d", (int)d->final_dtype);
    if (A->format != CNMF_DENSE && (d->pass_dtype != CNMF_F32 || d->final_dtype != CNMF_F32))
      return fail(h, CNMF_ENOTSUP, "reduced-precision passes need A dense on the device");
  }
  return CNMF_OK;
}

// -------------------------------------------------------------------------
// Workspace layout
// -------------------------------------------------------------------------
template <typename T>
struct SketchWs {
  T* Xop = nullptr;     // n x kkmax operand for A passes
  T* Zop = nullptr;     // m x kkmax operand for A^T passes
  T* Y = nullptr;       // max(m, n) x kkmax pass output
  T* Ppart = nullptr;   // splits partials
  double* Q64 = nullptr;
  double* Gp = nullptr;
  double* G = nullptr;
  double* Tinv = nullptr;
  // flags: [0], [1] breakdowns repaired per half (left, right chain),
  // [2] floored pivots of the ADMM solves, [3] unresolved breakdowns,
  // [4], [5] third CholeskyQR pass needed per half, [6], [7] alternating
  // NNLS: unfinished problems, largest number of active-set steps
  int* flags = nullptr;
  unsigned* counters = nullptr;
  double* orth_err = nullptr;
  uint64_t* mask = nullptr;    // decoupled columns of the first CholeskyQR pass (2 words per half)
  double* OmL = nullptr;       // n x k Omega_L drawn on the device (seeded sketches)
  double* OmR = nullptr;       // m x k Omega_R
  int32_t* srht_s = nullptr;   // sampled Hadamard columns of the SRHT test matrices (2 x 128)
  T* Lb = nullptr;      // m x k
  T* RTb = nullptr;     // n x k  (R^T)
  T* BTb = nullptr;     // n x k  (B^T)
  T* Acb = nullptr;     // m x k
  double* At = nullptr; // k x k
  int gparts = 0;
  size_t ppart_elems = 0;
  // reduced-precision passes: copies of A (m x ldo) and A^T (n x ldt),
  // padded with zeros to whole 128 x 128 tiles,
  // FP8 tile scales, transposed operands (kkmax x ldo / kkmax x ldt, 2-byte
  // slots) and their FP8 column scales (A passes [0, 128), A^T [128, 256))
  __hip_bfloat16* A16 = nullptr;
  __hip_bfloat16* At16 = nullptr;
  uint8_t* A8 = nullptr;
  uint8_t* At8 = nullptr;
  float* tscale = nullptr;
  int ntj = 0;
  int64_t ldo = 0, ldt = 0;
  uint8_t* XtN = nullptr;
  uint8_t* XtT = nullptr;
  float* cscale = nullptr;
  unsigned long long* cmax = nullptr;
  // FP32 / FP64 passes wider than 128 columns run one launch per chain
  // block through these tight buffers (max(m, n) x 128)
  T* Xg = nullptr;
  T* Yg = nullptr;
};

int gram_parts(int64_t rows) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, rows / 64)); }

template <typename T>
void layout_sketch(Arena& a, SketchWs<T>& w, int64_t m, int64_t n, int k, const std::vector<Pass>& passes,
                   bool want_ac, const cnmf_sketch_desc* d) {
  int kkmax = 16;
  size_t pmax = 0;
  bool need16 = false, need8 = false, wide = false;
  for (const Pass& p : passes) {
    kkmax = std::max(kkmax, p.kk);
    int64_t rows = p.dirN ? m : n, cols = p.dirN ? n : m;
    int s;
    int kl = p.kk;
    if (is_lowp(p.prec)) {
      s = choose_splits_lowp((int)rows, (int)cols, p.kk, lowp_es(p.prec));
      (p.prec == CNMF_BF16 ? need16 : need8) = true;
    } else {
      if (p.kk > 128) {
        kl = ru16(k);
        wide = true;
      }
      s = p.dirN ? choose_splits_n((int)m, (int)n, kl, sizeof(T)) : choose_splits_t((int)m, (int)n, kl, sizeof(T));
    }
    if (s > 1) pmax = std::max(pmax, (size_t)s * rows * kl);
  }
  const int64_t mx = std::max(m, n);
  w.Xop = a.take<T>((size_t)n * kkmax);
  w.Zop = a.take<T>((size_t)m * kkmax);
  w.Y = a.take<T>((size_t)mx * kkmax);
  w.ppart_elems = pmax;
  w.Ppart = a.take<T>(std::max<size_t>(pmax, 1));
  w.Q64 = a.take<double>((size_t)mx * kkmax);
  w.gparts = gram_parts(mx);
  w.Gp = a.take<double>((size_t)w.gparts * 2 * k * k);
  w.G = a.take<double>(2 * (size_t)k * k);
  w.Tinv = a.take<double>(2 * (size_t)k * k);
  w.flags = a.take<int>(8);
  w.counters = a.take<unsigned>(4);
  w.orth_err = a.take<double>(4);
  w.mask = a.take<uint64_t>(4);
  if ((d->sides & CNMF_LEFT) && !d->omega_left_dev) w.OmL = a.take<double>((size_t)n * k);
  if ((d->sides & CNMF_RIGHT) && !d->omega_right_dev) w.OmR = a.take<double>((size_t)m * k);
  w.srht_s = a.take<int32_t>(256);
  w.Lb = a.take<T>((size_t)m * k);
  w.RTb = a.take<T>((size_t)n * k);
  w.BTb = a.take<T>((size_t)n * k);
  w.Acb = want_ac ? a.take<T>((size_t)m * k) : nullptr;
  w.At = a.take<double>((size_t)k * k);
  if (need16 || need8) {
    w.ldo = lowp_pad(n);
    w.ldt = lowp_pad(m);
    if (need16) {
      w.A16 = a.take<__hip_bfloat16>((size_t)lowp_pad(m) * w.ldo);
      w.At16 = a.take<__hip_bfloat16>((size_t)lowp_pad(n) * w.ldt);
    }
    if (need8) {
      w.A8 = a.take<uint8_t>((size_t)lowp_pad(m) * w.ldo);
      w.At8 = a.take<uint8_t>((size_t)lowp_pad(n) * w.ldt);
      w.ntj = (int)((n + kFp8Tile - 1) / kFp8Tile);
      w.tscale = a.take<float>((size_t)w.ntj * ((m + kFp8Tile - 1) / kFp8Tile));
    }
    w.XtN = a.take<uint8_t>((size_t)kkmax * w.ldo * 2);
    w.XtT = a.take<uint8_t>((size_t)kkmax * w.ldt * 2);
    w.cscale = a.take<float>(512);
    w.cmax = a.take<unsigned long long>(128);
  }
  if (wide) {
    w.Xg = a.take<T>((size_t)mx * 128);
    w.Yg = a.take<T>((size_t)mx * 128);
  }
}

template <typename T>
struct AdmmWs {
  T* U = nullptr;
  T* Lam = nullptr;
  T* Vt = nullptr;
  T* Phit = nullptr;
  double* XY = nullptr;
  double* Pp = nullptr;
  double* Pred = nullptr;
  unsigned* counter = nullptr;
  int parts0 = 0, parts1 = 0;
  double* rpart = nullptr;
  int rparts = 0;
};

// Row-update blocks of one side: 64-row sweeps, at most 240 blocks, so that
// the blocks of one side are resident together beside the solve's block when
// each takes a whole CU (the split schedule's launches).
int uv_parts(int64_t rows) {
  const int64_t sweeps = std::max<int64_t>(1, (rows + 63) / 64);
  const int64_t per = (sweeps + 239) / 240;
  return (int)((sweeps + per - 1) / per);
}

template <typename T>
void layout_admm(Arena& a, AdmmWs<T>& w, int64_t m, int64_t n, int k, int r) {
  w.U = a.take<T>((size_t)m * r);
  w.Lam = a.take<T>((size_t)m * r);
  w.Vt = a.take<T>((size_t)n * r);
  w.Phit = a.take<T>((size_t)n * r);
  // Xt, Yt^T in FP64, then their zero-padded FP32 copies (2 x KP x RP floats)
  w.XY = a.take<double>(2 * (size_t)k * r + (size_t)((k + 15) / 16 * 16) * ((r + 15) / 16 * 16));
  w.parts0 = uv_parts(m);
  w.parts1 = uv_parts(n);
  w.Pp = a.take<double>((size_t)(w.parts0 + w.parts1) * k * r);
  w.Pred = a.take<double>(2 * (size_t)k * r);
  w.counter = a.take<unsigned>(4);
  w.rparts = residual_blocks((int)m, (int)n);
  w.rpart = a.take<double>(2 * (size_t)w.rparts);
}

cnmf_status ensure_ws(cnmf_handle* h, size_t bytes) {
  if (bytes <= h->ws_bytes) return CNMF_OK;
  if (h->ext_ws)
    return fail(h, CNMF_ENOMEM, "internal: request needs %zu workspace bytes, its block has %zu", bytes, h->ws_bytes);
  if (h->limit && bytes > h->limit)
    return fail(h, CNMF_ENOMEM, "workspace of %zu bytes exceeds the handle limit of %zu", bytes, h->limit);
  if (h->ws) {
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipFree(h->ws));
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(h, CNMF_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  h->ws = (char*)p;
  h->ws_bytes = bytes;
  return CNMF_OK;
}

// -------------------------------------------------------------------------
// Timing: stages 0 convert, 1 A X passes, 2 A^T Z passes, 3 orthonormalisation
// and small sketches, 4 iterations, 5 residual, 6 SPA.  With timing enabled
// every span is bracketed by two HIP events on the handle's stream.
// -------------------------------------------------------------------------
enum { ST_CONVERT = 0, ST_PASS_N = 1, ST_PASS_T = 2, ST_ORTH = 3, ST_ITER = 4, ST_RESID = 5, ST_SPA = 6 };

void timing_reset(cnmf_handle* h) {
  h->spans.clear();
  h->ev_next = 0;
  h->resolved = true;
  for (int i = 0; i < kStages; ++i) {
    h->stage_ms[i] = 0.0;
    h->stage_flops[i] = 0.0;
    h->stage_count[i] = 0;
  }
}

hipEvent_t next_event(cnmf_handle* h) {
  if (h->ev_next == h->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_next++];
}

struct Span {
  cnmf_handle* h;
  int stage;
  hipEvent_t a = nullptr;
  Span(cnmf_handle* hh, int st, double flops = 0.0) : h(hh), stage(st) {
    h->stage_flops[st] += flops;
    h->stage_count[st] += 1;
    if (h->timing) {
      a = next_event(h);
      if (a) hipEventRecord(a, h->stream);
    }
  }
  ~Span() {
    if (a) {
      hipEvent_t b = next_event(h);
      if (b) {
        hipEventRecord(b, h->stream);
        h->spans.push_back({stage, a, b});
        h->resolved = false;
      }
    }
  }
};

void timing_resolve(cnmf_handle* h) {
  if (h->resolved) return;
  if (!h->spans.empty()) hipEventSynchronize(h->spans.back().b);
  for (const auto& sp : h->spans) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) h->stage_ms[sp.stage] += ms;
  }
  h->resolved = true;
}

// -------------------------------------------------------------------------
// Orthonormalise nh column blocks [col0 + i*k, +k) of Y (rows x kk, already
// reduced) by CholeskyQR2; result in Q64 (same columns, FP64).
// Rank-deficient Y (k > rank A; plain CholeskyQR breaks down there):
//   pass 1 decouples the columns whose pivot is <= 1e-14 max diag(Y^T Y)
//     (dependent on the earlier columns to within the accuracy of the Gram)
//     and puts unit-scale Gaussian columns there;
//   pass 2 decouples the columns of Q1 with a pivot <= 1e-8 max diag: Q1's
//     independent columns are orthonormal to within rounding, so a column
//     it left in their span has a pivot at rounding level and is detected
//     reliably; they are replaced in the same way, and
//   pass 3, only for halves where pass 2 replaced a column (the kernels test
//     a device flag and return at once otherwise), orthonormalises the
//     completed matrix once more; a breakdown there, or a NaN pivot
//     anywhere, is unresolved (flags[3]).
// range(Q) contains range(Y) and Q^T Q = I.  The flags words [4], [5] hold
// the per-half "pass 3 needed" results of pass 2.
// -------------------------------------------------------------------------
template <typename T>
cnmf_status orth_blocks(cnmf_handle* h, SketchWs<T>& w, const T* Y, int rows, int kk, int col0, int nh, int k,
                        uint64_t seed, uint32_t id0) {
  hipStream_t st = h->stream;
  const int parts = std::min(w.gparts, std::max(1, rows / 32));
  int* need = w.flags + 4;
  CholOpts o{};
  o.repaired = w.flags;
  o.unresolved = w.flags + 3;
  o.unresolved_total = h->unresolved_dev;
  // pass 1: G = Y^T Y, T1, Q1 = Y T1^-1 (decoupled columns replaced)
  o.tau = 1e-14;
  o.mask = w.mask;
  HIPCHK(h, (launch_cross2<T, T>(Y, kk, col0, Y, kk, col0, k, nh, rows, k, k, w.Gp, parts, st)));
  HIPCHK(h, launch_gram_chol(w.Gp, parts, nh, k, w.G, w.Tinv, o, st));
  // apply writes Q64 columns col0 + h*k via an offset view
  HIPCHK(h, (launch_apply_tinv<T>(Y + col0, rows, kk, nh, k, w.Tinv, w.Q64 + col0, kk, w.mask, seed, id0, st)));
  // pass 2 on Q1
  o.tau = 1e-8;
  o.need = need;
  HIPCHK(h, (launch_cross2<double, double>(w.Q64, kk, col0, w.Q64, kk, col0, k, nh, rows, k, k, w.Gp, parts, st)));
  HIPCHK(h, launch_gram_chol(w.Gp, parts, nh, k, w.G, w.Tinv, o, st));
  HIPCHK(h, (launch_apply_tinv<double>(w.Q64 + col0, rows, kk, nh, k, w.Tinv, w.Q64 + col0, kk, w.mask, seed,
                                       id0 + 2, st)));
  // pass 3, conditional on pass 2 having replaced a column
  o.tau = 1e-14;
  o.mask = nullptr;
  o.need = nullptr;
  o.repaired = nullptr;
  o.run_if = need;
  HIPCHK(h, (launch_cross2<double, double>(w.Q64, kk, col0, w.Q64, kk, col0, k, nh, rows, k, k, w.Gp, parts, st,
                                           need)));
  HIPCHK(h, launch_gram_chol(w.Gp, parts, nh, k, w.G, w.Tinv, o, st));
  HIPCHK(h, (launch_apply_tinv<double>(w.Q64 + col0, rows, kk, nh, k, w.Tinv, w.Q64 + col0, kk, nullptr, 0, 0, st,
                                       need)));
  return CNMF_OK;
}

// Sketch driver for T = double (F64 input) or float (F32 input).
// -------------------------------------------------------------------------
// Products with A in its three formats.  Dense on the device: one streaming
// GEMM (split-K partials reduced in a fixed order).  Dense in host memory:
// the same GEMM on row blocks copied in on a second stream, two blocks in
// flight (block b + 2 is copied while block b + 1 is multiplied); A X writes
// each block's rows, A^T Z adds the blocks' products in block order.  CSR
// on the device: sparse products (A^T as CSR formed once per call).
// -------------------------------------------------------------------------
template <typename T>
struct AOpWs {
  T* stage[2] = {nullptr, nullptr};  // host format: staging blocks (brows x n, tight)
  int64_t brows = 0;
  int nblocks = 0;
  T* ysum = nullptr;                 // host format: one block's A_b^T Z_b (n x kkmax)
  T* hpart = nullptr;                // host format: split-K partials of a block's product
  double* rpart = nullptr;           // host format: residual partials of all blocks
  int rparts = 0;
  // CSR: A^T in CSR form
  int64_t* trow = nullptr;
  int32_t* tcol = nullptr;
  T* tval = nullptr;
  void* sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  int32_t* keys = nullptr;
  int32_t* perm = nullptr;
  int32_t* keys_out = nullptr;
  int32_t* perm_out = nullptr;
  int* bad = nullptr;                // column indices outside [0, n)
  double* gpart = nullptr;           // Gram partials of the residual (kCsrGramParts x 64 x 64)
  double* GU = nullptr;              // U^T U, V V^T (64 x 64 each)
  double* GV = nullptr;
  double* cpart = nullptr;           // residual partials over the nonzeros
  bool t_built = false;
};
constexpr int kCsrGramParts = 64;

int64_t host_block_rows(const cnmf_input* A) {
  const int64_t es = A->dtype == CNMF_F64 ? 8 : 4;
  int64_t b = A->block_rows;
  if (b <= 0) b = std::max<int64_t>(64, ((int64_t)64 << 20) / (A->n * es) / 64 * 64);
  return std::min<int64_t>(b, A->m);
}

template <typename T>
void layout_aop(Arena& a, AOpWs<T>& ao, const cnmf_input* A, int kkmax) {
  if (A->format == CNMF_DENSE_HOST) {
    ao.brows = host_block_rows(A);
    ao.nblocks = (int)((A->m + ao.brows - 1) / ao.brows);
    ao.stage[0] = a.take<T>((size_t)ao.brows * A->n);
    ao.stage[1] = a.take<T>((size_t)ao.brows * A->n);
    ao.ysum = a.take<T>((size_t)A->n * kkmax);
    // split-K partials of one block's product: the largest over the block
    // heights and operand widths (the split count grows as blocks shrink)
    size_t hp = 1;
    const int64_t last = A->m - (int64_t)(ao.nblocks - 1) * ao.brows;
    for (int64_t mb : {ao.brows, last})
      for (int kk = 16; kk <= std::min(kkmax, 128); kk += 16) {
        const size_t sn = choose_splits_n((int)mb, (int)A->n, kk, sizeof(T));
        const size_t stt = choose_splits_t((int)mb, (int)A->n, kk, sizeof(T));
        hp = std::max({hp, sn > 1 ? sn * mb * kk : 0, stt > 1 ? stt * A->n * kk : 0});
      }
    ao.hpart = a.take<T>(hp);
    int parts = 0;
    for (int b = 0; b < ao.nblocks; ++b) {
      const int64_t mb = std::min<int64_t>(ao.brows, A->m - (int64_t)b * ao.brows);
      parts += residual_blocks((int)mb, (int)A->n);
    }
    ao.rparts = parts;
    ao.rpart = a.take<double>(2 * (size_t)parts);
  } else if (A->format == CNMF_CSR) {
    const size_t nnz = (size_t)A->nnz;
    ao.trow = a.take<int64_t>((size_t)A->n + 1);
    ao.tcol = a.take<int32_t>(std::max<size_t>(nnz, 1));
    ao.tval = a.take<T>(std::max<size_t>(nnz, 1));
    ao.keys = a.take<int32_t>(std::max<size_t>(nnz, 1));
    ao.perm = a.take<int32_t>(std::max<size_t>(nnz, 1));
    ao.keys_out = a.take<int32_t>(std::max<size_t>(nnz, 1));
    ao.perm_out = a.take<int32_t>(std::max<size_t>(nnz, 1));
    ao.sort_tmp_bytes = csr_sort_temp_bytes((int)nnz, (int)A->n);
    ao.sort_tmp = a.take<char>(std::max<size_t>(ao.sort_tmp_bytes, 1));
    ao.bad = a.take<int>(1);
    ao.gpart = a.take<double>((size_t)kCsrGramParts * 64 * 64);
    ao.GU = a.take<double>(64 * 64);
    ao.GV = a.take<double>(64 * 64);
    ao.cpart = a.take<double>(2 * (size_t)csr_resid_blocks((int)A->m));
  }
}

// out (rows x kk) = A X (dirN; X n x kk) or A^T Z (Z m x kk) for a dense
// device A; k and nblk: the operand's chain blocks (k columns each), used when
// kk > 128 (the GEMM kernels take at most 128 columns).  Partial sums of
// split-K launches go through ppart; xg / yg hold one block's columns.
template <typename T>
cnmf_status dense_product(cnmf_handle* h, const T* Ap, int64_t lda, int m, int n, bool dirN, const T* op, int kk,
                          int k, int nblk, T* out, T* ppart, T* xg, T* yg) {
  hipStream_t st = h->stream;
  const int rows = dirN ? m : n, in_rows = dirN ? n : m;
  if (kk <= 128) {
    const int splits = dirN ? choose_splits_n(m, n, kk, sizeof(T)) : choose_splits_t(m, n, kk, sizeof(T));
    T* dst = splits > 1 ? ppart : out;
    if (dirN)
      HIPCHK(h, launch_gemm_n<T>(Ap, lda, m, n, op, kk, dst, splits, st));
    else
      HIPCHK(h, launch_gemm_t<T>(Ap, lda, m, n, op, kk, dst, splits, st));
    if (splits > 1) HIPCHK(h, launch_reduce_splits<T>(ppart, splits, rows, kk, out, st));
    return CNMF_OK;
  }
  // one product per chain block (k <= 128 columns each)
  const int kb = ru16(k);
  const int sb = dirN ? choose_splits_n(m, n, kb, sizeof(T)) : choose_splits_t(m, n, kb, sizeof(T));
  for (int b = 0; b < nblk; ++b) {
    const int col0 = b * k;
    if (kb != k) HIPCHK(h, launch_fill(xg, sizeof(T) * (size_t)in_rows * kb, st));
    HIPCHK(h, (launch_copy2d<T, T>(op + col0, kk, xg, kb, in_rows, k, 1.0, st)));
    T* db = sb > 1 ? ppart : yg;
    if (dirN)
      HIPCHK(h, launch_gemm_n<T>(Ap, lda, m, n, xg, kb, db, sb, st));
    else
      HIPCHK(h, launch_gemm_t<T>(Ap, lda, m, n, xg, kb, db, sb, st));
    if (sb > 1) HIPCHK(h, launch_reduce_splits<T>(ppart, sb, rows, kb, yg, st));
    HIPCHK(h, (launch_copy2d<T, T>(yg, kb, out + col0, kk, rows, k, 1.0, st)));
  }
  return CNMF_OK;
}

cnmf_status ensure_copy_stream(cnmf_handle* h) {
  if (h->copy_stream) return CNMF_OK;
  HIPCHK(h, hipStreamCreateWithFlags(&h->copy_stream, hipStreamNonBlocking));
  for (int i = 0; i < 2; ++i) {
    HIPCHK(h, hipEventCreateWithFlags(&h->stage_ready[i], hipEventDisableTiming));
    HIPCHK(h, hipEventCreateWithFlags(&h->stage_free[i], hipEventDisableTiming));
  }
  return CNMF_OK;
}

// Streams the row blocks of a host A through the staging buffers and calls
// body(b, stage, row0, rows) on the handle's stream for each, in order.
template <typename T, typename F>
cnmf_status host_blocks(cnmf_handle* h, const cnmf_input* A, AOpWs<T>& ao, F&& body) {
  cnmf_status s = ensure_copy_stream(h);
  if (s != CNMF_OK) return s;
  hipStream_t st = h->stream, cs = h->copy_stream;
  const int64_t m = A->m, n = A->n, es = sizeof(T);
  const char* src = (const char*)A->data_dev;
  // the stages may still be read by work already on the handle's stream
  HIPCHK(h, hipEventRecord(h->stage_free[0], st));
  HIPCHK(h, hipEventRecord(h->stage_free[1], st));
  auto copy_in = [&](int b) -> cnmf_status {
    const int sl = b & 1;
    const int64_t i0 = (int64_t)b * ao.brows, mb = std::min<int64_t>(ao.brows, m - i0);
    HIPCHK(h, hipStreamWaitEvent(cs, h->stage_free[sl], 0));
    HIPCHK(h, hipMemcpy2DAsync(ao.stage[sl], (size_t)(n * es), src + i0 * A->lda * es, (size_t)(A->lda * es),
                               (size_t)(n * es), (size_t)mb, hipMemcpyHostToDevice, cs));
    HIPCHK(h, hipEventRecord(h->stage_ready[sl], cs));
    return CNMF_OK;
  };
  s = copy_in(0);
  if (s == CNMF_OK && ao.nblocks > 1) s = copy_in(1);
  if (s != CNMF_OK) return s;
  for (int b = 0; b < ao.nblocks; ++b) {
    const int sl = b & 1;
    const int64_t i0 = (int64_t)b * ao.brows, mb = std::min<int64_t>(ao.brows, m - i0);
    HIPCHK(h, hipStreamWaitEvent(st, h->stage_ready[sl], 0));
    s = body(b, (const T*)ao.stage[sl], (int)i0, (int)mb);
    if (s != CNMF_OK) return s;
    HIPCHK(h, hipEventRecord(h->stage_free[sl], st));
    if (b + 2 < ao.nblocks) {
      s = copy_in(b + 2);
      if (s != CNMF_OK) return s;
    }
  }
  return CNMF_OK;
}

// CSR products: A X from the caller's rows; A^T Z from the transpose, built
// on the first A^T product of the call.  Column indices outside [0, n) are
// skipped and reported through the handle's unresolved count.
template <typename T>
cnmf_status csr_product(cnmf_handle* h, const cnmf_input* A, AOpWs<T>& ao, bool dirN, const T* op, int kk, T* out) {
  hipStream_t st = h->stream;
  const int m = (int)A->m, n = (int)A->n;
  const T* val = (const T*)A->data_dev;
  if (!ao.t_built) {
    HIPCHK(h, launch_fill(ao.bad, sizeof(int), st));
    HIPCHK(h, launch_csr_transpose<T>(A->rowptr_dev, A->colind_dev, val, m, n, A->nnz, ao.trow, ao.tcol, ao.tval,
                                      ao.keys, ao.perm, ao.keys_out, ao.perm_out, ao.sort_tmp, ao.sort_tmp_bytes,
                                      ao.bad, st));
    HIPCHK(h, launch_add_count(ao.bad, h->unresolved_dev, st));
    ao.t_built = true;
  }
  if (dirN)
    HIPCHK(h, launch_csr_spmm<T>(A->rowptr_dev, A->colind_dev, val, m, n, A->nnz, op, kk, out, st));
  else
    HIPCHK(h, launch_csr_spmm<T>(ao.trow, ao.tcol, ao.tval, n, m, A->nnz, op, kk, out, st));
  return CNMF_OK;
}

// out (rows x kk) = A X or A^T Z for any input format.
template <typename T>
cnmf_status a_product(cnmf_handle* h, const cnmf_input* A, AOpWs<T>& ao, bool dirN, const T* op, int kk, int k,
                      int nblk, T* out, T* ppart, T* xg, T* yg) {
  const int m = (int)A->m, n = (int)A->n;
  if (A->format == CNMF_DENSE)
    return dense_product<T>(h, (const T*)A->data_dev, A->lda, m, n, dirN, op, kk, k, nblk, out, ppart, xg, yg);
  if (A->format == CNMF_CSR) return csr_product<T>(h, A, ao, dirN, op, kk, out);
  // host: A X row block by row block; A^T Z as the block-ordered sum
  return host_blocks<T>(h, A, ao, [&](int b, const T* blk, int i0, int mb) -> cnmf_status {
    if (dirN)
      return dense_product<T>(h, blk, n, mb, n, true, op, kk, k, nblk, out + (int64_t)i0 * kk, ao.hpart, xg, yg);
    T* dst = b == 0 ? out : ao.ysum;
    cnmf_status s =
        dense_product<T>(h, blk, n, mb, n, false, op + (int64_t)i0 * kk, kk, k, nblk, dst, ao.hpart, xg, yg);
    if (s != CNMF_OK || b == 0) return s;
    HIPCHK(h, launch_add2d<T>(ao.ysum, kk, out, kk, n, kk, h->stream));
    return CNMF_OK;
  });
}

template <typename T>
cnmf_status csr_residual(cnmf_handle* h, const cnmf_input* A, AOpWs<T>& ao, const T* U, const T* Vt, int r,
                         double* out) {
  hipStream_t st = h->stream;
  const int m = (int)A->m, n = (int)A->n;
  if (r > 64) return fail(h, CNMF_ENOTSUP, "r > 64");
  HIPCHK(h, launch_csr_resid<T>(A->rowptr_dev, A->colind_dev, (const T*)A->data_dev, m, n, A->nnz, U, Vt, r,
                                ao.cpart, st));
  const int pu = std::min(kCsrGramParts, std::max(1, m / 32)), pv = std::min(kCsrGramParts, std::max(1, n / 32));
  HIPCHK(h, (launch_cross2<T, T>(U, r, 0, U, r, 0, 0, 1, m, r, r, ao.gpart, pu, st)));
  HIPCHK(h, launch_sum_parts(ao.gpart, pu, (int64_t)r * r, ao.GU, st));
  HIPCHK(h, (launch_cross2<T, T>(Vt, r, 0, Vt, r, 0, 0, 1, n, r, r, ao.gpart, pv, st)));
  HIPCHK(h, launch_sum_parts(ao.gpart, pv, (int64_t)r * r, ao.GV, st));
  HIPCHK(h, launch_csr_resid_finish(ao.cpart, csr_resid_blocks(m), ao.GU, ao.GV, r, out, st));
  return CNMF_OK;
}

// ||A - U V||_F / ||A||_F (U m x r, V^T n x r; ld r) into *out (FP64).
template <typename T>
cnmf_status a_residual(cnmf_handle* h, const cnmf_input* A, AOpWs<T>& ao, const T* U, const T* Vt, int r,
                       double* rpart, int rparts, double* out) {
  hipStream_t st = h->stream;
  const int m = (int)A->m, n = (int)A->n;
  if (A->format == CNMF_DENSE) {
    HIPCHK(h, launch_residual<T>((const T*)A->data_dev, A->lda, m, n, U, r, Vt, r, r, rpart, rparts, st));
    HIPCHK(h, launch_residual_finish(rpart, rparts, out, st));
    return CNMF_OK;
  }
  if (A->format == CNMF_CSR) return csr_residual<T>(h, A, ao, U, Vt, r, out);
  int off = 0;
  cnmf_status s = host_blocks<T>(h, A, ao, [&](int, const T* blk, int i0, int mb) -> cnmf_status {
    const int p = residual_blocks(mb, n);
    HIPCHK(h, launch_residual<T>(blk, n, mb, n, U + (int64_t)i0 * r, r, Vt, r, r, ao.rpart + 2 * (int64_t)off, p, st));
    off += p;
    return CNMF_OK;
  });
  if (s != CNMF_OK) return s;
  HIPCHK(h, launch_residual_finish(ao.rpart, ao.rparts, out, st));
  return CNMF_OK;
}

template <typename T>
cnmf_status run_sketch(cnmf_handle* h, const cnmf_input* A, const cnmf_sketch_desc* d, SketchWs<T>& w,
                       AOpWs<T>& ao, const std::vector<Pass>& passes, double* stats_dev) {
  hipStream_t st = h->stream;
  const int m = (int)A->m, n = (int)A->n, k = d->k;
  const T* Ap = (const T*)A->data_dev;
  const int64_t lda = A->lda;
  HIPCHK(h, launch_fill(w.flags, 8 * sizeof(int), st));
  HIPCHK(h, launch_fill(w.counters, 4 * sizeof(unsigned), st));

  // A pass multiplies an operand with one row per column of the matrix it
  // reads: FP32/FP64 operands are row-major (cols x kk), reduced-precision
  // operands transposed (kk x ld) in the pass type.
  auto operand_for = [&](const Pass& p) -> T* { return p.dirN ? w.Xop : w.Zop; };
  auto xt_for = [&](const Pass& p) -> uint8_t* { return p.dirN ? w.XtN : w.XtT; };
  auto xt_ld = [&](const Pass& p) -> int64_t { return p.dirN ? w.ldo : w.ldt; };
  auto scol_for = [&](const Pass& p) -> int { return p.dirN ? 0 : 256; };
  auto clear_operand = [&](const Pass& p) -> cnmf_status {
    const size_t cols = p.dirN ? n : m;
    if (is_lowp(p.prec))
      HIPCHK(h, launch_fill(xt_for(p), (size_t)lowp_es(p.prec) * p.kk * xt_ld(p), st));
    else
      HIPCHK(h, launch_fill(operand_for(p), sizeof(T) * cols * p.kk, st));
    return CNMF_OK;
  };
  // Q64 columns [c0, c0 + k) (rows x ldq) -> operand slot col of pass p
  auto store_operand = [&](const Pass& p, const double* Q, int rows, int ldq, int c0, int col) -> cnmf_status {
    if (is_lowp(p.prec))
      HIPCHK(h, launch_store_lowp(lowp_es(p.prec), Q + 0, rows, ldq, c0, k, xt_for(p), xt_ld(p), col, w.cscale,
                                  scol_for(p) + col, w.cmax, st));
    else
      HIPCHK(h, (launch_copy2d<double, T>(Q + c0, ldq, operand_for(p) + col, p.kk, rows, k, 1.0, st)));
    return CNMF_OK;
  };
#define RUN(expr)                 \
  do {                            \
    cnmf_status _s = (expr);      \
    if (_s != CNMF_OK) return _s; \
  } while (0)

  if (w.A16 || w.A8) {
    if constexpr (std::is_same<T, float>::value) {
      Span sp(h, ST_CONVERT);
      HIPCHK(h, launch_convert_lowp(Ap, lda, m, n, w.A16, w.At16, w.A8, w.At8, w.ldo, w.ldt, w.tscale, st));
    } else {
      return fail(h, CNMF_EINVAL, "internal: reduced-precision passes need an F32 input");
    }
  }
  // Gaussian test matrices (Alg. 1's first step) drawn on the device when
  // the caller gives none
  const double* omL = d->omega_left_dev;
  const double* omR = d->omega_right_dev;
  const bool srht = d->test_matrix == CNMF_TEST_SRHT;
  if (w.OmL) {
    if (srht)
      HIPCHK(h, launch_srht_fill(w.OmL, k, n, k, d->seed, kOmegaLeftId, w.srht_s, st));
    else
      HIPCHK(h, launch_gaussian_fill(w.OmL, k, n, k, d->seed, kOmegaLeftId, st));
    omL = w.OmL;
  }
  if (w.OmR) {
    if (srht)
      HIPCHK(h, launch_srht_fill(w.OmR, k, m, k, d->seed, kOmegaRightId, w.srht_s + 128, st));
    else
      HIPCHK(h, launch_gaussian_fill(w.OmR, k, m, k, d->seed, kOmegaRightId, st));
    omR = w.OmR;
  }
  // stage the first operands (Omegas) of the chains
  for (size_t pi = 0; pi < passes.size(); ++pi) {
    const Pass& p = passes[pi];
    bool zeroed = false;
    for (const Block& b : p.blocks) {
      if ((b.kind == L_RANGE || b.kind == R_RANGE) && b.step == 0) {
        if (!zeroed) {
          RUN(clear_operand(p));
          zeroed = true;
        }
        const double* om = b.kind == L_RANGE ? omL : omR;
        int rows = b.kind == L_RANGE ? n : m;
        RUN(store_operand(p, om, rows, k, 0, b.col0));
      }
    }
  }

  for (size_t pi = 0; pi < passes.size(); ++pi) {
    const Pass& p = passes[pi];
    const int rows = p.dirN ? m : n;
    T* op = operand_for(p);
    const bool lp = is_lowp(p.prec);
    const int splits = lp ? choose_splits_lowp(rows, p.dirN ? n : m, p.kk, lowp_es(p.prec)) : 1;
    {
      const double flops = 2.0 * m * n * (double)(k * (int)p.blocks.size());
      Span sp(h, p.dirN ? ST_PASS_N : ST_PASS_T, flops);
      if (lp) {
        if constexpr (std::is_same<T, float>::value) {
          const int es = lowp_es(p.prec);
          const void* M = es == 2 ? (p.dirN ? (const void*)w.A16 : (const void*)w.At16)
                                  : (p.dirN ? (const void*)w.A8 : (const void*)w.At8);
          HIPCHK(h, launch_gemm_lowp(es, M, p.dirN ? w.ldo : w.ldt, lowp_pad(rows), rows, p.dirN ? n : m, xt_for(p),
                                     xt_ld(p), p.kk,
                                     splits > 1 ? w.Ppart : w.Y, splits, w.tscale, w.ntj, p.dirN ? 0 : 1, st));
        }
      } else {
        RUN(a_product<T>(h, A, ao, p.dirN, op, p.kk, k, (int)p.blocks.size(), w.Y, w.Ppart, w.Xg, w.Yg));
      }
    }
    Span orth_span(h, ST_ORTH);
    if (lp && splits > 1) HIPCHK(h, launch_reduce_splits<T>(w.Ppart, splits, rows, p.kk, w.Y, st));

    // orthonormalise the range blocks (contiguous)
    int rcol0 = -1, nh = 0;
    for (const Block& b : p.blocks)
      if (b.kind == L_RANGE || b.kind == R_RANGE) {
        if (rcol0 < 0) rcol0 = b.col0;
        ++nh;
      }
    if (nh > 0) {
      cnmf_status s = orth_blocks<T>(h, w, w.Y, rows, p.kk, rcol0, nh, k, d->seed,
                                     kCompletionId0 + 4 * (uint32_t)pi);
      if (s != CNMF_OK) return s;
    }
    // route results
    const Pass* nx = pi + 1 < passes.size() ? &passes[pi + 1] : nullptr;
    bool nzeroed = false;
    auto zero_next = [&]() -> cnmf_status {
      if (nx && !nzeroed) {
        bool has_first = false;
        for (const Block& b : nx->blocks)
          if ((b.kind == L_RANGE || b.kind == R_RANGE) && b.step == 0) has_first = true;
        if (!has_first) RUN(clear_operand(*nx));
        nzeroed = true;
      }
      return CNMF_OK;
    };
    for (const Block& b : p.blocks) {
      if (b.kind == L_RANGE || b.kind == R_RANGE) {
        const bool isL = b.kind == L_RANGE;
        const bool last = b.step == 2 * d->q;
        // slot of this chain in the next pass
        int ncol = -1;
        if (nx)
          for (const Block& c : nx->blocks) {
            if (isL && (c.kind == L_RANGE || c.kind == L_B)) ncol = c.col0;
            if (!isL && (c.kind == R_RANGE || c.kind == R_AC)) ncol = c.col0;
          }
        if (ncol >= 0) {
          cnmf_status s = zero_next();
          if (s != CNMF_OK) return s;
          RUN(store_operand(*nx, w.Q64, rows, p.kk, b.col0, ncol));
        }
        if (last) {
          T* basis = isL ? w.Lb : w.RTb;
          HIPCHK(h, (launch_copy2d<double, T>(w.Q64 + b.col0, p.kk, basis, k, rows, k, 1.0, st)));
          if (stats_dev) {
            HIPCHK(h, (launch_cross2<double, double>(w.Q64, p.kk, b.col0, w.Q64, p.kk, b.col0, k, 1, rows, k, k, w.Gp,
                                                     std::min(w.gparts, std::max(1, rows / 32)), st)));
            HIPCHK(h, launch_sum_parts(w.Gp, std::min(w.gparts, std::max(1, rows / 32)), (int64_t)k * k, w.G, st));
            HIPCHK(h, launch_orth_error(w.G, k, w.orth_err + (isL ? 0 : 1), st));
          }
        }
      } else if (b.kind == L_B) {
        HIPCHK(h, (launch_copy2d<T, T>(w.Y + b.col0, p.kk, w.BTb, k, n, k, 1.0, st)));
      } else if (b.kind == R_AC) {
        HIPCHK(h, (launch_copy2d<T, T>(w.Y + b.col0, p.kk, w.Acb, k, m, k, 1.0, st)));
      }
    }
  }
  // At = L^T A R^T = B R^T = (B^T)^T R^T, a k x k product over n rows
  if ((d->sides & CNMF_BOTH) == CNMF_BOTH) {
    Span sp(h, ST_ORTH);
    int parts = std::min(w.gparts, std::max(1, n / 32));
    HIPCHK(h, (launch_cross2<T, T>(w.BTb, k, 0, w.RTb, k, 0, 0, 1, n, k, k, w.Gp, parts, st)));
    HIPCHK(h, launch_sum_parts(w.Gp, parts, (int64_t)k * k, w.At, st));
  }
#undef RUN
  return CNMF_OK;
}

template <typename T>
cnmf_status write_sketch_outputs(cnmf_handle* h, const cnmf_input* A, const cnmf_sketch_desc* d, SketchWs<T>& w,
                                 const cnmf_sketch_out* o) {
  if (!o) return CNMF_OK;
  hipStream_t st = h->stream;
  const int m = (int)A->m, n = (int)A->n, k = d->k;
  const bool L = d->sides & CNMF_LEFT, R = d->sides & CNMF_RIGHT;
  if (o->L_dev && L) HIPCHK(h, (launch_copy2d<T, T>(w.Lb, k, (T*)o->L_dev, k, m, k, 1.0, st)));
  if (o->R_dev && R) HIPCHK(h, (launch_transpose<T, T>(w.RTb, k, (T*)o->R_dev, n, n, k, st)));
  if (o->B_dev && L) HIPCHK(h, (launch_transpose<T, T>(w.BTb, k, (T*)o->B_dev, n, n, k, st)));
  if (o->At_dev && L && R) HIPCHK(h, (launch_copy2d<double, T>(w.At, k, (T*)o->At_dev, k, k, k, 1.0, st)));
  if (o->Ac_dev && R && w.Acb) HIPCHK(h, (launch_copy2d<T, T>(w.Acb, k, (T*)o->Ac_dev, k, m, k, 1.0, st)));
  if (o->stats_dev) {
    // stats: [0] max|L^T L - I|, [1] max|R R^T - I|, [2] breakdowns repaired,
    // [3] breakdowns unresolved
    HIPCHK(h, launch_fill(o->stats_dev, 4 * sizeof(double), st));
    if (L) HIPCHK(h, (launch_copy2d<double, double>(w.orth_err, 1, o->stats_dev, 1, 1, 1, 1.0, st)));
    if (R) HIPCHK(h, (launch_copy2d<double, double>(w.orth_err + 1, 1, o->stats_dev + 1, 1, 1, 1, 1.0, st)));
    HIPCHK(h, launch_flags_to_stats(w.flags, 2, o->stats_dev + 2, st));
    HIPCHK(h, launch_flags_to_stats(w.flags + 3, 1, o->stats_dev + 3, st));
  }
  return CNMF_OK;
}

int passes_kkmax(const std::vector<Pass>& passes) {
  int kk = 16;
  for (const Pass& p : passes) kk = std::max(kk, p.kk);
  return kk;
}

template <typename T>
cnmf_status do_sketch(cnmf_handle* h, const cnmf_input* A, const cnmf_sketch_desc* d, const cnmf_sketch_out* o,
                      bool want_ac) {
  std::vector<Pass> passes = plan_passes(d->k, d->q, d->sides, want_ac, d->pass_dtype, d->final_dtype);
  if (passes.empty()) return fail(h, CNMF_EINVAL, "internal: empty pass plan");
  Arena dry(nullptr);
  SketchWs<T> w;
  AOpWs<T> ao;
  layout_sketch<T>(dry, w, A->m, A->n, d->k, passes, want_ac, d);
  layout_aop<T>(dry, ao, A, passes_kkmax(passes));
  cnmf_status s = ensure_ws(h, dry.off);
  if (s != CNMF_OK) return s;
  Arena a(h->ws);
  layout_sketch<T>(a, w, A->m, A->n, d->k, passes, want_ac, d);
  layout_aop<T>(a, ao, A, passes_kkmax(passes));
  s = run_sketch<T>(h, A, d, w, ao, passes, o ? o->stats_dev : nullptr);
  if (s != CNMF_OK) return s;
  return write_sketch_outputs<T>(h, A, d, w, o);
}

// Buffers of the multiplicative / uncompressed iterations.
template <typename T>
struct IterWs {
  T* Xop = nullptr;    // n x kk operand (Y^T rows) for A passes
  T* Zop = nullptr;    // m x kk operand (X rows) for A^T passes
  T* Pn = nullptr;     // m x kk pass output
  T* Pt = nullptr;     // n x kk pass output
  T* Ppart = nullptr;  // split partials
  double* PpX = nullptr;
  double* PpY = nullptr;
  double* S = nullptr;
  double* Gp = nullptr;
  double* Gm = nullptr;
  int* hok = nullptr;     // alternating NNLS: Gm holds a checked G^-1
  int* floored = nullptr;  // floored pivots of the last small inverse
  double* Gt = nullptr;    // scratch of the small inverse: sym(S) + pen I and T^-1
  double* Tinv = nullptr;
  int kk = 16, bx = 1, by = 1;
};

int row_blocks(int64_t rows) { return (int)std::max<int64_t>(1, std::min<int64_t>(512, (rows + 63) / 64)); }

template <typename T>
void layout_iter(Arena& a, IterWs<T>& w, int64_t m, int64_t n, int k, int r, bool full) {
  w.kk = ru16(r);
  w.bx = row_blocks(m);
  w.by = row_blocks(n);
  const int k2 = full ? r : k;
  if (full) {
    w.Xop = a.take<T>((size_t)n * w.kk);
    w.Zop = a.take<T>((size_t)m * w.kk);
    w.Pn = a.take<T>((size_t)m * w.kk);
    w.Pt = a.take<T>((size_t)n * w.kk);
    int sn = choose_splits_n((int)m, (int)n, w.kk, sizeof(T)), stt = choose_splits_t((int)m, (int)n, w.kk, sizeof(T));
    size_t pm = std::max((size_t)(sn > 1 ? sn : 0) * m, (size_t)(stt > 1 ? stt : 0) * n) * w.kk;
    w.Ppart = a.take<T>(std::max<size_t>(pm, 1));
  }
  w.PpX = a.take<double>((size_t)w.bx * k2 * r);
  w.PpY = a.take<double>((size_t)w.by * k2 * r);
  w.S = a.take<double>((size_t)std::max(k2, r) * r);
  w.Gp = a.take<double>((size_t)r * r);
  w.Gm = a.take<double>((size_t)r * r);
  w.hok = a.take<int>(1);
  w.floored = a.take<int>(1);
  w.Gt = a.take<double>((size_t)r * r);
  w.Tinv = a.take<double>((size_t)r * r);
}

template <typename T>
cnmf_status pass_full(cnmf_handle* h, const cnmf_input* A, AOpWs<T>& ao, bool dirN, const T* op, int kk, T* out,
                      T* ppart) {
  Span sp(h, dirN ? ST_PASS_N : ST_PASS_T, 2.0 * A->m * A->n * (double)kk);
  // kk = r rounded up to 16 <= 64: one product
  return a_product<T>(h, A, ao, dirN, op, kk, kk, 1, out, ppart, nullptr, nullptr);
}

// A factorisation in four phases (the serving loop drives them separately):
// layout of the workspace, prologue (sketch, initial state and, for ADMM,
// the first partials), the iterations, and the epilogue (outputs, residual).
// The uncompressed comparators run on A itself (L = I, R = I); MU and
// alternating NNLS need Ac = A R^T besides B.
static bool full_method(int m) { return m == CNMF_ADMM_FULL || m == CNMF_MU_FULL || m == CNMF_ANLS_FULL; }
static bool method_wants_ac(int m) { return m == CNMF_MU || m == CNMF_ANLS; }

template <typename T>
struct FactState {
  std::vector<Pass> passes;
  bool full = false, want_ac = false;
  SketchWs<T> w;
  AdmmWs<T> aw;
  IterWs<T> iw;
  AOpWs<T> ao;
};

template <typename T>
cnmf_status fact_plan(cnmf_handle* h, const cnmf_factorize_desc* d, FactState<T>& f) {
  const cnmf_sketch_desc* sk = &d->sk;
  f.full = full_method(d->method);
  f.want_ac = method_wants_ac(d->method);
  if (!f.full) {
    f.passes = plan_passes(sk->k, sk->q, CNMF_BOTH, f.want_ac, sk->pass_dtype, sk->final_dtype);
    if (f.passes.empty()) return fail(h, CNMF_EINVAL, "internal: empty pass plan");
  }
  return CNMF_OK;
}

template <typename T>
void fact_layout(Arena& a, FactState<T>& f, int64_t m, int64_t n, const cnmf_factorize_desc* d,
                 const cnmf_input* A = nullptr) {
  const int k = d->sk.k, r = d->sk.r;
  if (!f.full)
    layout_sketch<T>(a, f.w, m, n, k, f.passes, f.want_ac, &d->sk);
  else
    f.w.flags = a.take<int>(8);
  layout_admm<T>(a, f.aw, m, n, k, r);
  if (d->method != CNMF_ADMM) layout_iter<T>(a, f.iw, m, n, k, r, f.full);
  if (A) layout_aop<T>(a, f.ao, A, std::max(f.full ? ru16(r) : 16, f.full ? 16 : passes_kkmax(f.passes)));
}

template <typename T>
AdmmJob admm_job_of(FactState<T>& f, const cnmf_input* A, const cnmf_factorize_desc* d) {
  const int m = (int)A->m, n = (int)A->n, k = d->sk.k, r = d->sk.r;
  AdmmJob J{};
  J.s0 = AdmmSide{f.w.Lb, k, f.aw.U, f.aw.Lam, r, m, d->lambda};
  J.s1 = AdmmSide{f.w.RTb, k, f.aw.Vt, f.aw.Phit, r, n, d->phi};
  J.At = f.w.At;
  J.XY = f.aw.XY;
  J.Pp = f.aw.Pp;
  J.Pred = f.aw.Pred;
  J.flags = f.w.flags + 2;
  J.lam = d->lambda;
  J.phi = d->phi;
  J.xi = d->xi;
  J.k = k;
  J.r = r;
  J.parts0 = f.aw.parts0;
  J.parts1 = f.aw.parts1;
  J.first = 1;
  return J;
}

template <typename T>
cnmf_status fact_prologue(cnmf_handle* h, const cnmf_input* A, const cnmf_factorize_desc* d,
                          const cnmf_factorize_out* o, FactState<T>& f) {
  const int m = (int)A->m, n = (int)A->n, k = d->sk.k, r = d->sk.r;
  hipStream_t st = h->stream;
  if (!f.full) {
    cnmf_status s = run_sketch<T>(h, A, &d->sk, f.w, f.ao, f.passes, o->sk_out.stats_dev);
    if (s != CNMF_OK) return s;
  } else {
    HIPCHK(h, launch_fill(f.w.flags, 8 * sizeof(int), st));
  }
  AdmmWs<T>& aw = f.aw;
  // state: U = U0, V^T = V0^T, Lam = Phi = 0
  HIPCHK(h, (launch_copy2d<double, T>(d->U0_dev, r, aw.U, r, m, r, 1.0, st)));
  HIPCHK(h, (launch_transpose<double, T>(d->V0_dev, n, aw.Vt, r, r, n, st)));
  HIPCHK(h, launch_fill(aw.Lam, sizeof(T) * (size_t)m * r, st));
  HIPCHK(h, launch_fill(aw.Phit, sizeof(T) * (size_t)n * r, st));
  HIPCHK(h, launch_fill(aw.counter, 4 * sizeof(unsigned), st));
  if (d->method == CNMF_ADMM) {
    AdmmJob J = admm_job_of(f, A, d);
    Span sp(h, ST_ITER);
    HIPCHK(h, launch_admm_uv<T>(J.s0, J.s1, 2, aw.XY, k, r, d->xi, 0, aw.Pp, aw.parts0, aw.parts1, st));
  }
  return CNMF_OK;
}

template <typename T>
cnmf_status fact_iterations(cnmf_handle* h, const cnmf_input* A, const cnmf_factorize_desc* d, FactState<T>& f) {
  const int m = (int)A->m, n = (int)A->n, k = d->sk.k, r = d->sk.r;
  hipStream_t st = h->stream;
  SketchWs<T>& w = f.w;
  AdmmWs<T>& aw = f.aw;
  IterWs<T>& iw = f.iw;
  auto row = [&](int rows, int blocks, const void* B1, int ldb1, const double* C, int k1, T* F, T* Mu,
                 const double* Gp, const double* Gm, const double* Minv, double pen, int method, const void* B2,
                 int k2, T* Op, double* Pp) -> cnmf_status {
    RowArgs ra{};
    ra.rows = rows;
    ra.k1 = k1;
    ra.r = r;
    ra.k2 = k2;
    ra.B1 = B1;
    ra.ldb1 = ldb1;
    ra.C = C;
    ra.F = F;
    ra.ldf = r;
    ra.Mu = Mu;
    ra.Gp = Gp;
    ra.Gm = Gm;
    ra.Minv = Minv;
    ra.pen = pen;
    ra.xi = d->xi;
    ra.eps = d->mu_eps;
    ra.method = method;
    ra.B2 = B2;
    ra.ldb2 = k;
    ra.Op = Op;
    ra.ldop = iw.kk;
    ra.Pp = Pp;
    HIPCHK(h, launch_nmf_row<T>(ra, blocks, st));
    return CNMF_OK;
  };
#define RUN(expr)                        \
  do {                                   \
    cnmf_status _s = (expr);             \
    if (_s != CNMF_OK) return _s;        \
  } while (0)

  if (d->method == CNMF_ADMM) {
    Span sp(h, ST_ITER, (double)d->iters * 4.0 * (double)(m + n) * k * r);
    AdmmJob J = admm_job_of(f, A, d);
    admm_job_prepare(J);
    AdmmHalf H{};
    H.s0 = J.s0;
    H.s1 = J.s1;
    H.At = J.At;
    H.Pred = J.Pred;
    H.XY = J.XY;
    H.Pp = J.Pp;
    H.flags = J.flags;
    H.lam = J.lam;
    H.phi = J.phi;
    H.xi = J.xi;
    H.k = k;
    H.r = r;
    H.parts0 = J.parts0;
    H.parts1 = J.parts1;
    H.rpb0 = J.rpb0;
    H.rpb1 = J.rpb1;
    // P_U, P_V of the initial U, V^T, then the first Xt (Yt^T from P_V / phi)
    if (d->iters > 0) {
      HIPCHK(h, launch_admm_reduce<T>(aw.Pp, aw.parts0, aw.parts1, k, r, 2, aw.Pred, st));
      H.solve = 1;
      H.pass = 0;
      H.first = 1;
      H.uv = 0;
      HIPCHK(h, launch_admm_half<T>(H, st));
    }
    H.first = 0;
    H.uv = 1;
    // From here on each solve's reduced partials are formed inside its own
    // launch where that pays (by workgroups beside the solve, which waits
    // for their count on aw.counter[0]; cleared by the prologue), else by
    // separate launches after each half; both sum in the same order.  P_V
    // of the first Yt^T solve is the one reduced above.
    const int nbh = (int)(((int64_t)k * r + 15) / 16);
    H.rgroups = admm_fused_reduce_groups(k, r, std::max(aw.parts0, aw.parts1));
    const bool fuse = H.rgroups > 0;
    const int nred = fuse ? (nbh + H.rgroups - 1) / H.rgroups : 0;
    unsigned signals = 0;
    H.ready = aw.counter;
    H.wait_fail = h->unresolved_dev + 1;
    for (int it = 0; it < d->iters; ++it) {
      const bool last = it + 1 == d->iters;
      H.mode = last ? 2 : 1;
      // Yt^T of this iteration (with P_V of the previous V-side row update)
      // beside the U-side row update (which needs Xt only)
      H.solve = 1;
      H.pass = 1;
      H.side = 0;
      H.nred = it > 0 ? nred : 0;
      signals += (unsigned)H.nred;
      H.ready_target = signals;
      HIPCHK(h, launch_admm_half<T>(H, st));
      if (!fuse && !last) HIPCHK(h, launch_admm_reduce<T>(aw.Pp, aw.parts0, aw.parts1, k, r, 0, aw.Pred, st));
      // the next iteration's Xt (with P_U of the U-side row update just
      // issued) beside the V-side row update
      H.solve = last ? 0 : 1;
      H.pass = 0;
      H.side = 1;
      H.nred = last ? 0 : nred;
      signals += (unsigned)H.nred;
      H.ready_target = signals;
      HIPCHK(h, launch_admm_half<T>(H, st));
      if (!fuse && !last) HIPCHK(h, launch_admm_reduce<T>(aw.Pp, aw.parts0, aw.parts1, k, r, 1, aw.Pred, st));
    }
  } else if (d->method == CNMF_MU) {
    Span sp(h, ST_ITER, (double)d->iters * (4.0 * (double)(m + n) * k * r + 4.0 * (double)(m + n) * r * r));
    // initial Yc^T = R V0^T
    RUN(row(n, iw.by, nullptr, 0, nullptr, k, aw.Vt, nullptr, nullptr, nullptr, nullptr, 0.0, 2, w.RTb, k, nullptr,
            iw.PpY));
    for (int it = 0; it < d->iters; ++it) {
      HIPCHK(h, launch_sum_parts(iw.PpY, iw.by, (int64_t)k * r, iw.S, st));
      HIPCHK(h, launch_nmf_small(iw.S, k, r, 0, 0.0, iw.Gp, iw.Gm, nullptr, st));
      RUN(row(m, iw.bx, w.Acb, k, iw.S, k, aw.U, nullptr, iw.Gp, iw.Gm, nullptr, 0.0, 0, w.Lb, k, nullptr, iw.PpX));
      HIPCHK(h, launch_sum_parts(iw.PpX, iw.bx, (int64_t)k * r, iw.S, st));
      HIPCHK(h, launch_nmf_small(iw.S, k, r, 0, 0.0, iw.Gp, iw.Gm, nullptr, st));
      RUN(row(n, iw.by, w.BTb, k, iw.S, k, aw.Vt, nullptr, iw.Gp, iw.Gm, nullptr, 0.0, 0, w.RTb, k, nullptr,
              iw.PpY));
    }
  } else if (d->method == CNMF_ANLS || d->method == CNMF_ANLS_FULL) {
    // alternating NNLS: per half-step the shared Gram G and the k x r (or
    // r x r) product C are formed from the other factor, every row is solved
    // to the end by the active-set kernel, and the row kernel's partial-sum
    // mode forms the next half-step's C from the new rows
    const bool cf = d->method == CNMF_ANLS;
    const int kk = iw.kk;
    int* info = w.flags + 6;
    HIPCHK(h, launch_fill(info, 2 * sizeof(int), st));
    auto half = [&](int rows, int blocks, const void* B1, int64_t ldb1, T* F, T* Op, const void* B2,
                    double* Pp) -> cnmf_status {
      AnlsArgs an{};
      an.rows = rows;
      an.r = r;
      an.k1 = cf ? k : r;
      an.B1 = B1;
      an.ldb1 = ldb1;
      an.C = cf ? iw.S : nullptr;
      an.G = cf ? iw.Gp : iw.S;
      an.H = iw.Gm;
      an.hok = iw.hok;
      an.F = F;
      an.ldf = r;
      an.Op = Op;
      an.ldop = kk;
      an.info = info;
      if (cf) HIPCHK(h, launch_nmf_small(iw.S, k, r, 3, 0.0, iw.Gp, nullptr, nullptr, st));
      // G^-1 and whether it checks out (the rows with few bound variables use it)
      HIPCHK(h, launch_spd_inverse(an.G, r, 0.0, iw.Gt, iw.Tinv, iw.Gm, iw.floored, iw.hok, st));
      HIPCHK(h, launch_anls_rows<T>(an, st));
      // partial sums of the next C over row slices (FP64 MFMA): B2^T F
      // (k x r) or the Gram F^T F
      const int parts = gram_parts(rows);
      if (cf)
        HIPCHK(h, (launch_cross2<T, T>((const T*)B2, k, 0, F, r, 0, 0, 1, rows, k, r, Pp, parts, st)));
      else
        HIPCHK(h, (launch_cross2<T, T>(F, r, 0, F, r, 0, 0, 1, rows, r, r, Pp, parts, st)));
      (void)blocks;
      return CNMF_OK;
    };
    const int px = gram_parts(m), py = gram_parts(n);
    if (cf) {
      Span sp(h, ST_ITER, (double)d->iters * 4.0 * (double)(m + n) * k * r);
      // initial Yc^T = R V0^T
      HIPCHK(h, (launch_cross2<T, T>(w.RTb, k, 0, aw.Vt, r, 0, 0, 1, n, k, r, iw.PpY, py, st)));
      for (int it = 0; it < d->iters; ++it) {
        HIPCHK(h, launch_sum_parts(iw.PpY, py, (int64_t)k * r, iw.S, st));
        RUN(half(m, iw.bx, w.Acb, k, aw.U, nullptr, w.Lb, iw.PpX));
        HIPCHK(h, launch_sum_parts(iw.PpX, px, (int64_t)k * r, iw.S, st));
        RUN(half(n, iw.by, w.BTb, k, aw.Vt, nullptr, w.RTb, iw.PpY));
      }
    } else {
      Span sp(h, ST_ITER, (double)d->iters * 4.0 * (double)m * n * r);
      HIPCHK(h, launch_fill(iw.Xop, sizeof(T) * (size_t)n * kk, st));
      HIPCHK(h, launch_fill(iw.Zop, sizeof(T) * (size_t)m * kk, st));
      HIPCHK(h, (launch_copy2d<T, T>(aw.Vt, r, iw.Xop, kk, n, r, 1.0, st)));
      // initial Gram of V0^T
      HIPCHK(h, (launch_cross2<T, T>(aw.Vt, r, 0, aw.Vt, r, 0, 0, 1, n, r, r, iw.PpY, py, st)));
      for (int it = 0; it < d->iters; ++it) {
        HIPCHK(h, launch_sum_parts(iw.PpY, py, (int64_t)r * r, iw.S, st));
        RUN(pass_full<T>(h, A, f.ao, true, iw.Xop, kk, iw.Pn, iw.Ppart));
        RUN(half(m, iw.bx, iw.Pn, kk, aw.U, iw.Zop, nullptr, iw.PpX));
        HIPCHK(h, launch_sum_parts(iw.PpX, px, (int64_t)r * r, iw.S, st));
        RUN(pass_full<T>(h, A, f.ao, false, iw.Zop, kk, iw.Pt, iw.Ppart));
        RUN(half(n, iw.by, iw.Pt, kk, aw.Vt, iw.Xop, nullptr, iw.PpY));
      }
    }
    // problems that did not finish reach cnmf_synchronize
    HIPCHK(h, launch_add_count(info, h->unresolved_dev, st));
  } else {
    // uncompressed comparators: L = I, R = I, two streaming passes per iteration
    const bool admm = d->method == CNMF_ADMM_FULL;
    // ADMM: Minv = (Gram + pen I)^-1 into Gp (floored pivots counted in
    // flags[2]); MU: the Gram's positive and negative parts into Gp, Gm
    auto small_step = [&](double pen) -> cnmf_status {
      if (admm) {
        HIPCHK(h, launch_spd_inverse(iw.S, r, pen, iw.Gt, iw.Tinv, iw.Gp, iw.floored, nullptr, st));
        HIPCHK(h, launch_add_count(iw.floored, w.flags + 2, st));
      } else {
        HIPCHK(h, launch_nmf_small(iw.S, r, r, 1, 0.0, iw.Gp, iw.Gm, nullptr, st));
      }
      return CNMF_OK;
    };
    const int kk = iw.kk;
    Span sp(h, ST_ITER, (double)d->iters * 4.0 * (double)m * n * r);
    HIPCHK(h, launch_fill(iw.Xop, sizeof(T) * (size_t)n * kk, st));
    HIPCHK(h, launch_fill(iw.Zop, sizeof(T) * (size_t)m * kk, st));
    HIPCHK(h, (launch_copy2d<T, T>(aw.Vt, r, iw.Xop, kk, n, r, 1.0, st)));
    // initial Gram of V0^T (= Yt^T for ADMM)
    RUN(row(n, iw.by, nullptr, 0, nullptr, r, aw.Vt, nullptr, nullptr, nullptr, nullptr, 0.0, 2, nullptr, r, nullptr,
            iw.PpY));
    for (int it = 0; it < d->iters; ++it) {
      HIPCHK(h, launch_sum_parts(iw.PpY, iw.by, (int64_t)r * r, iw.S, st));
      RUN(small_step(d->lambda));
      RUN(pass_full<T>(h, A, f.ao, true, iw.Xop, kk, iw.Pn, iw.Ppart));
      RUN(row(m, iw.bx, iw.Pn, kk, nullptr, r, aw.U, admm ? aw.Lam : nullptr, iw.Gp, iw.Gm, iw.Gp, d->lambda,
              admm ? 1 : 0, nullptr, r, iw.Zop, iw.PpX));
      HIPCHK(h, launch_sum_parts(iw.PpX, iw.bx, (int64_t)r * r, iw.S, st));
      RUN(small_step(d->phi));
      RUN(pass_full<T>(h, A, f.ao, false, iw.Zop, kk, iw.Pt, iw.Ppart));
      RUN(row(n, iw.by, iw.Pt, kk, nullptr, r, aw.Vt, admm ? aw.Phit : nullptr, iw.Gp, iw.Gm, iw.Gp, d->phi,
              admm ? 1 : 0, nullptr, r, iw.Xop, iw.PpY));
    }
  }
#undef RUN
  return CNMF_OK;
}

template <typename T>
cnmf_status fact_epilogue(cnmf_handle* h, const cnmf_input* A, const cnmf_factorize_desc* d,
                          const cnmf_factorize_out* o, FactState<T>& f) {
  const int m = (int)A->m, n = (int)A->n, r = d->sk.r;
  hipStream_t st = h->stream;
  AdmmWs<T>& aw = f.aw;
  if (o->U_dev) HIPCHK(h, (launch_copy2d<T, T>(aw.U, r, (T*)o->U_dev, r, m, r, 1.0, st)));
  if (o->V_dev) HIPCHK(h, (launch_transpose<T, T>(aw.Vt, r, (T*)o->V_dev, n, n, r, st)));
  if (o->rel_residual_dev) {
    Span sp(h, ST_RESID, 2.0 * m * n * (double)r);
    cnmf_status s = a_residual<T>(h, A, f.ao, aw.U, aw.Vt, r, aw.rpart, aw.rparts, o->rel_residual_dev);
    if (s != CNMF_OK) return s;
  }
  if (f.full) return CNMF_OK;
  return write_sketch_outputs<T>(h, A, &d->sk, f.w, &o->sk_out);
}

template <typename T>
cnmf_status do_factorize(cnmf_handle* h, const cnmf_input* A, const cnmf_factorize_desc* d,
                         const cnmf_factorize_out* o) {
  FactState<T> f;
  cnmf_status s = fact_plan<T>(h, d, f);
  if (s != CNMF_OK) return s;
  Arena dry(nullptr);
  fact_layout<T>(dry, f, A->m, A->n, d, A);
  s = ensure_ws(h, dry.off);
  if (s != CNMF_OK) return s;
  Arena a(h->ws);
  fact_layout<T>(a, f, A->m, A->n, d, A);
  s = fact_prologue<T>(h, A, d, o, f);
  if (s != CNMF_OK) return s;
  s = fact_iterations<T>(h, A, d, f);
  if (s != CNMF_OK) return s;
  return fact_epilogue<T>(h, A, d, o, f);
}

template <typename T>
size_t factorize_ws_bytes(const cnmf_input* A, const cnmf_factorize_desc* d) {
  FactState<T> f;
  if (fact_plan<T>(nullptr, d, f) != CNMF_OK) return 0;
  Arena dry(nullptr);
  fact_layout<T>(dry, f, A->m, A->n, d, A);
  return dry.off;
}

template <typename T>
cnmf_status do_select(cnmf_handle* h, const cnmf_input* A, const cnmf_sketch_desc* d, int64_t* K, double* score,
                      void* B_out) {
  std::vector<Pass> passes = plan_passes(d->k, d->q, d->sides, false, d->pass_dtype, d->final_dtype);
  const int m = (int)A->m, n = (int)A->n, k = d->k;
  Arena dry(nullptr);
  SketchWs<T> w;
  layout_sketch<T>(dry, w, m, n, k, passes, false, d);
  double* Bt64 = dry.take<double>((size_t)n * k);
  const int nblk = (n + 63) / 64;
  double* u = dry.take<double>(k);
  double* wb = dry.take<double>(nblk);
  int64_t* wi = dry.take<int64_t>(nblk);
  unsigned* ctr = dry.take<unsigned>(4);
  AOpWs<T> ao;
  layout_aop<T>(dry, ao, A, passes_kkmax(passes));
  cnmf_status s = ensure_ws(h, dry.off);
  if (s != CNMF_OK) return s;
  Arena a(h->ws);
  layout_sketch<T>(a, w, m, n, k, passes, false, d);
  Bt64 = a.take<double>((size_t)n * k);
  u = a.take<double>(k);
  wb = a.take<double>(nblk);
  wi = a.take<int64_t>(nblk);
  ctr = a.take<unsigned>(4);
  layout_aop<T>(a, ao, A, passes_kkmax(passes));
  hipStream_t st = h->stream;
  s = run_sketch<T>(h, A, d, w, ao, passes, nullptr);
  if (s != CNMF_OK) return s;
  HIPCHK(h, (launch_copy2d<T, double>(w.BTb, k, Bt64, k, n, k, 1.0, st)));
  {
    Span sp(h, ST_SPA);
    HIPCHK(h, launch_fill(ctr, 4 * sizeof(unsigned), st));
    for (int t = 0; t < d->r; ++t)
      HIPCHK(h, launch_spa_step(Bt64, n, k, k, t, K, score, u, wb, wi, ctr, nblk, st));
  }
  if (B_out) HIPCHK(h, (launch_transpose<T, T>(w.BTb, k, (T*)B_out, n, n, k, st)));
  return CNMF_OK;
}

}  // namespace

// ===========================================================================
// Hooks of the serving loop (server.cpp): one request run in phases inside a
// workspace block that the server owns.
// ===========================================================================
namespace cnmf {

cnmf_status serve_check(const cnmf_input* A, const cnmf_factorize_desc* d, const cnmf_factorize_out* o);

size_t serve_footprint(const cnmf_input* A, const cnmf_factorize_desc* d) {
  auto go = [&](auto tag) -> size_t {
    typedef decltype(tag) T;
    FactState<T> f;
    if (fact_plan<T>(nullptr, d, f) != CNMF_OK) return 0;
    Arena dry(nullptr);
    fact_layout<T>(dry, f, A->m, A->n, d);
    return dry.off;
  };
  return A->dtype == CNMF_F64 ? go(double{}) : go(float{});
}

cnmf_status serve_handle_create(int device, hipStream_t st, cnmf_handle** out) {
  cnmf_handle* h = new cnmf_handle();
  h->device = device;
  h->stream = st;
  h->ext_ws = true;
  timing_reset(h);
  *out = h;
  return CNMF_OK;
}

void serve_handle_destroy(cnmf_handle* h) {
  if (!h) return;
  for (hipEvent_t e : h->ev_pool) hipEventDestroy(e);
  delete h;
}

const char* serve_handle_error(const cnmf_handle* h) { return h->err.c_str(); }

// Batched (FP32 compressed ADMM with iterations): runs the prologue and
// fills *job; otherwise runs the whole request.  *batched says which.
cnmf_status serve_begin(cnmf_handle* h, char* ws, size_t ws_bytes, const cnmf_input* A, const cnmf_factorize_desc* d,
                        const cnmf_factorize_out* o, AdmmJob* job, bool* batched) {
  h->ws = ws;
  h->ws_bytes = ws_bytes;
  timing_reset(h);
  *batched = d->method == CNMF_ADMM && A->dtype == CNMF_F32 && d->iters > 0;
  if (!*batched) {
    if (A->dtype == CNMF_F64) return do_factorize<double>(h, A, d, o);
    return do_factorize<float>(h, A, d, o);
  }
  FactState<float> f;
  cnmf_status s = fact_plan<float>(h, d, f);
  if (s != CNMF_OK) return s;
  Arena dry(nullptr);
  fact_layout<float>(dry, f, A->m, A->n, d);
  s = ensure_ws(h, dry.off);
  if (s != CNMF_OK) return s;
  Arena a(h->ws);
  fact_layout<float>(a, f, A->m, A->n, d);
  s = fact_prologue<float>(h, A, d, o, f);
  if (s != CNMF_OK) return s;
  *job = admm_job_of(f, A, d);
  admm_job_prepare(*job);
  return CNMF_OK;
}

cnmf_status serve_end(cnmf_handle* h, char* ws, size_t ws_bytes, const cnmf_input* A, const cnmf_factorize_desc* d,
                      const cnmf_factorize_out* o) {
  h->ws = ws;
  h->ws_bytes = ws_bytes;
  FactState<float> f;
  cnmf_status s = fact_plan<float>(h, d, f);
  if (s != CNMF_OK) return s;
  Arena a(h->ws);
  fact_layout<float>(a, f, A->m, A->n, d);
  if (a.off > ws_bytes) return fail(h, CNMF_ENOMEM, "internal: workspace block too small");
  return fact_epilogue<float>(h, A, d, o, f);
}

}  // namespace cnmf

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* cnmf_version(void) { return "cnmf-mi355x 0.1"; }

const char* cnmf_status_string(cnmf_status s) {
  switch (s) {
    case CNMF_OK: return "ok";
    case CNMF_EINVAL: return "invalid argument";
    case CNMF_ENOMEM: return "out of device memory / workspace limit";
    case CNMF_EDEVICE: return "HIP device error";
    case CNMF_EBREAKDOWN: return "orthonormalisation breakdown";
    case CNMF_ENOTSUP: return "not supported";
    case CNMF_EBUSY: return "busy";
  }
  return "unknown status";
}

const char* cnmf_last_error(const cnmf_handle* h) { return h ? h->err.c_str() : g_noh_err.c_str(); }

cnmf_status cnmf_create(int device, void* hip_stream, size_t workspace_limit, cnmf_handle** out) {
  if (!out) return fail(nullptr, CNMF_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(nullptr, CNMF_EDEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(nullptr, CNMF_EINVAL, "device %d out of range [0, %d)", device, ndev);
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, CNMF_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  e = noalloc_scratch_init(device);
  if (e != hipSuccess)
    return fail(nullptr, CNMF_EDEVICE, "looking up the fixed scratch of cnmf_spa_noalloc failed: %s",
                hipGetErrorString(e));
  void* ud = nullptr;
  e = hipMalloc(&ud, 256);
  if (e != hipSuccess) return fail(nullptr, CNMF_ENOMEM, "hipMalloc(256) failed: %s", hipGetErrorString(e));
  e = launch_fill(ud, 256, (hipStream_t)hip_stream);
  if (e != hipSuccess) {
    hipFree(ud);
    return fail(nullptr, CNMF_EDEVICE, "clearing the breakdown counter failed: %s", hipGetErrorString(e));
  }
  cnmf_handle* h = new cnmf_handle();
  h->device = device;
  h->stream = (hipStream_t)hip_stream;
  h->limit = workspace_limit;
  h->unresolved_dev = (int*)ud;
  timing_reset(h);
  *out = h;
  return CNMF_OK;
}

cnmf_status cnmf_destroy(cnmf_handle* h) {
  if (!h) return CNMF_OK;
  hipSetDevice(h->device);
  hipStreamSynchronize(h->stream);
  if (h->ws) hipFree(h->ws);
  if (h->unresolved_dev) hipFree(h->unresolved_dev);
  if (h->copy_stream) {
    hipStreamSynchronize(h->copy_stream);
    hipStreamDestroy(h->copy_stream);
  }
  for (int i = 0; i < 2; ++i) {
    if (h->stage_ready[i]) hipEventDestroy(h->stage_ready[i]);
    if (h->stage_free[i]) hipEventDestroy(h->stage_free[i]);
  }
  for (hipEvent_t e : h->ev_pool) hipEventDestroy(e);
  delete h;
  return CNMF_OK;
}

cnmf_status cnmf_synchronize(cnmf_handle* h) {
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int words[2] = {0, 0};
  HIPCHK(h, hipMemcpy(words, h->unresolved_dev, sizeof(words), hipMemcpyDeviceToHost));
  const int unres = words[0];
  if (words[1]) {
    HIPCHK(h, launch_fill(h->unresolved_dev + 1, sizeof(int), h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return fail(h, CNMF_EDEVICE,
                "ADMM solves gave up waiting for the partial sums of their own launch %d time(s) (counted per "
                "waiting wave: the device did not run the launch's other workgroups within two seconds); the "
                "factors are not valid",
                words[1]);
  }
  if (unres) {
    HIPCHK(h, launch_fill(h->unresolved_dev, sizeof(int), h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return fail(h, CNMF_EBREAKDOWN,
                "%d CholeskyQR2 breakdown(s) not resolved by the fallback (NaN or Inf in the input, or a basis that "
                "stayed rank deficient)",
                unres);
  }
  return CNMF_OK;
}

cnmf_status cnmf_gaussian(cnmf_handle* h, uint64_t seed, int32_t matrix_id, int64_t rows, int32_t cols,
                          double* out_dev, int64_t ld) {
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  if (!out_dev) return fail(h, CNMF_EINVAL, "out_dev is NULL");
  if (rows < 0 || cols < 0 || ld < cols) return fail(h, CNMF_EINVAL, "bad shape rows=%lld cols=%d ld=%lld",
                                                      (long long)rows, cols, (long long)ld);
  if (rows > INT32_MAX / 2) return fail(h, CNMF_ENOTSUP, "rows above 2^30 are not supported");
  if (matrix_id < 0) return fail(h, CNMF_EINVAL, "matrix_id must be >= 0");
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, launch_gaussian_fill(out_dev, ld, (int)rows, cols, seed, (uint32_t)matrix_id, h->stream));
  return CNMF_OK;
}

cnmf_status cnmf_srht(cnmf_handle* h, uint64_t seed, int32_t matrix_id, int64_t rows, int32_t cols, double* out_dev,
                      int64_t ld) {
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  if (!out_dev) return fail(h, CNMF_EINVAL, "out_dev is NULL");
  if (rows < 1 || rows > INT32_MAX / 2) return fail(h, CNMF_EINVAL, "rows=%lld must be in [1, 2^30]", (long long)rows);
  int64_t p = 1;
  while (p < rows) p <<= 1;
  if (cols < 1 || cols > 128 || cols > p || ld < cols)
    return fail(h, CNMF_EINVAL, "cols=%d must be in [1, min(128, %lld)] and <= ld=%lld", cols, (long long)p,
                (long long)ld);
  if (matrix_id < 0) return fail(h, CNMF_EINVAL, "matrix_id must be >= 0");
  HIPCHK(h, hipSetDevice(h->device));
  cnmf_status s = ensure_ws(h, 128 * sizeof(int32_t));
  if (s != CNMF_OK) return s;
  HIPCHK(h, launch_srht_fill(out_dev, ld, (int)rows, cols, seed, (uint32_t)matrix_id, (int32_t*)h->ws, h->stream));
  return CNMF_OK;
}

cnmf_status cnmf_set_timing(cnmf_handle* h, int enable) {
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  h->timing = enable != 0;
  return CNMF_OK;
}

double cnmf_stage_ms(cnmf_handle* h, int stage) {
  if (!h || stage < 0 || stage >= kStages || !h->timing) return std::numeric_limits<double>::quiet_NaN();
  timing_resolve(h);
  return h->stage_count[stage] ? h->stage_ms[stage] : std::numeric_limits<double>::quiet_NaN();
}

double cnmf_stage_flops(cnmf_handle* h, int stage) {
  if (!h || stage < 0 || stage >= kStages) return 0.0;
  return h->stage_flops[stage];
}

int cnmf_stage_launches(cnmf_handle* h, int stage) {
  if (!h || stage < 0 || stage >= kStages) return 0;
  return h->stage_count[stage];
}

cnmf_status cnmf_sketch(cnmf_handle* h, const cnmf_input* A, const cnmf_sketch_desc* d, cnmf_sketch_out* out) {
  cnmf_status s = check_input(h, A);
  if (s != CNMF_OK) return s;
  s = check_sketch(h, A, d);
  if (s != CNMF_OK) return s;
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  HIPCHK(h, hipSetDevice(h->device));
  timing_reset(h);
  bool want_ac = out && out->Ac_dev && (d->sides & CNMF_RIGHT);
  if (A->dtype == CNMF_F64) return do_sketch<double>(h, A, d, out, want_ac);
  return do_sketch<float>(h, A, d, out, want_ac);
}

static cnmf_status check_factorize(cnmf_handle* h, const cnmf_input* A, const cnmf_factorize_desc* d) {
  if (!d) return fail(h, CNMF_EINVAL, "factorize descriptor is NULL");
  if (full_method(d->method)) {
    cnmf_sketch_desc sk = d->sk;  // only r and the precision matter
    sk.k = sk.r + 1 <= std::min(A->m, A->n) ? sk.r + 1 : sk.r;
    sk.sides = CNMF_LEFT;
    sk.q = 0;
    cnmf_status s = check_sketch(h, A, &sk);
    if (s != CNMF_OK) return s;
  } else {
    cnmf_status s = check_sketch(h, A, &d->sk);
    if (s != CNMF_OK) return s;
  }
  cnmf_status s = CNMF_OK;
  if (d->method < CNMF_ADMM || d->method > CNMF_ANLS_FULL) return fail(h, CNMF_EINVAL, "unknown method %d", d->method);
  if (!full_method(d->method) && d->sk.sides != CNMF_BOTH)
    return fail(h, CNMF_EINVAL, "compressed NMF needs sides = CNMF_BOTH");
  if (d->iters < 0) return fail(h, CNMF_EINVAL, "iters must be >= 0");
  if (d->method == CNMF_ADMM || d->method == CNMF_ADMM_FULL) {
    if (!(d->lambda > 0) || !(d->phi > 0) || !std::isfinite(d->lambda) || !std::isfinite(d->phi))
      return fail(h, CNMF_EINVAL, "lambda and phi must be finite and > 0");
    if (!(d->xi > 0) || !std::isfinite(d->xi)) return fail(h, CNMF_EINVAL, "xi must be finite and > 0");
  }
  if (!(d->mu_eps >= 0)) return fail(h, CNMF_EINVAL, "mu_eps must be >= 0");
  if (!d->U0_dev || !d->V0_dev) return fail(h, CNMF_EINVAL, "U0_dev and V0_dev are required");
  if (d->sk.r > 64) return fail(h, CNMF_ENOTSUP, "r=%d > 64 is not supported by the NMF iterations", d->sk.r);
  if (d->method == CNMF_ADMM && admm_solve_lds_bytes(d->sk.k, d->sk.r) > 160 * 1024)
    return fail(h, CNMF_ENOTSUP, "compressed ADMM at r=%d, k=%d needs more than 160 KiB of LDS (k <= 112 for r > 48)",
                d->sk.r, d->sk.k);
  return CNMF_OK;
}

}  // extern "C"

cnmf_status cnmf::serve_check(const cnmf_input* A, const cnmf_factorize_desc* d, const cnmf_factorize_out* o) {
  cnmf_status s = check_input(nullptr, A);
  if (s != CNMF_OK) return s;
  if (A->format != CNMF_DENSE) return fail(nullptr, CNMF_ENOTSUP, "the server takes dense device inputs");
  s = check_factorize(nullptr, A, d);
  if (s != CNMF_OK) return s;
  if (!o) return fail(nullptr, CNMF_EINVAL, "out is NULL");
  return CNMF_OK;
}

extern "C" {

cnmf_status cnmf_factorize(cnmf_handle* h, const cnmf_input* A, const cnmf_factorize_desc* d,
                           cnmf_factorize_out* out) {
  cnmf_status s = check_input(h, A);
  if (s != CNMF_OK) return s;
  s = check_factorize(h, A, d);
  if (s != CNMF_OK) return s;
  if (!out) return fail(h, CNMF_EINVAL, "out is NULL");
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  HIPCHK(h, hipSetDevice(h->device));
  timing_reset(h);
  if (A->dtype == CNMF_F64) return do_factorize<double>(h, A, d, out);
  return do_factorize<float>(h, A, d, out);
}

// A captured factorisation: every launch of one cnmf_factorize call,
// recorded on the handle's stream into a graph with a workspace of its own.
struct cnmf_graph {
  cnmf_handle* h = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipGraphExec_t exec = nullptr;
};

cnmf_status cnmf_factorize_capture(cnmf_handle* h, const cnmf_input* A, const cnmf_factorize_desc* d,
                                   const cnmf_factorize_out* out, cnmf_graph** graph) {
  cnmf_status s = check_input(h, A);
  if (s != CNMF_OK) return s;
  s = check_factorize(h, A, d);
  if (s != CNMF_OK) return s;
  if (!out || !graph) return fail(h, CNMF_EINVAL, "out and graph are required");
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  *graph = nullptr;
  if (!h->stream) return fail(h, CNMF_EINVAL, "capture needs a handle on a created stream (not the null stream)");
  if (A->format == CNMF_DENSE_HOST)
    return fail(h, CNMF_ENOTSUP, "inputs in host memory are streamed on a second stream: not captured");
  HIPCHK(h, hipSetDevice(h->device));
  const size_t bytes = std::max<size_t>(
      A->dtype == CNMF_F64 ? factorize_ws_bytes<double>(A, d) : factorize_ws_bytes<float>(A, d), kAlign);
  cnmf_graph* g = new cnmf_graph();
  g->h = h;
  hipError_t e = hipMalloc((void**)&g->ws, bytes);
  if (e != hipSuccess) {
    delete g;
    return fail(h, CNMF_ENOMEM, "graph workspace hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  g->ws_bytes = bytes;
  // record into the graph's own workspace (never grown), without timing events
  char* ws0 = h->ws;
  const size_t b0 = h->ws_bytes;
  const bool ext0 = h->ext_ws, tm0 = h->timing;
  h->ws = g->ws;
  h->ws_bytes = bytes;
  h->ext_ws = true;
  h->timing = false;
  timing_reset(h);
  hipGraph_t gr = nullptr;
  e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    s = A->dtype == CNMF_F64 ? do_factorize<double>(h, A, d, out) : do_factorize<float>(h, A, d, out);
    hipError_t e2 = hipStreamEndCapture(h->stream, &gr);
    if (s == CNMF_OK && e2 != hipSuccess) s = fail(h, CNMF_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e2));
  } else {
    s = fail(h, CNMF_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  h->ws = ws0;
  h->ws_bytes = b0;
  h->ext_ws = ext0;
  h->timing = tm0;
  if (s == CNMF_OK) {
    e = hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) s = fail(h, CNMF_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  if (gr) hipGraphDestroy(gr);
  if (s != CNMF_OK) {
    (void)hipGetLastError();
    hipFree(g->ws);
    delete g;
    return s;
  }
  *graph = g;
  return CNMF_OK;
}

cnmf_status cnmf_graph_launch(cnmf_graph* g) {
  if (!g) return fail(nullptr, CNMF_EINVAL, "graph is NULL");
  cnmf_handle* h = g->h;
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, hipGraphLaunch(g->exec, h->stream));
  return CNMF_OK;
}

cnmf_status cnmf_graph_destroy(cnmf_graph* g) {
  if (!g) return CNMF_OK;
  hipSetDevice(g->h->device);
  hipStreamSynchronize(g->h->stream);
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->ws) hipFree(g->ws);
  delete g;
  return CNMF_OK;
}

cnmf_status snmf_select(cnmf_handle* h, const cnmf_input* A, const cnmf_sketch_desc* d, int64_t* K_dev,
                        double* score_dev, void* B_dev) {
  cnmf_status s = check_input(h, A);
  if (s != CNMF_OK) return s;
  s = check_sketch(h, A, d);
  if (s != CNMF_OK) return s;
  if (!(d->sides & CNMF_LEFT)) return fail(h, CNMF_EINVAL, "SPA runs on B = Q^T A: sides must include CNMF_LEFT");
  if (!K_dev) return fail(h, CNMF_EINVAL, "K_dev is NULL");
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  HIPCHK(h, hipSetDevice(h->device));
  timing_reset(h);
  if (A->dtype == CNMF_F64) return do_select<double>(h, A, d, K_dev, score_dev, B_dev);
  return do_select<float>(h, A, d, K_dev, score_dev, B_dev);
}

static cnmf_status check_spa(cnmf_handle* h, const void* B_dev, cnmf_dtype dtype, int64_t k, int64_t n, int64_t ldb,
                             int32_t r, const int64_t* K_dev) {
  if (!B_dev || !K_dev) return fail(h, CNMF_EINVAL, "B_dev and K_dev are required");
  if (dtype != CNMF_F64 && dtype != CNMF_F32) return fail(h, CNMF_EINVAL, "B must be F64 or F32");
  if (k < 1 || n < 1 || ldb < n) return fail(h, CNMF_EINVAL, "bad B shape k=%lld n=%lld ldb=%lld", (long long)k, (long long)n, (long long)ldb);
  if (k > 128) return fail(h, CNMF_ENOTSUP, "k > 128 is not supported");
  if (n > INT32_MAX / 2) return fail(h, CNMF_ENOTSUP, "n above 2^30 is not supported");
  if (r < 1 || r > std::min<int64_t>(k, n)) return fail(h, CNMF_EINVAL, "r=%d must be in [1, min(k, n)]", r);
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  return CNMF_OK;
}

// SPA working storage (B^T in FP64, the unit pivot, per-block winners),
// laid out from `base` (NULL: sizing only); returns the bytes used.
struct SpaWs {
  double* Bt64;
  double* u;
  double* wb;
  int64_t* wi;
};
static size_t layout_spa(char* base, int64_t k, int64_t n, SpaWs& w) {
  const int nblk = (int)((n + 63) / 64);
  Arena a(base);
  w.Bt64 = a.take<double>((size_t)n * k);
  w.u = a.take<double>(k);
  w.wb = a.take<double>(nblk);
  w.wi = a.take<int64_t>(nblk);
  return a.off;
}

// Every word of the working storage is written before it is read (B^T by
// the transpose, u by step 0's pick, the winners by each step's norms), so
// nothing needs clearing.
static cnmf_status run_spa(cnmf_handle* h, const void* B_dev, cnmf_dtype dtype, int64_t k, int64_t n, int64_t ldb,
                           int32_t r, int64_t* K_dev, double* score_dev, const SpaWs& w) {
  hipStream_t st = h->stream;
  const int nblk = (int)((n + 63) / 64);
  if (dtype == CNMF_F64)
    HIPCHK(h, (launch_transpose<double, double>((const double*)B_dev, ldb, w.Bt64, k, (int)k, (int)n, st)));
  else
    HIPCHK(h, (launch_transpose<float, double>((const float*)B_dev, ldb, w.Bt64, k, (int)k, (int)n, st)));
  for (int t = 0; t < r; ++t)
    HIPCHK(h, launch_spa_step(w.Bt64, (int)n, (int)k, (int)k, t, K_dev, score_dev, w.u, w.wb, w.wi, nullptr, nblk,
                              st));
  return CNMF_OK;
}

cnmf_status cnmf_spa(cnmf_handle* h, const void* B_dev, cnmf_dtype dtype, int64_t k, int64_t n, int64_t ldb,
                     int32_t r, int64_t* K_dev, double* score_dev) {
  cnmf_status s = check_spa(h, B_dev, dtype, k, n, ldb, r, K_dev);
  if (s != CNMF_OK) return s;
  HIPCHK(h, hipSetDevice(h->device));
  SpaWs w;
  s = ensure_ws(h, layout_spa(nullptr, k, n, w));
  if (s != CNMF_OK) return s;
  layout_spa(h->ws, k, n, w);
  return run_spa(h, B_dev, dtype, k, n, ldb, r, K_dev, score_dev, w);
}

cnmf_status snmf_nnls(cnmf_handle* h, const void* B_dev, cnmf_dtype dtype, int64_t k, int64_t n, int64_t ldb,
                      int32_t r, const int64_t* K_dev, double* H_dev, int64_t ldh, int32_t* info_dev) {
  if (!B_dev || !K_dev || !H_dev) return fail(h, CNMF_EINVAL, "B_dev, K_dev and H_dev are required");
  if (dtype != CNMF_F64 && dtype != CNMF_F32) return fail(h, CNMF_EINVAL, "B must be F64 or F32");
  if (k < 1 || n < 1 || ldb < n) return fail(h, CNMF_EINVAL, "bad B shape k=%lld n=%lld ldb=%lld", (long long)k, (long long)n, (long long)ldb);
  if (k > 128) return fail(h, CNMF_ENOTSUP, "k > 128 is not supported");
  if (n > INT32_MAX / 2) return fail(h, CNMF_ENOTSUP, "n above 2^30 is not supported");
  if (r < 1 || r > std::min<int64_t>(k, n)) return fail(h, CNMF_EINVAL, "r=%d must be in [1, min(k, n)]", r);
  if (r > 64) return fail(h, CNMF_ENOTSUP, "r=%d > 64 is not supported", r);
  if (ldh < n) return fail(h, CNMF_EINVAL, "ldh (%lld) < n (%lld)", (long long)ldh, (long long)n);
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  HIPCHK(h, hipSetDevice(h->device));
  auto lay = [&](char* base, double** Bt, double** Cr, int** info) {
    Arena a(base);
    *Bt = a.take<double>((size_t)n * k);
    *Cr = a.take<double>((size_t)n * r);
    *info = a.take<int>(4);
    return a.off;
  };
  double *Bt, *Cr;
  int* info;
  cnmf_status s = ensure_ws(h, lay(nullptr, &Bt, &Cr, &info));
  if (s != CNMF_OK) return s;
  lay(h->ws, &Bt, &Cr, &info);
  int* inf = info_dev ? info_dev : info;
  hipStream_t st = h->stream;
  if (dtype == CNMF_F64)
    HIPCHK(h, (launch_transpose<double, double>((const double*)B_dev, ldb, Bt, k, (int)k, (int)n, st)));
  else
    HIPCHK(h, (launch_transpose<float, double>((const float*)B_dev, ldb, Bt, k, (int)k, (int)n, st)));
  HIPCHK(h, launch_fill(inf, 3 * sizeof(int), st));
  HIPCHK(h, launch_snmf_nnls(Bt, k, (int)n, (int)k, r, K_dev, Cr, H_dev, ldh, inf, st));
  return CNMF_OK;
}

cnmf_status cnmf_spa_noalloc(cnmf_handle* h, const void* B_dev, cnmf_dtype dtype, int64_t k, int64_t n,
                             int64_t ldb, int32_t r, int64_t* K_dev, double* score_dev) {
  cnmf_status s = check_spa(h, B_dev, dtype, k, n, ldb, r, K_dev);
  if (s != CNMF_OK) return s;
  SpaWs w;
  const size_t need = layout_spa(nullptr, k, n, w);
  if (need > kNoAllocScratchBytes)
    return fail(h, CNMF_ENOTSUP,
                "SPA of a %lld x %lld B needs %zu bytes of scratch; the fixed scratch holds %zu "
                "(about (k + 2) n <= 4.19e6 doubles); use cnmf_spa",
                (long long)k, (long long)n, need, kNoAllocScratchBytes);
  HIPCHK(h, hipSetDevice(h->device));
  char* base = (char*)noalloc_scratch(h->device);
  if (!base) return fail(h, CNMF_EDEVICE, "internal: the fixed scratch of device %d was not looked up", h->device);
  layout_spa(base, k, n, w);
  return run_spa(h, B_dev, dtype, k, n, ldb, r, K_dev, score_dev, w);
}

cnmf_status cnmf_range_product(cnmf_handle* h, const cnmf_input* A, int trans, const void* X_dev, int32_t kx,
                               void* Y_dev) {
  cnmf_status s = check_input(h, A);
  if (s != CNMF_OK) return s;
  if (A->format != CNMF_DENSE) return fail(h, CNMF_ENOTSUP, "cnmf_range_product takes a dense device A");
  if (trans != 0 && trans != 1) return fail(h, CNMF_EINVAL, "trans must be 0 or 1");
  if (!X_dev || !Y_dev) return fail(h, CNMF_EINVAL, "X_dev and Y_dev are required");
  if (kx < 1 || kx > 128) return fail(h, CNMF_EINVAL, "kx=%d must be in [1, 128]", kx);
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  HIPCHK(h, hipSetDevice(h->device));
  const int m = (int)A->m, n = (int)A->n, kk = ru16(kx);
  const int rows_in = trans ? m : n, rows_out = trans ? n : m;
  const size_t es = A->dtype == CNMF_F64 ? 8 : 4;
  const int splits = trans ? choose_splits_t(m, n, kk, (int)es) : choose_splits_n(m, n, kk, (int)es);
  Arena dry(nullptr);
  dry.take<char>((size_t)rows_in * kk * es);
  dry.take<char>((size_t)rows_out * kk * es);
  dry.take<char>((size_t)std::max(splits, 1) * rows_out * kk * es);
  s = ensure_ws(h, dry.off);
  if (s != CNMF_OK) return s;
  Arena a(h->ws);
  hipStream_t st = h->stream;
  auto run = [&](auto tag) -> cnmf_status {
    typedef decltype(tag) T;
    T* Xp = a.take<T>((size_t)rows_in * kk);
    T* Yp = a.take<T>((size_t)rows_out * kk);
    T* Pp = a.take<T>((size_t)std::max(splits, 1) * rows_out * kk);
    HIPCHK(h, launch_fill(Xp, sizeof(T) * (size_t)rows_in * kk, st));
    HIPCHK(h, (launch_copy2d<T, T>((const T*)X_dev, kx, Xp, kk, rows_in, kx, 1.0, st)));
    T* dst = splits > 1 ? Pp : Yp;
    if (trans)
      HIPCHK(h, launch_gemm_t<T>((const T*)A->data_dev, A->lda, m, n, Xp, kk, dst, splits, st));
    else
      HIPCHK(h, launch_gemm_n<T>((const T*)A->data_dev, A->lda, m, n, Xp, kk, dst, splits, st));
    if (splits > 1) HIPCHK(h, launch_reduce_splits<T>(Pp, splits, rows_out, kk, Yp, st));
    HIPCHK(h, (launch_copy2d<T, T>(Yp, kk, (T*)Y_dev, kx, rows_out, kx, 1.0, st)));
    return CNMF_OK;
  };
  if (A->dtype == CNMF_F64) return run(double{});
  return run(float{});
}

cnmf_status cnmf_range_product_lowp(cnmf_handle* h, const cnmf_input* A, int trans, cnmf_dtype pass_dtype,
                                    const double* X_dev, int32_t kx, float* Y_dev) {
  cnmf_status s = check_input(h, A);
  if (s != CNMF_OK) return s;
  if (A->format != CNMF_DENSE) return fail(h, CNMF_ENOTSUP, "reduced-precision passes take a dense device A");
  if (A->dtype != CNMF_F32) return fail(h, CNMF_EINVAL, "reduced-precision passes need an F32 input");
  if (pass_dtype != CNMF_BF16 && pass_dtype != CNMF_FP8_E4M3)
    return fail(h, CNMF_EINVAL, "pass_dtype must be CNMF_BF16 or CNMF_FP8_E4M3");
  if (trans != 0 && trans != 1) return fail(h, CNMF_EINVAL, "trans must be 0 or 1");
  if (!X_dev || !Y_dev) return fail(h, CNMF_EINVAL, "X_dev and Y_dev are required");
  if (kx < 1 || kx > 128) return fail(h, CNMF_EINVAL, "kx=%d must be in [1, 128]", kx);
  if (!h) return fail(nullptr, CNMF_EINVAL, "handle is NULL");
  HIPCHK(h, hipSetDevice(h->device));
  const int m = (int)A->m, n = (int)A->n, kk = ru16(kx);
  const int rows_out = trans ? n : m, cols = trans ? m : n;
  const int es = lowp_es(pass_dtype);
  const int64_t ldo = lowp_pad(n), ldt = lowp_pad(m);
  const int64_t ldm = trans ? ldt : ldo;
  const int ntj = (n + kFp8Tile - 1) / kFp8Tile, nti = (m + kFp8Tile - 1) / kFp8Tile;
  const int splits = choose_splits_lowp(rows_out, cols, kk, es);
  auto layout = [&](Arena& a, uint8_t** Mc, float** tsc, uint8_t** Xt, float** cs, float** Yp, float** Pp,
                    unsigned long long** cm) {
    *Mc = a.take<uint8_t>((size_t)es * lowp_pad(rows_out) * ldm);
    *tsc = a.take<float>((size_t)ntj * nti);
    *Xt = a.take<uint8_t>((size_t)es * kk * ldm);
    *cs = a.take<float>(128);
    *Yp = a.take<float>((size_t)rows_out * kk);
    *Pp = a.take<float>((size_t)std::max(splits, 1) * rows_out * kk);
    *cm = a.take<unsigned long long>(128);
  };
  uint8_t *Mc, *Xt;
  float *tsc, *cs, *Yp, *Pp;
  unsigned long long* cm;
  Arena dry(nullptr);
  layout(dry, &Mc, &tsc, &Xt, &cs, &Yp, &Pp, &cm);
  s = ensure_ws(h, dry.off);
  if (s != CNMF_OK) return s;
  Arena a(h->ws);
  layout(a, &Mc, &tsc, &Xt, &cs, &Yp, &Pp, &cm);
  hipStream_t st = h->stream;
  const float* Ap = (const float*)A->data_dev;
  // only the copy this direction reads is written
  __hip_bfloat16* c16 = es == 2 ? (__hip_bfloat16*)Mc : nullptr;
  uint8_t* c8 = es == 1 ? Mc : nullptr;
  HIPCHK(h, launch_convert_lowp(Ap, A->lda, m, n, trans ? nullptr : c16, trans ? c16 : nullptr, trans ? nullptr : c8,
                                trans ? c8 : nullptr, ldo, ldt, tsc, st));
  HIPCHK(h, launch_fill(Xt, (size_t)es * kk * ldm, st));
  HIPCHK(h, launch_store_lowp(es, X_dev, cols, kx, 0, kx, Xt, ldm, 0, cs, 0, cm, st));
  float* dst = splits > 1 ? Pp : Yp;
  HIPCHK(h, launch_gemm_lowp(es, Mc, ldm, lowp_pad(rows_out), rows_out, cols, Xt, ldm, kk, dst, splits, tsc, ntj,
                             trans, st));
  if (splits > 1) HIPCHK(h, launch_reduce_splits<float>(Pp, splits, rows_out, kk, Yp, st));
  if (es == 1) HIPCHK(h, launch_unscale_cols(Yp, rows_out, kk, kx, cs, st));
  HIPCHK(h, (launch_copy2d<float, float>(Yp, kk, Y_dev, kx, rows_out, kx, 1.0, st)));
  return CNMF_OK;
}

cnmf_status cnmf_workspace_bytes(int64_t m, int64_t n, const cnmf_factorize_desc* d, size_t* bytes) {
  if (!d || !bytes) return fail(nullptr, CNMF_EINVAL, "descriptor and bytes are required");
  if (m < 1 || n < 1) return fail(nullptr, CNMF_EINVAL, "m and n must be >= 1");
  const int k = d->sk.k, r = d->sk.r;
  if (r < 1 || k <= r || k > std::min<int64_t>(m, n) || k > 128)
    return fail(nullptr, CNMF_EINVAL, "need 1 <= r < k <= min(m, n), k <= 128");
  const bool f64 = d->sk.pass_dtype == CNMF_F64;
  const bool want_ac = method_wants_ac(d->method);
  const bool full = full_method(d->method);
  std::vector<Pass> passes = plan_passes(k, d->sk.q, d->sk.sides ? d->sk.sides : CNMF_BOTH, want_ac,
                                         d->sk.pass_dtype, d->sk.final_dtype);
  Arena dry(nullptr);
  auto go = [&](auto tag) {
    typedef decltype(tag) T;
    SketchWs<T> w;
    AdmmWs<T> aw;
    IterWs<T> iw;
    if (!full)
      layout_sketch<T>(dry, w, m, n, k, passes, want_ac, &d->sk);
    else
      dry.take<int>(8);
    layout_admm<T>(dry, aw, m, n, k, r);
    if (d->method != CNMF_ADMM) layout_iter<T>(dry, iw, m, n, k, r, full);
  };
  if (f64)
    go(double{});
  else
    go(float{});
  *bytes = dry.off;
  return CNMF_OK;
}

}  // extern "C"
