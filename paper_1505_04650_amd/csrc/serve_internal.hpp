// Hooks between the serving loop (server.cpp) and the request runtime
// (runtime.cpp), and the host-side admission policy shared by the server and
// its planning simulation.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>

#include "../../include/cnmf.h"
#include "cnmf_internal.hpp"

namespace cnmf {

// Synchronous checks of a factorisation request (thread-local error text).
cnmf_status serve_check(const cnmf_input* A, const cnmf_factorize_desc* d, const cnmf_factorize_out* o);
// Device workspace bytes of one request (the admission footprint).
size_t serve_footprint(const cnmf_input* A, const cnmf_factorize_desc* d);
// A handle whose workspace is supplied per call (never allocated).
cnmf_status serve_handle_create(int device, hipStream_t st, cnmf_handle** out);
void serve_handle_destroy(cnmf_handle* h);
const char* serve_handle_error(const cnmf_handle* h);
// FP32 compressed ADMM with iterations: prologue only, *job describes the
// iterations (*batched = true).  Any other request runs whole.
cnmf_status serve_begin(cnmf_handle* h, char* ws, size_t ws_bytes, const cnmf_input* A, const cnmf_factorize_desc* d,
                        const cnmf_factorize_out* o, AdmmJob* job, bool* batched);
// Outputs and residual of a batched request after its last iteration.
cnmf_status serve_end(cnmf_handle* h, char* ws, size_t ws_bytes, const cnmf_input* A, const cnmf_factorize_desc* d,
                      const cnmf_factorize_out* o);

// First-fit allocator of offsets in [0, capacity), 256-byte granules,
// coalescing neighbours on release.  Host-side bookkeeping of the server's
// device arena.
class BlockArena {
 public:
  static constexpr size_t kGranule = 256;
  explicit BlockArena(size_t capacity);
  static size_t round(size_t bytes) { return (bytes + kGranule - 1) / kGranule * kGranule; }
  bool alloc(size_t bytes, size_t* off);  // bytes already rounded
  void release(size_t off, size_t bytes);
  size_t capacity() const { return cap_; }
  size_t free_bytes() const { return free_total_; }
  size_t largest_free() const;

 private:
  size_t cap_;
  size_t free_total_;
  std::map<size_t, size_t> free_;  // offset -> size
};

// Admission (continuous batching by HBM footprint).  Requests wait in
// arrival order.  The head is admitted as soon as a block of its size is
// free.  While the head waits, a later request (within `window` places) may
// be admitted if it fits and the free bytes left afterwards still cover the
// head, at most `max_bypass` times per head; then the queue waits for the
// head.  Returns the index in `pending` to admit, or -1.
struct AdmissionState {
  int bypassed = 0;  // admissions that passed the current head
};
int pick_admission(const std::deque<size_t>& pending_bytes, const BlockArena& arena, int free_slots,
                   AdmissionState& st, int window = 32, int max_bypass = 64);

}  // namespace cnmf
