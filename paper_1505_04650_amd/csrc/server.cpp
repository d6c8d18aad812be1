// Serving loop: continuous batching of factorisation requests on one GPU.
//
// A request (A, r, k, q, initial factors, ADMM parameters) is submitted from
// any host thread and returns a ticket at once.  One dispatcher thread owns
// every HIP launch of the server:
//   * admission: requests wait in arrival order and are admitted when a
//     workspace block of their footprint fits in the server's device arena
//     (HBM budget) and an in-flight slot is free;
//   * prologue: the sketch (Alg. 1 and the small sketches), the initial
//     state and the first partials run on one of a few worker streams, so
//     the passes of new requests overlap the iterations of the others;
//   * batched iterations: every request whose prologue has finished joins
//     the batch; one batch step advances all of them by one ADMM iteration
//     (Appendix B, Alg. 3): the step's descriptor table is copied to the
//     device and three descriptor-driven kernels cover every job's blocks.
//     Either the grids are sized to the step (direct launches), or
//     (CNMF_SERVER_GRAPHS) fixed-grid kernels take the blocks from counters
//     in the table, and the copy and the three launches are captured once
//     per descriptor slot and shape class as a graph and replayed for every
//     step.  A request leaves the batch after its last iteration;
//   * epilogue: outputs and the FP64 residual on a worker stream.
// Each job in a batched launch runs the same per-request code as
// cnmf_factorize, so a result does not depend on the other requests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "serve_internal.hpp"

using namespace cnmf;

namespace cnmf {

BlockArena::BlockArena(size_t capacity) : cap_(capacity / kGranule * kGranule), free_total_(cap_) {
  if (cap_) free_[0] = cap_;
}

bool BlockArena::alloc(size_t bytes, size_t* off) {
  if (bytes == 0) bytes = kGranule;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes, noff = it->first + bytes;
      free_.erase(it);
      if (rest) free_[noff] = rest;
      free_total_ -= bytes;
      return true;
    }
  }
  return false;
}

void BlockArena::release(size_t off, size_t bytes) {
  if (bytes == 0) bytes = kGranule;
  auto it = free_.emplace(off, bytes).first;
  free_total_ += bytes;
  auto nx = std::next(it);
  if (nx != free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    free_.erase(nx);
  }
  if (it != free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      free_.erase(it);
    }
  }
}

size_t BlockArena::largest_free() const {
  size_t m = 0;
  for (const auto& kv : free_) m = std::max(m, kv.second);
  return m;
}

int pick_admission(const std::deque<size_t>& pending, const BlockArena& arena, int free_slots, AdmissionState& st,
                   int window, int max_bypass) {
  if (free_slots <= 0 || pending.empty()) return -1;
  const size_t head = pending.front();
  const size_t largest = arena.largest_free();
  if (head <= largest) return 0;
  if (st.bypassed >= max_bypass) return -1;
  const size_t free = arena.free_bytes();
  const int lim = std::min<int>((int)pending.size(), window + 1);
  for (int i = 1; i < lim; ++i) {
    const size_t b = pending[i];
    if (b <= largest && free >= b && free - b >= head) return i;
  }
  return -1;
}

}  // namespace cnmf

namespace {

enum ReqState { kQueued = 0, kPrologue = 1, kReady = 2, kActive = 3, kFinishing = 4, kDone = 5 };

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t ticket = 0;
  cnmf_input A{};
  cnmf_factorize_desc d{};
  cnmf_factorize_out o{};
  size_t bytes = 0, off = 0;
  int state = kQueued;
  cnmf_status status = CNMF_OK;
  cnmf_status begin_status = CNMF_OK;
  std::string err;
  hipEvent_t ev_in = nullptr, ev_ready = nullptr, ev_done = nullptr;
  AdmmJob job{};
  bool batched = false;
  int it = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

thread_local std::string g_server_err;

cnmf_status sfail(cnmf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_server_err = buf;
  return s;
}

constexpr int kRing = 3;  // descriptor buffers (at most 2 steps in flight)

}  // namespace

struct cnmf_server {
  int device = 0;
  size_t budget = 0;
  int max_batch = 0, nworkers = 0, max_inflight = 0;
  char* arena_dev = nullptr;
  BlockArena arena{0};
  hipStream_t batch_stream = nullptr;
  struct Worker {
    hipStream_t stream = nullptr;
    cnmf_handle* h = nullptr;
  };
  std::vector<Worker> workers;
  int next_worker = 0;
  // batched-step descriptors: [jobs x max_batch][uv_first x (max_batch + 1)][red_first x (max_batch + 1)]
  size_t desc_bytes = 0;
  char* desc_host[kRing] = {};
  char* desc_dev[kRing] = {};
  hipEvent_t step_ev[kRing] = {};
  long steps_issued = 0, steps_done = 0;
  // captured batch steps: (slot, k and r rounded up to 16) -> executable graph
  std::unordered_map<int, hipGraphExec_t> graphs;
  bool use_graphs = false;
  int max_steps_in_flight = 2;   // at most kRing - 1
  // shared with submitting threads (guarded by mu)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req*> pending;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  int admitted = 0;
  bool stopping = false;
  AdmissionState adm;
  cnmf_server_stats stats{};
  // dispatcher only
  std::vector<Req*> prologue, ready, active, finishing;
  std::thread th;
};

namespace {

// [BatchHeader][jobs x max_batch][uv_first x (max_batch + 1)][red_first x (max_batch + 1)]
constexpr size_t kOffJobs = 256;

size_t desc_layout(int max_batch, size_t* off_uv, size_t* off_red) {
  size_t o = kOffJobs + (size_t)max_batch * sizeof(AdmmJob);
  o = (o + 255) / 256 * 256;
  *off_uv = o;
  o += (size_t)(max_batch + 1) * sizeof(int);
  o = (o + 255) / 256 * 256;
  *off_red = o;
  o += (size_t)(max_batch + 1) * sizeof(int);
  return (o + 255) / 256 * 256;
}

// Under S->mu.
void finish_locked(cnmf_server* S, Req* r, cnmf_status st, const std::string& msg) {
  r->status = st;
  r->err = msg;
  r->state = kDone;
  r->t_done = now_ms();
  S->arena.release(r->off, r->bytes);
  S->admitted -= 1;
  if (st == CNMF_OK)
    S->stats.completed += 1;
  else
    S->stats.failed += 1;
}

void finish(cnmf_server* S, Req* r, cnmf_status st, const std::string& msg) {
  std::lock_guard<std::mutex> lk(S->mu);
  finish_locked(S, r, st, msg);
}

void set_state(cnmf_server* S, Req* r, int state) {
  std::lock_guard<std::mutex> lk(S->mu);
  r->state = state;
}

// Prologue (or the whole request) of r on the next worker stream.
void launch_begin(cnmf_server* S, Req* r) {
  cnmf_server::Worker& W = S->workers[S->next_worker];
  S->next_worker = (S->next_worker + 1) % S->nworkers;
  hipError_t e = hipSuccess;
  if (r->ev_in) e = hipStreamWaitEvent(W.stream, r->ev_in, 0);
  cnmf_status s = CNMF_EDEVICE;
  if (e == hipSuccess)
    s = serve_begin(W.h, S->arena_dev + r->off, r->bytes, &r->A, &r->d, &r->o, &r->job, &r->batched);
  r->begin_status = s;
  if (s != CNMF_OK) r->err = e == hipSuccess ? serve_handle_error(W.h) : hipGetErrorString(e);
  // the block is released only after everything enqueued for r has run
  e = hipEventRecord(r->ev_ready, W.stream);
  if (e != hipSuccess) {
    hipStreamSynchronize(W.stream);
    finish(S, r, CNMF_EDEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
    return;
  }
  S->prologue.push_back(r);
}

void launch_end(cnmf_server* S, Req* r, hipEvent_t after) {
  cnmf_server::Worker& W = S->workers[S->next_worker];
  S->next_worker = (S->next_worker + 1) % S->nworkers;
  hipError_t e = hipStreamWaitEvent(W.stream, after, 0);
  cnmf_status s = e == hipSuccess ? serve_end(W.h, S->arena_dev + r->off, r->bytes, &r->A, &r->d, &r->o)
                                  : CNMF_EDEVICE;
  if (s != CNMF_OK) {
    r->begin_status = s;
    r->err = e == hipSuccess ? serve_handle_error(W.h) : hipGetErrorString(e);
  }
  e = hipEventRecord(r->ev_done, W.stream);
  if (e != hipSuccess) {
    hipStreamSynchronize(W.stream);
    finish(S, r, CNMF_EDEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
    return;
  }
  set_state(S, r, kFinishing);
  S->finishing.push_back(r);
}

// One batched ADMM iteration for every active request.
bool batch_step(cnmf_server* S) {
  while (S->steps_done < S->steps_issued && hipEventQuery(S->step_ev[S->steps_done % kRing]) == hipSuccess)
    S->steps_done += 1;
  // join
  while (!S->ready.empty() && (int)S->active.size() < S->max_batch) {
    Req* r = S->ready.front();
    S->ready.erase(S->ready.begin());
    hipStreamWaitEvent(S->batch_stream, r->ev_ready, 0);
    set_state(S, r, kActive);
    S->active.push_back(r);
  }
  if (S->active.empty() || S->steps_issued - S->steps_done >= S->max_steps_in_flight) return false;
  const int slot = (int)(S->steps_issued % kRing);
  size_t off_uv, off_red;
  desc_layout(S->max_batch, &off_uv, &off_red);
  BatchHeader* hd = reinterpret_cast<BatchHeader*>(S->desc_host[slot]);
  AdmmJob* jobs = reinterpret_cast<AdmmJob*>(S->desc_host[slot] + kOffJobs);
  int* uvf = reinterpret_cast<int*>(S->desc_host[slot] + off_uv);
  int* rdf = reinterpret_cast<int*>(S->desc_host[slot] + off_red);
  int uv_total = 0, red_total = 0, max_k = 1, max_r = 1;
  size_t lds = 0;
  const int nj = (int)S->active.size();
  for (int j = 0; j < nj; ++j) {
    Req* r = S->active[j];
    jobs[j] = r->job;
    jobs[j].first = r->it == 0 ? 1 : 0;
    jobs[j].last = r->it + 1 == r->d.iters ? 1 : 0;
    uvf[j] = uv_total;
    rdf[j] = red_total;
    uv_total += admm_job_uv_blocks(r->job);
    red_total += admm_job_red_blocks(r->job);
    max_k = std::max(max_k, r->job.k);
    max_r = std::max(max_r, r->job.r);
    lds = std::max(lds, admm_job_solve_lds(r->job));
  }
  uvf[nj] = uv_total;
  rdf[nj] = red_total;
  *hd = BatchHeader{};
  hd->njobs = nj;
  hd->uv_total = uv_total;
  hd->red_total = red_total;
  // shape class: the launch configuration depends on k and r rounded up to 16
  const int KP = (max_k + 15) / 16 * 16, RP = (max_r + 15) / 16 * 16;
  const size_t uv_lds = admm_batch_uv_lds(KP, RP);
  const size_t solve_lds = std::min<size_t>(admm_solve_lds_bytes(KP, RP), 160 * 1024);
  const int grid_solve = S->max_batch;
  const int grid_red = 1024;
  const int grid_uv = 256 * (int)std::max<size_t>(1, std::min<size_t>(4, (160 * 1024) / uv_lds));
  hipError_t e = hipSuccess;
  auto enqueue = [&]() -> hipError_t {
    hipError_t x = hipMemcpyAsync(S->desc_dev[slot], S->desc_host[slot], S->desc_bytes, hipMemcpyHostToDevice,
                                  S->batch_stream);
    if (x == hipSuccess)
      x = launch_admm_step_fixed(S->desc_dev[slot], kOffJobs, off_uv, off_red, grid_solve, grid_red, grid_uv,
                                 uv_lds, solve_lds, S->batch_stream);
    return x;
  };
  bool replayed = false;
  if (lds > solve_lds || !S->use_graphs) {
    // direct launches sized to this batch (also when a job needs more LDS
    // than its class provides)
    e = hipMemcpyAsync(S->desc_dev[slot], S->desc_host[slot], S->desc_bytes, hipMemcpyHostToDevice,
                       S->batch_stream);
    if (e == hipSuccess)
      e = launch_admm_step_batch(reinterpret_cast<const AdmmJob*>(S->desc_dev[slot] + kOffJobs),
                                 reinterpret_cast<const int*>(S->desc_dev[slot] + off_uv),
                                 reinterpret_cast<const int*>(S->desc_dev[slot] + off_red), nj, uv_total, red_total,
                                 max_k, max_r, lds, S->batch_stream);
  } else {
    const int key = (slot * 16 + KP / 16) * 16 + RP / 16;
    auto it = S->graphs.find(key);
    if (it == S->graphs.end()) {
      // capture the copy and the three launches once for this slot and class
      hipGraph_t g = nullptr;
      hipGraphExec_t x = nullptr;
      e = hipStreamBeginCapture(S->batch_stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t e1 = enqueue();
        e = hipStreamEndCapture(S->batch_stream, &g);
        if (e1 != hipSuccess) e = e1;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (g) hipGraphDestroy(g);
      if (e == hipSuccess) {
        it = S->graphs.emplace(key, x).first;
        std::lock_guard<std::mutex> lk(S->mu);
        S->stats.graphs_built += 1;
      } else {
        // no graphs on this device or runtime: direct launches from now on
        (void)hipGetLastError();
        S->use_graphs = false;
        e = hipSuccess;
      }
    }
    if (S->use_graphs) {
      e = hipGraphLaunch(it->second, S->batch_stream);
      replayed = e == hipSuccess;
    } else {
      e = enqueue();
    }
  }
  if (e == hipSuccess) e = hipEventRecord(S->step_ev[slot], S->batch_stream);
  if (e != hipSuccess) {
    // nothing more can run for these requests: drain and fail them
    hipStreamSynchronize(S->batch_stream);
    for (Req* r : S->active) finish(S, r, CNMF_EDEVICE, std::string("batched step: ") + hipGetErrorString(e));
    S->active.clear();
    return true;
  }
  S->steps_issued += 1;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stats.batch_steps += 1;
    S->stats.graph_replays += replayed ? 1 : 0;
    S->stats.batched_iterations += nj;
    S->stats.max_batch_seen = std::max<int64_t>(S->stats.max_batch_seen, nj);
  }
  std::vector<Req*> keep;
  keep.reserve(S->active.size());
  for (Req* r : S->active) {
    r->it += 1;
    if (r->it >= r->d.iters)
      launch_end(S, r, S->step_ev[slot]);
    else
      keep.push_back(r);
  }
  S->active.swap(keep);
  return true;
}

void dispatcher(cnmf_server* S) {
  hipSetDevice(S->device);
  std::deque<size_t> sizes;
  for (;;) {
    bool progress = false;
    // retire finished requests
    for (size_t i = 0; i < S->finishing.size();) {
      Req* r = S->finishing[i];
      hipError_t q = hipEventQuery(r->ev_done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess)
        finish(S, r, CNMF_EDEVICE, hipGetErrorString(q));
      else
        finish(S, r, r->begin_status, r->err);
      S->finishing.erase(S->finishing.begin() + i);
      progress = true;
    }
    // prologues that have run
    for (size_t i = 0; i < S->prologue.size();) {
      Req* r = S->prologue[i];
      hipError_t q = hipEventQuery(r->ev_ready);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      S->prologue.erase(S->prologue.begin() + i);
      progress = true;
      if (q != hipSuccess) {
        finish(S, r, CNMF_EDEVICE, hipGetErrorString(q));
      } else if (r->begin_status != CNMF_OK || !r->batched) {
        finish(S, r, r->begin_status, r->err);
      } else {
        set_state(S, r, kReady);
        S->ready.push_back(r);
      }
    }
    // admission
    for (;;) {
      Req* r = nullptr;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        sizes.clear();
        for (size_t i = 0; i < S->pending.size() && i < 33; ++i) sizes.push_back(S->pending[i]->bytes);
        const int idx = pick_admission(sizes, S->arena, S->max_inflight - S->admitted, S->adm);
        if (idx < 0) break;
        r = S->pending[idx];
        if (!S->arena.alloc(r->bytes, &r->off)) break;  // cannot happen: the policy checked the block
        S->pending.erase(S->pending.begin() + idx);
        if (idx == 0)
          S->adm.bypassed = 0;
        else
          S->adm.bypassed += 1;
        S->admitted += 1;
        r->state = kPrologue;
        r->t_admit = now_ms();
        S->stats.peak_arena_bytes =
            std::max<uint64_t>(S->stats.peak_arena_bytes, S->arena.capacity() - S->arena.free_bytes());
      }
      launch_begin(S, r);
      progress = true;
    }
    if (batch_step(S)) progress = true;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->stopping && S->pending.empty() && S->admitted == 0) break;
    if (!progress) {
      if (S->admitted == 0 && S->pending.empty())
        S->cv.wait(lk, [&] { return S->stopping || !S->pending.empty(); });
      else
        S->cv.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

void destroy_server(cnmf_server* S) {
  for (auto& W : S->workers) {
    if (W.stream) hipStreamSynchronize(W.stream);
    serve_handle_destroy(W.h);
    if (W.stream) hipStreamDestroy(W.stream);
  }
  if (S->batch_stream) {
    hipStreamSynchronize(S->batch_stream);
    hipStreamDestroy(S->batch_stream);
  }
  for (auto& kv : S->graphs) hipGraphExecDestroy(kv.second);
  for (int i = 0; i < kRing; ++i) {
    if (S->step_ev[i]) hipEventDestroy(S->step_ev[i]);
    if (S->desc_host[i]) hipHostFree(S->desc_host[i]);
    if (S->desc_dev[i]) hipFree(S->desc_dev[i]);
  }
  for (auto& kv : S->reqs) {
    Req* r = kv.second;
    if (r->ev_in) hipEventDestroy(r->ev_in);
    if (r->ev_ready) hipEventDestroy(r->ev_ready);
    if (r->ev_done) hipEventDestroy(r->ev_done);
    delete r;
  }
  if (S->arena_dev) hipFree(S->arena_dev);
  delete S;
}

}  // namespace

extern "C" {

const char* cnmf_server_last_error(void) { return g_server_err.c_str(); }

cnmf_status cnmf_server_start(const cnmf_server_config* cfg, cnmf_server** out) {
  if (!cfg || !out) return sfail(CNMF_EINVAL, "cfg and out are required");
  *out = nullptr;
  if (cfg->hbm_budget_bytes < (1u << 20)) return sfail(CNMF_EINVAL, "hbm_budget_bytes must be at least 1 MiB");
  if (cfg->max_batch < 1 || cfg->max_batch > 4096) return sfail(CNMF_EINVAL, "max_batch must be in [1, 4096]");
  if (cfg->flags & ~(CNMF_SERVER_GRAPHS | CNMF_SERVER_ONE_STEP))
    return sfail(CNMF_EINVAL, "unknown server flags 0x%x", cfg->flags);
  if (cfg->workers < 1 || cfg->workers > 3)
    return sfail(CNMF_EINVAL, "workers must be in [1, 3] (one more stream runs the batched steps)");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return sfail(CNMF_EDEVICE, "no HIP device available");
  if (cfg->device < 0 || cfg->device >= ndev) return sfail(CNMF_EINVAL, "device %d out of range", cfg->device);
  int old = 0;
  hipGetDevice(&old);
  hipSetDevice(cfg->device);
  cnmf_server* S = new cnmf_server();
  S->device = cfg->device;
  S->budget = cfg->hbm_budget_bytes / BlockArena::kGranule * BlockArena::kGranule;
  S->max_batch = cfg->max_batch;
  S->nworkers = cfg->workers;
  S->use_graphs = (cfg->flags & CNMF_SERVER_GRAPHS) != 0;
  S->max_steps_in_flight = (cfg->flags & CNMF_SERVER_ONE_STEP) ? 1 : 2;
  S->max_inflight = cfg->max_batch + 2 * cfg->workers;
  S->arena = BlockArena(S->budget);
  auto bail = [&](cnmf_status st, const char* what, hipError_t e) {
    destroy_server(S);
    hipSetDevice(old);
    return sfail(st, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e = hipMalloc((void**)&S->arena_dev, S->budget);
  if (e != hipSuccess) return bail(CNMF_ENOMEM, "arena hipMalloc", e);
  e = hipStreamCreateWithFlags(&S->batch_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(CNMF_EDEVICE, "hipStreamCreate", e);
  S->workers.resize(S->nworkers);
  for (auto& W : S->workers) {
    e = hipStreamCreateWithFlags(&W.stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(CNMF_EDEVICE, "hipStreamCreate", e);
    serve_handle_create(S->device, W.stream, &W.h);
  }
  size_t a, b;
  S->desc_bytes = desc_layout(S->max_batch, &a, &b);
  for (int i = 0; i < kRing; ++i) {
    e = hipHostMalloc((void**)&S->desc_host[i], S->desc_bytes, hipHostMallocDefault);
    if (e != hipSuccess) return bail(CNMF_ENOMEM, "hipHostMalloc", e);
    e = hipMalloc((void**)&S->desc_dev[i], S->desc_bytes);
    if (e != hipSuccess) return bail(CNMF_ENOMEM, "descriptor hipMalloc", e);
    e = hipEventCreateWithFlags(&S->step_ev[i], hipEventDisableTiming);
    if (e != hipSuccess) return bail(CNMF_EDEVICE, "hipEventCreate", e);
  }
  e = admm_step_fixed_init();
  if (e != hipSuccess) return bail(CNMF_EDEVICE, "kernel attributes", e);
  S->th = std::thread(dispatcher, S);
  hipSetDevice(old);
  *out = S;
  return CNMF_OK;
}

cnmf_status cnmf_server_submit(cnmf_server* S, const cnmf_input* A, const cnmf_factorize_desc* d,
                               const cnmf_factorize_out* o, void* producer_stream, uint64_t* ticket) {
  if (!S || !ticket) return sfail(CNMF_EINVAL, "server and ticket are required");
  cnmf_status s = serve_check(A, d, o);
  if (s != CNMF_OK) return sfail(s, "%s", cnmf_last_error(nullptr));
  const size_t bytes = BlockArena::round(std::max<size_t>(serve_footprint(A, d), 1));
  if (bytes > S->budget)
    return sfail(CNMF_ENOMEM, "request needs %zu workspace bytes, the server's budget is %zu", bytes, S->budget);
  Req* r = new Req();
  r->A = *A;
  r->d = *d;
  r->o = *o;
  r->bytes = bytes;
  int old = 0;
  hipGetDevice(&old);
  hipSetDevice(S->device);
  hipError_t e = hipEventCreateWithFlags(&r->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev_ready, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev_done, hipEventDisableTiming);
  // the request's inputs were produced on producer_stream: its work so far
  // comes before the request's
  if (e == hipSuccess) e = hipEventRecord(r->ev_in, (hipStream_t)producer_stream);
  hipSetDevice(old);
  if (e != hipSuccess) {
    if (r->ev_in) hipEventDestroy(r->ev_in);
    if (r->ev_ready) hipEventDestroy(r->ev_ready);
    if (r->ev_done) hipEventDestroy(r->ev_done);
    delete r;
    return sfail(CNMF_EDEVICE, "event setup: %s", hipGetErrorString(e));
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) {
      hipEventDestroy(r->ev_in);
      hipEventDestroy(r->ev_ready);
      hipEventDestroy(r->ev_done);
      delete r;
      return sfail(CNMF_EBUSY, "the server is stopping");
    }
    r->ticket = S->next_ticket++;
    r->t_submit = now_ms();
    S->reqs[r->ticket] = r;
    S->pending.push_back(r);
    S->stats.submitted += 1;
    *ticket = r->ticket;
  }
  S->cv.notify_one();
  return CNMF_OK;
}

cnmf_status cnmf_server_poll(cnmf_server* S, uint64_t ticket, cnmf_ticket_info* info) {
  if (!S || !info) return sfail(CNMF_EINVAL, "server and info are required");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return sfail(CNMF_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  const Req* r = it->second;
  std::memset(info, 0, sizeof *info);
  info->state = r->state;
  info->done = r->state == kDone;
  info->status = r->state == kDone ? r->status : CNMF_OK;
  const double t = now_ms();
  info->queue_ms = (r->state >= kPrologue ? r->t_admit : t) - r->t_submit;
  info->total_ms = (r->state == kDone ? r->t_done : t) - r->t_submit;
  if (r->state == kDone && r->status != CNMF_OK)
    std::snprintf(info->message, sizeof info->message, "%s", r->err.c_str());
  return CNMF_OK;
}

cnmf_status cnmf_server_release(cnmf_server* S, uint64_t ticket) {
  if (!S) return sfail(CNMF_EINVAL, "server is NULL");
  Req* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return sfail(CNMF_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->state != kDone) return sfail(CNMF_EBUSY, "ticket %llu is not done", (unsigned long long)ticket);
    r = it->second;
    S->reqs.erase(it);
  }
  hipEventDestroy(r->ev_in);
  hipEventDestroy(r->ev_ready);
  hipEventDestroy(r->ev_done);
  delete r;
  return CNMF_OK;
}

cnmf_status cnmf_server_get_stats(cnmf_server* S, cnmf_server_stats* out) {
  if (!S || !out) return sfail(CNMF_EINVAL, "server and out are required");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  out->queued = (int64_t)S->pending.size();
  out->in_flight = S->admitted;
  out->arena_bytes = S->budget;
  out->arena_free_bytes = S->arena.free_bytes();
  return CNMF_OK;
}

cnmf_status cnmf_server_stop(cnmf_server* S) {
  if (!S) return CNMF_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  int old = 0;
  hipGetDevice(&old);
  hipSetDevice(S->device);
  destroy_server(S);
  hipSetDevice(old);
  return CNMF_OK;
}

// Host-only replay of the admission policy (no GPU): request i arrives at
// arrival_ms[i], needs bytes[i] of arena and, once admitted, occupies its
// slot for service_ms[i].  Outputs admit_ms[i] / done_ms[i] (-1: rejected,
// bytes above the budget) and the peak arena use.
cnmf_status cnmf_server_simulate(int32_t nreq, const double* arrival_ms, const uint64_t* bytes,
                                 const double* service_ms, uint64_t budget, int32_t max_inflight, double* admit_ms,
                                 double* done_ms, uint64_t* peak_bytes) {
  if (nreq < 0 || (nreq > 0 && (!arrival_ms || !bytes || !service_ms || !admit_ms || !done_ms)))
    return sfail(CNMF_EINVAL, "arrays are required");
  if (max_inflight < 1) return sfail(CNMF_EINVAL, "max_inflight must be >= 1");
  for (int i = 1; i < nreq; ++i)
    if (arrival_ms[i] < arrival_ms[i - 1]) return sfail(CNMF_EINVAL, "arrivals must be sorted");
  BlockArena arena(budget);
  AdmissionState adm;
  std::deque<int> pending;
  std::deque<size_t> sizes;
  struct Run {
    double end;
    int i;
    size_t off, bytes;
  };
  std::vector<Run> running;
  uint64_t peak = 0;
  int next = 0;
  double t = 0.0;
  for (int i = 0; i < nreq; ++i) admit_ms[i] = done_ms[i] = -1.0;
  while (next < nreq || !pending.empty() || !running.empty()) {
    // next event: an arrival or a completion
    double t_arr = next < nreq ? arrival_ms[next] : 1e300;
    double t_end = 1e300;
    for (const Run& r : running) t_end = std::min(t_end, r.end);
    if (t_arr == 1e300 && t_end == 1e300) break;  // only blocked requests left (cannot happen)
    t = std::min(t_arr, t_end);
    for (size_t j = 0; j < running.size();) {
      if (running[j].end <= t) {
        arena.release(running[j].off, running[j].bytes);
        done_ms[running[j].i] = running[j].end;
        running.erase(running.begin() + j);
      } else {
        ++j;
      }
    }
    while (next < nreq && arrival_ms[next] <= t) {
      const size_t b = BlockArena::round(std::max<uint64_t>(bytes[next], 1));
      if (b > arena.capacity())
        admit_ms[next] = -1.0;
      else
        pending.push_back(next);
      ++next;
    }
    for (;;) {
      sizes.clear();
      for (size_t j = 0; j < pending.size() && j < 33; ++j)
        sizes.push_back(BlockArena::round(std::max<uint64_t>(bytes[pending[j]], 1)));
      const int idx = pick_admission(sizes, arena, max_inflight - (int)running.size(), adm);
      if (idx < 0) break;
      const int i = pending[idx];
      size_t off;
      if (!arena.alloc(sizes[idx], &off)) break;
      pending.erase(pending.begin() + idx);
      adm.bypassed = idx == 0 ? 0 : adm.bypassed + 1;
      admit_ms[i] = t;
      running.push_back({t + service_ms[i], i, off, sizes[idx]});
      peak = std::max<uint64_t>(peak, arena.capacity() - arena.free_bytes());
    }
  }
  if (peak_bytes) *peak_bytes = peak;
  return CNMF_OK;
}

}  // extern "C"
