// Serving loop: similarity queries against a resident signature index, with
// memory-admitted continuous batching.
//
// A request is (query object, candidate ids on the host, threshold t).
// A scheduler thread owns the device:
//   - admission: a pending request is admitted (FIFO) when a slot is free and
//     its candidate ids fit in the device arena (first-fit allocator over a
//     budget fixed at creation); its ids are copied host -> device;
//   - iteration: every active request contributes its next chunk of
//     candidates (a fair share of the per-iteration budget) as one list of a
//     batched verification call (the graph-launched persistent kernels), so
//     requests that arrive while others run join at the next iteration and
//     their work shares the device;
//   - completion: accepted pairs of the iteration are copied back and
//     distributed to their requests; a request whose candidates are all done
//     is completed (host-visible) and its arena space freed.
// Two iterations are in flight at once: iteration i+1 is launched before the
// results of iteration i are read back.  Every candidate's decision depends on
// its own pair only, so a request's output does not depend on what it was
// batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace blsh {
int verify_batched(blsh_ctx *ctx, const blsh_list_desc *lists, int64_t n_lists, const uint32_t *cand, int64_t n_cand,
                   const blsh_sigs *jac, const blsh_sigs *cos, double eps, double delta, double gamma,
                   blsh_prior prior, int32_t kj, int32_t kc, blsh_result *res, int32_t *k_used, hipStream_t s,
                   int (*check_sigs_fn)(const blsh_sigs *, int, int *, int *), int mode);
int check_sigs_public(const blsh_sigs *s, int k, int *n_max_out, int *row_words);
}  // namespace blsh

using namespace blsh;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id;
  uint32_t query;
  double t;
  std::vector<uint32_t> cand;       // host copy (host submission)
  const uint32_t *d_src = nullptr;  // caller's device array (device submission)
  int64_t n;
  int64_t arena_off = -1;           // in uint32 units
  int64_t issued = 0, finished = 0; // candidates launched / completed
  std::vector<uint64_t> acc_idx;
  std::vector<float> acc_val;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int status = BLSH_OK;
  bool bad_id = false;              // a device-submitted id >= n_obj was seen
  bool done = false;
};

// first-fit allocator over [0, cap) in uint32 units
struct Arena {
  int64_t cap = 0;
  std::map<int64_t, int64_t> free_;   // offset -> size
  void init(int64_t c) { cap = c; free_.clear(); if (c > 0) free_[0] = c; }
  int64_t alloc(int64_t n) {
    if (n <= 0) n = 1;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const int64_t off = it->first, rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t n) {
    if (n <= 0) n = 1;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
    }
  }
};

struct Slice {        // one request's chunk inside an iteration
  Request *r;
  int64_t begin, len; // candidate range within the request
};

struct Iteration {
  std::vector<Slice> slices;
  std::vector<blsh_list_desc> lists;
  uint8_t *d_code = nullptr;
  uint64_t *d_acc_idx = nullptr;
  float *d_acc_val = nullptr;
  int64_t *d_n_acc = nullptr;
  uint64_t *d_sidx = nullptr;         // accepted pairs sorted by arena position
  float *d_sval = nullptr;
  int64_t acc_cap = 0;
  std::vector<uint64_t> h_idx;
  std::vector<float> h_val;
  hipEvent_t done{};
  bool busy = false;
};

}  // namespace

struct blsh_server {
  blsh_ctx *ctx = nullptr;
  blsh_sigs index{};
  blsh_server_config cfg{};
  hipStream_t stream{};
  hipStream_t post{};                 // sorts a finished iteration's pairs while the next one runs
  void *d_sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  int key_bits = 1;                   // arena positions < 2^key_bits
  uint32_t *d_arena = nullptr;
  Arena arena;
  Iteration iters[2];
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;
  std::vector<Request *> active;
  std::unordered_map<int64_t, std::unique_ptr<Request>> all;
  int64_t next_id = 1;
  bool stop = false;
  int fatal = BLSH_OK;
  std::thread th;
  Clock::time_point t0;
  int64_t iterations = 0;
  int64_t deferred = 0;   // admission rounds that left requests waiting (slots or memory)
  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

void iteration_free(Iteration &it) {
  if (it.d_code) hipFree(it.d_code);
  if (it.d_acc_idx) hipFree(it.d_acc_idx);
  if (it.d_acc_val) hipFree(it.d_acc_val);
  if (it.d_n_acc) hipFree(it.d_n_acc);
  if (it.d_sidx) hipFree(it.d_sidx);
  if (it.d_sval) hipFree(it.d_sval);
  if (it.done) hipEventDestroy(it.done);
}

// Launch one iteration over the active requests (caller holds no lock; the
// scheduler thread is the only user of `active` outside submit/poll).
int launch_iteration(blsh_server *S, Iteration &it, std::vector<Request *> &act) {
  it.slices.clear();
  it.lists.clear();
  int64_t budget = S->cfg.max_batch_candidates;
  std::vector<Request *> todo;
  for (Request *r : act)
    if (r->issued < r->n) todo.push_back(r);
  if (todo.empty()) return BLSH_OK;
  // fair share, remainder redistributed
  int64_t left = budget;
  for (size_t i = 0; i < todo.size() && left > 0; ++i) {
    Request *r = todo[i];
    const int64_t share = std::max<int64_t>(1, left / int64_t(todo.size() - i));
    const int64_t len = std::min(r->n - r->issued, share);
    it.slices.push_back({r, r->issued, len});
    blsh_list_desc d;
    d.measure = S->index.measure;
    d.t = r->t;
    d.query = r->query;
    d.offset = r->arena_off + r->issued;
    d.length = len;
    it.lists.push_back(d);
    r->issued += len;
    left -= len;
  }
  // codes are written at arena positions; the per-iteration code buffer covers the arena
  blsh_result res{};
  res.code = it.d_code;
  res.acc_idx = it.d_acc_idx;
  res.acc_val = it.d_acc_val;
  res.acc_capacity = it.acc_cap;
  res.n_accepted = it.d_n_acc;
  res.m_debug = nullptr;
  const blsh_sigs *jac = S->index.measure == BLSH_JACCARD ? &S->index : nullptr;
  const blsh_sigs *cos = S->index.measure == BLSH_COSINE ? &S->index : nullptr;
  int rc = verify_batched(S->ctx, it.lists.data(), int64_t(it.lists.size()), S->d_arena, S->arena.cap, jac, cos,
                          S->cfg.epsilon, S->cfg.delta, S->cfg.gamma, S->cfg.prior, S->cfg.k, S->cfg.k, &res, nullptr,
                          S->stream,
                          check_sigs_public, 0);
  if (rc) return rc;
  if (hipEventRecord(it.done, S->stream) != hipSuccess) return BLSH_EDEVICE;
  it.busy = true;
  return BLSH_OK;
}

// Device-to-host read on the server's second stream (non-blocking), so that
// the scheduler never waits on work of the null stream.
int read_back(blsh_server *S, void *dst, const void *src, size_t bytes) {
  if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, S->post) != hipSuccess ||
      hipStreamSynchronize(S->post) != hipSuccess)
    return BLSH_EDEVICE;
  return BLSH_OK;
}

// Device-submitted ids are checked by the kernels only: a bad id gets code
// 0xFF (no Algorithm 1 code reaches it: decisions 0-2 use at most 0xBF) and
// raises the context's status word (first error wins).  The word is shared by
// both in-flight iterations, so it only says that some iteration may hold a
// bad id; which request it belongs to is read from this iteration's own
// codes.  It is cleared only when no other iteration is in flight, so an error
// raised by the overlapping iteration is seen when that one finishes.
int check_device_ids(blsh_server *S, Iteration &it, bool other_busy) {
  bool dev = false;
  for (const Slice &sl : it.slices) dev |= sl.r->d_src != nullptr;
  if (!dev) return BLSH_OK;
  int32_t st = 0;
  if (read_back(S, &st, S->ctx->d_status, 4)) return BLSH_EDEVICE;
  if (st == BLSH_OK) return BLSH_OK;
  std::vector<uint8_t> code;
  for (const Slice &sl : it.slices) {
    if (!sl.r->d_src || sl.r->bad_id) continue;
    code.resize(size_t(sl.len));
    if (read_back(S, code.data(), it.d_code + sl.r->arena_off + sl.begin, size_t(sl.len))) return BLSH_EDEVICE;
    sl.r->bad_id = std::find(code.begin(), code.end(), uint8_t(0xFF)) != code.end();
  }
  if (!other_busy && (hipMemsetAsync(S->ctx->d_status, 0, 4, S->post) != hipSuccess ||
                      hipStreamSynchronize(S->post) != hipSuccess))
    return BLSH_EDEVICE;
  return BLSH_OK;
}

int finish_iteration(blsh_server *S, Iteration &it, bool other_busy) {
  if (!it.busy) return BLSH_OK;
  it.busy = false;
  if (hipEventSynchronize(it.done) != hipSuccess) return BLSH_EDEVICE;
  if (int rc = check_device_ids(S, it, other_busy)) return rc;
  int64_t n = 0;
  if (read_back(S, &n, it.d_n_acc, 8)) return BLSH_EDEVICE;
  if (n > it.acc_cap) return BLSH_ETRUNCATED;
  it.h_idx.resize(size_t(n));
  it.h_val.resize(size_t(n));
  if (n) {
    // the iteration's event has completed, so its pairs are ready for the other stream
    size_t tb = S->sort_tmp_bytes;
    if (int rc = sort_accepted(it.d_acc_idx, it.d_acc_val, it.d_sidx, it.d_sval, n, S->key_bits, S->d_sort_tmp, &tb,
                               S->post))
      return rc;
    if (hipMemcpyAsync(it.h_idx.data(), it.d_sidx, size_t(n) * 8, hipMemcpyDeviceToHost, S->post) != hipSuccess ||
        hipMemcpyAsync(it.h_val.data(), it.d_sval, size_t(n) * 4, hipMemcpyDeviceToHost, S->post) != hipSuccess ||
        hipStreamSynchronize(S->post) != hipSuccess)
      return BLSH_EDEVICE;
  }
  // slices are disjoint ranges of arena positions: each takes its range of the sorted pairs
  for (const Slice &sl : it.slices) {
    const uint64_t off = uint64_t(sl.r->arena_off), lo = off + uint64_t(sl.begin), hi = lo + uint64_t(sl.len);
    const auto b = std::lower_bound(it.h_idx.begin(), it.h_idx.end(), lo);
    const auto e = std::lower_bound(b, it.h_idx.end(), hi);
    std::vector<uint64_t> &ri = sl.r->acc_idx;
    const size_t at = ri.size();
    ri.resize(at + size_t(e - b));
    for (auto p = b; p != e; ++p) ri[at + size_t(p - b)] = *p - off;
    sl.r->acc_val.insert(sl.r->acc_val.end(), it.h_val.begin() + (b - it.h_idx.begin()),
                         it.h_val.begin() + (e - it.h_idx.begin()));
  }
  for (const Slice &sl : it.slices) sl.r->finished += sl.len;
  return BLSH_OK;
}

void scheduler(blsh_server *S) {
  hipSetDevice(S->ctx->device);
  int cur = 0;
  std::vector<Request *> act;
  for (;;) {
    std::vector<Request *> admitted;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        return S->stop || !S->pending.empty() || !act.empty() || S->iters[0].busy || S->iters[1].busy;
      });
      if (S->stop) break;
      // admission: FIFO while slots and arena space allow
      while (!S->pending.empty() && int(act.size() + admitted.size()) < S->cfg.max_active) {
        Request *r = S->pending.front();
        const int64_t off = S->arena.alloc(r->n);
        if (off < 0) break;
        r->arena_off = off;
        r->t_admit = S->now();
        admitted.push_back(r);
        S->pending.pop_front();
      }
      if (!S->pending.empty()) ++S->deferred;
    }
    // host ids: one copy each; device ids: one gather launch per kCopyJobs requests
    // (S->fatal is shared with the submitting threads: errors go through rc, set under the lock below)
    int rc = BLSH_OK;
    std::vector<CopyJob> jobs;
    for (Request *r : admitted) {
      if (r->n && r->d_src) {
        jobs.push_back({r->d_src, r->arena_off, r->n});
      } else if (r->n && hipMemcpyAsync(S->d_arena + r->arena_off, r->cand.data(), size_t(r->n) * 4,
                                        hipMemcpyHostToDevice, S->stream) != hipSuccess) {
        rc = BLSH_EDEVICE;
      }
      act.push_back(r);
    }
    for (size_t i = 0; i < jobs.size() && rc == BLSH_OK; i += kCopyJobs)
      if (gather_copy(jobs.data() + i, int(std::min<size_t>(kCopyJobs, jobs.size() - i)), S->d_arena, S->stream))
        rc = BLSH_EDEVICE;
    // launch the next iteration, then retire the previous one
    Iteration &nx = S->iters[cur];
    if (rc == BLSH_OK && !nx.busy) rc = launch_iteration(S, nx, act);
    Iteration &pv = S->iters[cur ^ 1];
    if (rc == BLSH_OK) rc = finish_iteration(S, pv, nx.busy);
    if (rc == BLSH_OK && !nx.busy) rc = finish_iteration(S, nx, false);   // nothing new was launched: drain
    cur ^= 1;
    ++S->iterations;
    // completions
    std::vector<Request *> keep;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (rc != BLSH_OK) S->fatal = rc;
      for (Request *r : act) {
        if (S->fatal != BLSH_OK || r->finished >= r->n) {
          r->done = true;
          r->status = S->fatal != BLSH_OK ? S->fatal : r->bad_id ? BLSH_EBADID : BLSH_OK;
          r->t_done = S->now();
          S->arena.release(r->arena_off, r->n);
          std::vector<uint32_t>().swap(r->cand);
        } else {
          keep.push_back(r);
        }
      }
    }
    act.swap(keep);
    S->cv_done.notify_all();
    if (S->fatal != BLSH_OK) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (Request *r : S->pending) { r->done = true; r->status = S->fatal; r->t_done = S->now(); }
      S->pending.clear();
      S->cv_done.notify_all();
    }
  }
}

}  // namespace

extern "C" {

int bayeslsh_server_create(blsh_ctx *ctx, const blsh_sigs *index, const blsh_server_config *cfg,
                           blsh_server **out) {
  if (!ctx || !index || !cfg || !out) return fail(BLSH_EINVAL, "null argument");
  *out = nullptr;
  int n_max = 0, rw = 0;
  const int k = cfg->k;
  int rc = check_sigs_public(index, k, &n_max, &rw);
  if (rc) return rc;
  if (cfg->max_active <= 0 || cfg->max_active > 65536) return fail(BLSH_EINVAL, "max_active must be in [1, 65536]");
  if (cfg->max_batch_candidates <= 0) return fail(BLSH_EINVAL, "max_batch_candidates must be positive");
  if (cfg->mem_budget_bytes < 1024) return fail(BLSH_EINVAL, "mem_budget_bytes too small");
  if (!(cfg->epsilon > 0 && cfg->epsilon < 1 && cfg->delta > 0 && cfg->delta < 1 && cfg->gamma > 0 && cfg->gamma < 1))
    return fail(BLSH_EINVAL, "epsilon, delta, gamma must be in (0,1)");
  auto S = std::make_unique<blsh_server>();
  S->ctx = ctx;
  S->index = *index;
  S->cfg = *cfg;
  BLSH_HIP(hipSetDevice(ctx->device));
  BLSH_HIP(hipMemset(ctx->d_status, 0, 4));   // the server owns the context from here on
  BLSH_HIP(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
  if (hipStreamCreateWithFlags(&S->post, hipStreamNonBlocking) != hipSuccess) {
    hipStreamDestroy(S->stream);
    return fail(BLSH_EDEVICE, "stream");
  }
  const int64_t words = int64_t(cfg->mem_budget_bytes / 4);
  while (S->key_bits < 64 && (int64_t(1) << S->key_bits) < words) ++S->key_bits;
  if (sort_accepted(nullptr, nullptr, nullptr, nullptr, cfg->max_batch_candidates, S->key_bits, nullptr,
                    &S->sort_tmp_bytes, S->post) != BLSH_OK ||
      hipMalloc(&S->d_sort_tmp, std::max<size_t>(S->sort_tmp_bytes, 256)) != hipSuccess) {
    hipStreamDestroy(S->post);
    hipStreamDestroy(S->stream);
    return fail(BLSH_ENOMEM, "sort buffer");
  }
  if (hipMalloc(&S->d_arena, size_t(words) * 4) != hipSuccess) {
    hipFree(S->d_sort_tmp);
    hipStreamDestroy(S->post);
    hipStreamDestroy(S->stream);
    return fail(BLSH_ENOMEM, "arena of %zu bytes", cfg->mem_budget_bytes);
  }
  S->arena.init(words);
  // code buffers are indexed by arena position: size them to the arena
  for (auto &it : S->iters) {
    it.acc_cap = cfg->max_batch_candidates;
    if (hipMalloc(&it.d_code, size_t(words)) != hipSuccess ||
        hipMalloc(&it.d_acc_idx, size_t(cfg->max_batch_candidates) * 8) != hipSuccess ||
        hipMalloc(&it.d_acc_val, size_t(cfg->max_batch_candidates) * 4) != hipSuccess ||
        hipMalloc(&it.d_n_acc, 256) != hipSuccess ||
        hipMalloc(&it.d_sidx, size_t(cfg->max_batch_candidates) * 8) != hipSuccess ||
        hipMalloc(&it.d_sval, size_t(cfg->max_batch_candidates) * 4) != hipSuccess ||
        hipEventCreateWithFlags(&it.done, hipEventDisableTiming) != hipSuccess) {
      for (auto &j : S->iters) iteration_free(j);
      hipFree(S->d_arena);
      hipFree(S->d_sort_tmp);
      hipStreamDestroy(S->post);
      hipStreamDestroy(S->stream);
      return fail(BLSH_ENOMEM, "iteration buffers");
    }
  }
  S->t0 = Clock::now();
  blsh_server *raw = S.release();
  raw->th = std::thread(scheduler, raw);
  *out = raw;
  return BLSH_OK;
}

double bayeslsh_server_clock(blsh_server *srv) { return srv ? srv->now() : 0.0; }

int bayeslsh_server_submit(blsh_server *srv, uint32_t query, const uint32_t *cand_host, int64_t n_cand, double t,
                           int64_t *request_id) {
  if (!srv || !request_id || n_cand < 0 || (n_cand > 0 && !cand_host)) return fail(BLSH_EINVAL, "bad argument");
  if (!(t > 0 && t < 1)) return fail(BLSH_EINVAL, "t must be in (0,1)");
  if (n_cand > srv->arena.cap) return fail(BLSH_ENOMEM, "request of %lld candidates exceeds the memory budget", (long long)n_cand);
  if (int64_t(query) >= srv->index.n_obj) return fail(BLSH_EINVAL, "query id %u >= n_obj", query);
  auto r = std::make_unique<Request>();
  r->query = query;
  r->t = t;
  r->n = n_cand;
  // copy first, then check the copy while it is still in cache (one pass over the caller's memory)
  r->cand.assign(cand_host, cand_host + n_cand);
  for (int64_t i = 0; i < n_cand; ++i)
    if (int64_t(r->cand[size_t(i)]) >= srv->index.n_obj)
      return fail(BLSH_EINVAL, "candidate %lld: id %u >= n_obj", (long long)i, r->cand[size_t(i)]);
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->fatal != BLSH_OK) return fail(srv->fatal, "server failed earlier");
  r->id = srv->next_id++;
  r->t_submit = srv->now();
  *request_id = r->id;
  srv->pending.push_back(r.get());
  srv->all[r->id] = std::move(r);
  srv->cv_work.notify_one();
  return BLSH_OK;
}

int bayeslsh_server_submit_device(blsh_server *srv, uint32_t query, const uint32_t *cand_dev, int64_t n_cand,
                                  double t, int64_t *request_id) {
  if (!srv || !request_id || n_cand < 0 || (n_cand > 0 && !cand_dev)) return fail(BLSH_EINVAL, "bad argument");
  if (!(t > 0 && t < 1)) return fail(BLSH_EINVAL, "t must be in (0,1)");
  if (n_cand > srv->arena.cap) return fail(BLSH_ENOMEM, "request of %lld candidates exceeds the memory budget", (long long)n_cand);
  if (int64_t(query) >= srv->index.n_obj) return fail(BLSH_EINVAL, "query id %u >= n_obj", query);
  if (n_cand > 0) {
    // the admission kernel reads cand_dev directly: it must be device memory of
    // the server's GPU that holds all n_cand ids (anything else would fault there)
    hipPointerAttribute_t at{};
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    void *p = const_cast<uint32_t *>(cand_dev);
    const bool ok = hipPointerGetAttributes(&at, p) == hipSuccess && at.type == hipMemoryTypeDevice &&
                    at.device == srv->ctx->device && hipMemGetAddressRange(&base, &size, p) == hipSuccess &&
                    uintptr_t(p) + uint64_t(n_cand) * 4 <= uintptr_t(base) + size;
    if (!ok) {
      (void)hipGetLastError();   // a failed query leaves the runtime's last error set
      return fail(BLSH_EINVAL, "cand_dev is not device memory of the server's GPU holding %lld ids",
                  (long long)n_cand);
    }
  }
  auto r = std::make_unique<Request>();
  r->query = query;
  r->t = t;
  r->n = n_cand;
  r->d_src = cand_dev;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->fatal != BLSH_OK) return fail(srv->fatal, "server failed earlier");
  r->id = srv->next_id++;
  r->t_submit = srv->now();
  *request_id = r->id;
  srv->pending.push_back(r.get());
  srv->all[r->id] = std::move(r);
  srv->cv_work.notify_one();
  return BLSH_OK;
}

static void fill_result(const Request *r, blsh_request_result *out) {
  out->n_candidates = r->n;
  out->n_accepted = int64_t(r->acc_idx.size());
  out->acc_idx_host = r->acc_idx.data();
  out->acc_val_host = r->acc_val.data();
  out->submit_time_s = r->t_submit;
  out->admit_time_s = r->t_admit;
  out->done_time_s = r->t_done;
  out->status = r->status;
}

int bayeslsh_server_poll(blsh_server *srv, int64_t request_id, blsh_request_result *out) {
  if (!srv || !out) return fail(BLSH_EINVAL, "bad argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(request_id);
  if (it == srv->all.end()) return fail(BLSH_EINVAL, "unknown request %lld", (long long)request_id);
  if (!it->second->done) return BLSH_EAGAIN;
  fill_result(it->second.get(), out);
  return it->second->status;
}

int bayeslsh_server_wait(blsh_server *srv, int64_t request_id, blsh_request_result *out) {
  if (!srv || !out) return fail(BLSH_EINVAL, "bad argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->all.find(request_id);
  if (it == srv->all.end()) return fail(BLSH_EINVAL, "unknown request %lld", (long long)request_id);
  Request *r = it->second.get();
  srv->cv_done.wait(lk, [&] { return r->done; });
  fill_result(r, out);
  return r->status;
}

int bayeslsh_server_release(blsh_server *srv, int64_t request_id) {
  if (!srv) return fail(BLSH_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(request_id);
  if (it == srv->all.end() || !it->second->done) return fail(BLSH_EINVAL, "request not finished or unknown");
  srv->all.erase(it);
  return BLSH_OK;
}

int bayeslsh_server_stats(blsh_server *srv, int64_t *iterations_host, int64_t *pending_host, int64_t *active_host,
                          int64_t *deferred_host) {
  if (!srv) return fail(BLSH_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (iterations_host) *iterations_host = srv->iterations;
  if (deferred_host) *deferred_host = srv->deferred;
  if (pending_host) *pending_host = int64_t(srv->pending.size());
  if (active_host) {
    int64_t a = 0;
    for (auto &kv : srv->all) a += (!kv.second->done && kv.second->arena_off >= 0);
    *active_host = a;
  }
  return BLSH_OK;
}

void bayeslsh_server_destroy(blsh_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->th.joinable()) srv->th.join();
  hipSetDevice(srv->ctx->device);
  hipStreamSynchronize(srv->stream);
  hipStreamSynchronize(srv->post);
  for (auto &it : srv->iters) iteration_free(it);
  if (srv->d_arena) hipFree(srv->d_arena);
  if (srv->d_sort_tmp) hipFree(srv->d_sort_tmp);
  hipStreamDestroy(srv->post);
  hipStreamDestroy(srv->stream);
  delete srv;
}

}  // extern "C"
