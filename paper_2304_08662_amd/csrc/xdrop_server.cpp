// Continuous-batching server for X-Drop seed extension.
//
// Requests (host sequences, seeds and a scoring scheme) are admitted against
// a device-memory budget: their packed sequences are copied into a resident
// device arena as space frees up.  A worker thread groups admitted requests
// that share a scoring scheme into micro-batches and launches each on one of
// several streams (one library context per stream), so the work of requests
// that arrive while others run overlaps on the device.  A micro-batch needs
// no copy of the sequences: its offsets point into the arena (a gap entry
// separates requests that are not adjacent), and its seeds are renumbered to
// those offsets.  Completion is tracked with events; results come back
// through pinned host memory and each request's arena space is released.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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

#include "xdrop.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  uint64_t ticket = 0;
  int alphabet = 0;
  std::vector<uint8_t> seqs;     // packed stream of the request
  std::vector<int64_t> offsets;  // n_seqs + 1, request-local symbols
  std::vector<xdrop_seed> seeds;
  xdrop_scoring sc{};
  std::vector<int32_t> matrix;
  size_t arena_off = 0, arena_bytes = 0;  // placement in the arena
  std::vector<xdrop_result> results;
  bool done = false;
  int status = XDROP_OK;
};

// First-fit allocator over [0, cap) (host bookkeeping of device ranges).
class Arena {
 public:
  explicit Arena(size_t cap) : cap_(cap) { free_[0] = cap; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
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
  size_t cap() const { return cap_; }

 private:
  size_t cap_, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Slot {  // one stream with its context and staging buffers
  hipStream_t stream = nullptr;
  xdrop_ctx* ctx = nullptr;
  hipEvent_t done = nullptr;
  int64_t* d_offsets = nullptr;
  xdrop_seed* d_seeds = nullptr;
  xdrop_result* d_results = nullptr;
  int64_t* h_offsets = nullptr;  // pinned
  xdrop_seed* h_seeds = nullptr;
  xdrop_result* h_results = nullptr;
  bool busy = false;
  std::vector<std::shared_ptr<Req>> batch;
  std::vector<int32_t> first_seed;  // per request: start in the batch
  int32_t n_seeds = 0;
};

bool same_scoring(const Req& a, const Req& b) {
  return a.alphabet == b.alphabet && a.sc.alphabet_size == b.sc.alphabet_size &&
         a.sc.match == b.sc.match && a.sc.mismatch == b.sc.mismatch &&
         a.sc.gap == b.sc.gap && a.sc.X == b.sc.X && a.matrix == b.matrix;
}

}  // namespace

struct xdrop_server {
  int device = 0;
  size_t budget = 0;
  int max_inflight = 256;
  int32_t max_batch_seeds = 1 << 16;
  int32_t max_batch_seqs = 1 << 17;
  uint8_t* d_arena = nullptr;
  std::unique_ptr<Arena> arena;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Req>> pending;    // waiting for arena space
  std::deque<std::shared_ptr<Req>> admitted;   // in the arena, not launched
  std::unordered_map<uint64_t, std::shared_ptr<Req>> all;
  uint64_t next_ticket = 1;
  int inflight = 0;  // admitted or running requests
  bool stop = false;
  int sticky = XDROP_OK;
  std::thread worker;

  void run();
  bool launch(Slot& s, std::vector<std::shared_ptr<Req>>& batch);
  void finish(Slot& s);
};

bool xdrop_server::launch(Slot& s, std::vector<std::shared_ptr<Req>>& batch) {
  // merged offsets: arena-absolute symbol offsets, a gap entry between
  // requests that are not adjacent, and a last entry covering the arena
  const int alpha = batch[0]->alphabet;
  const int64_t spb = alpha == XDROP_DNA2 ? 4 : 1;  // symbols per byte
  int32_t nseq = 0, nseed = 0;
  int64_t* off = s.h_offsets;
  int64_t max_end = 0;
  s.first_seed.clear();
  for (auto& r : batch) {
    const int64_t base = (int64_t)r->arena_off * spb;
    const int32_t first = nseq;
    const int32_t rn = (int32_t)r->offsets.size() - 1;
    for (int32_t i = 0; i <= rn; ++i) off[nseq + i] = base + r->offsets[i];
    max_end = std::max(max_end, base + r->offsets[rn]);
    nseq += rn + 1;  // the request's end entry starts a gap pseudo-sequence
    s.first_seed.push_back(nseed);
    for (const auto& sd : r->seeds) {
      xdrop_seed t = sd;
      t.q = sd.q >= 0 && sd.q < rn ? sd.q + first : -1;
      t.t = sd.t >= 0 && sd.t < rn ? sd.t + first : -1;
      s.h_seeds[nseed++] = t;
    }
  }
  // the last entry bounds the readable stream: past every request's end
  off[nseq] = std::max(max_end, off[nseq - 1]);
  s.n_seeds = nseed;
  s.batch = batch;
  hipError_t e = hipMemcpyAsync(s.d_offsets, s.h_offsets,
                                (size_t)(nseq + 1) * sizeof(int64_t),
                                hipMemcpyHostToDevice, s.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.d_seeds, s.h_seeds, (size_t)nseed * sizeof(xdrop_seed),
                       hipMemcpyHostToDevice, s.stream);
  if (e != hipSuccess) return false;
  xdrop_scoring sc = batch[0]->sc;
  sc.matrix = batch[0]->matrix.empty() ? nullptr : batch[0]->matrix.data();
  int rc = xdrop_extend_batch(s.ctx, d_arena, s.d_offsets, nseq, s.d_seeds,
                              nseed, &sc, nullptr, s.d_results, s.stream);
  if (rc != XDROP_OK) return false;
  e = hipMemcpyAsync(s.h_results, s.d_results,
                     (size_t)nseed * sizeof(xdrop_result),
                     hipMemcpyDeviceToHost, s.stream);
  if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
  if (e != hipSuccess) return false;
  s.busy = true;
  return true;
}

void xdrop_server::finish(Slot& s) {
  std::vector<std::shared_ptr<Req>> b;
  b.swap(s.batch);
  {
    std::lock_guard<std::mutex> lk(mu);
    for (size_t i = 0; i < b.size(); ++i) {
      auto& r = b[i];
      const int32_t f = s.first_seed[i];
      r->results.assign(s.h_results + f, s.h_results + f + r->seeds.size());
      arena->release(r->arena_off, r->arena_bytes);
      r->seqs.clear();
      r->seqs.shrink_to_fit();
      r->done = true;
      --inflight;
    }
    s.busy = false;
  }
  cv_done.notify_all();
  cv_work.notify_all();
}

void xdrop_server::run() {
  (void)hipSetDevice(device);
  std::vector<std::shared_ptr<Req>> to_copy;
  for (;;) {
    // 1. admission: FIFO, as long as arena space and in-flight slots allow
    to_copy.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop) break;
      while (!pending.empty() && inflight < max_inflight) {
        auto& r = pending.front();
        size_t off;
        if (!arena->alloc(r->arena_bytes, &off)) break;
        r->arena_off = off;
        to_copy.push_back(r);
        admitted.push_back(r);
        pending.pop_front();
        ++inflight;
      }
    }
    for (auto& r : to_copy) {
      // staged through the copy in host memory (synchronous for pageable)
      hipError_t e = hipMemcpy(d_arena + r->arena_off, r->seqs.data(),
                               r->seqs.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        sticky = XDROP_E_DEVICE;
      }
    }
    // 2. completions
    bool progressed = !to_copy.empty();
    for (auto& s : slots) {
      if (s.busy && hipEventQuery(s.done) == hipSuccess) {
        finish(s);
        progressed = true;
      }
    }
    // 3. launches: micro-batches of admitted requests with one scoring
    for (auto& s : slots) {
      if (s.busy) continue;
      std::vector<std::shared_ptr<Req>> batch;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (admitted.empty()) break;
        int32_t ns = 0, nq = 0;
        auto it = admitted.begin();
        while (it != admitted.end()) {
          auto& r = *it;
          const int32_t rs = (int32_t)r->seeds.size();
          const int32_t rq = (int32_t)r->offsets.size();
          if (!batch.empty() &&
              (!same_scoring(*batch[0], *r) || ns + rs > max_batch_seeds ||
               nq + rq + 1 > max_batch_seqs)) {
            ++it;
            continue;
          }
          batch.push_back(r);
          ns += rs;
          nq += rq;
          it = admitted.erase(it);
          if (ns >= max_batch_seeds) break;
        }
      }
      if (batch.empty()) break;
      if (!launch(s, batch)) {
        std::lock_guard<std::mutex> lk(mu);
        sticky = XDROP_E_DEVICE;
        for (auto& r : batch) {
          r->status = XDROP_E_DEVICE;
          r->done = true;
          arena->release(r->arena_off, r->arena_bytes);
          --inflight;
        }
        cv_done.notify_all();
      }
      progressed = true;
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(mu);
      bool any_busy = false;
      for (auto& s : slots) any_busy |= s.busy;
      if (any_busy)
        cv_work.wait_for(lk, std::chrono::microseconds(20));
      else if (pending.empty() && admitted.empty())
        cv_work.wait_for(lk, std::chrono::milliseconds(5),
                         [&] { return stop || !pending.empty(); });
    }
  }
  for (auto& s : slots)
    if (s.busy) {
      (void)hipEventSynchronize(s.done);
      finish(s);
    }
}

extern "C" {

int xdrop_server_create(int device, size_t hbm_budget_bytes,
                        const xdrop_server_opts* opts, xdrop_server** out) {
  if (!out) return XDROP_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return XDROP_E_INVALID;
  if (opts && (opts->max_inflight < 0 || opts->streams < 0 ||
               opts->streams > 16 || opts->arena_mib < 0))
    return XDROP_E_INVALID;
  const int nslots = opts && opts->streams ? opts->streams : 4;
  // per stream: staging of one micro-batch and one library context
  const size_t per_slot = (size_t)40 << 20;
  if (hbm_budget_bytes < nslots * per_slot + ((size_t)1 << 20))
    return XDROP_E_BUDGET;
  size_t arena_bytes = hbm_budget_bytes - nslots * per_slot;
  if (opts && opts->arena_mib) {
    if (((size_t)opts->arena_mib << 20) > arena_bytes) return XDROP_E_BUDGET;
    arena_bytes = (size_t)opts->arena_mib << 20;
  }
  auto* s = new (std::nothrow) xdrop_server();
  if (!s) return XDROP_E_NOMEM;
  s->device = device;
  s->budget = hbm_budget_bytes;
  if (opts && opts->max_inflight > 0) s->max_inflight = opts->max_inflight;
  if (hipSetDevice(device) != hipSuccess) {
    delete s;
    return XDROP_E_DEVICE;
  }
  if (hipMalloc(&s->d_arena, arena_bytes) != hipSuccess) {
    delete s;
    return XDROP_E_NOMEM;
  }
  s->arena.reset(new Arena(arena_bytes));
  s->slots.resize(nslots);
  for (auto& sl : s->slots) {
    bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) ==
                  hipSuccess &&
              hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) ==
                  hipSuccess &&
              xdrop_ctx_create(device, nullptr, &sl.ctx) == XDROP_OK &&
              hipMalloc(&sl.d_offsets, (size_t)(s->max_batch_seqs + 1) * 8) ==
                  hipSuccess &&
              hipMalloc(&sl.d_seeds, (size_t)s->max_batch_seeds *
                                         sizeof(xdrop_seed)) == hipSuccess &&
              hipMalloc(&sl.d_results, (size_t)s->max_batch_seeds *
                                           sizeof(xdrop_result)) ==
                  hipSuccess &&
              hipHostMalloc(&sl.h_offsets,
                            (size_t)(s->max_batch_seqs + 1) * 8) ==
                  hipSuccess &&
              hipHostMalloc(&sl.h_seeds, (size_t)s->max_batch_seeds *
                                             sizeof(xdrop_seed)) ==
                  hipSuccess &&
              hipHostMalloc(&sl.h_results, (size_t)s->max_batch_seeds *
                                               sizeof(xdrop_result)) ==
                  hipSuccess;
    if (!ok) {
      s->stop = true;
      xdrop_server_destroy(s);
      return XDROP_E_NOMEM;
    }
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return XDROP_OK;
}

int xdrop_server_submit(xdrop_server* s, const xdrop_request* r,
                        uint64_t* ticket) {
  if (!s || !r || !ticket) return XDROP_E_INVALID;
  if (r->n_seqs < 0 || r->n_seeds < 0 || (r->n_seqs > 0 && !r->offsets) ||
      (r->n_seeds > 0 && !r->seeds))
    return XDROP_E_INVALID;
  const xdrop_scoring& sc = r->scoring;
  if (sc.alphabet != XDROP_DNA2 && sc.alphabet != XDROP_BYTE)
    return XDROP_E_INVALID;
  if (sc.alphabet == XDROP_DNA2 ? sc.alphabet_size != 4
                                : (sc.alphabet_size < 1 || sc.alphabet_size > 32))
    return XDROP_E_INVALID;
  if (sc.gap > 0 || sc.X < 0) return XDROP_E_INVALID;
  if (r->n_seqs + 1 > s->max_batch_seqs || r->n_seeds > s->max_batch_seeds)
    return XDROP_E_BUDGET;
  for (int32_t i = 0; i < r->n_seqs; ++i)
    if (r->offsets[i] < 0 || r->offsets[i + 1] < r->offsets[i])
      return XDROP_E_INVALID;
  if (r->n_seqs > 0 && r->offsets[0] != 0) return XDROP_E_INVALID;
  auto q = std::make_shared<Req>();
  q->alphabet = sc.alphabet;
  const int64_t syms = r->n_seqs > 0 ? r->offsets[r->n_seqs] : 0;
  const size_t bytes = sc.alphabet == XDROP_DNA2 ? (size_t)((syms + 15) / 16) * 4
                                                 : (size_t)((syms + 3) / 4) * 4;
  q->arena_bytes = bytes + 64;
  if (q->arena_bytes > s->arena->cap()) return XDROP_E_BUDGET;
  q->seqs.assign(r->seqs, r->seqs + bytes);
  if (r->n_seqs > 0)
    q->offsets.assign(r->offsets, r->offsets + r->n_seqs + 1);
  else
    q->offsets.assign(1, 0);
  q->seeds.assign(r->seeds, r->seeds + r->n_seeds);
  q->sc = sc;
  if (sc.matrix)
    q->matrix.assign(sc.matrix, sc.matrix + sc.alphabet_size * sc.alphabet_size);
  q->sc.matrix = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->sticky != XDROP_OK) return s->sticky;
    q->ticket = s->next_ticket++;
    *ticket = q->ticket;
    s->all[q->ticket] = q;
    if (q->seeds.empty()) {
      q->done = true;  // nothing to compute
    } else {
      s->pending.push_back(q);
    }
  }
  s->cv_work.notify_all();
  return XDROP_OK;
}

static int take_result(xdrop_server* s, uint64_t ticket, xdrop_result* out,
                       std::unique_lock<std::mutex>& lk, bool block,
                       int64_t timeout_ns) {
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return XDROP_E_INVALID;
  auto r = it->second;
  if (!r->done && block) {
    auto pred = [&] { return r->done; };
    if (timeout_ns < 0)
      s->cv_done.wait(lk, pred);
    else
      s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), pred);
  }
  if (!r->done) return XDROP_PENDING;
  if (out && !r->results.empty())
    std::memcpy(out, r->results.data(), r->results.size() * sizeof(xdrop_result));
  const int st = r->status;
  s->all.erase(it);
  return st;
}

int xdrop_server_poll(xdrop_server* s, uint64_t ticket, xdrop_result* out) {
  if (!s) return XDROP_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  return take_result(s, ticket, out, lk, false, 0);
}

int xdrop_server_wait(xdrop_server* s, uint64_t ticket, xdrop_result* out,
                      int64_t timeout_ns) {
  if (!s) return XDROP_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  return take_result(s, ticket, out, lk, true, timeout_ns);
}

int xdrop_server_destroy(xdrop_server* s) {
  if (!s) return XDROP_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  for (auto& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.ctx) xdrop_ctx_destroy(sl.ctx);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.d_offsets) (void)hipFree(sl.d_offsets);
    if (sl.d_seeds) (void)hipFree(sl.d_seeds);
    if (sl.d_results) (void)hipFree(sl.d_results);
    if (sl.h_offsets) (void)hipHostFree(sl.h_offsets);
    if (sl.h_seeds) (void)hipHostFree(sl.h_seeds);
    if (sl.h_results) (void)hipHostFree(sl.h_results);
  }
  if (s->d_arena) (void)hipFree(s->d_arena);
  delete s;
  return XDROP_OK;
}

}  // extern "C"
