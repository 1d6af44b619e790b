// Continuous-batching server for X-Drop seed extension.
//
// Sequences live in a resident device arena, admitted against a memory
// budget.  They arrive in sets: a request's own sequences form a set that
// lives as long as the request, and a caller can register a set once
// (xdrop_server_put_sequences) and let any number of requests seed against
// it, so a sequence crosses the host link once however many seeds use it
// (the paper keeps sequences apart from the seed tuples that refer to them
// and partitions comparisons so that sequences are shared; Sec. 4.1.1,
// Sec. 4.3).  The caller's thread copies a set into pinned staging memory at
// submission; the worker thread places it in the arena as space frees up
// and moves it to the device with an asynchronous copy on a copy stream, so
// no copy waits on the worker.  Requests whose sequences are resident are
// grouped by scoring scheme into micro-batches and launched on several
// streams (one library context per stream): requests that arrive while
// others run are admitted and their work overlaps on the device.  A
// micro-batch copies no sequence: its offsets point into the arena (each set
// once, a gap entry after each), its seeds are renumbered to those offsets.
// Completion is tracked with events; results come back through pinned host
// memory, and a set's arena space is released when its last user is done.
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
#include <unordered_set>
#include <vector>

#include "xdrop.h"

namespace {

constexpr size_t NONE = ~size_t(0);

// First-fit allocator over [0, cap) (host bookkeeping of device or pinned
// ranges, 256-byte granules).
class Arena {
 public:
  explicit Arena(size_t cap) : cap_(cap) { if (cap) free_[0] = cap; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
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
  size_t cap_;
  std::map<size_t, size_t> free_;
};

// Sequences of one set: a request's own, or registered for many requests.
struct SeqSet {
  uint64_t id = 0;  // 0: a request's own sequences
  int alphabet = 0;
  std::vector<int64_t> offsets;  // n_seqs + 1, set-local symbols
  size_t bytes = 0;              // packed bytes on the device
  size_t arena_off = 0, arena_bytes = 0;
  size_t pin_off = NONE;          // host copy in pinned staging, or
  std::vector<uint8_t> pageable;  // in ordinary memory (staging was full)
  bool placed = false, resident = false, released = false;
  int users = 0;  // requests not finished that use the set
};

struct Req {
  uint64_t ticket = 0;
  std::shared_ptr<SeqSet> set;  // the sequences the seeds index
  std::vector<xdrop_seed> seeds;
  xdrop_scoring sc{};
  std::vector<int32_t> matrix;
  std::vector<xdrop_result> results;
  bool done = false;
  int status = XDROP_OK;
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

struct CopyRound {  // sets moved to the device by one event
  hipEvent_t ev = nullptr;
  std::vector<std::shared_ptr<SeqSet>> sets;
};

bool same_scoring(const Req& a, const Req& b) {
  return a.sc.alphabet == b.sc.alphabet &&
         a.sc.alphabet_size == b.sc.alphabet_size &&
         a.sc.match == b.sc.match && a.sc.mismatch == b.sc.mismatch &&
         a.sc.gap == b.sc.gap && a.sc.X == b.sc.X && a.matrix == b.matrix;
}

size_t packed_bytes(int alphabet, int64_t syms) {
  return alphabet == XDROP_DNA2 ? (size_t)((syms + 15) / 16) * 4
                                : (size_t)((syms + 3) / 4) * 4;
}

}  // namespace

struct xdrop_server {
  int device = 0;
  int max_inflight = 256;
  int32_t max_batch_seeds = 1 << 16;
  int32_t max_batch_seqs = 1 << 17;
  uint8_t* d_arena = nullptr;
  std::unique_ptr<Arena> arena;
  uint8_t* h_stage = nullptr;  // pinned staging of sets not yet copied
  std::unique_ptr<Arena> stage;
  hipStream_t copy_stream = nullptr;
  std::vector<hipEvent_t> free_events;
  std::deque<CopyRound> copies;  // in flight (worker thread only)
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<SeqSet>> to_place;  // waiting for arena space
  std::deque<std::shared_ptr<Req>> waiting;      // sequences not resident yet
  std::deque<std::shared_ptr<Req>> ready;        // resident, not launched
  std::unordered_map<uint64_t, std::shared_ptr<Req>> all;
  std::unordered_map<uint64_t, std::shared_ptr<SeqSet>> sets;
  uint64_t next_ticket = 1, next_set = 1;
  int inflight = 0;  // requests admitted to run, not finished
  int busy_slots = 0;
  bool stop = false;
  int sticky = XDROP_OK;
  xdrop_server_counters st{};
  std::thread worker;

  void run();
  bool launch(Slot& s, std::vector<std::shared_ptr<Req>>& batch);
  void finish(Slot& s);
  void drop_user(const std::shared_ptr<SeqSet>& set);  // under mu
  void free_set(SeqSet& set);                          // under mu
  std::shared_ptr<SeqSet> make_set(int alphabet, const uint8_t* seqs,
                                   const int64_t* offsets, int32_t n_seqs);
};

void xdrop_server::free_set(SeqSet& set) {
  if (set.placed) arena->release(set.arena_off, set.arena_bytes);
  set.placed = false;
  if (set.pin_off != NONE) stage->release(set.pin_off, set.bytes);
  set.pin_off = NONE;
  set.pageable.clear();
  set.pageable.shrink_to_fit();
  if (set.id) sets.erase(set.id);
}

void xdrop_server::drop_user(const std::shared_ptr<SeqSet>& set) {
  if (--set->users == 0 && set->released) free_set(*set);
}

// A set with its sequences copied from the caller: into pinned staging if
// it has room (the worker then moves them with an asynchronous copy), else
// into ordinary memory.
std::shared_ptr<SeqSet> xdrop_server::make_set(int alphabet,
                                               const uint8_t* seqs,
                                               const int64_t* offsets,
                                               int32_t n_seqs) {
  auto set = std::make_shared<SeqSet>();
  set->alphabet = alphabet;
  if (n_seqs > 0)
    set->offsets.assign(offsets, offsets + n_seqs + 1);
  else
    set->offsets.assign(1, 0);
  set->bytes = packed_bytes(alphabet, set->offsets.back());
  set->arena_bytes = set->bytes + 64;
  size_t off = NONE;
  if (set->bytes) {
    std::lock_guard<std::mutex> lk(mu);
    if (!stage->alloc(set->bytes, &off)) off = NONE;
  }
  if (off != NONE) {
    std::memcpy(h_stage + off, seqs, set->bytes);  // (the range is ours)
    set->pin_off = off;
  } else if (set->bytes) {
    set->pageable.assign(seqs, seqs + set->bytes);
  }
  return set;
}

bool xdrop_server::launch(Slot& s, std::vector<std::shared_ptr<Req>>& batch) {
  // merged offsets: arena-absolute symbol offsets of each set once, a gap
  // entry after each, and a last entry covering every set
  const int alpha = batch[0]->sc.alphabet;
  const int64_t spb = alpha == XDROP_DNA2 ? 4 : 1;  // symbols per byte
  int32_t nseq = 0, nseed = 0;
  int64_t* off = s.h_offsets;
  int64_t max_end = 0;
  std::unordered_map<const SeqSet*, int32_t> first_seq;
  s.first_seed.clear();
  for (auto& r : batch) {
    const SeqSet* set = r->set.get();
    const int32_t rn = (int32_t)set->offsets.size() - 1;
    auto f = first_seq.find(set);
    int32_t first;
    if (f == first_seq.end()) {
      const int64_t base = (int64_t)set->arena_off * spb;
      first = nseq;
      for (int32_t i = 0; i <= rn; ++i) off[nseq + i] = base + set->offsets[i];
      max_end = std::max(max_end, base + set->offsets[rn]);
      nseq += rn + 1;  // the set's end entry starts a gap pseudo-sequence
      first_seq[set] = first;
    } else {
      first = f->second;
    }
    s.first_seed.push_back(nseed);
    for (const auto& sd : r->seeds) {
      xdrop_seed t = sd;
      t.q = sd.q >= 0 && sd.q < rn ? sd.q + first : -1;
      t.t = sd.t >= 0 && sd.t < rn ? sd.t + first : -1;
      s.h_seeds[nseed++] = t;
    }
  }
  // the last entry bounds the readable stream: past every set's end
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
      drop_user(r->set);
      r->set.reset();
      r->done = true;
      --inflight;
      ++st.requests_done;
    }
    s.busy = false;
    --busy_slots;
  }
  cv_done.notify_all();
  cv_work.notify_all();
}

void xdrop_server::run() {
  (void)hipSetDevice(device);
  std::vector<std::shared_ptr<SeqSet>> to_copy;
  for (;;) {
    bool progressed = false;
    // 1. placement: sets in arrival order, as arena space allows
    to_copy.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop) break;
      while (!to_place.empty()) {
        auto& set = to_place.front();
        if (set->released && set->users == 0) {  // dropped before placement
          free_set(*set);
          to_place.pop_front();
          continue;
        }
        size_t off;
        if (!arena->alloc(set->arena_bytes, &off)) break;
        set->arena_off = off;
        set->placed = true;
        to_copy.push_back(set);
        to_place.pop_front();
      }
    }
    // 2. asynchronous copies of the placed sets on the copy stream (from
    // pinned staging; a set held in ordinary memory is staged by the
    // runtime), one event per round
    if (!to_copy.empty()) {
      CopyRound round;
      hipError_t e = hipSuccess;
      for (auto& set : to_copy) {
        const uint8_t* src = set->pin_off != NONE ? h_stage + set->pin_off
                                                  : set->pageable.data();
        if (set->bytes && e == hipSuccess)
          e = hipMemcpyAsync(d_arena + set->arena_off, src, set->bytes,
                             hipMemcpyHostToDevice, copy_stream);
        round.sets.push_back(set);
      }
      if (free_events.empty()) {
        hipEvent_t ev;
        if (e == hipSuccess)
          e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) free_events.push_back(ev);
      }
      if (e == hipSuccess) {
        round.ev = free_events.back();
        free_events.pop_back();
        e = hipEventRecord(round.ev, copy_stream);
      }
      if (e != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        sticky = XDROP_E_DEVICE;
      }
      copies.push_back(std::move(round));
      progressed = true;
    }
    // 3. copies done: the sets are resident
    while (!copies.empty() && copies.front().ev &&
           hipEventQuery(copies.front().ev) == hipSuccess) {
      CopyRound round = std::move(copies.front());
      copies.pop_front();
      free_events.push_back(round.ev);
      std::lock_guard<std::mutex> lk(mu);
      for (auto& set : round.sets) {
        set->resident = true;
        st.h2d_bytes += (int64_t)set->bytes;
        if (set->pin_off != NONE) stage->release(set->pin_off, set->bytes);
        set->pin_off = NONE;
        set->pageable.clear();
        set->pageable.shrink_to_fit();
        if (set->released && set->users == 0) free_set(*set);
      }
      progressed = true;
    }
    // 4. admission: requests whose sequences are resident, in arrival
    // order, as far as the in-flight limit allows
    {
      std::lock_guard<std::mutex> lk(mu);
      for (auto it = waiting.begin();
           it != waiting.end() && inflight < max_inflight;) {
        if ((*it)->set->resident) {
          if (busy_slots > 0) ++st.admitted_while_busy;
          ready.push_back(*it);
          it = waiting.erase(it);
          ++inflight;
          progressed = true;
        } else {
          ++it;
        }
      }
    }
    // 5. completions
    for (auto& s : slots) {
      if (s.busy && hipEventQuery(s.done) == hipSuccess) {
        finish(s);
        progressed = true;
      }
    }
    // 6. launches: micro-batches of ready requests with one scoring
    for (auto& s : slots) {
      if (s.busy) continue;
      std::vector<std::shared_ptr<Req>> batch;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (ready.empty()) break;
        int32_t ns = 0, nq = 0;
        std::unordered_set<const SeqSet*> in_batch;
        auto it = ready.begin();
        while (it != ready.end()) {
          auto& r = *it;
          const int32_t rs = (int32_t)r->seeds.size();
          const int32_t rq = in_batch.count(r->set.get())
                                 ? 0 : (int32_t)r->set->offsets.size();
          if (!batch.empty() &&
              (!same_scoring(*batch[0], *r) || ns + rs > max_batch_seeds ||
               nq + rq + 1 > max_batch_seqs)) {
            ++it;
            continue;
          }
          batch.push_back(r);
          in_batch.insert(r->set.get());
          ns += rs;
          nq += rq;
          it = ready.erase(it);
          if (ns >= max_batch_seeds) break;
        }
        if (!batch.empty()) {
          ++busy_slots;
          ++st.batches_launched;
          st.max_batches_in_flight =
              std::max<int64_t>(st.max_batches_in_flight, busy_slots);
        }
      }
      if (batch.empty()) break;
      if (!launch(s, batch)) {
        std::lock_guard<std::mutex> lk(mu);
        sticky = XDROP_E_DEVICE;
        --busy_slots;
        for (auto& r : batch) {
          r->status = XDROP_E_DEVICE;
          r->done = true;
          drop_user(r->set);
          r->set.reset();
          --inflight;
        }
        cv_done.notify_all();
      }
      progressed = true;
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(mu);
      if (busy_slots > 0 || !copies.empty())
        cv_work.wait_for(lk, std::chrono::microseconds(20));
      else if (to_place.empty() && waiting.empty() && ready.empty())
        cv_work.wait_for(lk, std::chrono::milliseconds(5), [&] {
          return stop || !to_place.empty() || !waiting.empty();
        });
    }
  }
  for (auto& s : slots)
    if (s.busy) {
      (void)hipEventSynchronize(s.done);
      finish(s);
    }
  (void)hipStreamSynchronize(copy_stream);
  for (auto& round : copies)
    if (round.ev) free_events.push_back(round.ev);
  copies.clear();
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
               opts->streams > 16 || opts->arena_mib < 0 ||
               opts->staging_mib < 0))
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
  const size_t stage_bytes =
      (size_t)(opts && opts->staging_mib ? opts->staging_mib : 64) << 20;
  auto* s = new (std::nothrow) xdrop_server();
  if (!s) return XDROP_E_NOMEM;
  s->device = device;
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
  if (hipHostMalloc(&s->h_stage, stage_bytes, hipHostMallocDefault) !=
          hipSuccess ||
      hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) !=
          hipSuccess) {
    s->stop = true;
    xdrop_server_destroy(s);
    return XDROP_E_NOMEM;
  }
  s->stage.reset(new Arena(stage_bytes));
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

static int check_set_args(xdrop_server* s, int alphabet,
                          const int64_t* offsets, int32_t n_seqs) {
  if (alphabet != XDROP_DNA2 && alphabet != XDROP_BYTE) return XDROP_E_INVALID;
  if (n_seqs < 0 || (n_seqs > 0 && !offsets)) return XDROP_E_INVALID;
  if (n_seqs + 1 > s->max_batch_seqs) return XDROP_E_BUDGET;
  for (int32_t i = 0; i < n_seqs; ++i)
    if (offsets[i] < 0 || offsets[i + 1] < offsets[i]) return XDROP_E_INVALID;
  if (n_seqs > 0 && offsets[0] != 0) return XDROP_E_INVALID;
  const int64_t syms = n_seqs > 0 ? offsets[n_seqs] : 0;
  if (packed_bytes(alphabet, syms) + 64 > s->arena->cap()) return XDROP_E_BUDGET;
  return XDROP_OK;
}

int xdrop_server_put_sequences(xdrop_server* s, const uint8_t* seqs,
                               const int64_t* offsets, int32_t n_seqs,
                               int32_t alphabet, uint64_t* set_id) {
  if (!s || !set_id) return XDROP_E_INVALID;
  int rc = check_set_args(s, alphabet, offsets, n_seqs);
  if (rc != XDROP_OK) return rc;
  const int64_t syms = n_seqs > 0 ? offsets[n_seqs] : 0;
  if (syms > 0 && !seqs) return XDROP_E_INVALID;
  auto set = s->make_set(alphabet, seqs, offsets, n_seqs);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->sticky != XDROP_OK) {
      s->free_set(*set);
      return s->sticky;
    }
    set->id = s->next_set++;
    *set_id = set->id;
    s->sets[set->id] = set;
    s->to_place.push_back(set);
  }
  s->cv_work.notify_all();
  return XDROP_OK;
}

int xdrop_server_release_sequences(xdrop_server* s, uint64_t set_id) {
  if (!s) return XDROP_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->sets.find(set_id);
  if (it == s->sets.end() || it->second->released) return XDROP_E_INVALID;
  auto set = it->second;
  set->released = true;
  // freed now if resident and unused; a set still waiting for space or
  // being copied is freed by the worker when that step ends
  if (set->users == 0 && set->resident) s->free_set(*set);
  return XDROP_OK;
}

int xdrop_server_submit(xdrop_server* s, const xdrop_request* r,
                        uint64_t* ticket) {
  if (!s || !r || !ticket) return XDROP_E_INVALID;
  if (r->n_seeds < 0 || (r->n_seeds > 0 && !r->seeds)) return XDROP_E_INVALID;
  const xdrop_scoring& sc = r->scoring;
  if (sc.alphabet != XDROP_DNA2 && sc.alphabet != XDROP_BYTE)
    return XDROP_E_INVALID;
  if (sc.alphabet == XDROP_DNA2 ? sc.alphabet_size != 4
                                : (sc.alphabet_size < 1 || sc.alphabet_size > 32))
    return XDROP_E_INVALID;
  if (sc.gap > 0 || sc.X < 0) return XDROP_E_INVALID;
  if (r->n_seeds > s->max_batch_seeds) return XDROP_E_BUDGET;
  auto q = std::make_shared<Req>();
  std::shared_ptr<SeqSet> own;
  if (!r->seq_set) {
    int rc = check_set_args(s, sc.alphabet, r->offsets, r->n_seqs);
    if (rc != XDROP_OK) return rc;
    const int64_t syms = r->n_seqs > 0 ? r->offsets[r->n_seqs] : 0;
    if (syms > 0 && !r->seqs) return XDROP_E_INVALID;
    own = s->make_set(sc.alphabet, r->seqs, r->offsets, r->n_seqs);
    own->released = true;  // lives as long as the request
  }
  q->seeds.assign(r->seeds, r->seeds + r->n_seeds);
  q->sc = sc;
  if (sc.matrix)
    q->matrix.assign(sc.matrix, sc.matrix + sc.alphabet_size * sc.alphabet_size);
  q->sc.matrix = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->sticky != XDROP_OK) {
      if (own) s->free_set(*own);
      return s->sticky;
    }
    if (own) {
      q->set = own;
    } else {
      auto it = s->sets.find(r->seq_set);
      if (it == s->sets.end() || it->second->released ||
          it->second->alphabet != sc.alphabet)
        return XDROP_E_INVALID;
      q->set = it->second;
      // the bytes of the sequences the seeds use that this request does not
      // copy
      const auto& off = q->set->offsets;
      const int32_t ns = (int32_t)off.size() - 1;
      std::unordered_set<int32_t> used;
      for (const auto& z : q->seeds) {
        if (z.q >= 0 && z.q < ns) used.insert(z.q);
        if (z.t >= 0 && z.t < ns) used.insert(z.t);
      }
      for (int32_t i : used)
        s->st.reused_bytes +=
            (int64_t)packed_bytes(sc.alphabet, off[i + 1] - off[i]);
    }
    q->set->users++;
    q->ticket = s->next_ticket++;
    *ticket = q->ticket;
    s->all[q->ticket] = q;
    ++s->st.requests_submitted;
    if (q->seeds.empty()) {
      q->done = true;  // nothing to compute
      s->drop_user(q->set);
      q->set.reset();
    } else {
      if (own) s->to_place.push_back(own);
      s->waiting.push_back(q);
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

int xdrop_server_stats(xdrop_server* s, xdrop_server_counters* out) {
  if (!s || !out) return XDROP_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->batches_in_flight = s->busy_slots;
  return XDROP_OK;
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
  if (s->copy_stream) {
    (void)hipStreamSynchronize(s->copy_stream);
    (void)hipStreamDestroy(s->copy_stream);
  }
  for (auto ev : s->free_events) (void)hipEventDestroy(ev);
  if (s->h_stage) (void)hipHostFree(s->h_stage);
  if (s->d_arena) (void)hipFree(s->d_arena);
  delete s;
  return XDROP_OK;
}

}  // extern "C"
