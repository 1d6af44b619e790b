// Host side of the X-Drop library: argument checks, workspace, launch
// sequence, autotuning and graph replay.  The C ABI is declared in
// include/xdrop.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "xdrop.h"
#include "xdrop_internal.h"

using namespace xd;

struct GraphEntry {
  // launch inputs the captured graph is valid for
  const void* seqs;
  const void* offsets;
  const void* seeds;
  void* results;
  int32_t n_seqs, n_seeds;
  xdrop_scoring sc;
  std::vector<int32_t> matrix;
  xdrop_options opts;
  hipStream_t stream;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Tuned launch options apply to batches of one alphabet, X class and batch
// size class: the launch form is chosen on the host before any device data
// is read, and these are what the host knows.  X stands in for the band
// width (the tile), the batch size for how many waves the queue feeds (the
// form and the chunk).
struct TuneKey {
  int alphabet, x_class, size_class;
  bool operator==(const TuneKey& o) const {
    return alphabet == o.alphabet && x_class == o.x_class &&
           size_class == o.size_class;
  }
};
struct TunedEntry {
  TuneKey key;
  xdrop_options opts;
};

struct xdrop_ctx {
  int device = 0;
  int num_cu = 0;
  int sticky = XDROP_OK;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int32_t* counters = nullptr;
  int32_t* gen_scratch = nullptr;
  int gen_slots = 32;
  int32_t* last_counters = nullptr;  // counters of the last batch
  int32_t last_combine_blocks = 0;    // its combine blocks (tier counts)
  char* scratch = nullptr;  // the device's fixed scratch (allocation-free
                            // entry point)
  int pair_blocks_per_cu[2] = {0, 0};   // two rows per wave
  int rows4_blocks_per_cu[2] = {0, 0};  // four rows per wave
  int block_blocks_per_cu[2] = {0, 0};
  int dual_blocks_per_cu[2] = {0, 0};
  int blocks_per_cu[2] = {0, 0};  // [alphabet]
  std::string arch;  // gfx name of the device (tuning cache key)
  std::vector<TunedEntry> tuned;  // xdrop_autotune / xdrop_load_tuning
  std::vector<GraphEntry> graphs;
  // phase timing (xdrop_ctx_set_timing): one set of events around the
  // launch phases per batch, summed by xdrop_last_timing
  bool timing = false;
  std::vector<std::array<hipEvent_t, 6>> ev_sets;
  size_t ev_used = 0;
};

namespace {

constexpr size_t ALIGN = 256;

constexpr size_t align_up(size_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

struct Layout {
  size_t items, order, gen_q, dev_q, esc_q, bad, total;
};

Layout layout(int32_t n_items, int32_t n_seqs) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes > 0 ? bytes : 1);
    return o;
  };
  const size_t ni = (size_t)std::max(n_items, 1);
  L.items = take(ni * sizeof(ItemResult));
  L.order = take(ni * 4);
  L.gen_q = take(ni * 4);
  L.dev_q = take(ni * 4);
  L.esc_q = take(ni * 4);
  L.bad = take((size_t)std::max(n_seqs, 1));
  L.total = off;
  return L;
}

int fail(xdrop_ctx* c, hipError_t e) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return XDROP_E_NOMEM;
  if (c) c->sticky = XDROP_E_DEVICE;
  return XDROP_E_DEVICE;
}

#define HIP_OK(expr)                     \
  do {                                   \
    hipError_t e_ = (expr);              \
    if (e_ != hipSuccess) return fail(c, e_); \
  } while (0)

// Scoring checks and the kernel-side constants.
int fill_scoring(const xdrop_scoring* sc, Params& P) {
  if (!sc) return XDROP_E_INVALID;
  if (sc->alphabet != XDROP_DNA2 && sc->alphabet != XDROP_BYTE)
    return XDROP_E_INVALID;
  if (sc->gap > 0 || sc->gap < -MAX_ENTRY || sc->X < 0) return XDROP_E_INVALID;
  const int A = sc->alphabet_size;
  if (sc->alphabet == XDROP_DNA2 && A != 4) return XDROP_E_INVALID;
  if (sc->alphabet == XDROP_BYTE && (A < 1 || A > TABLE_DIM))
    return XDROP_E_INVALID;
  std::vector<int32_t> M((size_t)A * A);
  if (sc->matrix) {
    for (int i = 0; i < A * A; ++i) M[i] = sc->matrix[i];
  } else {
    for (int i = 0; i < A; ++i)
      for (int j = 0; j < A; ++j)
        M[(size_t)i * A + j] = i == j ? sc->match : sc->mismatch;
  }
  int max_abs = 0;
  for (int32_t v : M) {
    if (v > MAX_ENTRY || v < -MAX_ENTRY) return XDROP_E_INVALID;
    max_abs = std::max(max_abs, std::abs(v));
  }
  const int g = sc->gap;
  P.alphabet = sc->alphabet;
  P.gap = g;
  P.X = std::min(sc->X, X_CLAMP);
  P.max_abs = max_abs + 2 * std::abs(g);
  if (P.max_abs == 0) P.max_abs = 1;
  std::memset(P.table, 0, sizeof(P.table));
  if (sc->alphabet == XDROP_DNA2) {
    // the 2-bit path compares codes: the matrix must be match / mismatch
    const int32_t mt = M[0], mm = M[1];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        if (M[i * 4 + j] != (i == j ? mt : mm)) return XDROP_E_INVALID;
    P.mat_s = mt - 2 * g;
    P.mis_s = mm - 2 * g;
  } else {
    P.mat_s = P.mis_s = 0;
    for (int i = 0; i < A; ++i)
      for (int j = 0; j < A; ++j)
        P.table[i * TABLE_DIM + j] = (int16_t)(M[(size_t)i * A + j] - 2 * g);
  }
  return XDROP_OK;
}

int check_options(const xdrop_options* o) {
  if (!o) return XDROP_OK;
  if (o->variant < 0 || o->variant > XDROP_VARIANT_ROWS16)
    return XDROP_E_INVALID;
  const int t = o->tile;
  if (!(t == 0 || t == 1 || t == 2 || t == 4 || t == 8))
    return XDROP_E_INVALID;
  if (o->chunk < 0 || o->chunk > 64) return XDROP_E_INVALID;
  if (o->band_cap < 0 || o->order < 0 || o->order > 1 ||
      o->waves_per_cu < 0 || o->waves_per_cu > 64)
    return XDROP_E_INVALID;
  return XDROP_OK;
}

int x_class(int32_t X) { return X < 24 ? 0 : X < 100 ? 1 : 2; }
int size_class(int32_t n_seeds) {
  return n_seeds < 2048 ? 0 : n_seeds < 32768 ? 1 : n_seeds < 524288 ? 2 : 3;
}
TuneKey tune_key(const xdrop_scoring* sc, int32_t n_seeds) {
  return TuneKey{sc->alphabet == XDROP_BYTE ? 1 : 0, x_class(sc->X),
                 size_class(n_seeds)};
}

// Options of a batch: the caller's, over the tuned entry of the batch's key
// (if any), over the defaults.
xdrop_options resolve(const xdrop_ctx* c, const xdrop_scoring* sc,
                      const xdrop_options* o, int32_t n_seeds) {
  xdrop_options r{};
  const TuneKey k = tune_key(sc, n_seeds);
  for (const auto& t : c->tuned)
    if (t.key == k) r = t.opts;
  if (o) {
    if (o->variant) r.variant = o->variant;
    if (o->tile) r.tile = o->tile;
    if (o->chunk) r.chunk = o->chunk;
    r.band_cap = o->band_cap;
    r.order = o->order;
    if (o->waves_per_cu) r.waves_per_cu = o->waves_per_cu;
  }
  // the row kernels keep no per-antidiagonal band width: a band cap runs on
  // the wave kernel
  if ((r.variant == XDROP_VARIANT_PAIR || r.variant == XDROP_VARIANT_DUAL16 ||
       r.variant == XDROP_VARIANT_ROWS16) &&
      r.band_cap > 0)
    r.variant = XDROP_VARIANT_WAVE;
  if (!r.tile) r.tile = 1;
  return r;
}

// The automatic choices that depend on the batch size: the queue chunk (one
// extension per claim while the batch fills the persistent grid at most a
// few times over, where longest-first balance matters most; up to 8 per
// claim for large batches, fewer contended atomics on the queue head) and
// the form (a batch within one wave of the persistent grid starts every
// extension at once: the plain form, one launched wave per extension, then
// does the same work without the queue and the longest-first order).
void finalize(const xdrop_ctx* c, int alphabet, int32_t n_items,
              xdrop_options& o) {
  const int64_t waves = (int64_t)c->num_cu * c->blocks_per_cu[alphabet] * WPB;
  if (!o.chunk)
    o.chunk = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>(8, n_items / (waves * 8)));
  if (o.variant == XDROP_VARIANT_AUTO)
    o.variant = (o.waves_per_cu == 0 && (int64_t)n_items <= waves)
                    ? XDROP_VARIANT_PLAIN : XDROP_VARIANT_WAVE;
}

void drop_graphs(xdrop_ctx* c);

// Device buffers of the launch sequence.  Graphs captured earlier hold the
// old workspace address, so a move drops them.
int ensure_workspace(xdrop_ctx* c, size_t bytes, hipStream_t st) {
  if (!c->counters) {
    // zeroed once here (a kernel on the batch's stream, never inside a
    // capture: graphs are recorded after this call); from then on the last
    // kernel of every batch leaves them zero for the next one
    HIP_OK(hipMalloc(&c->counters, C_COUNT * sizeof(int32_t)));
    HIP_OK(launch_reset(c->counters, st));
  }
  if (!c->gen_scratch) {
    HIP_OK(hipMalloc(&c->gen_scratch,
                     (size_t)c->gen_slots * 3 * GEN_CAP * sizeof(int32_t)));
  }
  if (bytes > c->ws_bytes) {
    drop_graphs(c);
    if (c->ws) HIP_OK(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
    size_t want = bytes + bytes / 4;
    HIP_OK(hipMalloc(&c->ws, want));
    c->ws_bytes = want;
  }
  return XDROP_OK;
}

// Device buffers one batch runs on: the context's workspace, or the fixed
// scratch of the allocation-free entry point.
struct Workspace {
  char* ws;              // Layout regions (items, order, queues, symbols)
  int32_t* counters;     // C_COUNT counters
  int32_t* gen_scratch;  // device-memory tier rings, gen_slots of them
  int gen_slots;
  bool reset;            // zero the counters first (they hold another
                         // call's values)
};

// Enqueue the whole launch sequence of one batch on `st`.  fixed == nullptr:
// the context's workspace, grown on demand; otherwise the given buffers,
// and nothing is allocated.
int enqueue(xdrop_ctx* c, const uint8_t* d_seqs, const int64_t* d_offsets,
            int32_t n_seqs, const xdrop_seed* d_seeds, int32_t n_seeds,
            const xdrop_scoring* sc, const xdrop_options* opts,
            xdrop_result* d_results, hipStream_t st,
            const Workspace* fixed = nullptr) {
  Params P;
  std::memset(&P, 0, sizeof(P));
  int rc = fill_scoring(sc, P);
  if (rc != XDROP_OK) return rc;
  rc = check_options(opts);
  if (rc != XDROP_OK) return rc;
  if (n_seeds < 0 || n_seqs < 0 || n_seeds > (1 << 29)) return XDROP_E_INVALID;
  if (n_seeds == 0) return XDROP_OK;
  if (!d_seqs || !d_offsets || !d_seeds || !d_results || n_seqs == 0)
    return XDROP_E_INVALID;
  xdrop_options o = resolve(c, sc, opts, n_seeds);
  // the 16-bit kernel only where its relative scores are exact
  if (o.variant == XDROP_VARIANT_DUAL16 && !dual_exact(P))
    o.variant = XDROP_VARIANT_WAVE;
  const int32_t n_items = 2 * n_seeds;
  Layout L = layout(n_items, n_seqs);
  Workspace W;
  if (fixed) {
    W = *fixed;
  } else {
    rc = ensure_workspace(c, L.total, st);
    if (rc != XDROP_OK) return rc;
    W = Workspace{(char*)c->ws, c->counters, c->gen_scratch, c->gen_slots,
                  false};
  }
  char* ws = W.ws;
  c->last_counters = W.counters;
  c->last_combine_blocks = combine_blocks(n_seeds);

  P.seqs = (const uint32_t*)d_seqs;
  P.offsets = d_offsets;
  P.seeds = (const int32_t*)d_seeds;
  P.items = (ItemResult*)(ws + L.items);
  P.counters = W.counters;
  P.gen_queue = (int32_t*)(ws + L.gen_q);
  P.dev_queue = (int32_t*)(ws + L.dev_q);
  P.esc_queue = (int32_t*)(ws + L.esc_q);
  P.gen_scratch = W.gen_scratch;
  P.n_seqs = n_seqs;
  P.n_seeds = n_seeds;
  P.n_items = n_items;
  P.tile = o.tile;
  finalize(c, P.alphabet, n_items, o);
  P.chunk = o.chunk;
  P.band_cap = o.band_cap;
  P.gen_slots = W.gen_slots;
  const bool plain = o.variant == XDROP_VARIANT_PLAIN;
  P.flags = plain ? F_PLAIN : 0;

  hipEvent_t* ev = nullptr;
  if (c->timing && !fixed) {  // (event creation is left to the other path)
    if (c->ev_used == c->ev_sets.size()) {
      std::array<hipEvent_t, 6> set{};
      for (auto& e : set) HIP_OK(hipEventCreate(&e));
      c->ev_sets.push_back(set);
    }
    ev = c->ev_sets[c->ev_used].data();
  }
  const bool timed = ev != nullptr;
  if (timed) HIP_OK(hipEventRecord(ev[0], st));
  if (W.reset) HIP_OK(launch_reset(W.counters, st));
  // (the counters were left zero by the previous batch's combine kernel)
  if (P.alphabet == 1) {
    P.seq_bad = (const uint8_t*)(ws + L.bad);
    HIP_OK(launch_validate(d_seqs, d_offsets, n_seqs, P.seeds, n_seeds,
                           sc->alphabet_size, (uint8_t*)(ws + L.bad),
                           std::min(c->num_cu * 64, (n_seqs + 15) / 16 + 1),
                           st));
  }
  if (o.order == 0 && !plain) {
    int32_t* ord = (int32_t*)(ws + L.order);
    HIP_OK(launch_order(P.seeds, d_offsets, n_seqs, n_items, W.counters, ord,
                        c->num_cu, st));
    P.order = ord;
    P.flags |= F_ORDERED;
  }
  const int a = P.alphabet;
  auto persistent_grid = [&]() {
    int bpc = c->blocks_per_cu[a];
    if (o.waves_per_cu > 0)
      bpc = std::max(1, std::min(bpc, (o.waves_per_cu + WPB - 1) / WPB));
    return c->num_cu * bpc;
  };
  if (timed) HIP_OK(hipEventRecord(ev[1], st));
  if (o.variant == XDROP_VARIANT_WORKGROUP) {
    // every extension on the workgroup tier
    HIP_OK(launch_fill_queue(P.order, n_items, P.gen_queue, W.counters,
                             C_GEN_TAIL, st));
    if (timed) HIP_OK(hipEventRecord(ev[2], st));
    if (timed) HIP_OK(hipEventRecord(ev[3], st));
  } else if (o.variant == XDROP_VARIANT_DUAL16) {
    // two extensions per wave in 16-bit halves; bands that fill a half's
    // window are handed on to the wave kernel
    const int pairs = (n_items + 1) / 2;
    const int dgrid = std::min(c->num_cu * c->dual_blocks_per_cu[a],
                               (pairs + WPB - 1) / WPB);
    HIP_OK(launch_dual(P, dgrid, st));
    if (timed) HIP_OK(hipEventRecord(ev[2], st));
    Params Q = P;
    Q.flags |= F_ESC;
    HIP_OK(launch_wave(Q, persistent_grid(), st));
    if (timed) HIP_OK(hipEventRecord(ev[3], st));
  } else if (o.variant == XDROP_VARIANT_PAIR ||
             o.variant == XDROP_VARIANT_ROWS16) {
    // two (four) extensions per wave in rows of 32 (16) lanes; bands that
    // fill a row are handed on to the wave kernel
    const int rows = o.variant == XDROP_VARIANT_PAIR ? 2 : 4;
    const int per_cu = rows == 2 ? c->pair_blocks_per_cu[a]
                                 : c->rows4_blocks_per_cu[a];
    const int waves = (n_items + rows - 1) / rows;
    const int pgrid = std::min(c->num_cu * per_cu, (waves + WPB - 1) / WPB);
    HIP_OK(launch_rows(P, rows, pgrid, st));
    if (timed) HIP_OK(hipEventRecord(ev[2], st));
    Params Q = P;
    Q.flags |= F_ESC;
    HIP_OK(launch_wave(Q, persistent_grid(), st));
    if (timed) HIP_OK(hipEventRecord(ev[3], st));
  } else {
    int grid;
    if (plain)
      grid = (n_items + WPB - 1) / WPB;
    else
      grid = std::min(persistent_grid(),
                      (n_items + WPB * o.chunk - 1) / (WPB * o.chunk));
    HIP_OK(launch_wave(P, grid, st));
    if (timed) HIP_OK(hipEventRecord(ev[2], st));
    if (timed) HIP_OK(hipEventRecord(ev[3], st));
  }
  // extensions whose band outgrew one wave's window: the block tier, and
  // beyond 2,048 cells the device-memory tier (both leave at once when
  // nothing was handed to them)
  HIP_OK(launch_block(P, std::min(c->num_cu * c->block_blocks_per_cu[a],
                                  n_items), st));
  HIP_OK(launch_general(P, W.gen_slots, st));
  if (timed) HIP_OK(hipEventRecord(ev[4], st));
  HIP_OK(launch_combine(P, d_results, st));
  if (timed) {
    HIP_OK(hipEventRecord(ev[5], st));
    ++c->ev_used;
  }
  return XDROP_OK;
}

}  // namespace

extern "C" {

const char* xdrop_strerror(int s) {
  switch (s) {
    case XDROP_OK: return "ok";
    case XDROP_E_INVALID: return "invalid argument";
    case XDROP_E_RANGE: return "seed or score out of range";
    case XDROP_E_NOMEM: return "out of memory";
    case XDROP_E_DEVICE: return "device error";
    case XDROP_E_BUDGET: return "request exceeds the memory budget";
    case XDROP_E_SYMBOL: return "symbol outside the alphabet";
    case XDROP_BAND_OVERFLOW: return "band wider than the cap";
    case XDROP_PENDING: return "pending";
    case XDROP_E_SCRATCH:
      return "batch larger than the fixed scratch of the allocation-free "
             "entry point";
    default: return "unknown status";
  }
}

int xdrop_ctx_create(int device, const xdrop_ctx_opts* opts,
                     xdrop_ctx** out) {
  if (!out) return XDROP_E_INVALID;
  *out = nullptr;
  if (opts && (opts->device_tier_slots < 0 || opts->device_tier_slots > 1024))
    return XDROP_E_INVALID;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return XDROP_E_INVALID;
  xdrop_ctx* c = new (std::nothrow) xdrop_ctx();
  if (!c) return XDROP_E_NOMEM;
  c->device = device;
  if (opts && opts->device_tier_slots) c->gen_slots = opts->device_tier_slots;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return XDROP_E_DEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return XDROP_E_DEVICE;
  }
  c->num_cu = prop.multiProcessorCount;
  c->arch = prop.gcnArchName;
  c->arch = c->arch.substr(0, c->arch.find(':'));
  // occupancy of every kernel form, queried once here (the launch paths then
  // make no runtime queries, under graph capture or otherwise)
  for (int a = 0; a < 2; ++a) {
    c->blocks_per_cu[a] = wave_blocks_per_cu(a);
    c->pair_blocks_per_cu[a] = rows_blocks_per_cu(a, 2);
    c->rows4_blocks_per_cu[a] = rows_blocks_per_cu(a, 4);
    c->block_blocks_per_cu[a] = block_blocks_per_cu(a);
    c->dual_blocks_per_cu[a] = dual_blocks_per_cu(a);
  }
  // the address of this device's fixed scratch, for the allocation-free
  // entry point
  void* sp = nullptr;
  if (noalloc_scratch(device, &sp) != hipSuccess || !sp) {
    delete c;
    return XDROP_E_DEVICE;
  }
  c->scratch = (char*)sp;
  *out = c;
  return XDROP_OK;
}

int xdrop_ctx_destroy(xdrop_ctx* c) {
  if (!c) return XDROP_E_INVALID;
  (void)hipSetDevice(c->device);
  for (auto& g : c->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  if (c->ws) (void)hipFree(c->ws);
  if (c->counters) (void)hipFree(c->counters);
  if (c->gen_scratch) (void)hipFree(c->gen_scratch);
  for (auto& set : c->ev_sets)
    for (auto& e : set) (void)hipEventDestroy(e);
  delete c;
  return XDROP_OK;
}

int xdrop_extend_batch(xdrop_ctx* c, const uint8_t* d_seqs,
                       const int64_t* d_offsets, int32_t n_seqs,
                       const xdrop_seed* d_seeds, int32_t n_seeds,
                       const xdrop_scoring* scoring, const xdrop_options* opts,
                       xdrop_result* d_results, void* stream) {
  if (!c) return XDROP_E_INVALID;
  if (c->sticky != XDROP_OK) return c->sticky;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, hipErrorInvalidDevice);
  return enqueue(c, d_seqs, d_offsets, n_seqs, d_seeds, n_seeds, scoring,
                 opts, d_results, (hipStream_t)stream);
}

int xdrop_extend_batch_noalloc(xdrop_ctx* c, const uint8_t* d_seqs,
                               const int64_t* d_offsets, int32_t n_seqs,
                               const xdrop_seed* d_seeds, int32_t n_seeds,
                               const xdrop_scoring* scoring,
                               const xdrop_options* opts,
                               xdrop_result* d_results, void* stream) {
  if (!c) return XDROP_E_INVALID;
  if (c->sticky != XDROP_OK) return c->sticky;
  if (n_seeds < 0 || n_seqs < 0) return XDROP_E_INVALID;
  if (n_seeds > XDROP_NOALLOC_MAX_SEEDS || n_seqs > XDROP_NOALLOC_MAX_SEQS)
    return XDROP_E_SCRATCH;
  // scratch: counters | device-memory tier rings | Layout regions
  constexpr size_t CNT = align_up(C_COUNT * sizeof(int32_t));
  constexpr int SLOTS = 4;
  constexpr size_t RINGS = (size_t)SLOTS * 3 * GEN_CAP * sizeof(int32_t);
  const Layout L = layout(2 * n_seeds, n_seqs);
  if (CNT + RINGS + L.total > NOALLOC_BYTES) return XDROP_E_SCRATCH;
  static_assert(C_COUNT * sizeof(int32_t) <= CNT, "counter block");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, hipErrorInvalidDevice);
  const Workspace W{c->scratch + CNT + RINGS, (int32_t*)c->scratch,
                    (int32_t*)(c->scratch + CNT), SLOTS, true};
  return enqueue(c, d_seqs, d_offsets, n_seqs, d_seeds, n_seeds, scoring,
                 opts, d_results, (hipStream_t)stream, &W);
}

int xdrop_ctx_set_timing(xdrop_ctx* c, int32_t on) {
  if (!c) return XDROP_E_INVALID;
  (void)hipSetDevice(c->device);
  c->timing = on != 0;
  c->ev_used = 0;
  return XDROP_OK;
}

int xdrop_last_timing(xdrop_ctx* c, float* ms, int32_t n,
                      int32_t* batches) {
  if (!c || !ms || n < 0) return XDROP_E_INVALID;
  for (int i = 0; i < n; ++i) ms[i] = 0.f;
  if (batches) *batches = (int32_t)c->ev_used;
  if (!c->ev_used) return XDROP_E_INVALID;
  HIP_OK(hipEventSynchronize(c->ev_sets[c->ev_used - 1][5]));
  for (size_t b = 0; b < c->ev_used; ++b)
    for (int i = 0; i < n && i < 5; ++i) {
      float t = 0.f;
      HIP_OK(hipEventElapsedTime(&t, c->ev_sets[b][i], c->ev_sets[b][i + 1]));
      ms[i] += t;
    }
  c->ev_used = 0;
  return XDROP_OK;
}

int xdrop_last_stats(xdrop_ctx* c, int64_t* counts, int32_t n_counts) {
  if (!c || !counts || n_counts < 0) return XDROP_E_INVALID;
  std::vector<int32_t> h((size_t)N_TIERS * MAX_COMBINE_BLOCKS, 0);
  const int nb = c->last_counters ? c->last_combine_blocks : 0;
  if (nb > 0 &&
      hipMemcpy(h.data(), c->last_counters + C_PART,
                (size_t)N_TIERS * nb * sizeof(int32_t),
                hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, hipErrorUnknown);
  for (int i = 0; i < n_counts; ++i) {
    int64_t sum = 0;
    if (i < N_TIERS)
      for (int b = 0; b < nb; ++b) sum += h[(size_t)N_TIERS * b + i];
    counts[i] = sum;
  }
  return XDROP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ graphs
namespace {

bool same_scoring(const GraphEntry& g, const xdrop_scoring* sc) {
  if (g.sc.alphabet != sc->alphabet || g.sc.alphabet_size != sc->alphabet_size ||
      g.sc.match != sc->match || g.sc.mismatch != sc->mismatch ||
      g.sc.gap != sc->gap || g.sc.X != sc->X)
    return false;
  if ((sc->matrix == nullptr) != g.matrix.empty()) return false;
  if (sc->matrix) {
    const size_t n = (size_t)sc->alphabet_size * sc->alphabet_size;
    if (g.matrix.size() != n) return false;
    for (size_t i = 0; i < n; ++i)
      if (g.matrix[i] != sc->matrix[i]) return false;
  }
  return true;
}

bool same_opts(const xdrop_options& a, const xdrop_options& b) {
  return a.variant == b.variant && a.tile == b.tile && a.chunk == b.chunk &&
         a.band_cap == b.band_cap && a.order == b.order &&
         a.waves_per_cu == b.waves_per_cu;
}

void drop_graphs(xdrop_ctx* c) {
  for (auto& g : c->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  c->graphs.clear();
}

}  // namespace

extern "C" int xdrop_extend_batch_graph(
    xdrop_ctx* c, const uint8_t* d_seqs, const int64_t* d_offsets,
    int32_t n_seqs, const xdrop_seed* d_seeds, int32_t n_seeds,
    const xdrop_scoring* sc, const xdrop_options* opts,
    xdrop_result* d_results, void* stream) {
  if (!c) return XDROP_E_INVALID;
  if (c->sticky != XDROP_OK) return c->sticky;
  hipStream_t st = (hipStream_t)stream;
  if (!st) return XDROP_E_INVALID;  // the legacy stream cannot be captured
  Params tmp;
  int rc = fill_scoring(sc, tmp);
  if (rc != XDROP_OK) return rc;
  rc = check_options(opts);
  if (rc != XDROP_OK) return rc;
  if (n_seeds < 0 || n_seqs < 0 || n_seeds > (1 << 29)) return XDROP_E_INVALID;
  if (n_seeds == 0) return XDROP_OK;
  if (!d_seqs || !d_offsets || !d_seeds || !d_results || n_seqs == 0)
    return XDROP_E_INVALID;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, hipErrorInvalidDevice);
  const xdrop_options o = resolve(c, sc, opts, n_seeds);
  for (auto& g : c->graphs) {
    if (g.seqs == d_seqs && g.offsets == d_offsets && g.seeds == d_seeds &&
        g.results == d_results && g.n_seqs == n_seqs &&
        g.n_seeds == n_seeds && g.stream == st && same_scoring(g, sc) &&
        same_opts(g.opts, o)) {
      HIP_OK(hipGraphLaunch(g.exec, st));
      return XDROP_OK;
    }
  }
  // everything that allocates or queries happens before the capture
  Layout L = layout(2 * n_seeds, n_seqs);
  rc = ensure_workspace(c, L.total, st);  // (drops the graphs if it moves)
  if (rc != XDROP_OK) return rc;
  GraphEntry g;
  g.seqs = d_seqs; g.offsets = d_offsets; g.seeds = d_seeds;
  g.results = d_results; g.n_seqs = n_seqs; g.n_seeds = n_seeds;
  g.sc = *sc;
  if (sc->matrix)
    g.matrix.assign(sc->matrix,
                    sc->matrix + (size_t)sc->alphabet_size * sc->alphabet_size);
  g.sc.matrix = nullptr;
  g.opts = o;
  g.stream = st;
  HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  rc = enqueue(c, d_seqs, d_offsets, n_seqs, d_seeds, n_seeds, sc, &o,
               d_results, st);
  hipGraph_t graph = nullptr;
  hipError_t ce = hipStreamEndCapture(st, &graph);
  if (rc != XDROP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ce != hipSuccess) return fail(c, ce);
  hipGraphExec_t exec = nullptr;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(c, ie);
  }
  g.graph = graph;
  g.exec = exec;
  c->graphs.push_back(std::move(g));
  if (c->graphs.size() > 64) {  // bounded cache: drop the oldest
    auto& old = c->graphs.front();
    (void)hipGraphExecDestroy(old.exec);
    (void)hipGraphDestroy(old.graph);
    c->graphs.erase(c->graphs.begin());
  }
  HIP_OK(hipGraphLaunch(exec, st));
  return XDROP_OK;
}

// ------------------------------------------------------------------ tuning
namespace {

// Mean extension length m + n of a batch (host copies of its offsets and
// seeds; recorded with the tuned choice).
int mean_extension_length(const int64_t* d_offsets, int32_t n_seqs,
                          const xdrop_seed* d_seeds, int32_t n_seeds,
                          double* out) {
  std::vector<int64_t> off((size_t)n_seqs + 1);
  std::vector<xdrop_seed> sd((size_t)n_seeds);
  if (hipMemcpy(off.data(), d_offsets, off.size() * sizeof(int64_t),
                hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(sd.data(), d_seeds, sd.size() * sizeof(xdrop_seed),
                hipMemcpyDeviceToHost) != hipSuccess)
    return XDROP_E_DEVICE;
  double sum = 0;
  for (const auto& z : sd) {
    if (z.q < 0 || z.q >= n_seqs || z.t < 0 || z.t >= n_seqs) continue;
    sum += (double)(off[z.q + 1] - off[z.q]) +
           (double)(off[z.t + 1] - off[z.t]) - 2.0 * z.k;
  }
  *out = sum / (2.0 * std::max(n_seeds, 1));
  return XDROP_OK;
}

void set_tuned(xdrop_ctx* c, const TuneKey& k, const xdrop_options& o) {
  for (auto& t : c->tuned)
    if (t.key == k) {
      t.opts = o;
      return;
    }
  c->tuned.push_back(TunedEntry{k, o});
}

}  // namespace

extern "C" int xdrop_autotune(xdrop_ctx* c, const uint8_t* d_seqs,
                              const int64_t* d_offsets, int32_t n_seqs,
                              const xdrop_seed* d_seeds, int32_t n_seeds,
                              const xdrop_scoring* sc,
                              xdrop_result* d_results, void* stream,
                              const char* cache_path,
                              xdrop_options* best_out) {
  if (!c || !sc) return XDROP_E_INVALID;
  if (c->sticky != XDROP_OK) return c->sticky;
  if (n_seeds <= 0 || n_seqs <= 0 || !d_offsets || !d_seeds)
    return XDROP_E_INVALID;
  Params tmp;
  int rc = fill_scoring(sc, tmp);
  if (rc != XDROP_OK) return rc;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, hipErrorInvalidDevice);
  hipStream_t st = (hipStream_t)stream;
  const TuneKey key = tune_key(sc, n_seeds);
  // candidates: the row forms (tile and chunk of the wave kernel that takes
  // the extensions it hands on), the persistent wave form (tile x chunk),
  // the plain form (tile), the workgroup form; every field is set, so no
  // tuned entry applies while they are timed
  std::vector<xdrop_options> cand;
  const int tiles[] = {1, 2, 4, 8};
  const int chunks[] = {1, 2, 4, 8, 16, 32, 64};
  for (int v : {XDROP_VARIANT_PAIR, XDROP_VARIANT_ROWS16})
    for (int ch : {4, 16}) {
      xdrop_options o{};
      o.variant = v; o.tile = 1; o.chunk = ch;
      cand.push_back(o);
    }
  for (int t : tiles)
    for (int ch : chunks) {
      xdrop_options o{};
      o.variant = XDROP_VARIANT_WAVE; o.tile = t; o.chunk = ch;
      cand.push_back(o);
    }
  for (int t : tiles) {
    xdrop_options o{};
    o.variant = XDROP_VARIANT_PLAIN; o.tile = t; o.chunk = 1;
    cand.push_back(o);
  }
  {
    xdrop_options o{};
    o.variant = XDROP_VARIANT_WORKGROUP; o.tile = 1; o.chunk = 1;
    cand.push_back(o);
  }
  if (dual_exact(tmp))
    for (int ch : {1, 8}) {
      xdrop_options o{};
      o.variant = XDROP_VARIANT_DUAL16; o.tile = 1; o.chunk = ch;
      cand.push_back(o);
    }
  double mean_len = 0;
  rc = mean_extension_length(d_offsets, n_seqs, d_seeds, n_seeds, &mean_len);
  if (rc != XDROP_OK) return fail(c, hipErrorUnknown);
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  float best_ms = 1e30f, plain_ms = 0.f;
  xdrop_options best{};
  for (const auto& o : cand) {
    // one warm run, then the median of three timed runs (one if slow)
    rc = enqueue(c, d_seqs, d_offsets, n_seqs, d_seeds, n_seeds, sc, &o,
                 d_results, st);
    if (rc != XDROP_OK) break;
    float t[3];
    int reps = 3;
    for (int r = 0; r < reps; ++r) {
      HIP_OK(hipEventRecord(e0, st));
      rc = enqueue(c, d_seqs, d_offsets, n_seqs, d_seeds, n_seeds, sc, &o,
                   d_results, st);
      if (rc != XDROP_OK) break;
      HIP_OK(hipEventRecord(e1, st));
      HIP_OK(hipEventSynchronize(e1));
      HIP_OK(hipEventElapsedTime(&t[r], e0, e1));
      if (r == 0 && t[0] > 3.0f * best_ms) { reps = 1; break; }
    }
    if (rc != XDROP_OK) break;
    std::sort(t, t + reps);
    const float ms = t[reps / 2];
    if (o.variant == XDROP_VARIANT_PLAIN && o.tile == 1) plain_ms = ms;
    if (ms < best_ms) { best_ms = ms; best = o; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != XDROP_OK) return rc;
  set_tuned(c, key, best);
  if (best_out) *best_out = best;
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (!f) return XDROP_E_INVALID;
    std::fprintf(f,
                 "{\"arch\": \"%s\", \"alphabet\": %d, \"x_class\": %d, "
                 "\"size_class\": %d, \"variant\": %d, \"tile\": %d, "
                 "\"chunk\": %d, \"waves_per_cu\": %d, \"X\": %d, "
                 "\"n_seeds\": %d, \"mean_extension_length\": %.1f, "
                 "\"ms\": %.4f, \"plain_ms\": %.4f}\n",
                 c->arch.c_str(), key.alphabet, key.x_class, key.size_class,
                 best.variant, best.tile, best.chunk, best.waves_per_cu,
                 sc->X, n_seeds, mean_len, best_ms, plain_ms);
    std::fclose(f);
  }
  return XDROP_OK;
}

namespace {
bool json_int(const std::string& line, const char* key, int* out) {
  const std::string k = std::string("\"") + key + "\":";
  size_t p = line.find(k);
  if (p == std::string::npos) return false;
  return std::sscanf(line.c_str() + p + k.size(), " %d", out) == 1;
}
bool json_str(const std::string& line, const char* key, std::string* out) {
  const std::string k = std::string("\"") + key + "\": \"";
  size_t p = line.find(k);
  if (p == std::string::npos) return false;
  p += k.size();
  const size_t e = line.find('"', p);
  if (e == std::string::npos) return false;
  *out = line.substr(p, e - p);
  return true;
}
}  // namespace

extern "C" int xdrop_load_tuning(xdrop_ctx* c, const char* cache_path) {
  if (!c || !cache_path) return XDROP_E_INVALID;
  FILE* f = std::fopen(cache_path, "r");
  if (!f) return XDROP_E_INVALID;
  char buf[1024];
  int loaded = 0;
  while (std::fgets(buf, sizeof(buf), f)) {
    const std::string line(buf);
    // every key of an entry must be present; entries of another device
    // architecture are skipped
    std::string arch;
    TuneKey k{};
    xdrop_options o{};
    if (!json_str(line, "arch", &arch) || arch != c->arch ||
        !json_int(line, "alphabet", &k.alphabet) ||
        !json_int(line, "x_class", &k.x_class) ||
        !json_int(line, "size_class", &k.size_class) ||
        !json_int(line, "variant", &o.variant) ||
        !json_int(line, "tile", &o.tile) ||
        !json_int(line, "chunk", &o.chunk) ||
        !json_int(line, "waves_per_cu", &o.waves_per_cu))
      continue;
    if (k.alphabet < 0 || k.alphabet > 1 || k.x_class < 0 || k.x_class > 2 ||
        k.size_class < 0 || k.size_class > 3 || o.variant == 0 ||
        check_options(&o) != XDROP_OK)
      continue;
    set_tuned(c, k, o);  // a later line of the same key replaces an earlier
    ++loaded;
  }
  std::fclose(f);
  return loaded ? XDROP_OK : XDROP_E_INVALID;
}

extern "C" int xdrop_resolve_options(xdrop_ctx* c, const xdrop_scoring* sc,
                                     int32_t n_seeds,
                                     const xdrop_options* opts,
                                     xdrop_options* out) {
  if (!c || !sc || !out || n_seeds < 0) return XDROP_E_INVALID;
  Params tmp;
  int rc = fill_scoring(sc, tmp);
  if (rc != XDROP_OK) return rc;
  rc = check_options(opts);
  if (rc != XDROP_OK) return rc;
  xdrop_options o = resolve(c, sc, opts, n_seeds);
  if (o.variant == XDROP_VARIANT_DUAL16 && !dual_exact(tmp))
    o.variant = XDROP_VARIANT_WAVE;
  finalize(c, sc->alphabet == XDROP_BYTE ? 1 : 0, 2 * n_seeds, o);
  *out = o;
  return XDROP_OK;
}
