// Runtime of the CPU build of the library's HIP sources (test
// infrastructure; see hip/hip_runtime.h).
//
// Threads of a block are fibers on one OS thread, switched by a small
// register-saving routine.  A fiber runs until it reaches a cross-lane
// operation or a block barrier; the 64 lanes of a wave meet there, the last
// one to arrive evaluates the operation for the whole wave, and all continue.
// A lane that reaches a different cross-lane operation than the rest of its
// wave, or a block that can make no progress, aborts the process with a
// report (the GPU would hang or compute garbage there).  Blocks of a launch
// run on a pool of OS threads; launches run to completion before they
// return, except while their stream is captured into a graph.
#include <hip/hip_runtime.h>
#include <sys/mman.h>
#include <time.h>

#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

extern "C" void emu_swap(void** save_sp, void* new_sp);
asm(R"(
.text
.globl emu_swap
.type emu_swap,@function
emu_swap:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
.size emu_swap, .-emu_swap
)");

namespace emu {

[[noreturn]] static void die(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "emu: ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
  std::fflush(stderr);
  std::abort();
}

constexpr size_t STACK = 256 << 10;
constexpr int MAX_THREADS = 1024;

enum Kind { K_BALLOT = 1, K_DPP, K_READLANE, K_READFIRST, K_BPERM, K_SYNC };

struct Fiber {
  void* sp = nullptr;
  char* stack = nullptr;
  Idx tid{};
  int wave = 0, lane = 0;
  bool done = false;
  uint64_t ncoll = 0;  // cross-lane operations taken
};

struct Wave {
  int64_t in[64], in2[64], out[64];
  int arrived = 0;
  uint64_t gen = 0;
  int kind = 0;
  uint64_t seq = 0;
  int ctrl = 0, rm = 0, bm = 0;
  bool bc = false;
};

struct Block {
  Idx bidx{}, bdim{}, gdim{};
  int n = 0;
  Fiber fibers[MAX_THREADS];
  Wave waves[MAX_THREADS / 64];
  int bar_arrived = 0;
  uint64_t bar_gen = 0;
  void* sched_sp = nullptr;
  Fiber* cur = nullptr;
  bool progress = false;
  KernelThunk fn = nullptr;
  void* args = nullptr;
};

static thread_local Block* g_blk = nullptr;
static std::atomic<uint64_t> g_block_gen{0};
static thread_local uint64_t g_cur_gen = 0;  // this OS thread's block
static thread_local std::vector<std::pair<void*, uint64_t>> g_shared;

void shared_decl(void* p, size_t n) {
  for (auto& e : g_shared)
    if (e.first == p) {
      if (e.second == g_cur_gen) return;
      e.second = g_cur_gen;
      goto fill;
    }
  g_shared.emplace_back(p, g_cur_gen);
fill:
  // a different pattern per block: nothing may depend on it
  uint64_t x = g_cur_gen * 0x9E3779B97F4A7C15ull + 0x5A5A5A5A5A5A5A5Aull;
  unsigned char* q = (unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    x ^= x << 13; x ^= x >> 7; x ^= x << 17;
    q[i] = (unsigned char)x;
  }
}

Fiber* cur() { return g_blk->cur; }
const Idx& thread_idx() { return g_blk->cur->tid; }
const Idx& block_idx() { return g_blk->bidx; }
const Idx& block_dim() { return g_blk->bdim; }
const Idx& grid_dim() { return g_blk->gdim; }
int lane() { return g_blk->cur->lane; }

static void yield() {
  Block* b = g_blk;
  emu_swap(&b->cur->sp, b->sched_sp);
}

static void fiber_main() {
  Block* b = g_blk;
  b->fn(b->args);
  b->cur->done = true;
  b->progress = true;
  yield();
  die("finished fiber resumed");
}

static void init_fiber(Fiber& f) {
  if (!f.stack) {
    void* p = mmap(nullptr, STACK, PROT_READ | PROT_WRITE,
                   MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (p == MAP_FAILED) die("stack mmap failed");
    f.stack = (char*)p;
  }
  uintptr_t top = ((uintptr_t)(f.stack + STACK)) & ~(uintptr_t)15;
  uintptr_t* sp = (uintptr_t*)(top - 16);
  sp[0] = (uintptr_t)&fiber_main;  // return address of the first switch
  for (int i = 1; i <= 6; ++i) sp[-i] = 0;  // rbp rbx r12-r15
  f.sp = (void*)(sp - 6);
  f.done = false;
  f.ncoll = 0;
}

static void run_block(Block& b) {
  g_blk = &b;
  g_cur_gen = ++g_block_gen;
  for (int i = 0; i < b.n; ++i) {
    Fiber& f = b.fibers[i];
    f.tid = Idx{(unsigned)(i % b.bdim.x), (unsigned)(i / b.bdim.x % b.bdim.y),
                (unsigned)(i / (b.bdim.x * b.bdim.y))};
    f.wave = i / 64;
    f.lane = i % 64;
    init_fiber(f);
  }
  for (int w = 0; w < (b.n + 63) / 64; ++w) {
    b.waves[w].arrived = 0;
    b.waves[w].gen = 0;
  }
  b.bar_arrived = 0;
  int live = b.n;
  while (live > 0) {
    bool any = false;
    for (int i = 0; i < b.n; ++i) {
      Fiber& f = b.fibers[i];
      if (f.done) continue;
      b.cur = &f;
      b.progress = false;
      emu_swap(&b.sched_sp, f.sp);
      if (b.progress) any = true;
      if (f.done) --live;
    }
    if (!any) {
      for (int w = 0; w < (b.n + 63) / 64; ++w) {
        int done = 0;
        for (int l = 0; l < 64 && w * 64 + l < b.n; ++l)
          done += b.fibers[w * 64 + l].done;
        std::fprintf(stderr,
                     "emu: block (%u) wave %d: %d lanes finished, %d at a "
                     "cross-lane operation (kind %d), barrier %d/%d\n",
                     b.bidx.x, w, done, b.waves[w].arrived, b.waves[w].kind,
                     b.bar_arrived, b.n);
      }
      die("no progress: lanes of a wave diverged at a cross-lane operation "
          "or a barrier");
    }
  }
  g_blk = nullptr;
}

// The calling lane's part of a cross-lane operation; the last lane of the
// wave to arrive evaluates it.
template <class F>
static int64_t collective(int kind, int64_t v, int64_t v2, F&& eval) {
  Block* b = g_blk;
  Fiber* f = b->cur;
  if ((b->n & 63) != 0) die("block size %d is not a multiple of 64", b->n);
  Wave& w = b->waves[f->wave];
  if (w.arrived == 0) {
    w.kind = kind;
    w.seq = f->ncoll;
  } else if (w.kind != kind || w.seq != f->ncoll) {
    die("divergent cross-lane operation: block %u wave %d lane %d takes "
        "kind %d (#%llu) while the wave is at kind %d (#%llu)",
        b->bidx.x, f->wave, f->lane, kind, (unsigned long long)f->ncoll,
        w.kind, (unsigned long long)w.seq);
  }
  ++f->ncoll;
  w.in[f->lane] = v;
  w.in2[f->lane] = v2;
  b->progress = true;
  const uint64_t g = w.gen;
  if (++w.arrived == 64) {
    eval(w);
    w.arrived = 0;
    ++w.gen;
  } else {
    while (w.gen == g) yield();
    b->progress = true;
  }
  return w.out[f->lane];
}

uint64_t ballot(bool p) {
  return (uint64_t)collective(K_BALLOT, p ? 1 : 0, 0, [](Wave& w) {
    uint64_t m = 0;
    for (int l = 0; l < 64; ++l)
      if (w.in[l]) m |= 1ull << l;
    for (int l = 0; l < 64; ++l) w.out[l] = (int64_t)m;
  });
}

// Source lane of a DPP move for lane l, -1 if none.
static int dpp_src(int ctrl, int l) {
  const int r = l & ~15, p = l & 15;
  if (ctrl <= 0xFF) return (l & ~3) | ((ctrl >> (2 * (l & 3))) & 3);
  if (ctrl >= 0x101 && ctrl <= 0x10F) {
    const int n = ctrl - 0x100;
    return p + n < 16 ? l + n : -1;
  }
  if (ctrl >= 0x111 && ctrl <= 0x11F) {
    const int n = ctrl - 0x110;
    return p - n >= 0 ? l - n : -1;
  }
  if (ctrl >= 0x121 && ctrl <= 0x12F) {
    const int n = ctrl - 0x120;
    return r + ((p - n + 16) & 15);
  }
  switch (ctrl) {
    case 0x130: return l + 1 < 64 ? l + 1 : -1;   // wave_shl:1
    case 0x134: return (l + 1) & 63;              // wave_rol:1
    case 0x138: return l >= 1 ? l - 1 : -1;       // wave_shr:1
    case 0x13C: return (l + 63) & 63;             // wave_ror:1
    case 0x140: return r + 15 - p;                // row_mirror
    case 0x141: return (l & ~7) + 7 - (l & 7);    // row_half_mirror
    case 0x142: return r >= 16 ? r - 1 : -1;      // row_bcast:15
    case 0x143: return r >= 32 ? 31 : -1;         // row_bcast:31
  }
  die("DPP control 0x%x not modelled", ctrl);
}

int dpp(int old, int src, int ctrl, int rm, int bm, bool bc, bool) {
  Block* b = g_blk;
  Wave& w0 = b->waves[b->cur->wave];
  (void)w0;
  return (int)collective(K_DPP, src, old, [=](Wave& w) {
    for (int l = 0; l < 64; ++l) {
      const int row = l >> 4, bank = (l >> 2) & 3;
      if (!((rm >> row) & 1) || !((bm >> bank) & 1)) {
        w.out[l] = w.in2[l];
        continue;
      }
      const int s = dpp_src(ctrl, l);
      w.out[l] = s < 0 ? (bc ? 0 : w.in2[l]) : w.in[s];
    }
  });
}

int readlane(int v, int l) {
  return (int)collective(K_READLANE, v, l, [](Wave& w) {
    for (int i = 1; i < 64; ++i)
      if (w.in2[i] != w.in2[0]) die("readlane with a lane index that differs across the wave");
    const int64_t x = w.in[w.in2[0] & 63];
    for (int i = 0; i < 64; ++i) w.out[i] = x;
  });
}

int readfirstlane(int v) {
  return (int)collective(K_READFIRST, v, 0, [](Wave& w) {
    for (int i = 0; i < 64; ++i) w.out[i] = w.in[0];
  });
}

int bpermute(int addr, int v) {
  return (int)collective(K_BPERM, v, addr, [](Wave& w) {
    for (int i = 0; i < 64; ++i) w.out[i] = w.in[(w.in2[i] >> 2) & 63];
  });
}

void wave_sync() {
  collective(K_SYNC, 0, 0, [](Wave& w) {
    for (int i = 0; i < 64; ++i) w.out[i] = 0;
  });
}

void syncthreads() {
  Block* b = g_blk;
  b->progress = true;
  const uint64_t g = b->bar_gen;
  if (++b->bar_arrived == b->n) {
    b->bar_arrived = 0;
    ++b->bar_gen;
  } else {
    while (b->bar_gen == g) yield();
    b->progress = true;
  }
}

// ------------------------------------------------------------ launches
static int pool_threads() {
  static int n = [] {
    const char* e = std::getenv("XDROP_EMU_THREADS");
    int v = e ? std::atoi(e) : (int)std::thread::hardware_concurrency();
    return v < 1 ? 1 : v;
  }();
  return n;
}

static thread_local Block* t_block = nullptr;

void launch(KernelThunk fn, void* args, dim3 grid, dim3 block) {
  const int nthr = (int)(block.x * block.y * block.z);
  if (nthr <= 0 || nthr > MAX_THREADS) die("block of %d threads", nthr);
  const long nblk = (long)grid.x * grid.y * grid.z;
  if (nblk <= 0) return;
  std::atomic<long> next{0};
  auto worker = [&]() {
    if (!t_block) t_block = new Block();
    Block& b = *t_block;
    for (;;) {
      const long i = next.fetch_add(1);
      if (i >= nblk) break;
      b.bidx = Idx{(unsigned)(i % grid.x), (unsigned)(i / grid.x % grid.y),
                   (unsigned)(i / ((long)grid.x * grid.y))};
      b.bdim = Idx{block.x, block.y, block.z};
      b.gdim = Idx{grid.x, grid.y, grid.z};
      b.n = nthr;
      b.fn = fn;
      b.args = args;
      run_block(b);
    }
  };
  const int nt = (int)std::min<long>(pool_threads(), nblk);
  if (nt <= 1) {
    worker();
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(worker);
  for (auto& t : th) t.join();
}

}  // namespace emu

// ------------------------------------------------------------ runtime API
struct emu_event {
  std::chrono::steady_clock::time_point t;
  bool recorded = false;
};
struct Op {
  void (*run)(void*);
  void* ctx;
  void (*drop)(void*);
};
struct emu_stream {
  bool capturing = false;
  std::vector<Op> ops;
};
struct emu_graph {
  std::vector<Op> ops;
};

namespace emu {
void submit(hipStream_t s, void (*run)(void*), void* ctx,
            void (*drop)(void*)) {
  if (s && s->capturing) {
    s->ops.push_back(Op{run, ctx, drop});
    return;
  }
  run(ctx);
  drop(ctx);
}
}  // namespace emu

static std::mutex g_alloc_mu;
static int g_device = 0;

hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDevice(int* d) { *d = g_device; return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d) {
  if (d != 0) return hipErrorInvalidDevice;
  std::memset(p, 0, sizeof(*p));
  const char* e = std::getenv("XDROP_EMU_CUS");
  p->multiProcessorCount = e ? std::atoi(e) : 4;
  std::strcpy(p->gcnArchName, "gfx950-emu");
  p->totalGlobalMem = (size_t)1 << 34;
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
  std::lock_guard<std::mutex> g(g_alloc_mu);
  void* q = std::aligned_alloc(256, (n + 255) & ~(size_t)255);
  if (!q) return hipErrorOutOfMemory;
  std::memset(q, 0xA5, n);  // device memory starts with garbage
  *p = q;
  return hipSuccess;
}
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k,
                          hipStream_t) {
  return hipMemcpy(d, s, n, k);
}
hipError_t hipMemset(void* d, int v, size_t n) { std::memset(d, v, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { return hipMemset(d, v, n); }
hipError_t hipStreamCreate(hipStream_t* s) { *s = new emu_stream(); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { return hipStreamCreate(s); }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new emu_event(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
static void rec_event(void* p) {
  auto* e = (emu_event*)p;
  e->t = std::chrono::steady_clock::now();
  e->recorded = true;
}
static void no_drop(void*) {}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  emu::submit(s, &rec_event, e, &no_drop);
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s || s->capturing) return hipErrorInvalidValue;
  s->capturing = true;
  s->ops.clear();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  if (!s || !s->capturing) return hipErrorInvalidValue;
  s->capturing = false;
  *g = new emu_graph{std::move(s->ops)};
  s->ops.clear();
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*,
                               size_t) {
  *e = g;  // the executable shares the recorded launches
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto& op : e->ops) op.run(op.ctx);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  for (auto& op : g->ops) op.drop(op.ctx);
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "emu error"; }

// v_writelane_b32 of the library's kernels: lane `lane` takes `val`.
extern "C" int xd_writelane_i32(int val, int lane, int old) {
  return emu::lane() == lane ? val : old;
}

// Per-extension trace of the wave kernel: (end state, tier) of each item of
// the last batches, read with emu_trace_read.
static std::vector<int32_t> g_trace;
static std::mutex g_trace_mu;
void emu_item_done(int item, int r, int tier) {
  if (emu::lane() != 0) return;
  std::lock_guard<std::mutex> g(g_trace_mu);
  if ((size_t)item >= g_trace.size()) g_trace.resize(item + 1, -1);
  g_trace[item] = r * 100 + tier;
}
extern "C" int emu_trace_read(int32_t* out, int n) {
  std::lock_guard<std::mutex> g(g_trace_mu);
  int k = 0;
  for (; k < n && (size_t)k < g_trace.size(); ++k) out[k] = g_trace[k];
  g_trace.clear();
  return k;
}
