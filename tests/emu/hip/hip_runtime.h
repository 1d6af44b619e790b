// CPU build of the library's HIP sources (test infrastructure only).
//
// This header stands in for <hip/hip_runtime.h> when tests/emu/build.py
// compiles the kernel and host sources of the library with the host compiler.
// Every GPU thread becomes a fiber; the 64 lanes of a wavefront meet at every
// cross-lane operation (DPP moves, ballots, lane reads, ds_bpermute), which
// the runtime (emu_runtime.cpp) evaluates over the whole wave once all 64
// lanes have arrived, so each lane sees what the hardware would give it.
// A lane that skips a cross-lane operation the others take (divergence)
// stops the run with a report instead of hanging.  Device memory is host
// memory; launches run to completion before they return.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <tuple>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static thread_local
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(s) (&(s))

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint2 {
  uint32_t x, y;
};
struct alignas(16) uint4 {
  uint32_t x, y, z, w;
};
struct int4 {
  int x, y, z, w;
};
inline int4 make_int4(int x, int y, int z, int w) { return int4{x, y, z, w}; }

namespace emu {
struct Idx {
  unsigned x, y, z;
};
struct Fiber;
Fiber* cur();
const Idx& thread_idx();
const Idx& block_idx();
const Idx& block_dim();
const Idx& grid_dim();
int lane();
// cross-lane operations (evaluated over the whole wave)
uint64_t ballot(bool p);
int dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bc,
        bool old_defined);
int readlane(int v, int l);
int readfirstlane(int v);
int bpermute(int addr, int v);
// the lanes of a wave execute in lockstep: LDS written before this point by
// any lane is visible to every lane after it
void wave_sync();
void syncthreads();
using KernelThunk = void (*)(void*);
void launch(KernelThunk fn, void* args, dim3 grid, dim3 block);
// a block's shared variable, filled with garbage when the block's first
// thread reaches its declaration (as on the GPU, where LDS starts with
// whatever the previous workgroup left)
void shared_decl(void* p, size_t n);
}  // namespace emu

// trace hook (tests/emu/build.py inserts the calls)
void emu_item_done(int item, int r, int tier);

#define threadIdx (emu::thread_idx())
#define blockIdx (emu::block_idx())
#define blockDim (emu::block_dim())
#define gridDim (emu::grid_dim())

inline uint64_t __ballot(int p) { return emu::ballot(p != 0); }
inline void __syncthreads() { emu::syncthreads(); }

#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) \
  emu::dpp((old), (src), (ctrl), (rm), (bm), (bc), true)
#define __builtin_amdgcn_mov_dpp(src, ctrl, rm, bm, bc) \
  emu::dpp(0x5eadbeef, (src), (ctrl), (rm), (bm), (bc), false)
#define __builtin_amdgcn_readlane(v, l) emu::readlane((v), (l))
#define __builtin_amdgcn_readfirstlane(v) emu::readfirstlane((v))
#define __builtin_amdgcn_ds_bpermute(a, v) emu::bpermute((a), (v))
#define __builtin_amdgcn_wave_barrier() emu::wave_sync()
#define __builtin_amdgcn_inverse_ballot_w64(m) \
  ((((uint64_t)(m)) >> emu::lane()) & 1u)

inline uint32_t emu_alignbit(uint32_t hi, uint32_t lo, uint32_t sh) {
  const uint64_t v = ((uint64_t)hi << 32) | lo;
  return (uint32_t)(v >> (sh & 31));
}
inline uint32_t emu_ubfe(uint32_t v, uint32_t off, uint32_t w) {
  off &= 31;
  w &= 31;
  if (w == 0) return 0;
  if (off + w < 32) return (v << (32 - off - w)) >> (32 - w);
  return v >> off;
}
inline int emu_sbfe(int v, uint32_t off, uint32_t w) {
  off &= 31;
  w &= 31;
  if (w == 0) return 0;
  if (off + w < 32) return (int)((uint32_t)v << (32 - off - w)) >> (32 - w);
  return v >> off;
}
// v_perm_b32: byte i of the result chosen by byte i of sel from the eight
// bytes of {s0, s1} (s1 the low four); 12 gives 0x00, 13 and above 0xff,
// 8..11 the sign of a 16-bit half (not used by the library)
inline uint32_t emu_perm(uint32_t s0, uint32_t s1, uint32_t sel) {
  const uint64_t v = ((uint64_t)s0 << 32) | s1;
  uint32_t r = 0;
  for (int i = 0; i < 4; ++i) {
    const uint32_t b = (sel >> (8 * i)) & 0xFF;
    uint32_t o;
    if (b < 8) o = (uint32_t)(v >> (8 * b)) & 0xFF;
    else if (b == 12) o = 0;
    else if (b >= 13) o = 0xFF;
    else std::abort();
    r |= o << (8 * i);
  }
  return r;
}
// v_ffbl_b32 / v_ffbh_u32: lowest / highest set bit (counted from the
// top for ffbh), 0xffffffff for 0
inline uint32_t emu_ffbl_32(uint32_t x) { return x ? (uint32_t)__builtin_ctz(x) : 0xffffffffu; }
inline uint32_t emu_ffbh_32(uint32_t x) { return x ? (uint32_t)__builtin_clz(x) : 0xffffffffu; }
#define __builtin_amdgcn_alignbit(hi, lo, sh) emu_alignbit((hi), (lo), (sh))
#define __builtin_amdgcn_perm(s0, s1, sel) emu_perm((s0), (s1), (sel))
#define __builtin_amdgcn_ubfe(v, o, w) emu_ubfe((v), (o), (w))
#define __builtin_amdgcn_sbfe(v, o, w) emu_sbfe((v), (o), (w))

template <class A, class B>
inline std::common_type_t<A, B> min(A a, B b) {
  using T = std::common_type_t<A, B>;
  return (T)a < (T)b ? (T)a : (T)b;
}
template <class A, class B>
inline std::common_type_t<A, B> max(A a, B b) {
  using T = std::common_type_t<A, B>;
  return (T)a > (T)b ? (T)a : (T)b;
}

template <class T>
inline T atomicAdd(T* p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
template <class T>
inline T atomicExch(T* p, T v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }
template <class T>
inline T atomicMax(T* p, T v) {
  T o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (o < v && !__atomic_compare_exchange_n(p, &o, v, false,
                                               __ATOMIC_SEQ_CST,
                                               __ATOMIC_SEQ_CST)) {
  }
  return o;
}
template <class T>
inline T atomicMin(T* p, T v) {
  T o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (o > v && !__atomic_compare_exchange_n(p, &o, v, false,
                                               __ATOMIC_SEQ_CST,
                                               __ATOMIC_SEQ_CST)) {
  }
  return o;
}
#define __HIP_MEMORY_SCOPE_WAVEFRONT 1
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __HIP_MEMORY_SCOPE_SYSTEM 4
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), (order))
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), (order))
#define __hip_atomic_fetch_add(p, v, order, scope) \
  __atomic_fetch_add((p), (v), (order))
inline void __threadfence() { __atomic_thread_fence(__ATOMIC_SEQ_CST); }

// ------------------------------------------------------------ runtime API
typedef int hipError_t;
enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorMemoryAllocation = 2,
  hipErrorInvalidDevice = 101,
  hipErrorNotReady = 600,
  hipErrorUnknown = 999
};
typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
typedef struct emu_graph* hipGraph_t;
typedef struct emu_graph* hipGraphExec_t;
typedef struct emu_graph_node* hipGraphNode_t;
enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
};
enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
};
#define hipStreamNonBlocking 1
#define hipEventDisableTiming 2
#define hipHostMallocDefault 0
struct hipDeviceProp_t {
  int multiProcessorCount;
  char gcnArchName[256];
  size_t totalGlobalMem;
};

hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int* d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
hipError_t hipMalloc(void** p, size_t n);
template <class T>
inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags = 0);
template <class T>
inline hipError_t hipHostMalloc(T** p, size_t n, unsigned flags = 0) {
  return hipHostMalloc((void**)p, n, flags);
}
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k,
                          hipStream_t st = nullptr);
hipError_t hipMemset(void* d, int v, size_t n);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st = nullptr);
hipError_t hipStreamCreate(hipStream_t* s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags = 0);
hipError_t hipDeviceSynchronize();
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetLastError();
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*,
                               size_t);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGetSymbolAddress(void** p, const void* sym);
template <class T>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, T,
                                                               int, size_t) {
  *n = 2;
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t e);

namespace emu {
// A launch either runs now or, while its stream is being captured, is
// recorded for hipGraphLaunch.
void submit(hipStream_t s, void (*run)(void*), void* ctx, void (*drop)(void*));
template <class... A>
struct LaunchBox {
  void (*kern)(A...);
  std::tuple<A...> args;
  dim3 grid, block;
};
template <class... A>
void run_box(void* p) {
  auto* b = (LaunchBox<A...>*)p;
  struct Thunk {
    static void call(void* q) {
      auto* bb = (LaunchBox<A...>*)q;
      std::apply(bb->kern, bb->args);
    }
  };
  launch(&Thunk::call, b, b->grid, b->block);
}
template <class... A>
void drop_box(void* p) { delete (LaunchBox<A...>*)p; }
template <class... A, class... B>
void launch_kernel(void (*k)(A...), dim3 g, dim3 b, hipStream_t s, B&&... args) {
  auto* box = new LaunchBox<A...>{k, std::tuple<A...>((A)args...), g, b};
  submit(s, &run_box<A...>, box, &drop_box<A...>);
}
}  // namespace emu
#define hipLaunchKernelGGL(kern, grid, block, shmem, stream, ...) \
  emu::launch_kernel((kern), dim3(grid), dim3(block), (hipStream_t)(stream), ##__VA_ARGS__)
