// X-Drop seed extension kernels for gfx950 (CDNA4, wave64).
//
// One extension E(a, b) is the antidiagonal sweep of the paper's Sec. 3 /
// Algorithm 1: cells (x, y) with d = x + y are filled antidiagonal by
// antidiagonal from the two previous ones (three rolling antidiagonals);
// a cell below T - X (T = best score of all earlier antidiagonals, strict '<')
// is set to -infinity (Sec. 2.2 X-Drop rule); the band [lo_d, hi_d] is the
// span reachable from the finite cells of antidiagonals d-1 and d-2, and the
// sweep stops once both hold no finite cell.
//
// MI355X mapping (what differs from the paper's IPU codelet):
//  * one wavefront per extension; the band window of 64*C cells lives in
//    VGPRs, lane l holding window positions l*C .. l*C+C-1 (blocked), so the
//    x-1 neighbour is the previous register of the same lane except for j = 0,
//    which comes from lane l-1 by one DPP wave_shr:1 per antidiagonal;
//  * values are kept in the frame V = S - gap*d, which removes both gap adds:
//      V_d[x] = max(V_{d-1}[x-1], V_{d-1}[x], V_{d-2}[x-1] + sim - 2*gap);
//  * pruning, the running best T (wave max reduction only on antidiagonals
//    where some lane beats T, detected with a ballot) and the finite range
//    (L, U) come from per-register ballots;
//  * the window slides up by whole lanes when the band reaches its top, by as
//    many as the dead lanes below the band allow; when the band is wider than
//    the window the tile widens in place (C -> 2C, registers redistributed
//    with ds_bpermute) up to C = 8 (512 cells); wider bands go to a
//    workgroup tier that spreads the window over the registers of four
//    wavefronts (up to 2,048 cells), and beyond that to a tier with rings in
//    device memory;
//  * for C = 1 and 2, blocks of antidiagonals run in unrolled interior loops
//    on the finite-lane masks, with the live-span count formed per block on
//    the vector unit (fast_interior, fast_interior_multi);
//  * sequences stream through per-wave LDS rings (2-bit DNA or byte codes),
//    read backwards for left extensions (the paper's op() transform);
//  * extensions are pulled from a device queue by persistent waves, or for a
//    batch that starts at once, one launched wave per extension.
// All arithmetic is int32 integer VALU/SALU; no MFMA.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "xdrop_internal.h"

#ifndef XD_KB1
#define XD_KB1 48  // antidiagonals per block of the one-cell loop (DNA)
#endif
#ifndef XD_KB1B
#define XD_KB1B 60  // ... for byte codes (48: 0.4% slower on protein-500k)
#endif
#ifndef XD_KB2
#define XD_KB2 48  // antidiagonals per block of the two-cell loop (DNA)
#endif
#ifndef XD_KB2B
#define XD_KB2B 56  // ... for byte codes (48 and 60: 0.15% slower on protein-500k)
#endif
#ifndef XD_G2
#define XD_G2 2  // guard lanes of the two-cell loop
#endif
#ifndef XD_PRE
#define XD_PRE 24  // byte codes: slide early with fewer free lanes than G + this
#endif
#ifndef XD_MINSL
#define XD_MINSL 1  // ... by at least this many lanes (4 and 2: 0.3% slower)
#endif
namespace xd {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// The LDS copy of the byte-code score table has rows of TAB_LD words (33):
// with rows of 32, the bank of entry (q, c) would be fixed by the target code
// c alone, so lanes reading different rows at one code would meet in a bank;
// the odd stride spreads (q, c) over the banks.
constexpr int TAB_LD = TABLE_DIM + 1;
constexpr int TAB_WORDS = TABLE_DIM * TAB_LD;
__device__ __forceinline__ void fill_tab(int* tab, const Params& P) {
  for (int i = threadIdx.x; i < TAB_WORDS; i += blockDim.x) {
    const int q = i / TAB_LD, c = i - q * TAB_LD;
    tab[i] = c < TABLE_DIM ? P.table[q * TABLE_DIM + c] : 0;
  }
}

// Hide a value's origin from the optimiser (no instruction is emitted), so
// that it cannot turn the operations that follow into longer forms: a
// scalar (s) or vector (v) register.
__device__ __forceinline__ void opaque_s(uint32_t& v) { asm("" : "+s"(v)); }
__device__ __forceinline__ void opaque_v(int& v) { asm("" : "+v"(v)); }
// The same as a volatile statement: the instructions that form v stay ahead
// of the branches that follow (the compiler may not sink them past one).
__device__ __forceinline__ void pin_v(int& v) { asm volatile("" : "+v"(v)); }

// Lane l receives lane l-1's value; lane 0 receives `fill`.
__device__ __forceinline__ int wave_shr1(int v, int fill) {
  return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xf, 0xf, false);
}
// Lane l receives lane l-1's value; lane 0 receives 0 (bound control: no
// register holding the fill value to set first).
__device__ __forceinline__ int wave_shr1_z(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true);
}
// The lowest / highest set bit of each lane's word, 0xffffffff for a zero
// word (v_ffbl_b32, v_ffbh_u32).  Written out: the compiler's bit scans with
// a fallback for zero add a compare and a select to each, eight vector
// instructions per block of the sweeps.
__device__ __forceinline__ uint32_t ffbl32(uint32_t x) {
  uint32_t r;
  asm("v_ffbl_b32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}
__device__ __forceinline__ uint32_t ffbh32(uint32_t x) {
  uint32_t r;
  asm("v_ffbh_u32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}
// Lane l receives lane l+1's value; lane 63 receives `fill`.
__device__ __forceinline__ int wave_shl1(int v, int fill) {
  return __builtin_amdgcn_update_dpp(fill, v, 0x130, 0xf, 0xf, false);
}

// Maximum over the wave, returned as a uniform value.  (Each permutation
// gives every lane a source, so bound_ctrl changes nothing; it lets the
// compiler fold each move into its max.)
__device__ __forceinline__ int wave_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, true));
  int r0 = __builtin_amdgcn_readlane(v, 0);
  int r1 = __builtin_amdgcn_readlane(v, 16);
  int r2 = __builtin_amdgcn_readlane(v, 32);
  int r3 = __builtin_amdgcn_readlane(v, 48);
  // (the row maxima are combined on the scalar unit, not moved back into
  // vector registers for a three-input max)
  uint32_t a = (uint32_t)max(r0, r1), b = (uint32_t)max(r2, r3);
  opaque_s(a);
  opaque_s(b);
  return max((int)a, (int)b);
}

// v_writelane_b32: lane `lane` of `old` takes the uniform value `val`.  This
// compiler has no source-level builtin for it; the declaration binds the
// function to the target intrinsic's own name.
extern "C" __device__ int xd_writelane_i32(int val, int lane, int old) __asm(
    "llvm.amdgcn.writelane.i32");

// Sums of the lanes of each row of 16, in every lane of the row.
__device__ __forceinline__ int row_sums(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);
  return v;
}

// Sum of lanes 0..31 (a uniform value).
__device__ __forceinline__ int sum_lanes_0_31(int v) {
  v = row_sums(v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16);
}

// Sum of all 64 lanes (a uniform value).
__device__ __forceinline__ int sum_lanes(int v) {
  v = row_sums(v);
  return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
         (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

__device__ __forceinline__ uint64_t ballot(bool p) {
  return __ballot(p);
}

__device__ __forceinline__ int uni(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// Minimum / maximum of wave-uniform values.  The readfirstlane keeps the
// compiler from fusing nested uniform min/max into VALU min3/max3, whose
// results would pull the whole scalar state of the sweep into VGPRs.
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = (uint32_t)uni((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)uni((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int smin(int a, int b) { return uni(min(a, b)); }
__device__ __forceinline__ int smax(int a, int b) { return uni(max(a, b)); }

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo,
                                           uint32_t sh) {
  return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// Reverse the sixteen 2-bit fields of a word.
__device__ __forceinline__ uint32_t rev2(uint32_t v) {
  uint32_t r = __builtin_bitreverse32(v);
  return ((r >> 1) & 0x55555555u) | ((r & 0x55555555u) << 1);
}

// Packed sequence stream; word reads are clamped to the stream, so reads
// past either end of a sequence return other symbols (never used by a finite
// cell) instead of leaving the buffer.
struct Src {
  const uint32_t* w;
  int64_t tw;  // readable words
};

__device__ __forceinline__ Src make_src(const Params& P) {
  const int64_t syms = P.offsets[P.n_seqs];
  Src s;
  s.w = P.seqs;
  s.tw = P.alphabet == 0 ? (syms + 15) >> 4 : (syms + 3) >> 2;
  if (s.tw < 1) s.tw = 1;
  return s;
}

__device__ __forceinline__ uint32_t load_word(const Src& S, int64_t w) {
  w = w < 0 ? 0 : (w >= S.tw ? S.tw - 1 : w);
  return S.w[w];
}

// ------------------------------------------------------------------ rings
// A ring holds elements [loaded - RS, loaded) of one extension sequence
// (element e = source symbol start + dir * e), element e at position
// e mod RS.  Extra words past the end mirror the first words so that reads
// of a few consecutive words never wrap.
// RS elements, filled by NT threads (thread l writes the l-th piece of a
// fill).
template <int ALPHA, int RS_, int NT>
struct RingT;

template <int RS_, int NT>
struct RingT<0, RS_, NT> {  // 2-bit DNA
  static constexpr int RS = RS_;           // elements
  static constexpr int RW = RS / 16;       // words
  static constexpr int MIRROR = 1;
  static constexpr int WORDS = RW + MIRROR;
  static constexpr int CH = 16 * NT;       // elements per fill (16 per thread)

  __device__ static void fill(uint32_t* ring, const Src& S, int64_t start,
                              int dir, int c0, int l) {
    int64_t e0 = (int64_t)c0 + 16 * l;
    uint32_t v;
    if (dir > 0) {
      int64_t p = start + e0;
      int64_t w = p >> 4;
      uint32_t sh = (uint32_t)(p & 15) * 2;
      v = funnel(load_word(S, w + 1), load_word(S, w), sh);
    } else {
      int64_t p = start - e0 - 15;
      int64_t w = p >> 4;
      uint32_t sh = (uint32_t)(p & 15) * 2;
      v = rev2(funnel(load_word(S, w + 1), load_word(S, w), sh));
    }
    int wi = ((c0 >> 4) + l) & (RW - 1);
    ring[wi] = v;
    if (wi < MIRROR) ring[RW + wi] = v;
  }
  // 2*C bits: element e0 + k at bits 2k (k < C <= 16).
  __device__ static uint32_t read(const uint32_t* ring, int e0) {
    int pos = e0 & (RS - 1);
    int w = pos >> 4;
    uint32_t sh = (uint32_t)(pos & 15) * 2;
    return funnel(ring[w + 1], ring[w], sh);
  }
};

template <int RS_, int NT>
struct RingT<1, RS_, NT> {  // one byte per code
  static constexpr int RS = RS_;
  static constexpr int RW = RS / 4;
  // reads of up to 8 words, and the per-lane code reads of the one- and
  // two-cell loops up to a block's length + 2 bytes past a position
  static constexpr int KMAX = XD_KB1B > XD_KB2B ? XD_KB1B : XD_KB2B;
  static constexpr int MIRROR = (KMAX + 6) / 4 > 9 ? (KMAX + 6) / 4 : 9;
  static constexpr int WORDS = RW + MIRROR;
  static constexpr int CH = 8 * NT;        // elements per fill (8 per thread)

  __device__ static void fill(uint32_t* ring, const Src& S, int64_t start,
                              int dir, int c0, int l) {
    int64_t e0 = (int64_t)c0 + 8 * l;
    uint32_t v0, v1;
    if (dir > 0) {
      int64_t p = start + e0;
      int64_t w = p >> 2;
      uint32_t sh = (uint32_t)(p & 3) * 8;
      uint32_t w0 = load_word(S, w), w1 = load_word(S, w + 1),
               w2 = load_word(S, w + 2);
      v0 = funnel(w1, w0, sh);
      v1 = funnel(w2, w1, sh);
    } else {
      int64_t p = start - e0 - 7;
      int64_t w = p >> 2;
      uint32_t sh = (uint32_t)(p & 3) * 8;
      uint32_t w0 = load_word(S, w), w1 = load_word(S, w + 1),
               w2 = load_word(S, w + 2);
      uint32_t lo = funnel(w1, w0, sh), hi = funnel(w2, w1, sh);
      v0 = __builtin_bswap32(hi);
      v1 = __builtin_bswap32(lo);
    }
    // (codes above 31 are invalid input, reported by the symbol check; kept
    // below 32 here so that every score-table index stays in its row)
    v0 &= 0x1F1F1F1Fu;
    v1 &= 0x1F1F1F1Fu;
    int wi = ((c0 >> 2) + 2 * l) & (RW - 1);
    ring[wi] = v0;
    ring[wi + 1] = v1;
    if (wi < MIRROR) ring[RW + wi] = v0;
    if (wi + 1 < MIRROR) ring[RW + wi + 1] = v1;
  }
  // NW words: element e0 + k at byte k (k < 4*NW).
  template <int NW>
  __device__ static void read(const uint32_t* ring, int e0, uint32_t (&out)[NW]) {
    int pos = e0 & (RS - 1);
    int w = pos >> 2;
    uint32_t sh = (uint32_t)(pos & 3) * 8;
    uint32_t prev = ring[w];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      uint32_t nx = ring[w + i + 1];
      out[i] = funnel(nx, prev, sh);
      prev = nx;
    }
  }
};

// The rings of one wavefront: 4,096 DNA codes or 2,048 byte codes.
template <int ALPHA>
using Ring = RingT<ALPHA, ALPHA == 0 ? 4096 : 2048, WAVE>;

// ------------------------------------------------------------------ state
// Scalar (wave-uniform) state of one extension.
struct Ext {
  int m, n;           // lengths of a and b
  int64_t a_start, b_start;
  int a_dir, b_dir;
  int d;              // next antidiagonal to compute
  int base;           // window position 0 is x = base
  int T, bx, by;      // best score (S frame) and its cell
  int L1, U1;         // finite range of d-1 (L1 > U1: no finite cell)
  int L2, U2;         // finite range of d-2
  int64_t W;          // live-span cells so far
  int loaded_a, loaded_b;  // ring fill levels (elements)
  // queue of the target codes that enter the window at lane 0, one per
  // antidiagonal: b[qi], b[qi+1], ... with the next code in the low bits
  uint64_t q;
  int qn;             // codes left in q
  int qi;             // element index of the next code
};

// Keep the scalar state in SGPRs: every field is the same in all lanes.
__device__ __forceinline__ void make_uniform(Ext& e) {
  e.d = uni(e.d);
  e.base = uni(e.base);
  e.T = uni(e.T);
  e.bx = uni(e.bx);
  e.by = uni(e.by);
  e.L1 = uni(e.L1);
  e.U1 = uni(e.U1);
  e.L2 = uni(e.L2);
  e.U2 = uni(e.U2);
  e.loaded_a = uni(e.loaded_a);
  e.loaded_b = uni(e.loaded_b);
  e.qn = uni(e.qn);
  e.qi = uni(e.qi);
}

enum { R_CONT = 0, R_DONE = 1, R_ESC = 2, R_CAP = 3 };

template <int ALPHA>
struct WaveLds {
  uint32_t ra[Ring<ALPHA>::WORDS];
  uint32_t rb[Ring<ALPHA>::WORDS];
};

template <int ALPHA>
__device__ __forceinline__ void cover_a(Ext& e, WaveLds<ALPHA>& w,
                                        const Src& P, int need_hi) {
  // make elements up to need_hi available (the ring keeps the RS below)
  while (e.loaded_a <= need_hi) {
    Ring<ALPHA>::fill(w.ra, P, e.a_start, e.a_dir, e.loaded_a, lane_id());
    e.loaded_a += Ring<ALPHA>::CH;
  }
  __builtin_amdgcn_wave_barrier();
}

template <int ALPHA>
__device__ __forceinline__ void cover_b(Ext& e, WaveLds<ALPHA>& w,
                                        const Src& P, int need_hi) {
  while (e.loaded_b <= need_hi) {
    Ring<ALPHA>::fill(w.rb, P, e.b_start, e.b_dir, e.loaded_b, lane_id());
    e.loaded_b += Ring<ALPHA>::CH;
  }
  __builtin_amdgcn_wave_barrier();
}

// Symbols of a lane's C cells.  Query codes (A) depend only on the window
// (base, C) and are read from the ring when it moves; target codes (B) move
// by one cell per antidiagonal: cell j takes cell j-1's code, cell 0 takes
// cell C-1 of the lane below, and lane 0 takes the next code of the queue.
// DNA: 2-bit codes, cell j at bits [30-2j, 32-2j) of one word.
// Bytes: cell j at byte 4*NB-1-j of NB words (cell 0 in the top byte);
// the query side keeps 32 * code per cell (row offset of the score table).
template <int ALPHA, int C>
struct Syms;

template <int C>
struct Syms<0, C> {
  static constexpr int QBITS = 2, QCODES = 16;
  uint32_t a, b;
  __device__ void load_a(const WaveLds<0>& w, int base) {
    a = rev2(Ring<0>::read(w.ra, base + lane_id() * C - 1));
  }
  __device__ void load_b(const WaveLds<0>& w, int d, int base) {
    const int yb = d - base - lane_id() * C - 1;
    b = Ring<0>::read(w.rb, yb - C + 1) << (32 - 2 * C);
  }
  // codes of the next antidiagonal; `in` = the code entering at lane 0
  __device__ void advance(uint32_t in) {
    const uint32_t below = (uint32_t)wave_shr1((int)b, (int)(in << (32 - 2 * C)));
    b = funnel(below >> (32 - 2 * C), b, 2);
  }
  __device__ int sim(int j, const Params& P, const int*) const {
    return (((a ^ b) >> (30 - 2 * j)) & 3u) ? P.mis_s : P.mat_s;
  }
  // 16 codes from element e0 (next code lowest)
  __device__ static uint64_t queue(const WaveLds<0>& w, int e0) {
    return (uint64_t)(uint32_t)uni((int)Ring<0>::read(w.rb, e0));
  }
};

template <int C>
struct Syms<1, C> {
  static constexpr int QBITS = 8, QCODES = 8;
  static constexpr int NB = (C + 3) / 4;
  int row[C];
  uint32_t b[NB];
  __device__ void load_a(const WaveLds<1>& w, int base) {
    uint32_t v[NB];
    Ring<1>::read<NB>(w.ra, base + lane_id() * C - 1, v);
#pragma unroll
    for (int j = 0; j < C; ++j)
      row[j] = (int)((v[j >> 2] >> (8 * (j & 3))) & 31u) * TAB_LD;
  }
  __device__ void load_b(const WaveLds<1>& w, int d, int base) {
    const int yb = d - base - lane_id() * C - 1;
    Ring<1>::read<NB>(w.rb, yb - C + 1, b);
    if constexpr (C < 4) b[0] <<= 8 * (4 - C);
  }
  __device__ void advance(uint32_t in) {
    if constexpr (NB == 1) {
      const uint32_t below =
          (uint32_t)wave_shr1((int)b[0], (int)(in << (8 * (4 - C))));
      b[0] = funnel(below >> (8 * (4 - C)), b[0], 8);
    } else {
      const uint32_t below = (uint32_t)wave_shr1((int)b[0], (int)in);
#pragma unroll
      for (int k = 0; k < NB - 1; ++k) b[k] = funnel(b[k + 1], b[k], 8);
      b[NB - 1] = funnel(below, b[NB - 1], 8);
    }
  }
  __device__ int sim(int j, const Params&, const int* tab) const {
    constexpr int NBY = 4 * NB;
    const int k = NBY - 1 - j;  // byte index of cell j
    const int code = (int)((b[k >> 2] >> (8 * (k & 3))) & 31u);
    return tab[row[j] + code];
  }
  // 8 codes from element e0 (next code lowest)
  __device__ static uint64_t queue(const WaveLds<1>& w, int e0) {
    uint32_t v[2];
    Ring<1>::read<2>(w.rb, e0, v);
    return ((uint64_t)(uint32_t)uni((int)v[1]) << 32) |
           (uint32_t)uni((int)v[0]);
  }
};

// Window contents after the window or the tile changed: query codes, target
// codes of antidiagonal e.d, and an empty code queue.
template <int ALPHA, int C>
__device__ __forceinline__ void reload_syms(Ext& e, Syms<ALPHA, C>& sy,
                                            WaveLds<ALPHA>& w, const Src& S) {
  cover_a<ALPHA>(e, w, S, e.base + 64 * C - 2);
  cover_b<ALPHA>(e, w, S, e.d - e.base - 1);
  sy.load_a(w, e.base);
  sy.load_b(w, e.d, e.base);
  e.qi = e.d - e.base;  // code entering lane 0 for antidiagonal e.d + 1
  e.qn = 0;
}

// ------------------------------------------------------------------ window
enum { MV_NONE = 0, MV_MOVED = 1, MV_ESC = 2 };

// Keeps the band of antidiagonal e.d inside the window, given the finite
// ranges [La, Ua] of e.d - 1 and [Lb, Ub] of e.d - 2 (A and B hold those
// antidiagonals).  If the band can reach past the top, the window slides up
// by as many whole lanes as the dead cells below the band allow (cells below
// min(La, Lb) are -infinity on both) and the symbols are reloaded; MV_ESC
// when not even one lane is free (the caller widens the tile).
template <int ALPHA, int C>
__device__ __forceinline__ int window_move(Ext& e, int (&A)[C], int (&B)[C],
                                           Syms<ALPHA, C>& sy,
                                           WaveLds<ALPHA>& w, const Src& S,
                                           int La, int Lb, int Ua, int Ub) {
  constexpr int LOG2C = C == 1 ? 0 : C == 2 ? 1 : C == 4 ? 2 : 3;
  const int hi_next = smin(smax(Ua, Ub) + 1, smin(e.m, e.d));
  if (hi_next <= e.base + 64 * C - 1) return MV_NONE;
  const int sl = (smin(La, Lb) - e.base) >> LOG2C;
  if (sl < 1) return MV_ESC;
  const int src = lane_id() + sl;
  const bool in = src < 64;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int pa = __builtin_amdgcn_ds_bpermute((src & 63) << 2, A[j]);
    const int pb = __builtin_amdgcn_ds_bpermute((src & 63) << 2, B[j]);
    A[j] = in ? pa : NEG;
    B[j] = in ? pb : NEG;
  }
  e.base += sl << LOG2C;
  reload_syms<ALPHA, C>(e, sy, w, S);
  return MV_MOVED;
}

// ------------------------------------------------------------------ step
// Computes antidiagonal e.d.  On entry A holds d-1 and B holds d-2; on exit
// A holds d and B holds d-1.  The body is straight-line code with three
// rarely taken uniform branches (a new best score, a window move, a refill
// of the target-code queue) and one exit value, so that the compiler keeps
// the sweep state in SGPRs.
template <int ALPHA, int C>
__device__ __forceinline__ int step(Ext& e, int (&A)[C], int (&B)[C],
                                    Syms<ALPHA, C>& sy, WaveLds<ALPHA>& w,
                                    const int* tab, const Params& P,
                                    const Src& S) {
  constexpr int LOG2C = C == 1 ? 0 : C == 2 ? 1 : C == 4 ? 2 : 3;
  const int lane = lane_id();
  const int d = e.d;

  // span of this antidiagonal (live-span count, band cap); an empty range
  // (DEAD_L, DEAD_U) drops out of the min / max
  const int lo = smax(smin(e.L1, e.L2 + 1), smax(0, d - e.n));
  const int hi = smin(smax(e.U1, e.U2) + 1, smin(e.m, d));
  const int width = hi - lo + 1;
  if (width > 0) e.W += width;
  const bool cap_hit = P.band_cap > 0 && width > P.band_cap;

  // neighbours from the lane below (window position l*C - 1)
  const int up0 = wave_shr1(A[C - 1], NEG);
  const int dg0 = wave_shr1(B[C - 1], NEG);

  // prune threshold in the V frame: S >= T - X  <=>  V >= T - X - gap*d
  const int thr = smax(e.T - P.X - P.gap * d, THR_FLOOR);
  // window positions p with y > n (p < pmin) or x > m (p > pmin + span)
  // are outside the matrix
  const int pmin = d - e.n - e.base;
  const uint32_t span = (uint32_t)(e.m - e.base - pmin);

  int v[C];
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const int up = j ? A[j - 1] : up0;
    const int dg = j ? B[j - 1] : dg0;
    v[j] = max(max(up, A[j]), dg + sy.sim(j, P, tab));
  }
  uint64_t msk[C];
  uint64_t any = 0;
  int lm = NEG;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const bool f = v[j] >= thr && (uint32_t)(lane * C + j - pmin) <= span;
    v[j] = f ? v[j] : NEG;
    msk[j] = ballot(f);
    any |= msk[j];
    lm = max(lm, v[j]);
  }
#pragma unroll
  for (int j = 0; j < C; ++j) { B[j] = A[j]; A[j] = v[j]; }

  // running best (S frame value T <=> V frame value T - gap*d); the wave
  // maximum is needed only when some lane beats T, and is one readlane when
  // a single lane does
  const int Tv = e.T - P.gap * d;
  const uint64_t imp = ballot(lm > Tv);
  if (imp) {
    int wm, l0;
    if (__builtin_popcountll(imp) == 1) {
      l0 = __builtin_ctzll(imp);
      wm = __builtin_amdgcn_readlane(lm, l0);
    } else {
      wm = uni(wave_max(lm));
      l0 = __builtin_ctzll(ballot(lm == wm));
    }
    int js = 0;
    if constexpr (C > 1) {
      int jf = C - 1;
#pragma unroll
      for (int j = C - 1; j >= 0; --j)
        if (A[j] == wm) jf = j;
      js = __builtin_amdgcn_readlane(jf, l0);
    }
    e.T = wm + P.gap * d;
    e.bx = e.base + l0 * C + js;
    e.by = d - e.bx;
  }

  // finite range of d
  int L0 = DEAD_L, U0 = DEAD_U;
  if (any) {
    const int llo = __builtin_ctzll(any);
    const int lhi = 63 - __builtin_clzll(any);
    int jlo = 0, jhi = 0;
    if constexpr (C > 1) {
#pragma unroll
      for (int j = C - 1; j >= 0; --j)
        if ((msk[j] >> llo) & 1) jlo = j;
#pragma unroll
      for (int j = 0; j < C; ++j)
        if ((msk[j] >> lhi) & 1) jhi = j;
    }
    L0 = e.base + (llo << LOG2C) + jlo;
    U0 = e.base + (lhi << LOG2C) + jhi;
  }

  const int L1 = e.L1, U1 = e.U1;
  e.L2 = L1; e.U2 = U1;
  e.L1 = L0; e.U1 = U0;
  e.d = d + 1;
  int r = R_CONT;
  if ((!any && L1 > U1) || d >= e.m + e.n) r = R_DONE;

  // keep the next antidiagonal's band inside the window
  int mv = MV_NONE;
  if (r == R_CONT) mv = window_move<ALPHA, C>(e, A, B, sy, w, S, L0, L1, U0, U1);
  if (mv == MV_ESC) {
    r = R_ESC;
  } else if (r == R_CONT && mv == MV_NONE) {
    // target codes of the next antidiagonal: one code enters at lane 0
    if (e.qn == 0) {
      cover_b<ALPHA>(e, w, S, e.qi + Syms<ALPHA, C>::QCODES - 1);
      e.q = Syms<ALPHA, C>::queue(w, e.qi);
      e.qn = Syms<ALPHA, C>::QCODES;
    }
    const uint32_t in =
        (uint32_t)(e.q & ((1u << Syms<ALPHA, C>::QBITS) - 1));
    e.q >>= Syms<ALPHA, C>::QBITS;
    e.qn -= 1;
    e.qi += 1;
    sy.advance(in);
  }
  if (cap_hit) r = R_CAP;
  make_uniform(e);
  return r;
}

// ------------------------------------------------------------------ interior

// A value that the compiler keeps in a VGPR (a loop-invariant operand of a
// per-lane select, which may not read two SGPRs).
__device__ __forceinline__ int in_vgpr(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0xE4, 0xf, 0xf, false);
}

// Lean sweep for one cell per lane.  The band bookkeeping runs on the
// finite-lane ballots M1, M2 of the last two antidiagonals instead of on
// scalar ranges (positions relative to the window base):
//   lo_d = max(ctz(M1 | M2 << 1), d - n - base),
//   hi_d = min(64 - clz(M1 | M2), m - base),
// where the clamps matter only near the matrix edges; blocks of XD_KB1
// (DNA) or XD_KB1B (byte codes) antidiagonals that stay clear of both edges skip them and the per-lane
// edge masks.  The live-span count
// sum(hi_d - lo_d + 1) is formed once per block on the vector unit from the
// masks, which the block keeps in lanes of two registers.  The top G lanes
// (8 for DNA, 4 for byte codes) stay -infinity at the start of every group
// of G antidiagonals (the
// band grows by at most one lane per antidiagonal, so the top lane is still
// -infinity G - 1 antidiagonals later): the neighbour exchange is then a
// wave rotation that brings -infinity to lane 0, and the band is tested
// against the top only every G-th antidiagonal.  When the band reaches lane
// 64 - G the window slides up in place by the dead lanes below the band.
// DNA scores come from per-block match words (bit 2k of lane l: the codes
// of cell base + l agree on antidiagonal d + k); byte codes are read per
// lane from the ring and index the score table.  The loop computes
// antidiagonals up to m + n and returns R_DONE after the last one or after
// two dead antidiagonals; it hands over to the generic step (state as that
// step expects) when the band fills the window, and returns R_ESC when the
// window can neither slide nor stay.
template <int ALPHA>
__device__ __forceinline__ int fast_interior(Ext& e, int (&A)[1], int (&B)[1],
                                             Syms<ALPHA, 1>& sy,
                                             WaveLds<ALPHA>& w,
                                             const int* tab, const Params& P,
                                             const Src& S) {
  int base = e.base;
  if (P.band_cap > 0) return R_CONT;
  const int d_last = e.m + e.n;  // antidiagonals this loop may compute
  if (e.d > d_last) return R_CONT;
  uint64_t m1 = e.L1 > e.U1 ? 0
                : (1ull << (e.L1 - base)) | (1ull << (e.U1 - base));
  uint64_t m2 = e.L2 > e.U2 ? 0
                : (1ull << (e.L2 - base)) | (1ull << (e.U2 - base));
  if ((m1 | m2) == 0) return R_CONT;
  // leading zeros of M1 | M2 (never both zero inside the loop)
  int cz = (int)__builtin_clzll(m1 | m2);
  const int d0 = e.d;
  const int d_end = smin(d_last, d0 + (1 << 20));  // 32-bit sums exact
  // every finite V lies in [-2^28, 2^28] and T's frame value tv in
  // [0, 2^28] (value bound checked per extension), so capping X at 2^29
  // prunes exactly the same cells and keeps tv - X above the floor
  const int gap = P.gap, X = smin(P.X, 1 << 29);
  const int m = e.m, n = e.n;
  const int lane = lane_id();
  const int vmat = in_vgpr(P.mat_s), vmis = in_vgpr(P.mis_s);
  // DNA: the query code of each lane copied into all 16 code slots of a
  // word; bytes: the byte offset of the lane's row of the score table (row
  // = query code, 32 entries of 4 bytes)
  uint32_t fa = 0;
  auto load_fa = [&]() {
    if constexpr (ALPHA == 0) {
      fa = (Ring<0>::read(w.ra, base + lane - 1) & 3u) * 0x55555555u;
    } else {
      uint32_t t[1];
      Ring<1>::read<1>(w.ra, base + lane - 1, t);
      fa = (t[0] & 31u) * (4 * TAB_LD);
    }
  };
  // bytes: score of the lane's cell for target code c
  auto score = [&](uint32_t c) {
    return *reinterpret_cast<const int*>(
        reinterpret_cast<const char*>(tab) + fa + (c << 2));
  };
  load_fa();
  int d = d0;
  int tv = e.T - gap * d0;  // best score in the frame of antidiagonal d
  // per lane: the sum over the blocks of its antidiagonal's 65 - live-span
  // cells (lanes 2 .. KB + 1); summed over the wave once, after the loop
  int vacc = 0;
  // last new best: its antidiagonal, its x, and its lane (folded into x
  // once per block: base moves only between blocks); T itself follows from
  // tv, which is T in the frame of the next antidiagonal
  int bd = -1, bxa = 0, bln = 0;
  int pm = 0, mrel = 0;     // d - n - base, m - base (edge clamps and masks)
  uint64_t in_m = 0;        // edge blocks: the lanes with x <= m
  int rem = 0;              // edge blocks: d_end - d
  // antidiagonals per block (the block's fixed work, some 60 vector
  // instructions, spreads over its steps; 48 measured 3-5% faster than 32,
  // and 60 another 0.4% for byte codes, whose blocks need no whole match
  // words): DNA reads KB / 16 match words, bytes take their codes from the
  // ring
  constexpr int KB = ALPHA == 1 ? XD_KB1B : XD_KB1;
  static_assert((ALPHA == 1 || KB % 16 == 0) && KB + 2 <= 64,
                "whole DNA match words; the masks of a block fit in 64 lanes");
  // top lanes kept -infinity between the tests against the top, which run
  // with the dead test every G-th antidiagonal.  Fewer tests cost a smaller
  // window: DNA bands are narrow and its chains long (8: dna-tail 6.05 ->
  // 5.70 ms, dna-1k 0.158 -> 0.150), protein bands wider (4: 2 and 8 were
  // 1.5% and 3.4% slower on protein-500k)
  constexpr int G = ALPHA == 0 ? 8 : 4;
  static_assert(KB % G == 0, "tests fall on the same steps in every block");
  uint32_t mw[KB / 16] = {};  // DNA: match words of the block (16 steps each)
  // finite-lane masks of the block's antidiagonals for the live-span count,
  // kept in lanes of two registers (low and high words): lanes 0 and 1 hold
  // the two antidiagonals before the block, lane k + 2 the block's k-th
  int ml = 0, mh = 0;
  // bytes: the ring position of the lane's target code on the block's first
  // antidiagonal (cell base + l of antidiagonal d + k takes b[d + k - base -
  // l - 1], k bytes further on: an immediate offset of the read); the score
  // of the next antidiagonal and the codes of the two after it are read
  // ahead of their use
  const uint8_t* cp = reinterpret_cast<const uint8_t*>(w.rb);
  int sc_next = 0;
  uint32_t cd1 = 0, cd2 = 0;

  // Antidiagonal d + k from prev (d+k-1) and pp (d+k-2), with their
  // finite-lane masks mp and mpp; pp and mpp receive d + k (the two
  // antidiagonals and their masks swap roles every step).  True (k = G - 1
  // mod G) when the band reached lane 64 - G or after two dead
  // antidiagonals, or (edge blocks) at the last antidiagonal of the range;
  // the reason is read from the masks and d after the block.  (Two dead
  // antidiagonals may be followed by up to G - 1 more, dead as well, that
  // add no live-span cell.)  d itself moves once per block.
  auto body = [&](auto edge_tag, auto g_tag, int& prev, int& pp,
                  const uint64_t& mp, uint64_t& mpp, int k) -> bool {
    constexpr bool EDGE = decltype(edge_tag)::value;
    constexpr int GG = decltype(g_tag)::value;  // G, or 1 (narrow top room)
    const int thr = tv - X;
    int sim;
    if constexpr (ALPHA == 0) {
      // -1: match
      int t = __builtin_amdgcn_sbfe((int)mw[k >> 4], 2 * (k & 15), 1);
      opaque_v(t);  // keeps the bit select one v_bfi (not compare + select)
      sim = (t & vmat) | (~t & vmis);
      opaque_v(sim);  // (the select stays whole, so the add below is VOP2)
    } else {
      sim = sc_next;
      sc_next = score(cd1);
      cd1 = cd2;
      // (the load's zero extension stays with it: left to the block after
      // the improvement branch, it becomes a separate mask there)
      int c3 = cp[k + 3];
      opaque_v(c3);
      cd2 = (uint32_t)c3;
    }
    // (every lane of a wave rotation has a source, so bound_ctrl changes
    // nothing; it lets the compiler fold the move into its user, a VOP2
    // add and max here: the inner max is kept apart from the outer, which
    // would otherwise make a three-input max that takes no DPP operand)
    const int up = __builtin_amdgcn_update_dpp(0, prev, 0x13C, 0xf, 0xf, true);
    const int dg = __builtin_amdgcn_update_dpp(0, pp, 0x13C, 0xf, 0xf, true);
    int uh = max(up, prev);
    opaque_v(uh);
    const int v = max(uh, dg + sim);
    uint64_t fm = ballot(v >= thr);
    if constexpr (EDGE) {
      // y > n below pm + k, x > m above mrel (block mask).  Byte codes form
      // pm + k on the scalar unit: the compiler would otherwise compare
      // lane - k with pm, one more vector instruction per edge step (0.15%
      // on protein-500k; DNA's latency-bound chain lost as much).
      if constexpr (ALPHA == 1) {
        uint32_t pk = (uint32_t)(pm + k);
        opaque_s(pk);
        fm &= ballot(lane >= (int)pk) & in_m;
      } else {
        fm &= ballot(lane >= pm + k) & in_m;
      }
    }
    const int vn = __builtin_amdgcn_inverse_ballot_w64(fm) ? v : NEG;
    // away from the edges a cell with v > tv >= thr is finite, so the
    // improvement test need not wait for the select
    const int vi = EDGE ? vn : v;
    const uint64_t imp = ballot(vi > tv);
    // (the select before the improvement branch: the next antidiagonal's
    // neighbour moves then need not wait for it after the branch)
    int vk = vn;
    pin_v(vk);
    pp = vk;
    // (T improves on a large share of the antidiagonals, a third of the
    // one-cell steps of protein-500k, so the update is laid out inline: kept
    // apart, each improvement cost two taken branches, 0.35% of the tuned
    // protein-500k time.  The two-cell loop, whose steps improve T less
    // often, keeps it apart)
    if (imp != 0) {
      // usually a single lane beats T: its value is the new best
      int l0 = __builtin_ctzll(imp);
      int wm = __builtin_amdgcn_readlane(vi, l0);
      uint32_t nimp = (uint32_t)__builtin_popcountll(imp);
      opaque_s(nimp);  // (one s_bcnt1, not a 64-bit x & (x - 1))
      if (nimp > 1) {
        wm = uni(wave_max(vi));
        l0 = __builtin_ctzll(ballot(vi == wm));
      }
      tv = wm;  // T, bx, by are formed on hand-over
      bd = d + k;
      bln = l0;
    }
    mpp = fm;
    ml = xd_writelane_i32((int)(uint32_t)fm, k + 2, ml);
    mh = xd_writelane_i32((int)(uint32_t)(fm >> 32), k + 2, mh);
    tv -= gap;
    if ((k & (GG - 1)) == GG - 1) {
      const uint64_t o = mp | fm;
      if (o == 0) return true;
      // one of the top GG lanes finite; tested on the high word, since a
      // 64-bit compare would run on the vector unit
      uint32_t hw = (uint32_t)(o >> 32);
      opaque_s(hw);
      if (hw >= (1u << (32 - GG))) return true;
    }
    if constexpr (EDGE) {
      if (k >= rem) return true;  // d + k is d_end
    }
    return false;
  };

  // x (mask m1) holds d-1 and y (mask m2) holds d-2 at the start of a block
  int x = A[0], y = B[0];
  while (d <= d_end) {
    // byte codes: a band with fewer than G free lanes above it after the
    // slide runs a block with one guard lane, tested every antidiagonal (a
    // band that fills the window goes to the generic step, which widens the
    // tile).  Protein bands hover near the window's width: this replaced a
    // hand-over to the generic step and back for 14% of protein-500k's
    // extensions, 8.7 times each (10.22 -> 9.67 ms).  DNA bands are narrow;
    // there the extra block copy cost 5-9% (register allocation), so DNA
    // hands over as before.
    // Byte codes also slide early: a band with fewer than G + XD_PRE free
    // lanes above it would likely reach the top within the block, which then
    // ends early (protein-500k: 0.5% with blocks of 48 and a margin of 16,
    // another 0.6% with blocks of 60 and a margin of 24, where margins of
    // 24 to 40 measure the same; DNA's narrow bands lost 1-2%).
    constexpr int EARLY = ALPHA == 1 ? XD_PRE : 0;
    bool tight = false;
    if (cz < G + EARLY) {
      // the band reached lane 64 - G: slide the window up by the lanes
      // below the lowest finite cell of d-1 and d-2 (they are -infinity on
      // both)
      const int sl = __builtin_ctzll(m1 | m2);
      if (cz < G && cz + sl < (ALPHA == 1 ? 1 : G)) break;
      if (cz < G ? (ALPHA == 0 || sl > 0) : sl >= XD_MINSL) {
        const int src = lane + sl;
        const bool in = src < 64;
        const int pn = __builtin_amdgcn_ds_bpermute((src & 63) << 2, x);
        const int po = __builtin_amdgcn_ds_bpermute((src & 63) << 2, y);
        x = in ? pn : NEG;
        y = in ? po : NEG;
        m1 >>= sl;
        m2 >>= sl;
        cz += sl;
        base += sl;
        cover_a<ALPHA>(e, w, S, base + 62);
        load_fa();
      }
      if constexpr (ALPHA == 1) tight = cz < G;
    }
    pm = d - n - base;
    mrel = m - base;
    rem = d_end - d;
    in_m = ballot(lane <= mrel);
    const int e0 = d - base;
    cover_b<ALPHA>(e, w, S, e0 + KB - 1);
    if constexpr (ALPHA == 0) {
      // codes of b[e0 - lane - 1 + k], k < KB, against the lane's query code
#pragma unroll
      for (int h = 0; h < KB / 16; ++h) {
        const uint32_t xw = Ring<0>::read(w.rb, e0 - lane - 1 + 16 * h) ^ fa;
        mw[h] = ~(xw | (xw >> 1)) & 0x55555555u;
      }
    } else {
      // (reads up to KB + 2 bytes past a position of the ring, which its
      // mirror words cover; codes past those covered belong to no block step)
      cp = reinterpret_cast<const uint8_t*>(w.rb) +
           ((e0 - lane - 1) & (Ring<1>::RS - 1));
      sc_next = score(cp[0]);
      cd1 = cp[1];
      cd2 = cp[2];
    }
    ml = xd_writelane_i32((int)(uint32_t)m2, 0, ml);
    mh = xd_writelane_i32((int)(uint32_t)(m2 >> 32), 0, mh);
    ml = xd_writelane_i32((int)(uint32_t)m1, 1, ml);
    mh = xd_writelane_i32((int)(uint32_t)(m1 >> 32), 1, mh);
    int nk = KB;  // antidiagonals computed by the block
    bool newest_in_y = false;
    auto run_block = [&](auto edge_tag, auto g_tag) {
#pragma unroll
      for (int k = 0; k < KB; k += 2) {
        if (body(edge_tag, g_tag, x, y, m1, m2, k)) {
          nk = k + 1; newest_in_y = true; return;
        }
        if (body(edge_tag, g_tag, y, x, m2, m1, k + 1)) { nk = k + 2; return; }
      }
    };
    if (ALPHA == 1 && tight)  // (its own copy with the edge masks)
      run_block(std::true_type{}, std::integral_constant<int, 1>{});
    else if (pm + KB - 1 <= 0 && mrel >= 63 && rem >= KB - 1)
      run_block(std::false_type{}, std::integral_constant<int, G>{});
    else
      run_block(std::true_type{}, std::integral_constant<int, G>{});
    {
      // live-span cells of the block's antidiagonals, one per lane k + 2,
      // from the masks of the two antidiagonals before each (lanes k + 1 and
      // k): 65 - |[max(lo, d - n - base), min(hi, m - base)]| with
      // lo = ctz(M1 | M2 << 1), hi = 64 - clz(M1 | M2) (M2 never holds lane
      // 63, so neither search comes up empty unless both masks are zero: an
      // antidiagonal after two dead ones, with no live-span cell)
      const uint32_t al = (uint32_t)wave_shr1_z(ml), ah = (uint32_t)wave_shr1_z(mh);
      const uint32_t bl = (uint32_t)wave_shr1_z((int)al), bh = (uint32_t)wave_shr1_z((int)ah);
      const uint32_t cl = al | (bl << 1);
      const uint32_t ch = ah | __builtin_amdgcn_alignbit(bh, bl, 31);
      const uint32_t ctz = min(ffbl32(cl), ffbl32(ch) | 32u);
      const uint32_t clz = min(ffbh32(ah | bh), ffbh32(al | bl) | 32u);
      const int kk = lane - 2;
      const int lo = max((int)ctz, pm + kk);
      const int hi = min(64 - (int)clz, mrel);
      const bool live = (al | ah | bl | bh) != 0;
      const int cnt = (kk >= 0 && kk < nk)
                          ? (live ? 65 - max(hi - lo + 1, 0) : 65) : 0;
      // (lanes 2 .. KB + 1 hold counts)
      vacc += cnt;
    }
    if (bd >= d) bxa = base + bln;  // a new best in this block
    d += nk;
    if (newest_in_y) {
      const int t = x;
      x = y;
      y = t;
    }
    // the masks again from the cells (a cell is finite exactly when it is not
    // -infinity): the block's many ends then need not carry them, which
    // would cost register moves on every block
    m1 = ballot(x != NEG);
    m2 = ballot(y != NEG);
    cz = (int)__builtin_clzg(m1 | m2, 64);
    if ((m1 | m2) == 0) break;  // two dead antidiagonals
  }
  A[0] = x;
  B[0] = y;

  e.base = base;
  e.d = d;
  const uint32_t acc =
      (uint32_t)(KB + 2 <= 32 ? sum_lanes_0_31(vacc) : sum_lanes(vacc));
  e.W += (int64_t)65 * (d - d0) - (int64_t)acc;
  e.T = tv + gap * d;
  if (bd >= 0) {
    e.bx = bxa;
    e.by = bd - bxa;
  }
  // finished: two dead antidiagonals (every later cell is -infinity) or the
  // last antidiagonal of the matrix computed
  int r = R_DONE;
  if ((m1 | m2) != 0 && d <= e.m + e.n) {
    e.L1 = m1 ? base + __builtin_ctzll(m1) : DEAD_L;
    e.U1 = m1 ? base + 63 - __builtin_clzll(m1) : DEAD_U;
    e.L2 = m2 ? base + __builtin_ctzll(m2) : DEAD_L;
    e.U2 = m2 ? base + 63 - __builtin_clzll(m2) : DEAD_U;
    r = R_CONT;
    const int mv = window_move<ALPHA, 1>(e, A, B, sy, w, S, e.L1, e.L2, e.U1,
                                         e.U2);
    if (mv == MV_ESC) r = R_ESC;
    else if (mv == MV_NONE) reload_syms<ALPHA, 1>(e, sy, w, S);
  }
  make_uniform(e);
  return r;
}

// The same loop for C = 2 cells per lane (cell j of lane l is window
// position 2l + j), with one finite-lane mask per register (M_j: the lanes
// whose cell j is finite).  The top two lanes (positions 124..127) stay
// -infinity at the start of every pair of antidiagonals, so the rotation
// brings -infinity to cell 0 of lane 0 and the band is tested against the
// top (and for two dead antidiagonals) only every second antidiagonal; the
// window slides up in place by whole lanes.  Edge blocks mask cells outside
// the matrix.  Live-span cells are counted per block on the vector unit from
// the masks kept in lanes (as in the one-cell loop), with
//   L = min_j 2 ctz(M_j) + j,  U = max_j 2 (63 - clz(M_j)) + j.
template <int ALPHA, int C>
__device__ __forceinline__ int fast_interior_multi(Ext& e, int (&A)[C],
                                                   int (&B)[C],
                                                   Syms<ALPHA, C>& sy,
                                                   WaveLds<ALPHA>& w,
                                                   const int* tab,
                                                   const Params& P,
                                                   const Src& S) {
  static_assert(C == 2, "two cells per lane");
  // top lanes kept -infinity between the tests against the top, which run
  // with the dead test every G2-th antidiagonal
  constexpr int G2 = XD_G2;
  static_assert(XD_KB2 % G2 == 0 && XD_KB2B % G2 == 0,
                "tests fall on the same steps in every block");
  int base = e.base;
  if (P.band_cap > 0) return R_CONT;
  const int d_last = e.m + e.n - 1;
  if (e.d > d_last) return R_CONT;
  const int lane = lane_id();
  // finite-lane masks of d-1 (x) and d-2 (y), from the cells (a cell is
  // finite exactly when it is not -infinity)
  uint64_t mx0 = ballot(A[0] != NEG), mx1 = ballot(A[1] != NEG);
  uint64_t my0 = ballot(B[0] != NEG), my1 = ballot(B[1] != NEG);
  if ((mx0 | mx1 | my0 | my1) == 0) return R_CONT;
  const int d0 = e.d;
  const int d_end = smin(d_last, d0 + (1 << 20));  // 32-bit sums exact
  const int gap = P.gap, X = smin(P.X, 1 << 29);  // see fast_interior
  const int m = e.m, n = e.n;
  const int vmat = in_vgpr(P.mat_s), vmis = in_vgpr(P.mis_s);
  // cell j of lane l is x = base + 2l + j and takes a[x - 1] and
  // b[d - x - 1]: DNA keeps bare codes of both (the target codes move one
  // cell up per antidiagonal); bytes keep the byte offset of the score
  // table's row for a[x - 1] and read b[d - x - 1] from the ring per lane
  // (cell 0 at an immediate offset per antidiagonal, cell 1 the code cell 0
  // had one antidiagonal before)
  int fa[C], fb[C] = {};
  auto load_fa = [&]() {
    const int sa = base + lane * C - 1;
    if constexpr (ALPHA == 0) {
      const uint32_t wa = Ring<0>::read(w.ra, sa);
#pragma unroll
      for (int j = 0; j < C; ++j) fa[j] = (int)((wa >> (2 * j)) & 3u);
    } else {
      uint32_t ta[1];
      Ring<1>::read<1>(w.ra, sa, ta);
#pragma unroll
      for (int j = 0; j < C; ++j)
        fa[j] = (int)((ta[0] >> (8 * j)) & 31u) * (4 * TAB_LD);
    }
  };
  load_fa();
  if constexpr (ALPHA == 0) {
    const int sb = d0 - base - lane * C - C;  // b index of cell C-1
    const uint32_t wb = Ring<0>::read(w.rb, sb);
#pragma unroll
    for (int j = 0; j < C; ++j) fb[j] = (int)((wb >> (2 * (C - 1 - j))) & 3u);
  }
  // bytes: the lane's ring position of cell 0's code on the block's first
  // antidiagonal; the two cells' scores of the next antidiagonal, cell 0's
  // code on the current one and its codes of the two after the next are
  // read ahead of their use (as in the one-cell loop)
  const uint8_t* cp = reinterpret_cast<const uint8_t*>(w.rb);
  int sc0 = 0, sc1 = 0;
  uint32_t ccur = 0, cd1 = 0, cd2 = 0;
  auto score = [&](int f, uint32_t c) {
    return *reinterpret_cast<const int*>(
        reinterpret_cast<const char*>(tab) + f + (c << 2));
  };
  int d = d0;
  int tv = e.T - gap * d0;  // best score in the frame of antidiagonal d
  int vacc = 0;  // per lane: live-span cells of its antidiagonals (see
                 // fast_interior), summed over the wave after the loop
  int tbest = 0, bd = -1, bxa = 0;
  int pm = 0, mrel = 0;     // edge blocks: d - n - base, m - base
  int rem = 0;              // edge blocks: d_end - d
  uint64_t in_m0 = 0, in_m1 = 0;  // edge blocks: lanes whose cell j has x <= m
  // masks of the block's antidiagonals in lanes (lane k + 2: the block's
  // k-th; lanes 0 and 1: the two before it), per register j and word
  int ml0 = 0, mh0 = 0, ml1 = 0, mh1 = 0;

  // antidiagonal d + k from prev (d+k-1, masks mp0/mp1) and pp (d+k-2,
  // masks mpp0/mpp1); pp and its masks receive d + k.  True (odd k only)
  // after two dead antidiagonals or when the band reached lane 62, or (edge
  // blocks) at the last antidiagonal of the range.
  auto body = [&](auto edge_tag, int (&prev)[C], int (&pp)[C],
                  const uint64_t& mp0, const uint64_t& mp1, uint64_t& mpp0,
                  uint64_t& mpp1, int in, int k) -> bool {
    constexpr bool EDGE = decltype(edge_tag)::value;
    const int thr = tv - X;
    int v[C];
#pragma unroll
    for (int j = C - 1; j >= 0; --j) {
      const int up = j ? prev[j - 1]
                       : __builtin_amdgcn_mov_dpp(prev[C - 1], 0x13C, 0xf,
                                                  0xf, false);
      const int dg = j ? pp[j - 1]
                       : __builtin_amdgcn_mov_dpp(pp[C - 1], 0x13C, 0xf, 0xf,
                                                  false);
      int sim;
      if constexpr (ALPHA == 0) sim = fa[j] == fb[j] ? vmat : vmis;
      else sim = j == 0 ? sc0 : sc1;
      v[j] = max(max(up, prev[j]), dg + sim);
    }
    if constexpr (ALPHA == 1) {
      // next antidiagonal: cell 1 takes cell 0's current code
      sc1 = score(fa[1], ccur);
      ccur = cd1;
      sc0 = score(fa[0], cd1);
      cd1 = cd2;
      int c3 = cp[k + 3];
      opaque_v(c3);  // (the load's zero extension stays with it)
      cd2 = (uint32_t)c3;
    }
    uint64_t f[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      f[j] = ballot(v[j] >= thr);
      if constexpr (EDGE) {
        // y > n below pm + k (pm + k - j formed on the scalar unit: the
        // compiler would otherwise form lane * C - k on the vector unit),
        // x > m above mrel (block masks)
        uint32_t pk = (uint32_t)(pm + k - j);
        opaque_s(pk);
        f[j] &= ballot(lane * C >= (int)pk) & (j ? in_m1 : in_m0);
      }
    }
    int vn[C];
#pragma unroll
    for (int j = 0; j < C; ++j)
      vn[j] = __builtin_amdgcn_inverse_ballot_w64(f[j]) ? v[j] : NEG;
    // away from the edges a cell with v > tv >= thr is finite
    const int lm = EDGE ? max(vn[0], vn[1]) : max(v[0], v[1]);
    const uint64_t imp = ballot(lm > tv);
#pragma unroll
    for (int j = 0; j < C; ++j) pp[j] = vn[j];
    if (__builtin_expect(imp != 0, 0)) {
      int l0 = __builtin_ctzll(imp);
      int wm = __builtin_amdgcn_readlane(lm, l0);
      uint32_t nimp = (uint32_t)__builtin_popcountll(imp);
      opaque_s(nimp);
      if (nimp > 1) {
        wm = uni(wave_max(lm));
        l0 = __builtin_ctzll(ballot(lm == wm));
      }
      // lowest x of the lane: cell 0 if it holds the maximum
      const int jf = __builtin_amdgcn_readlane(pp[0] == wm ? 0 : 1, l0);
      tv = wm;
      tbest = wm;  // T, bx, by are formed on hand-over
      bd = d + k;
      bxa = base + (l0 << 1) + jf;
    }
    mpp0 = f[0];
    mpp1 = f[1];
    ml0 = xd_writelane_i32((int)(uint32_t)f[0], k + 2, ml0);
    mh0 = xd_writelane_i32((int)(uint32_t)(f[0] >> 32), k + 2, mh0);
    ml1 = xd_writelane_i32((int)(uint32_t)f[1], k + 2, ml1);
    mh1 = xd_writelane_i32((int)(uint32_t)(f[1] >> 32), k + 2, mh1);
    tv -= gap;
    if constexpr (ALPHA == 0) {
      // the target codes move one cell up; lane 0 takes `in`
      const int top = fb[C - 1];
#pragma unroll
      for (int j = C - 1; j > 0; --j) fb[j] = fb[j - 1];
      fb[0] = __builtin_amdgcn_update_dpp(in, top, 0x138, 0xf, 0xf, false);
    }
    if ((k & (G2 - 1)) == G2 - 1) {
      const uint64_t o = mp0 | mp1 | f[0] | f[1];
      if (o == 0) return true;
      uint32_t hw = (uint32_t)(o >> 32);  // the top G2 lanes (see fast_interior)
      opaque_s(hw);
      if (hw >= (1u << (32 - G2))) return true;
    }
    if constexpr (EDGE) {
      if (k >= rem) return true;  // d + k is d_end
    }
    return false;
  };
  // blocks of QB antidiagonals; the codes entering lane 0 during a block
  // are read from the ring at its start (QB / 16 words of DNA codes, QB / 4
  // words of byte codes)
  constexpr int QB = ALPHA == 1 ? XD_KB2B : XD_KB2;
  static_assert((ALPHA == 1 || QB % 16 == 0) && QB + 2 <= 64 &&
                    QB + 3 <= 4 * Ring<1>::MIRROR,
                "whole DNA code words; the masks of a block fit in 64 lanes; "
                "byte reads stay within the ring's mirror words");
  int x[C], y[C];
#pragma unroll
  for (int j = 0; j < C; ++j) { x[j] = A[j]; y[j] = B[j]; }
  while (d <= d_end) {
    {
      const uint64_t o = mx0 | mx1 | my0 | my1;
      if ((uint32_t)(o >> 32) >= (1u << (32 - G2))) {
        // the band reached lane 62: slide the window up by the whole lanes
        // below the lowest finite cell of d-1 and d-2
        const int sl = __builtin_ctzll(o);
        if (sl < G2) break;
        const int src = lane + sl;
        const bool in = src < 64;
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const int pn = __builtin_amdgcn_ds_bpermute((src & 63) << 2, x[j]);
          const int po = __builtin_amdgcn_ds_bpermute((src & 63) << 2, y[j]);
          // DNA: target codes move with their cells; stray codes at the
          // top lanes are not used before they have moved out (see
          // fast_interior)
          if constexpr (ALPHA == 0)
            fb[j] = __builtin_amdgcn_ds_bpermute((src & 63) << 2, fb[j]);
          x[j] = in ? pn : NEG;
          y[j] = in ? po : NEG;
        }
        mx0 >>= sl; mx1 >>= sl; my0 >>= sl; my1 >>= sl;
        base += sl << 1;
        cover_a<ALPHA>(e, w, S, base + 2 * 64 - 2);
        load_fa();
      }
    }
    pm = d - n - base;
    mrel = m - base;
    rem = d_end - d;
    in_m0 = ballot(lane * C <= mrel);
    in_m1 = ballot(lane * C + 1 <= mrel);
    const int e0 = d - base;
    cover_b<ALPHA>(e, w, S, e0 + QB - 1);
    constexpr int NQ = ALPHA == 0 ? QB / 16 : 1;
    uint32_t qw[NQ] = {};
    if constexpr (ALPHA == 0) {
#pragma unroll
      for (int i = 0; i < NQ; ++i)
        qw[i] = (uint32_t)in_vgpr((int)Ring<0>::read(w.rb, e0 + 16 * i));
    } else {
      // (reads up to QB + 2 bytes past a ring position, which the mirror
      // words cover)
      const uint8_t* rbb = reinterpret_cast<const uint8_t*>(w.rb);
      cp = rbb + ((e0 - 2 * lane - 1) & (Ring<1>::RS - 1));
      ccur = cp[0];
      sc0 = score(fa[0], ccur);
      sc1 = score(fa[1], rbb[(e0 - 2 * lane - 2) & (Ring<1>::RS - 1)]);
      cd1 = cp[1];
      cd2 = cp[2];
    }
    ml0 = xd_writelane_i32((int)(uint32_t)my0, 0, ml0);
    mh0 = xd_writelane_i32((int)(uint32_t)(my0 >> 32), 0, mh0);
    ml1 = xd_writelane_i32((int)(uint32_t)my1, 0, ml1);
    mh1 = xd_writelane_i32((int)(uint32_t)(my1 >> 32), 0, mh1);
    ml0 = xd_writelane_i32((int)(uint32_t)mx0, 1, ml0);
    mh0 = xd_writelane_i32((int)(uint32_t)(mx0 >> 32), 1, mh0);
    ml1 = xd_writelane_i32((int)(uint32_t)mx1, 1, ml1);
    mh1 = xd_writelane_i32((int)(uint32_t)(mx1 >> 32), 1, mh1);
    int nk = QB;  // antidiagonals computed by the block
    bool newest_in_y = false;
    auto run_block = [&](auto edge_tag) {
#pragma unroll
      for (int k = 0; k < QB; k += 2) {
        const int in0 = ALPHA == 0
            ? (int)__builtin_amdgcn_ubfe(qw[k >> 4], 2 * (k & 15), 2) : 0;
        const int in1 = ALPHA == 0
            ? (int)__builtin_amdgcn_ubfe(qw[(k + 1) >> 4], 2 * ((k + 1) & 15), 2)
            : 0;
        if (body(edge_tag, x, y, mx0, mx1, my0, my1, in0, k)) {
          nk = k + 1; newest_in_y = true; return;
        }
        if (body(edge_tag, y, x, my0, my1, mx0, mx1, in1, k + 1)) {
          nk = k + 2; return;
        }
      }
    };
    if (pm + QB - 1 <= 0 && mrel >= 2 * 64 - 1 && rem >= QB - 1)
      run_block(std::false_type{});
    else
      run_block(std::true_type{});
    {
      // live-span cells of the block's antidiagonals (see fast_interior):
      // lane k + 2 forms antidiagonal k's span from the finite ranges of the
      // antidiagonals in lanes k + 1 (a) and k (b)
      auto range = [&](uint32_t l0, uint32_t h0, uint32_t l1, uint32_t h1,
                       int& L, int& U) {
        const uint32_t c0 = min(ffbl32(l0), ffbl32(h0) | 32u);
        const uint32_t c1 = min(ffbl32(l1), ffbl32(h1) | 32u);
        const uint32_t z0 = min(ffbh32(h0), ffbh32(l0) | 32u);
        const uint32_t z1 = min(ffbh32(h1), ffbh32(l1) | 32u);
        // (an empty mask gives c = z = 2^32 - 1: L above, U below any cell)
        L = (int)min(min(c0, 64u) * 2, min(c1, 64u) * 2 + 1);
        U = max(c0 >= 64u ? -1 : (int)(63 - z0) * 2,
                c1 >= 64u ? -1 : (int)(63 - z1) * 2 + 1);
      };
      int La, Ua, Lb, Ub;
      range((uint32_t)wave_shr1_z(ml0), (uint32_t)wave_shr1_z(mh0),
            (uint32_t)wave_shr1_z(ml1), (uint32_t)wave_shr1_z(mh1), La, Ua);
      range((uint32_t)wave_shr1_z(wave_shr1_z(ml0)),
            (uint32_t)wave_shr1_z(wave_shr1_z(mh0)),
            (uint32_t)wave_shr1_z(wave_shr1_z(ml1)),
            (uint32_t)wave_shr1_z(wave_shr1_z(mh1)), Lb, Ub);
      const int kk = lane - 2;
      const int lo = max(min(La, Lb + 1), pm + kk);
      const int hi = min(max(Ua, Ub) + 1, mrel);
      const bool live = Ua >= 0 || Ub >= 0;
      const int cnt = (kk >= 0 && kk < nk && live) ? max(hi - lo + 1, 0) : 0;
      // (lanes 2 .. QB + 1 hold counts)
      vacc += cnt;
    }
    d += nk;
    if (newest_in_y) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int t = x[j];
        x[j] = y[j];
        y[j] = t;
      }
    }
    mx0 = ballot(x[0] != NEG); mx1 = ballot(x[1] != NEG);
    my0 = ballot(y[0] != NEG); my1 = ballot(y[1] != NEG);
    if ((mx0 | mx1 | my0 | my1) == 0) break;  // two dead antidiagonals
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    A[j] = x[j];
    B[j] = y[j];
  }
  e.base = base;
  e.d = d;
  e.W += (int64_t)(uint32_t)(QB + 2 <= 32 ? sum_lanes_0_31(vacc)
                                          : sum_lanes(vacc));
  if (bd >= 0) {
    e.T = tbest + gap * bd;
    e.bx = bxa;
    e.by = bd - bxa;
  }

  auto lo_of = [&](uint64_t m0, uint64_t m1) {
    return smin(m0 ? 2 * __builtin_ctzll(m0) : DEAD_L,
                m1 ? 2 * __builtin_ctzll(m1) + 1 : DEAD_L);
  };
  auto hi_of = [&](uint64_t m0, uint64_t m1) {
    return smax(m0 ? 2 * (63 - __builtin_clzll(m0)) : DEAD_U,
                m1 ? 2 * (63 - __builtin_clzll(m1)) + 1 : DEAD_U);
  };
  const bool lx = (mx0 | mx1) != 0, ly = (my0 | my1) != 0;
  e.L1 = lx ? base + lo_of(mx0, mx1) : DEAD_L;
  e.U1 = lx ? base + hi_of(mx0, mx1) : DEAD_U;
  e.L2 = ly ? base + lo_of(my0, my1) : DEAD_L;
  e.U2 = ly ? base + hi_of(my0, my1) : DEAD_U;
  int r = R_CONT;
  const int mv = window_move<ALPHA, C>(e, A, B, sy, w, S, e.L1, e.L2, e.U1,
                                       e.U2);
  if (mv == MV_ESC) r = R_ESC;
  else if (mv == MV_NONE) reload_syms<ALPHA, C>(e, sy, w, S);
  make_uniform(e);
  return r;
}

// Redistribute a window of C cells per lane into 2C cells per lane
// (same base; the upper half of the new window starts at -infinity).
template <int C>
__device__ __forceinline__ void widen(const int (&src)[C], int (&dst)[2 * C]) {
  const int lane = lane_id();
#pragma unroll
  for (int j = 0; j < 2 * C; ++j) {
    const int sl = 2 * lane + j / C;
    const int v = __builtin_amdgcn_ds_bpermute((sl & 63) << 2, src[j % C]);
    dst[j] = sl < 64 ? v : NEG;
  }
}

// Runs tier C (64*C cells per window) and widens in place (C -> 2C) while
// the band outgrows the window, up to CMAX.  A holds d-1 and B holds d-2 on
// entry.  The first call may ask for a wider starting tile (start > C); the
// state is then still the initial one and is widened before any step.
template <int ALPHA, int C, int CMAX>
__device__ __forceinline__ int run_tier(Ext& e, int (&A)[C], int (&B)[C], WaveLds<ALPHA>& w,
                        const int* tab, const Params& P, const Src& S,
                        int start, int& tier_out) {
  int r = R_ESC;
  if (start <= C) {
    Syms<ALPHA, C> sy;
    reload_syms<ALPHA, C>(e, sy, w, S);
    make_uniform(e);
    do {
      if constexpr (C == 1) {
        r = fast_interior<ALPHA>(e, A, B, sy, w, tab, P, S);
        if (r != R_CONT) break;
      } else if constexpr (C == 2) {
        r = fast_interior_multi<ALPHA, C>(e, A, B, sy, w, tab, P, S);
        if (r != R_CONT) break;
      }
      r = step<ALPHA, C>(e, A, B, sy, w, tab, P, S);
    } while (r == R_CONT);
  }
  if constexpr (C < CMAX) {
    if (r == R_ESC) {
      int N1[2 * C], N2[2 * C];
      widen<C>(A, N1);
      widen<C>(B, N2);
      return run_tier<ALPHA, 2 * C, CMAX>(e, N1, N2, w, tab, P, S, start,
                                          tier_out);
    }
  }
  tier_out = C;
  return r;
}

template <int ALPHA, int CMIN, int CMAX>
__device__ __forceinline__ int start_tier(Ext& e, WaveLds<ALPHA>& w, const int* tab,
                          const Params& P, const Src& S, int start,
                          int& tier_out) {
  int A[CMIN], B[CMIN];
#pragma unroll
  for (int j = 0; j < CMIN; ++j) { A[j] = NEG; B[j] = NEG; }
  if (lane_id() == 0) A[0] = 0;  // S(0,0) = 0 at window position 0
  return run_tier<ALPHA, CMIN, CMAX>(e, A, B, w, tab, P, S, start, tier_out);
}

// ------------------------------------------------------------------ items
struct ItemSetup {
  int status;
  Ext e;
};

__device__ __forceinline__ ItemSetup setup_item(const Params& P, int item) {
  ItemSetup s;
  s.status = S_OK;
  const int seed = item >> 1;
  const int right = item & 1;
  const int* sd = P.seeds + 5 * (int64_t)seed;
  // wave-uniform loads: readfirstlane keeps them (and the state derived
  // from them) in SGPRs
  const int q = uni(sd[0]), t = uni(sd[1]), qp = uni(sd[2]),
            tp = uni(sd[3]), k = uni(sd[4]);
  Ext& e = s.e;
  e.m = e.n = 0;
  if (q < 0 || q >= P.n_seqs || t < 0 || t >= P.n_seqs) {
    s.status = S_RANGE;
    return s;
  }
  const int64_t oq = uni64(P.offsets[q]), lq = uni64(P.offsets[q + 1]) - oq;
  const int64_t ot = uni64(P.offsets[t]), lt = uni64(P.offsets[t + 1]) - ot;
  if (k < 0 || qp < 0 || tp < 0 || qp + (int64_t)k > lq ||
      tp + (int64_t)k > lt) {
    s.status = S_RANGE;
    return s;
  }
  if (P.seq_bad && (uni(P.seq_bad[q]) == 2 || uni(P.seq_bad[t]) == 2)) {
    s.status = S_SYMBOL;
    return s;
  }
  int64_t m, n;
  if (!right) {
    m = qp; n = tp;
    e.a_start = oq + qp - 1; e.b_start = ot + tp - 1;
    e.a_dir = -1; e.b_dir = -1;
  } else {
    m = lq - qp - k; n = lt - tp - k;
    e.a_start = oq + qp + k; e.b_start = ot + tp + k;
    e.a_dir = 1; e.b_dir = 1;
  }
  if ((m + n) * (int64_t)P.max_abs > VALUE_LIMIT ||
      k * (int64_t)P.max_abs > VALUE_LIMIT) {
    s.status = S_RANGE;
    return s;
  }
  e.m = (int)m; e.n = (int)n;
  e.d = 1; e.base = 0;
  e.T = 0; e.bx = 0; e.by = 0;
  e.L1 = 0; e.U1 = 0;            // antidiagonal 0: S(0,0) = 0
  e.L2 = DEAD_L; e.U2 = DEAD_U;  // antidiagonal -1: empty
  e.W = 1;
  e.loaded_a = 0; e.loaded_b = 0;
  e.q = 0; e.qn = 0; e.qi = 0;
  return s;
}

__device__ __forceinline__ int tier_index(int C) {
  return C == 1 ? 0 : C == 2 ? 1 : C == 4 ? 2 : C == 8 ? 3 : 4;
}  // the block tier counts at index 5, the device-memory tier at 6, the
   // two-extension 16-bit kernel at 7

template <int ALPHA, int CMIN, int CMAX>
__device__ __forceinline__ void run_item(const Params& P, const Src& S, int item,
                         WaveLds<ALPHA>& w, const int* tab) {
  ItemSetup s = setup_item(P, item);
  ItemResult res;
  res.best = 0; res.x = 0; res.y = 0; res.status = s.status; res.cells = 0;
  res.tier = -1; res.pad = 0;
  bool handed_on = false;
  if (s.status == S_OK) {
    Ext& e = s.e;
    int r = R_DONE, tier = CMIN;
    if (e.m + e.n != 0) {
      const int start = CMIN > P.tile ? CMIN : P.tile;
      r = start_tier<ALPHA, CMIN, CMAX>(e, w, tab, P, S, start, tier);
    }
    if (r == R_ESC) {
      // band wider than the widest register window of one wave: restart the
      // extension on the block tier
      handed_on = true;
      if (lane_id() == 0) {
        const int slot = atomicAdd(P.counters + C_GEN_TAIL, 1);
        P.gen_queue[slot] = item;
      }
    } else if (r == R_CAP) {
      res.status = S_BAND;
    } else {
      res.best = e.T; res.x = e.bx; res.y = e.by; res.cells = e.W;
      res.tier = tier_index(tier);
    }
  }
  if (!handed_on && lane_id() == 0) P.items[item] = res;
}

// Persistent wave kernel: extensions of the batch pulled from the queue in
// chunks of P.chunk (or, in the plain form, one per launched wave), tiles of
// 1..CMAX cells per lane.  Occupancy targets, measured: six waves per SIMD
// for DNA (the compiler then keeps the kernel within 80 registers per lane;
// the one-cell loop, bound by issue with dependent steps, gains from the
// sixth wave) and seven for byte codes (72 registers, a few spills outside
// the sweep; 2.5% faster on protein-500k, while seven cost DNA 2%).
template <int ALPHA, int CMAX>
__global__ __launch_bounds__(WAVE * WPB) __attribute__((amdgpu_waves_per_eu(ALPHA == 1 ? 7 : 6)))
void xd_wave_kernel(Params P) {
  constexpr int CMIN = 1;
  __shared__ WaveLds<ALPHA> lds[WPB];
  __shared__ int tab[ALPHA == 1 ? TAB_WORDS : 1];
  if constexpr (ALPHA == 1) {
    fill_tab(tab, P);
    __syncthreads();
  }
  const int wid = threadIdx.x >> 6;
  WaveLds<ALPHA>& w = lds[wid];
  const Src S = make_src(P);
  if (P.flags & F_PLAIN) {
    const int idx = uni(blockIdx.x * WPB + wid);
    if (idx < P.n_items)
      run_item<ALPHA, CMIN, CMAX>(
          P, S, (P.flags & F_ORDERED) ? uni(P.order[idx]) : idx, w, tab);
    return;
  }
  // the extensions handed on by the row or 16-bit kernels, or the whole batch
  const bool esc = (P.flags & F_ESC) != 0;
  const int n_items =
      esc ? uni(__hip_atomic_load(P.counters + C_ESC_TAIL, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT))
          : P.n_items;
  if (esc && n_items == 0) return;  // nothing was handed on
  int cur = 0, end = 0;
  for (;;) {
    if (cur >= end) {
      // (a wave that finds the queue drained leaves without touching the
      // contended head)
      if (esc && uni(__hip_atomic_load(P.counters + C_ESC_HEAD,
                                       __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT)) >= n_items)
        break;
      int c = 0;
      if (lane_id() == 0)
        c = atomicAdd(P.counters + (esc ? C_ESC_HEAD : C_HEAD), P.chunk);
      cur = uni(c);
      end = min(cur + P.chunk, n_items);
      if (cur >= n_items) break;
    }
    const int idx = cur++;
    const int item = esc ? uni(P.esc_queue[idx])
                     : (P.flags & F_ORDERED) ? uni(P.order[idx]) : idx;
    run_item<ALPHA, CMIN, CMAX>(P, S, item, w, tab);
  }
}

// ------------------------------------------------------------------ rows
// Several extensions per wavefront for narrow bands: the 64 lanes form R
// rows of W = 64 / R lanes (R = 2: 32-cell windows, the pair form; R = 4:
// 16-lane rows), each row one extension with one cell per lane (lane W*h + p
// holds window position p of row h), so every vector instruction of the
// sweep serves R extensions.  Each row keeps its own antidiagonal, window
// and scalar state, and takes the next extension from the queue when its
// own ends.  The sweep is the one-cell loop of the wave kernel on R windows:
//  * blocks of RKB antidiagonals on finite-lane ballots, whose W-bit fields
//    are the rows' masks; blocks clear of the matrix edges of every row skip
//    the edge masks;
//  * the top G lanes of each row are -infinity at the start of every group
//    of G antidiagonals, so the wave rotation brings -infinity to each row's
//    lane 0, and the band is tested against the top every G-th step; a band
//    that reaches the top slides its row's window up in place (`ds_bpermute`
//    within the row);
//  * thresholds are per lane: a lane compares v - T0 of its row (T in the
//    frame of the block's first antidiagonal) with two running scalars that
//    move by -gap per antidiagonal;
//  * a new best is found for every row at once: each lane takes the
//    maximum of its row's improving cells (DPP maxima within the row) and
//    the lowest lane among equals from one ballot, and keeps step, lane and
//    value for its row in three registers until the block ends (per-row
//    scalar bookkeeping in the steps had spilled the scalar registers);
//  * the test of every fourth step is one check over the 64-bit mask: a
//    live row with no finite lane in the last two antidiagonals (a zero
//    W-bit field, idle rows filled with ones) or a finite top lane;
//  * live-span cells are counted per block and row from the masks kept in
//    lanes of two registers (the ballot's low and high words);
//  * byte scores come from per-lane ring reads at immediate offsets, DNA
//    scores from per-block match words;
//  * the state a block does not touch stays in LDS between blocks, so the
//    block keeps its scalar registers for the sweep.
// Each row's sequences stream through rings of their own, half the size of
// the wave kernel's (a row's window is at most 32 cells).  An extension
// whose band fills its row (W - G cells) is handed on to the wave kernel,
// which restarts it.

// Rings of one row: 2,048 DNA codes or 1,024 byte codes.
template <int ALPHA>
using RowRing = RingT<ALPHA, ALPHA == 0 ? 2048 : 1024, WAVE>;

template <int ALPHA>
struct RowWin {
  uint32_t ra[RowRing<ALPHA>::WORDS];
  uint32_t rb[RowRing<ALPHA>::WORDS];
};

// State of a row's extension that the sweep does not touch between block
// boundaries.
struct RowCold {
  int64_t a_start, b_start, W;  // sources, live-span cells so far
  int a_dir, b_dir, loaded_a, loaded_b;  // ring levels
  int bd, bxa, tbest;  // last new best: antidiagonal (-1: none), x, V value
};

template <int ALPHA, int R>
struct RowLds {
  RowWin<ALPHA> h[R];
  RowCold c[R];
};

// Uniform state of one row's extension kept in scalar registers.
struct RowHot {
  int item;         // -1: none
  int m, n;         // lengths
  int d, base;      // next antidiagonal, window position 0 = x of base
  int tv0;          // T in the V frame of antidiagonal d
  uint32_t m1, m2;  // finite lanes of d - 1 and d - 2
};

// Fills a row's ring up to element need_hi (the ring keeps the RS below).
template <int ALPHA>
__device__ __forceinline__ void row_cover(uint32_t* ring, const Src& S,
                                          int64_t start, int dir, int& loaded,
                                          int need_hi) {
  while (loaded <= need_hi) {
    RowRing<ALPHA>::fill(ring, S, start, dir, loaded, lane_id());
    loaded += RowRing<ALPHA>::CH;
  }
  __builtin_amdgcn_wave_barrier();
}

// Every lane: the maximum of v over the lanes of its row (rows of W lanes).
template <int W>
__device__ __forceinline__ int row_max_v(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xf, 0xf, false));
  // (each 16-lane hardware row now holds its maximum in every lane)
  if constexpr (W == 16) return v;
  const int lo = smax(__builtin_amdgcn_readlane(v, 0),
                      __builtin_amdgcn_readlane(v, 16));
  const int hi = smax(__builtin_amdgcn_readlane(v, 32),
                      __builtin_amdgcn_readlane(v, 48));
  return lane_id() < 32 ? lo : hi;
}

// The lane's row's entry of a per-row array.
template <int R>
__device__ __forceinline__ int row_sel(const int (&a)[R], int hf) {
  if constexpr (R == 2)
    return hf ? a[1] : a[0];
  else
    return (hf & 2) ? ((hf & 1) ? a[3] : a[2]) : ((hf & 1) ? a[1] : a[0]);
}

constexpr int RKB = 48;  // antidiagonals per block of the row sweep

// Result of a finished row's extension (tier: 4 for two rows, 8 for four).
__device__ __forceinline__ void row_finish(const Params& P, const RowHot& H,
                                           const RowCold& c, int gap,
                                           int tier) {
  ItemResult r;
  r.status = S_OK;
  r.cells = uni64(c.W);
  r.tier = tier; r.pad = 0;
  const int bd = uni(c.bd);
  if (bd >= 0) {
    const int bxa = uni(c.bxa);
    r.best = uni(c.tbest) + gap * bd;
    r.x = bxa;
    r.y = bd - bxa;
  } else {
    r.best = 0; r.x = 0; r.y = 0;
  }
  if (lane_id() == 0) P.items[H.item] = r;
}

template <int ALPHA, int R>
__device__ __forceinline__ void run_rows(const Params& P, const Src& S,
                                         RowLds<ALPHA, R>& L, const int* tab) {
  constexpr int W = WAVE / R;
  constexpr int KB = RKB;
  static_assert(KB % 16 == 0 && KB + 2 <= 64, "match words; mask lanes");
  constexpr int G = 4;
  constexpr uint32_t RM = (uint32_t)((1ull << W) - 1);  // row bits
  constexpr int TIER = R == 2 ? 4 : 8;  // result tier index
  constexpr int BIG = 1 << 29;  // T of an idle row: no cell passes
  // the top G lanes of every row; the lowest and highest lane of every row
  constexpr uint64_t TOPS = R == 2 ? 0xF0000000F0000000ull
                                   : 0xF000F000F000F000ull;
  constexpr uint64_t LOW1 = R == 2 ? 0x0000000100000001ull
                                   : 0x0001000100010001ull;
  constexpr uint64_t HIGH1 = LOW1 << (W - 1);
  static_assert(R == 2 || R == 4, "rows of 32 or 16 lanes");
  static_assert(RowRing<ALPHA>::RS >= KB + 34 + RowRing<ALPHA>::CH,
                "a fill keeps the codes a block still reads");
  const int lane = lane_id();
  const int hf = lane / W, p = lane % W;
  const int gap = P.gap, X = smin(P.X, 1 << 29);  // see fast_interior
  const int vmat = in_vgpr(P.mat_s), vmis = in_vgpr(P.mis_s);
  RowHot H[R];
#pragma unroll
  for (int h = 0; h < R; ++h) {
    H[h].item = -1;
    H[h].m1 = H[h].m2 = 0;  // (idle rows: no lanes)
    H[h].d = H[h].base = H[h].m = H[h].n = 0;
    H[h].tv0 = 0;
  }
  int x = NEG, y = NEG;  // antidiagonals d-1 and d-2 of the lane's row
  // DNA: the lane's query code in all 16 code slots of a word; bytes: the
  // byte offset of its score-table row
  uint32_t fa = 0;
  auto load_fa = [&](int h) {
    const uint32_t* ra = L.h[h].ra;
    uint32_t f;
    if constexpr (ALPHA == 0) {
      f = (RowRing<0>::read(ra, H[h].base + p - 1) & 3u) * 0x55555555u;
    } else {
      uint32_t t[1];
      RowRing<1>::read<1>(ra, H[h].base + p - 1, t);
      f = (t[0] & 31u) * (4 * TAB_LD);
    }
    fa = hf == h ? f : fa;
  };
  auto score = [&](uint32_t c) {
    return *reinterpret_cast<const int*>(
        reinterpret_cast<const char*>(tab) + fa + (c << 2));
  };
  bool drained = false;
  int cur = 0, end = 0;  // queue slots claimed, P.chunk at a time
  for (;;) {
    // idle rows take the next extensions
#pragma unroll
    for (int h = 0; h < R; ++h) {
      while (H[h].item < 0 && !drained) {
        if (cur >= end) {
          int c = 0;
          if (lane == 0) c = atomicAdd(P.counters + C_PAIR_HEAD, P.chunk);
          cur = uni(c);
          end = min(cur + P.chunk, P.n_items);
          if (cur >= P.n_items) { drained = true; break; }
        }
        const int c = cur++;
        const int item = (P.flags & F_ORDERED) ? uni(P.order[c]) : c;
        ItemSetup st = setup_item(P, item);
        if (st.status != S_OK || st.e.m + st.e.n == 0) {
          ItemResult r;
          r.best = 0; r.x = 0; r.y = 0; r.status = st.status;
          r.cells = st.status == S_OK ? 1 : 0;
          r.tier = st.status == S_OK ? TIER : -1; r.pad = 0;
          if (lane == 0) P.items[item] = r;
          continue;
        }
        RowHot& Hh = H[h];
        Hh.item = item;
        Hh.m = st.e.m; Hh.n = st.e.n;
        Hh.d = 1; Hh.base = 0;
        Hh.tv0 = -gap;  // T = 0 in the frame of antidiagonal 1
        Hh.m1 = 1;  // antidiagonal 0: S(0,0) = 0 at window position 0
        Hh.m2 = 0;
        x = hf == h ? (p == 0 ? 0 : NEG) : x;
        y = hf == h ? NEG : y;
        int la = 0;
        row_cover<ALPHA>(L.h[h].ra, S, st.e.a_start, st.e.a_dir, la, W - 2);
        RowCold& rc = L.c[h];
        rc.a_start = st.e.a_start; rc.b_start = st.e.b_start; rc.W = 1;
        rc.a_dir = st.e.a_dir; rc.b_dir = st.e.b_dir;
        rc.loaded_a = la; rc.loaded_b = 0;
        rc.bd = -1; rc.bxa = 0; rc.tbest = 0;
        __builtin_amdgcn_wave_barrier();
        load_fa(h);
      }
    }
    // idle rows' lanes (all bits of their mask fields)
    uint64_t idle = 0;
#pragma unroll
    for (int h = 0; h < R; ++h)
      if (H[h].item < 0) idle |= (uint64_t)RM << (W * h);
    if (idle == ~0ull) break;

    // ---- one block of antidiagonals of every row
    int pm[R], mrel[R], e0[R], tvr[R];
    int remmin = KB;  // antidiagonals left after d, over the live rows
    bool edge = false;
#pragma unroll
    for (int h = 0; h < R; ++h) {
      RowHot& Hh = H[h];
      if (Hh.item < 0) {
        pm[h] = -KB; mrel[h] = W - 1; e0[h] = 0;
        tvr[h] = BIG;
        continue;
      }
      pm[h] = Hh.d - Hh.n - Hh.base;
      mrel[h] = Hh.m - Hh.base;
      const int rem = Hh.m + Hh.n - Hh.d;
      remmin = smin(remmin, rem);
      tvr[h] = Hh.tv0;
      if (!(pm[h] + KB - 1 <= 0 && mrel[h] >= W - 1 && rem >= KB - 1))
        edge = true;
      e0[h] = Hh.d - Hh.base;
      RowCold& rc = L.c[h];
      int lb = uni(rc.loaded_b);
      if (lb <= e0[h] + KB - 1) {
        row_cover<ALPHA>(L.h[h].rb, S, uni64(rc.b_start), uni(rc.b_dir), lb,
                         e0[h] + KB - 1);
        rc.loaded_b = lb;
      }
    }
    // per lane: its row's values
    const int pq = p - row_sel<R>(pm, hf);  // y <= n from step pq on
    const uint64_t in_m = ballot(p <= row_sel<R>(mrel, hf));
    int tv0_v = row_sel<R>(tvr, hf);
    const int e0_l = row_sel<R>(e0, hf);
    uint32_t mw[KB / 16] = {};  // DNA: match words of the block
    const uint32_t* rb_l = L.h[0].rb;
#pragma unroll
    for (int h = 1; h < R; ++h) rb_l = hf == h ? L.h[h].rb : rb_l;
    const uint8_t* cp = reinterpret_cast<const uint8_t*>(rb_l);
    int sc_next = 0;
    uint32_t cd1 = 0, cd2 = 0;
    if constexpr (ALPHA == 0) {
#pragma unroll
      for (int i = 0; i < KB / 16; ++i) {
        const uint32_t xw = RowRing<0>::read(rb_l, e0_l - p - 1 + 16 * i) ^ fa;
        mw[i] = ~(xw | (xw >> 1)) & 0x55555555u;
      }
    } else {
      // (reads up to KB + 2 bytes past a position of the ring, which its
      // mirror words cover; codes past those covered belong to no step)
      cp += (e0_l - p - 1) & (RowRing<1>::RS - 1);
      sc_next = score(cp[0]);
      cd1 = cp[1];
      cd2 = cp[2];
    }
    // finite-lane masks of the block's antidiagonals, the ballot's low word
    // in lanes of ml and its high word in lanes of mh: lanes 0 and 1 the two
    // antidiagonals before the block, lane k + 2 the k-th
    uint64_t a1 = 0, a2 = 0;
#pragma unroll
    for (int h = 0; h < R; ++h) {
      a1 |= (uint64_t)H[h].m1 << (W * h);
      a2 |= (uint64_t)H[h].m2 << (W * h);
    }
    int ml = 0, mh = 0;
    ml = xd_writelane_i32((int)(uint32_t)a2, 0, ml);
    mh = xd_writelane_i32((int)(uint32_t)(a2 >> 32), 0, mh);
    ml = xd_writelane_i32((int)(uint32_t)a1, 1, ml);
    mh = xd_writelane_i32((int)(uint32_t)(a1 >> 32), 1, mh);
    // new bests of the block, per lane for its row: step (-1: none), lane,
    // V value
    int bk_v = -1, bln_v = 0, tb_v = 0;
    int nk = KB;
    bool newest_in_y = false;
    // running -k * gap and -k * gap - X of step k (set for k = -1)
    uint32_t ck = (uint32_t)gap, thc = (uint32_t)(gap - X);
    // antidiagonal d_h + k of every row from prev (d-1, masks mp) and pp
    // (d-2, masks mpp); pp and mpp receive d.  True when a live row's band
    // reached its top lanes or had two dead antidiagonals (tested every G),
    // or at a row's last antidiagonal (edge blocks).
    auto body = [&](auto edge_tag, int& prev, int& pp, const uint64_t& mp,
                    uint64_t& mpp, int k) -> bool {
      constexpr bool EDGE = decltype(edge_tag)::value;
      int sim;
      if constexpr (ALPHA == 0) {
        int t = __builtin_amdgcn_sbfe((int)mw[k >> 4], 2 * (k & 15), 1);
        opaque_v(t);  // (one v_bfi below, not compare + select)
        sim = (t & vmat) | (~t & vmis);
        opaque_v(sim);
      } else {
        sim = sc_next;
        sc_next = score(cd1);
        cd1 = cd2;
        int c3 = cp[k + 3];  // (zero extension kept with the load)
        opaque_v(c3);
        cd2 = (uint32_t)c3;
      }
      const int up = __builtin_amdgcn_update_dpp(0, prev, 0x13C, 0xf, 0xf, true);
      const int dg = __builtin_amdgcn_update_dpp(0, pp, 0x13C, 0xf, 0xf, true);
      int uh = max(up, prev);
      opaque_v(uh);
      const int v = max(uh, dg + sim);
      // T of the lane's row at this antidiagonal is T0 + ck (ck and the
      // threshold kept as running scalars, which the compiler would
      // otherwise precompute for every step of the block)
      ck -= gap;
      thc -= gap;
      opaque_s(ck);
      opaque_s(thc);
      const int t = v - tv0_v;
      uint64_t fm = ballot(t >= (int)thc);
      if constexpr (EDGE)  // y > n below pm + k, x > m above mrel
        fm &= ballot(pq >= k) & in_m;
      const int vn = __builtin_amdgcn_inverse_ballot_w64(fm) ? v : NEG;
      uint64_t imp = ballot(t > (int)ck);
      if constexpr (EDGE) imp &= fm;
      int vk = vn;
      pin_v(vk);
      pp = vk;
      if (__builtin_expect(imp != 0, 0)) {
        // every row at once: its highest improving cell, the lowest lane
        // among equals (the rows' improving cells are above all others)
        const int vi = __builtin_amdgcn_inverse_ballot_w64(imp) ? vn : NEG;
        const int wm = row_max_v<W>(vi);
        const uint64_t eq = ballot(vi == wm);
        const int l0 = __builtin_ctz((uint32_t)(eq >> (W * hf)) | 0x80000000u);
        if (wm != NEG) {
          tv0_v = wm - (int)ck;
          bk_v = k;
          bln_v = l0;
          tb_v = wm;
        }
      }
      mpp = fm;
      ml = xd_writelane_i32((int)(uint32_t)fm, k + 2, ml);
      mh = xd_writelane_i32((int)(uint32_t)(fm >> 32), k + 2, mh);
      bool stop = false;
      if ((k & (G - 1)) == G - 1) {
        // a live row with no finite lane in the two antidiagonals (a zero
        // W-bit field of o, idle rows filled), or finite top lanes
        const uint64_t o = mp | fm, oi = o | idle;
        if ((((oi - LOW1) & ~oi & HIGH1) | (o & TOPS)) != 0) stop = true;
      }
      if constexpr (EDGE)
        if (k >= remmin) stop = true;
      return stop;
    };
    auto run_block = [&](auto edge_tag) {
#pragma unroll
      for (int k = 0; k < KB; k += 2) {
        if (body(edge_tag, x, y, a1, a2, k)) {
          nk = k + 1; newest_in_y = true; return;
        }
        if (body(edge_tag, y, x, a2, a1, k + 1)) { nk = k + 2; return; }
      }
    };
    if (edge) run_block(std::true_type{});
    else run_block(std::false_type{});
    if (newest_in_y) {
      const int t = x;
      x = y;
      y = t;
    }
    // live-span cells of the block's antidiagonals per row: lane k + 2
    // forms antidiagonal k's span from the masks of the two before it (lanes
    // k + 1 and k): lo = ctz(M1 | M2 << 1), hi = index of the top bit of
    // M1 | M2, plus 1 (M2 never holds the row's top lane), clamped to the
    // matrix
    const uint32_t al = (uint32_t)wave_shr1(ml, 0), ah = (uint32_t)wave_shr1(mh, 0);
    const uint32_t bl = (uint32_t)wave_shr1((int)al, 0), bh = (uint32_t)wave_shr1((int)ah, 0);
    const int kk = lane - 2;
    int64_t acc[R];
#pragma unroll
    for (int h = 0; h < R; ++h) {
      if (H[h].item >= 0) {  // (recomputed: not kept over the block)
        uint32_t dh = (uint32_t)H[h].d;
        opaque_s(dh);
        pm[h] = (int)dh - H[h].n - H[h].base;
        mrel[h] = H[h].m - H[h].base;
      }
      const int sh = (h * W) & 31;
      const uint32_t a = ((h * W < 32 ? al : ah) >> sh) & RM;
      const uint32_t b = ((h * W < 32 ? bl : bh) >> sh) & RM;
      const int lo = max((int)__builtin_ctzg(a | (b << 1), 32), pm[h] + kk);
      const int hi = min(32 - (int)__builtin_clzg(a | b, 32), mrel[h]);
      const int cnt = (kk >= 0 && kk < nk && (a | b) != 0) ? max(hi - lo + 1, 0)
                                                          : 0;
      acc[h] = sum_lanes(cnt);
    }
    // ---- after the block: advance and see to each row
    const uint64_t f1 = ballot(x != NEG), f2 = ballot(y != NEG);
#pragma unroll
    for (int h = 0; h < R; ++h) {
      RowHot& Hh = H[h];
      if (Hh.item < 0) continue;
      RowCold& rc = L.c[h];
      const int bk = __builtin_amdgcn_readlane(bk_v, W * h);
      if (bk >= 0) {  // a new best in this block
        rc.bd = Hh.d + bk;
        rc.bxa = Hh.base + __builtin_amdgcn_readlane(bln_v, W * h);
        rc.tbest = __builtin_amdgcn_readlane(tb_v, W * h);
      }
      Hh.d += nk;
      rc.W = uni64(rc.W) + acc[h];
      // T in the frame of the next antidiagonal
      Hh.tv0 = __builtin_amdgcn_readlane(tv0_v, W * h) - nk * gap;
      Hh.m1 = (uint32_t)(f1 >> (W * h)) & RM;
      Hh.m2 = (uint32_t)(f2 >> (W * h)) & RM;
      const uint32_t o = Hh.m1 | Hh.m2;
      if (o == 0 || Hh.d > Hh.m + Hh.n) {
        __builtin_amdgcn_wave_barrier();
        row_finish(P, Hh, rc, gap, TIER);
        Hh.item = -1;
        Hh.m1 = Hh.m2 = 0;
        x = hf == h ? NEG : x;
        y = hf == h ? NEG : y;
        continue;
      }
      const int cz = (int)__builtin_clz(o) - (32 - W);  // free lanes on top
      if (cz < G) {
        // the band reached the top lanes: slide the window up by the lanes
        // below its lowest finite cell, or hand the extension on
        const int sl = (int)__builtin_ctz(o);
        if (cz + sl < G) {
          if (lane == 0) {
            const int slot = atomicAdd(P.counters + C_ESC_TAIL, 1);
            P.esc_queue[slot] = Hh.item;
          }
          Hh.item = -1;
          Hh.m1 = Hh.m2 = 0;
          x = hf == h ? NEG : x;
          y = hf == h ? NEG : y;
          continue;
        }
        const int src = lane + sl;
        const bool inw = p + sl < W;
        const int px = __builtin_amdgcn_ds_bpermute((src & 63) << 2, x);
        const int py = __builtin_amdgcn_ds_bpermute((src & 63) << 2, y);
        x = hf == h ? (inw ? px : NEG) : x;
        y = hf == h ? (inw ? py : NEG) : y;
        Hh.m1 >>= sl;
        Hh.m2 >>= sl;
        Hh.base += sl;
        int la = uni(rc.loaded_a);
        if (la <= Hh.base + W - 2) {
          row_cover<ALPHA>(L.h[h].ra, S, uni64(rc.a_start), uni(rc.a_dir), la,
                           Hh.base + W - 2);
          rc.loaded_a = la;
        }
        __builtin_amdgcn_wave_barrier();
        load_fa(h);
      }
    }
  }
}

// Persistent row kernel: R rows per wave take extensions of the
// (longest-first) order from the device queue as they become free.
template <int ALPHA, int R>
__global__ __launch_bounds__(WAVE * WPB) void xd_rows_kernel(Params P) {
  __shared__ RowLds<ALPHA, R> lds[WPB];
  __shared__ int tab[ALPHA == 1 ? TAB_WORDS : 1];
  if constexpr (ALPHA == 1) {
    fill_tab(tab, P);
    __syncthreads();
  }
  const int wid = threadIdx.x >> 6;
  const Src S = make_src(P);
  run_rows<ALPHA, R>(P, S, lds[wid], tab);
}

// ------------------------------------------------------------------ dual16
// Two extensions per wavefront in the two 16-bit halves of every register
// (the paper changed the ALU type of its inner loop for dual issue, Sec.
// 4.1.4; here packed 16-bit integer operations do the work of two
// extensions at once): lane l holds window position l of extension 0 in the
// low half and of extension 1 in the high half, one cell per lane each, and
// one v_pk_max_i16 / v_pk_add_i16 advances both.  Scores are kept relative:
// a register half holds V - off_h (V = S - gap*d, as in the wave kernel),
// and after every block of antidiagonals each half is rebased so that its
// best score sits at 0; every finite value then stays within
// [-X - 3*max_abs, 33*max_abs], which the host checks fits 16 bits (else
// the batch runs on the int32 wave kernel).  -infinity is -32768 and the
// adds saturate, so it stays below every threshold.  Each half runs its own
// extension at its own antidiagonal and window; when one ends, that half
// takes the next extension from the queue while the other goes on.  The
// band bookkeeping follows the one-cell loop of the wave kernel (finite-lane
// ballots, four guard lanes at the window top, the window sliding up in
// place); a band that fills the window is handed on to the wave kernel,
// which restarts the extension.
typedef short xd_short2 __attribute__((ext_vector_type(2)));
typedef unsigned short xd_ushort2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_add_sat(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(
      uint32_t, __builtin_elementwise_add_sat(__builtin_bit_cast(xd_short2, a),
                                              __builtin_bit_cast(xd_short2, b)));
}
__device__ __forceinline__ uint32_t pk_sub_sat(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(
      uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(xd_short2, a),
                                              __builtin_bit_cast(xd_short2, b)));
}
__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(
      uint32_t, __builtin_elementwise_max(__builtin_bit_cast(xd_short2, a),
                                          __builtin_bit_cast(xd_short2, b)));
}
__device__ __forceinline__ uint32_t pack16(int lo, int hi) {
  return ((uint32_t)lo & 0xFFFFu) | ((uint32_t)hi << 16);
}
__device__ __forceinline__ int half16(uint32_t v, int h) {
  return h ? (int)(short)(v >> 16) : (int)(short)v;
}

constexpr int NEG16 = -32768;
constexpr uint32_t NEG2 = 0x80008000u;
// the host runs a batch here only if X + DUAL_SPAN * max_abs fits 16 bits
constexpr int DUAL_SPAN = 40;

template <int ALPHA>
struct DualLds {
  WaveLds<ALPHA> h[2];
};

// Uniform state of one half's extension.
struct DualHalf {
  Ext e;        // lengths, sources, ring levels, d, base (other fields unused)
  int item;     // -1: none
  int off;      // register half = V - off
  int tv;       // T in the frame of antidiagonal e.d, relative (V - off)
  int bd, bln;  // last new best: antidiagonal and lane (bd < 0: none yet)
  int bxa;      // its x
  uint64_t m1, m2;  // finite lanes of e.d - 1 and e.d - 2
};

// Starts `item` in half h (registers x: antidiagonal 0, y: antidiagonal -1).
// Returns false (result written, half left idle) for an extension that
// needs no sweep or has a bad seed.
template <int ALPHA>
__device__ __forceinline__ bool dual_start(const Params& P, const Src& S,
                                           int item, int h, DualHalf& H,
                                           WaveLds<ALPHA>& w, uint32_t& x,
                                           uint32_t& y, uint32_t& fa2,
                                           uint32_t& fb2) {
  const int lane = lane_id();
  ItemSetup st = setup_item(P, item);
  if (st.status != S_OK || st.e.m + st.e.n == 0) {
    ItemResult r;
    r.best = 0; r.x = 0; r.y = 0; r.status = st.status;
    r.cells = st.status == S_OK ? 1 : 0;
    r.tier = st.status == S_OK ? 7 : -1; r.pad = 0;
    if (lane == 0) P.items[item] = r;
    return false;
  }
  H.e = st.e;
  H.item = item;
  H.off = 0;
  H.tv = -P.gap;  // T = 0 in the frame of antidiagonal 1
  H.bd = -1; H.bln = 0; H.bxa = 0;
  H.m1 = 1;  // antidiagonal 0: S(0,0) = 0 at lane 0
  H.m2 = 0;
  const uint32_t hm = h ? 0xFFFF0000u : 0x0000FFFFu;
  x = (x & ~hm) | ((lane == 0 ? 0u : NEG2) & hm);
  y = (y & ~hm) | (NEG2 & hm);
  cover_a<ALPHA>(H.e, w, S, 62);
  cover_b<ALPHA>(H.e, w, S, 0);
  if constexpr (ALPHA == 1) {
    uint32_t t[1];
    Ring<1>::read<1>(w.ra, lane - 1, t);
    const uint32_t fa = (t[0] & 31u) << 6;  // byte offset of the table row
    Ring<1>::read<1>(w.rb, -lane, t);       // b[d - base - lane - 1], d = 1
    const uint32_t fb = (t[0] & 31u) << 1;
    fa2 = (fa2 & ~hm) | ((fa << (16 * h)) & hm);
    fb2 = (fb2 & ~hm) | ((fb << (16 * h)) & hm);
  } else {
    const uint32_t fa = (Ring<0>::read(w.ra, lane - 1) & 3u) * 0x55555555u;
    fa2 = h ? fa2 : fa;  // (DNA: query codes of half h kept in fa2 / fb2)
    fb2 = h ? fa : fb2;
  }
  return true;
}

template <int ALPHA>
__device__ __forceinline__ void run_dual(const Params& P, const Src& S,
                                         DualLds<ALPHA>& L,
                                         const int16_t* tab16) {
  const int lane = lane_id();
  const int gap = P.gap, X = P.X;
  DualHalf H[2];
  H[0].item = H[1].item = -1;
  uint32_t x = NEG2, y = NEG2;  // x: antidiagonal d-1, y: d-2 (both halves)
  uint32_t fa2 = 0, fb2 = 0;    // bytes: table row / column offsets;
                                // DNA: query codes of half 0 / half 1
  bool drained = false;
  constexpr int KB = 32;        // antidiagonals per block
  constexpr int G = 4;          // guard lanes at the window top
  const uint32_t vmat2 = (uint32_t)in_vgpr((int)pack16(P.mat_s, P.mat_s));
  const uint32_t vmis2 = (uint32_t)in_vgpr((int)pack16(P.mis_s, P.mis_s));
  int cur = 0, end = 0;  // slots claimed from the queue, P.chunk at a time
  for (;;) {
    // idle halves take the next extensions
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      while (H[h].item < 0 && !drained) {
        if (cur >= end) {
          int c = 0;
          if (lane == 0) c = atomicAdd(P.counters + C_HEAD, P.chunk);
          cur = uni(c);
          end = min(cur + P.chunk, P.n_items);
          if (cur >= P.n_items) { drained = true; break; }
        }
        const int c = cur++;
        const int item = (P.flags & F_ORDERED) ? uni(P.order[c]) : c;
        dual_start<ALPHA>(P, S, item, h, H[h], L.h[h], x, y, fa2, fb2);
      }
    }
    const bool live0 = H[0].item >= 0, live1 = H[1].item >= 0;
    if (!live0 && !live1) break;
    // ---- one block of antidiagonals for both halves
    int pm[2], mrel[2], rem[2], d0[2];
    bool edge = false;
    uint32_t qw[2][8];   // bytes: codes entering lane 0, per half
    uint32_t mw[2][2];   // DNA: match words per half
    uint32_t mp2[4];     // DNA: steps 8i .. 8i + 7, half 0 low, half 1 high
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      DualHalf& Hh = H[h];
      d0[h] = Hh.e.d;
      if (Hh.item < 0) {
        pm[h] = 0; mrel[h] = 63; rem[h] = KB;
#pragma unroll
        for (int i = 0; i < 8; ++i) qw[h][i] = 0;
        mw[h][0] = mw[h][1] = 0;
        continue;
      }
      pm[h] = Hh.e.d - Hh.e.n - Hh.e.base;
      mrel[h] = Hh.e.m - Hh.e.base;
      rem[h] = Hh.e.m + Hh.e.n - Hh.e.d;  // antidiagonals left after d
      if (!(pm[h] + KB - 1 <= 0 && mrel[h] >= 63 && rem[h] >= KB - 1))
        edge = true;
      const int e0 = Hh.e.d - Hh.e.base;
      cover_b<ALPHA>(Hh.e, L.h[h], S, e0 + KB - 1);
      if constexpr (ALPHA == 1) {
        // codes doubled (byte offsets of table columns; codes < 32, so no
        // byte carries into the next)
        Ring<1>::read<8>(L.h[h].rb, e0, qw[h]);
#pragma unroll
        for (int i = 0; i < 8; ++i)
          qw[h][i] = (uint32_t)in_vgpr((int)((qw[h][i] & 0x1F1F1F1Fu) << 1));
      } else {
        const uint32_t fa = h ? fb2 : fa2;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const uint32_t xw =
              Ring<0>::read(L.h[h].rb, e0 - lane - 1 + 16 * i) ^ fa;
          mw[h][i] = ~(xw | (xw >> 1)) & 0x55555555u;
        }
      }
    }
    // an idle half (all -infinity) never passes its threshold and never
    // improves: its T sits at the top of the 16-bit range
    int tv0 = live0 ? H[0].tv : 0x7FFF, tv1 = live1 ? H[1].tv : 0x7FFF;
    if constexpr (ALPHA == 0) {
      // low 16 bits of half 0's word beside those of half 1's (steps 0-7 of
      // the word), then the high 16 bits (steps 8-15)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        mp2[2 * i] = __builtin_amdgcn_perm(mw[1][i], mw[0][i], 0x05040100u);
        mp2[2 * i + 1] = __builtin_amdgcn_perm(mw[1][i], mw[0][i], 0x07060302u);
      }
    }
    uint64_t a1[2] = {H[0].m1, H[1].m1}, a2[2] = {H[0].m2, H[1].m2};
    int bd[2] = {H[0].bd, H[1].bd}, bln[2] = {H[0].bln, H[1].bln};
    // finite-lane masks of the block's antidiagonals for the live-span
    // count, per half in lanes of two registers (low and high words): lanes
    // 0 and 1 the two antidiagonals before the block, lane k + 2 the k-th
    int ml[2] = {0, 0}, mh[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      ml[h] = xd_writelane_i32((int)(uint32_t)a2[h], 0, ml[h]);
      mh[h] = xd_writelane_i32((int)(uint32_t)(a2[h] >> 32), 0, mh[h]);
      ml[h] = xd_writelane_i32((int)(uint32_t)a1[h], 1, ml[h]);
      mh[h] = xd_writelane_i32((int)(uint32_t)(a1[h] >> 32), 1, mh[h]);
    }
    const uint32_t xhi = ((uint32_t)X << 16) | 0xFFFFu;
    int nk = KB;
    bool newest_in_y = false;
    // antidiagonal d_h + k of both halves: prev (d-1, masks mp), pp (d-2,
    // masks mpp) -> pp, mpp.  True when a live half's band reached the guard
    // lanes, or it had two dead antidiagonals (tested every G), or at its
    // last antidiagonal (edge blocks).
    auto body = [&](auto edge_tag, uint32_t& prev, uint32_t& pp,
                    uint64_t (&mp)[2], uint64_t (&mpp)[2], int k) -> bool {
      constexpr bool EDGE = decltype(edge_tag)::value;
      const uint32_t thr2 = pack16(tv0 - X, tv1 - X);
      uint32_t sim2;
      if constexpr (ALPHA == 1) {
        const uint32_t a2v = fa2 + fb2;  // (no carry between the halves)
        const int s0 = tab16[(a2v & 0xFFFFu) >> 1];
        const int s1 = tab16[a2v >> 17];
        sim2 = pack16(s0, s1);
      } else {
        // match bit of both halves to bit 15 of each, then spread it over
        // the half: 0xFFFF on a match
        const uint32_t sh = (uint32_t)(15 - 2 * (k & 7));
        int sel = (int)__builtin_bit_cast(
            uint32_t, __builtin_bit_cast(xd_ushort2, mp2[k >> 3]) << (unsigned short)sh);
        sel = (int)__builtin_bit_cast(
            uint32_t, __builtin_bit_cast(xd_short2, (uint32_t)sel) >> (short)15);
        opaque_v(sel);  // (one v_bfi below, not compares and selects)
        sim2 = (vmat2 & (uint32_t)sel) | (vmis2 & ~(uint32_t)sel);
      }
      const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)prev, 0x13C, 0xf, 0xf, false);
      const uint32_t dg = (uint32_t)__builtin_amdgcn_mov_dpp((int)pp, 0x13C, 0xf, 0xf, false);
      const uint32_t v = pk_max(pk_max(up, prev), pk_add_sat(dg, sim2));
      // per half v - thr: not negative exactly when the cell survives (and
      // exact up to X + max_abs, far below the 16-bit limit)
      const uint32_t r = pk_sub_sat(v, thr2);
      uint64_t f0 = ballot((int)(short)r >= 0);
      uint64_t f1 = ballot((int)r >= 0);
      uint32_t vn;
      if constexpr (EDGE) {
        // cells outside the matrix: y > n below pm, x > m above mrel
        f0 &= ballot((uint32_t)(lane - (pm[0] + k)) <= (uint32_t)(mrel[0] - (pm[0] + k)));
        f1 &= ballot((uint32_t)(lane - (pm[1] + k)) <= (uint32_t)(mrel[1] - (pm[1] + k)));
        const uint32_t keep =
            (__builtin_amdgcn_inverse_ballot_w64(f0) ? 0x0000FFFFu : 0u) |
            (__builtin_amdgcn_inverse_ballot_w64(f1) ? 0xFFFF0000u : 0u);
        vn = (v & keep) | (NEG2 & ~keep);
      } else {
        int neg = (int)__builtin_bit_cast(
            uint32_t, __builtin_bit_cast(xd_short2, r) >> (short)15);
        opaque_v(neg);  // (one v_bfi, not compares and selects per half)
        vn = (v & ~(uint32_t)neg) | (NEG2 & (uint32_t)neg);
      }
      // a new best: v > tv, i.e. v - thr > X
      uint64_t i0 = ballot((int)(short)r > X);
      uint64_t i1 = ballot((int)r > (int)xhi);  // (signed: high half > X)
      if constexpr (EDGE) {
        i0 &= f0;
        i1 &= f1;
      }
      pp = vn;
      if (__builtin_expect((i0 | i1) != 0, 0)) {
        const uint64_t im[2] = {i0, i1};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (!im[h]) continue;
          const int hv = half16(vn, h);
          int l0 = __builtin_ctzll(im[h]);
          int wm = __builtin_amdgcn_readlane(hv, l0);
          if (__builtin_popcountll(im[h]) > 1) {
            wm = uni(wave_max(hv));
            l0 = __builtin_ctzll(ballot(hv == wm));
          }
          if (h) tv1 = wm; else tv0 = wm;
          bd[h] = d0[h] + k;
          bln[h] = l0;
        }
      }
      mpp[0] = f0;
      mpp[1] = f1;
      ml[0] = xd_writelane_i32((int)(uint32_t)f0, k + 2, ml[0]);
      mh[0] = xd_writelane_i32((int)(uint32_t)(f0 >> 32), k + 2, mh[0]);
      ml[1] = xd_writelane_i32((int)(uint32_t)f1, k + 2, ml[1]);
      mh[1] = xd_writelane_i32((int)(uint32_t)(f1 >> 32), k + 2, mh[1]);
      tv0 -= gap;
      tv1 -= gap;
      if constexpr (ALPHA == 1) {
        // byte k&3 of half 0's word to byte 0, of half 1's to byte 2, zeros
        // elsewhere (v_perm_b32 selector 0x0c gives a zero byte)
        const uint32_t in2 = __builtin_amdgcn_perm(
            qw[1][k >> 2], qw[0][k >> 2],
            (uint32_t)(k & 3) | 0x0C000000u | ((uint32_t)(4 + (k & 3)) << 16) |
                0x0C00u);
        fb2 = (uint32_t)__builtin_amdgcn_update_dpp((int)in2, (int)fb2, 0x138,
                                                   0xf, 0xf, false);
      }
      bool stop = false;
      if ((k & (G - 1)) == G - 1) {
        const uint64_t o0 = mp[0] | f0, o1 = mp[1] | f1;
        if ((live0 && o0 == 0) || (live1 && o1 == 0)) stop = true;
        // one of the top G lanes finite (an idle half has none)
        uint32_t hw = (uint32_t)((o0 | o1) >> 32);
        opaque_s(hw);
        if (hw >= (1u << (32 - G))) stop = true;
      }
      if constexpr (EDGE) {
        if ((live0 && k >= rem[0]) || (live1 && k >= rem[1])) stop = true;
      }
      return stop;
    };
    auto run_block = [&](auto edge_tag) {
#pragma unroll
      for (int k = 0; k < KB; k += 2) {
        if (body(edge_tag, x, y, a1, a2, k)) {
          nk = k + 1; newest_in_y = true; return;
        }
        if (body(edge_tag, y, x, a2, a1, k + 1)) { nk = k + 2; return; }
      }
    };
    if (edge) run_block(std::true_type{});
    else run_block(std::false_type{});
    if (newest_in_y) {
      const uint32_t t = x;
      x = y;
      y = t;
    }
    // live-span cells of the block's antidiagonals per half: lane k + 2
    // forms antidiagonal k's span from the masks of the two before it (lanes
    // k + 1 and k), clamped to the matrix
    int64_t acc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t al = (uint32_t)wave_shr1(ml[h], 0), ah = (uint32_t)wave_shr1(mh[h], 0);
      const uint32_t bl = (uint32_t)wave_shr1((int)al, 0), bh = (uint32_t)wave_shr1((int)ah, 0);
      const uint32_t cl = al | (bl << 1);
      const uint32_t ch = ah | __builtin_amdgcn_alignbit(bh, bl, 31);
      const uint32_t cz = min((uint32_t)__builtin_ctzg(cl, -1),
                              (uint32_t)__builtin_ctzg(ch, -1) | 32u);
      const uint32_t lz = min((uint32_t)__builtin_clzg(ah | bh, -1),
                              (uint32_t)__builtin_clzg(al | bl, -1) | 32u);
      const int kk = lane - 2;
      const int lo = max((int)cz, pm[h] + kk);
      const int hi = min(64 - (int)lz, mrel[h]);
      const bool live = (al | ah | bl | bh) != 0;
      const int cnt = (kk >= 0 && kk < nk && live) ? max(hi - lo + 1, 0) : 0;
      acc[h] = sum_lanes(cnt);
    }
    // ---- after the block: advance, rebase, and see to each half
    const int tvs[2] = {tv0, tv1};
    uint32_t delta2 = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      DualHalf& Hh = H[h];
      if (Hh.item < 0) continue;
      Hh.e.d += nk;
      Hh.e.W += acc[h];
      if (bd[h] >= d0[h]) Hh.bxa = Hh.e.base + bln[h];  // a new best here
      Hh.bd = bd[h];
      Hh.bln = bln[h];
      // rebase: the half's best score at 0
      Hh.off += tvs[h];
      Hh.tv = 0;
      delta2 |= ((uint32_t)tvs[h] & 0xFFFFu) << (16 * h);
    }
    x = pk_sub_sat(x, delta2);
    y = pk_sub_sat(y, delta2);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      DualHalf& Hh = H[h];
      if (Hh.item < 0) continue;
      const uint32_t hm = h ? 0xFFFF0000u : 0x0000FFFFu;
      Hh.m1 = ballot(half16(x, h) != NEG16);
      Hh.m2 = ballot(half16(y, h) != NEG16);
      const bool dead = (Hh.m1 | Hh.m2) == 0;
      const bool last = Hh.e.d > Hh.e.m + Hh.e.n;
      if (dead || last) {
        // finished: T in the S frame from the relative frame value
        ItemResult r;
        r.status = S_OK;
        r.cells = Hh.e.W;
        r.tier = 7; r.pad = 0;
        if (Hh.bd >= 0) {
          r.best = Hh.off + gap * Hh.e.d;  // (tv = 0 after the rebase)
          r.x = Hh.bxa;
          r.y = Hh.bd - Hh.bxa;
        } else {
          r.best = 0; r.x = 0; r.y = 0;
        }
        if (lane == 0) P.items[Hh.item] = r;
        Hh.item = -1;
        x = (x & ~hm) | (NEG2 & hm);
        y = (y & ~hm) | (NEG2 & hm);
        continue;
      }
      const uint64_t o = Hh.m1 | Hh.m2;
      const int cz = (int)__builtin_clzll(o);
      if (cz < G) {
        // the band reached the guard lanes: slide the half's window up by
        // the lanes below its lowest finite cell, or hand the extension on
        const int sl = (int)__builtin_ctzll(o);
        if (cz + sl < G) {
          if (lane == 0) {
            const int slot = atomicAdd(P.counters + C_ESC_TAIL, 1);
            P.esc_queue[slot] = Hh.item;
          }
          Hh.item = -1;
          x = (x & ~hm) | (NEG2 & hm);
          y = (y & ~hm) | (NEG2 & hm);
          continue;
        }
        const int src = lane + sl;
        const bool in = src < 64;
        const uint32_t px = (uint32_t)__builtin_amdgcn_ds_bpermute((src & 63) << 2, (int)x);
        const uint32_t py = (uint32_t)__builtin_amdgcn_ds_bpermute((src & 63) << 2, (int)y);
        x = (x & ~hm) | ((in ? px : NEG2) & hm);
        y = (y & ~hm) | ((in ? py : NEG2) & hm);
        if constexpr (ALPHA == 1) {
          // target codes move with their cells (stray codes at the top lanes
          // are not used before they have moved out)
          const uint32_t pb = (uint32_t)__builtin_amdgcn_ds_bpermute((src & 63) << 2, (int)fb2);
          fb2 = (fb2 & ~hm) | (pb & hm);
        }
        Hh.m1 >>= sl;
        Hh.m2 >>= sl;
        Hh.e.base += sl;
        cover_a<ALPHA>(Hh.e, L.h[h], S, Hh.e.base + 62);
        if constexpr (ALPHA == 1) {
          uint32_t t[1];
          Ring<1>::read<1>(L.h[h].ra, Hh.e.base + lane - 1, t);
          const uint32_t fa = (t[0] & 31u) << 6;
          fa2 = (fa2 & ~hm) | ((fa << (16 * h)) & hm);
        } else {
          const uint32_t fa =
              (Ring<0>::read(L.h[h].ra, Hh.e.base + lane - 1) & 3u) * 0x55555555u;
          if (h) fb2 = fa; else fa2 = fa;
        }
      }
      make_uniform(Hh.e);
      Hh.off = uni(Hh.off);
      Hh.bd = uni(Hh.bd);
      Hh.bln = uni(Hh.bln);
      Hh.bxa = uni(Hh.bxa);
    }
  }
}

template <int ALPHA>
__global__ __launch_bounds__(WAVE * WPB) void xd_dual_kernel(Params P) {
  __shared__ DualLds<ALPHA> lds[WPB];
  __shared__ int16_t tab16[ALPHA == 1 ? TABLE_DIM * TABLE_DIM : 1];
  if constexpr (ALPHA == 1) {
    for (int i = threadIdx.x; i < TABLE_DIM * TABLE_DIM; i += blockDim.x)
      tab16[i] = P.table[i];
    __syncthreads();
  }
  const int wid = threadIdx.x >> 6;
  const Src S = make_src(P);
  run_dual<ALPHA>(P, S, lds[wid], tab16);
}

// ------------------------------------------------------------------ block
// Workgroup tier for bands wider than one wavefront's register window: the
// paper's memory-restricted band (two antidiagonals of at most delta_b cells
// kept in fast memory and updated in place, Sec. 3 and Alg. 1) with the
// window spread over the registers of BT_WAVES wavefronts.  Thread
// t = wave * 64 + lane holds window positions t*C .. t*C+C-1 of the current
// antidiagonal (A) and the one before it (B); computing antidiagonal d
// overwrites B in place.  Per antidiagonal the waves meet at one barrier:
// before it each wave publishes, in LDS slots indexed by d mod 4, the value
// of its top cell (the x-1 neighbour of the next wave's lane 0) and its part
// of the reductions (its best cell if it beats T, its finite range); after it
// every wave combines the BT_WAVES records into T, the end cell and the
// finite range.  Sequences stream through workgroup LDS rings.  The window
// slides by whole threads and widens in place (C = 4 -> 8, 1,024 -> 2,048
// cells) through an LDS exchange buffer; a band wider than 2,048 cells moves
// to the device-memory tier.
constexpr int BT_WAVES = 4;
constexpr int BT_NT = BT_WAVES * WAVE;

template <int ALPHA>
using BRing = RingT<ALPHA, ALPHA == 0 ? 8192 : 4096, BT_NT>;
// a fill must never overwrite codes the 2,048-cell window still reads
static_assert(BRing<0>::CH + 2048 - 1 <= BRing<0>::RS, "DNA block ring");
static_assert(BRing<1>::CH + 2048 - 1 <= BRing<1>::RS, "byte block ring");

template <int ALPHA>
struct BlockLds {
  uint32_t ra[BRing<ALPHA>::WORDS];
  uint32_t rb[BRing<ALPHA>::WORDS];
  int xa[BT_NT * 8], xb[BT_NT * 8];  // slide / widen exchange
  int top[4][BT_WAVES];              // top cell of each wave, by d mod 4
  int4 red[2][BT_WAVES];             // best value, its x, L, U; by d mod 2
  int item;
};

// Make ring elements up to need_hi available (all threads fill, then meet).
template <int ALPHA>
__device__ __forceinline__ void bcover(int& loaded, uint32_t* ring,
                                       const Src& S, int64_t start, int dir,
                                       int need_hi) {
  if (loaded > need_hi) return;  // (uniform)
  do {
    BRing<ALPHA>::fill(ring, S, start, dir, loaded, (int)threadIdx.x);
    loaded += BRing<ALPHA>::CH;
  } while (loaded <= need_hi);
  __syncthreads();
}

// Query codes of a thread's C cells (they change only with the window base)
// and the scores of its cells on one antidiagonal.
template <int ALPHA, int C>
struct BCodes;

template <int C>
struct BCodes<0, C> {
  uint32_t qa;  // cell j's query code at bits 2j
  __device__ void load(const uint32_t* ra, int base) {
    qa = BRing<0>::read(ra, base + (int)threadIdx.x * C - 1);
  }
  // yb: target element of cell 0 (cell j takes yb - j)
  __device__ void sims(const uint32_t* rb, int yb, const Params& P,
                       const int*, int (&s)[C]) const {
    const uint32_t bw = BRing<0>::read(rb, yb - C + 1);  // yb-C+1+k at 2k
#pragma unroll
    for (int j = 0; j < C; ++j)
      s[j] = (((qa >> (2 * j)) ^ (bw >> (2 * (C - 1 - j)))) & 3u) ? P.mis_s
                                                                  : P.mat_s;
  }
};

template <int C>
struct BCodes<1, C> {
  static constexpr int NB = (C + 3) / 4;
  int row[C];  // TAB_LD * query code
  __device__ void load(const uint32_t* ra, int base) {
    uint32_t v[NB];
    BRing<1>::read<NB>(ra, base + (int)threadIdx.x * C - 1, v);
#pragma unroll
    for (int j = 0; j < C; ++j)
      row[j] = (int)((v[j >> 2] >> (8 * (j & 3))) & 31u) * TAB_LD;
  }
  __device__ void sims(const uint32_t* rb, int yb, const Params&,
                       const int* tab, int (&s)[C]) const {
    uint32_t v[NB];
    BRing<1>::read<NB>(rb, yb - C + 1, v);
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = C - 1 - j;
      s[j] = tab[row[j] + (int)((v[k >> 2] >> (8 * (k & 3))) & 31u)];
    }
  }
};

// Lane 63 of every wave publishes its top cells of A (antidiagonal d-1) and
// B (d-2) after the window changed, then the workgroup meets.
template <int ALPHA, int C>
__device__ __forceinline__ void bpublish(const Ext& e, const int (&A)[C],
                                         const int (&B)[C],
                                         BlockLds<ALPHA>& L) {
  const int wv = (int)threadIdx.x >> 6;
  if (lane_id() == 63) {
    L.top[(e.d - 1) & 3][wv] = A[C - 1];
    L.top[(e.d - 2) & 3][wv] = B[C - 1];
  }
  __syncthreads();
}

// Window positions p <- p + sl*C (thread t takes thread t+sl's cells).
template <int C>
__device__ __forceinline__ void bslide(int (&A)[C], int (&B)[C], int* xa,
                                       int* xb, int sl) {
  const int t = (int)threadIdx.x;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    xa[t * C + j] = A[j];
    xb[t * C + j] = B[j];
  }
  __syncthreads();
  const int src = t + sl;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    A[j] = src < BT_NT ? xa[src * C + j] : NEG;
    B[j] = src < BT_NT ? xb[src * C + j] : NEG;
  }
}

// C -> 2C cells per thread, same base (the upper half starts at -infinity).
template <int C>
__device__ __forceinline__ void bwiden(const int (&A)[C], const int (&B)[C],
                                       int (&NA)[2 * C], int (&NB)[2 * C],
                                       int* xa, int* xb) {
  const int t = (int)threadIdx.x;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    xa[t * C + j] = A[j];
    xb[t * C + j] = B[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 2 * C; ++j) {
    const int p = t * 2 * C + j;
    NA[j] = p < BT_NT * C ? xa[p] : NEG;
    NB[j] = p < BT_NT * C ? xb[p] : NEG;
  }
}

// Antidiagonal e.d of the block tier (A: d-1, B: d-2 on entry; d, d-1 on
// exit).  Returns R_CONT, R_DONE, R_CAP or R_ESC (the band needs a wider
// window); every thread returns the same value.
template <int ALPHA, int C>
__device__ __forceinline__ int bstep(Ext& e, int (&A)[C], int (&B)[C],
                                     BCodes<ALPHA, C>& cq, BlockLds<ALPHA>& L,
                                     const int* tab, const Params& P,
                                     const Src& S) {
  constexpr int NC = BT_NT * C;
  constexpr int LOG2C = C == 4 ? 2 : 3;
  const int t = (int)threadIdx.x, lane = t & 63, wv = t >> 6;
  const int d = e.d;
  const int lo = smax(smin(e.L1, e.L2 + 1), smax(0, d - e.n));
  const int hi = smin(smax(e.U1, e.U2) + 1, smin(e.m, d));
  const int width = hi - lo + 1;
  if (width > 0) e.W += width;
  if (P.band_cap > 0 && width > P.band_cap) return R_CAP;

  bcover<ALPHA>(e.loaded_b, L.rb, S, e.b_start, e.b_dir, d - e.base - 1);
  int s[C];
  cq.sims(L.rb, d - e.base - t * C - 1, P, tab, s);
  // x-1 neighbours of cell 0: the thread below, or for lane 0 the top cell
  // of the wave below (published on the antidiagonal it belongs to)
  const int fu = wv ? L.top[(d - 1) & 3][wv - 1] : NEG;
  const int fd = wv ? L.top[(d - 2) & 3][wv - 1] : NEG;
  const int up0 = wave_shr1(A[C - 1], fu);
  const int dg0 = wave_shr1(B[C - 1], fd);
  const int thr = smax(e.T - P.X - P.gap * d, THR_FLOOR);
  const int pmin = d - e.n - e.base;
  const uint32_t span = (uint32_t)(e.m - e.base - pmin);
  int v[C];
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const int up = j ? A[j - 1] : up0;
    const int dg = j ? B[j - 1] : dg0;
    v[j] = max(max(up, A[j]), dg + s[j]);
  }
  uint64_t msk[C];
  uint64_t any = 0;
  int lm = NEG;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const bool f = v[j] >= thr && (uint32_t)(t * C + j - pmin) <= span;
    v[j] = f ? v[j] : NEG;
    msk[j] = ballot(f);
    any |= msk[j];
    lm = max(lm, v[j]);
  }
#pragma unroll
  for (int j = 0; j < C; ++j) { B[j] = A[j]; A[j] = v[j]; }
  if (lane == 63) L.top[d & 3][wv] = A[C - 1];

  // this wave's part of the reductions
  const int Tv = e.T - P.gap * d;
  const uint64_t imp = ballot(lm > Tv);
  int wm = NEG, wx = 0x7fffffff;
  if (imp) {
    int l0;
    if (__builtin_popcountll(imp) == 1) {
      l0 = __builtin_ctzll(imp);
      wm = __builtin_amdgcn_readlane(lm, l0);
    } else {
      wm = uni(wave_max(lm));
      l0 = __builtin_ctzll(ballot(lm == wm));
    }
    int jf = C - 1;
#pragma unroll
    for (int j = C - 1; j >= 0; --j)
      if (A[j] == wm) jf = j;
    wx = e.base + ((wv * 64 + l0) << LOG2C) + __builtin_amdgcn_readlane(jf, l0);
  }
  int wl = DEAD_L, wu = DEAD_U;
  if (any) {
    const int llo = __builtin_ctzll(any);
    const int lhi = 63 - __builtin_clzll(any);
    int jlo = 0, jhi = 0;
#pragma unroll
    for (int j = C - 1; j >= 0; --j)
      if ((msk[j] >> llo) & 1) jlo = j;
#pragma unroll
    for (int j = 0; j < C; ++j)
      if ((msk[j] >> lhi) & 1) jhi = j;
    wl = e.base + ((wv * 64 + llo) << LOG2C) + jlo;
    wu = e.base + ((wv * 64 + lhi) << LOG2C) + jhi;
  }
  if (lane == 0) L.red[d & 1][wv] = make_int4(wm, wx, wl, wu);
  __syncthreads();
  // all waves: best (lowest wave first on ties: its x is lower), range
  int gm = NEG, gx = 0, gl = DEAD_L, gu = DEAD_U;
#pragma unroll
  for (int k = 0; k < BT_WAVES; ++k) {
    const int4 r = L.red[d & 1][k];
    if (r.x > gm) { gm = r.x; gx = r.y; }
    gl = min(gl, r.z);
    gu = max(gu, r.w);
  }
  gm = uni(gm); gx = uni(gx); gl = uni(gl); gu = uni(gu);
  if (gm > Tv) {
    e.T = gm + P.gap * d;
    e.bx = gx;
    e.by = d - gx;
  }
  const int L1 = e.L1, U1 = e.U1;
  e.L2 = L1; e.U2 = U1;
  e.L1 = gl; e.U1 = gu;
  e.d = d + 1;
  int r = R_CONT;
  if ((gl > gu && L1 > U1) || d >= e.m + e.n) r = R_DONE;
  if (r == R_CONT) {
    // keep the next antidiagonal's band inside the window
    const int hi_next = smin(smax(gu, U1) + 1, smin(e.m, d + 1));
    if (hi_next > e.base + NC - 1) {
      const int sl = (smin(gl, L1) - e.base) >> LOG2C;  // whole threads
      if (sl < 1) {
        r = R_ESC;
      } else {
        bslide<C>(A, B, L.xa, L.xb, sl);
        e.base += sl << LOG2C;
        bcover<ALPHA>(e.loaded_a, L.ra, S, e.a_start, e.a_dir,
                      e.base + NC - 2);
        cq.load(L.ra, e.base);
        bpublish<ALPHA, C>(e, A, B, L);
      }
    }
  }
  make_uniform(e);
  return r;
}

template <int ALPHA, int C, int CMAX>
__device__ __forceinline__ int run_btier(Ext& e, int (&A)[C], int (&B)[C],
                                         BlockLds<ALPHA>& L, const int* tab,
                                         const Params& P, const Src& S,
                                         int& tier_out) {
  BCodes<ALPHA, C> cq;
  bcover<ALPHA>(e.loaded_a, L.ra, S, e.a_start, e.a_dir,
                e.base + BT_NT * C - 2);
  cq.load(L.ra, e.base);
  bpublish<ALPHA, C>(e, A, B, L);
  int r;
  do {
    r = bstep<ALPHA, C>(e, A, B, cq, L, tab, P, S);
  } while (r == R_CONT);
  if constexpr (C < CMAX) {
    if (r == R_ESC) {
      int NA[2 * C], NB[2 * C];
      bwiden<C>(A, B, NA, NB, L.xa, L.xb);
      return run_btier<ALPHA, 2 * C, CMAX>(e, NA, NB, L, tab, P, S, tier_out);
    }
  }
  tier_out = C;
  return r;
}

// One extension on the block tier (all threads of the workgroup).
template <int ALPHA>
__device__ __forceinline__ void run_bitem(const Params& P, const Src& S,
                                          int item, BlockLds<ALPHA>& L,
                                          const int* tab) {
  ItemSetup s = setup_item(P, item);
  ItemResult res;
  res.best = 0; res.x = 0; res.y = 0; res.status = s.status; res.cells = 0;
  res.tier = -1; res.pad = 0;
  bool handed_on = false;
  if (s.status == S_OK) {
    Ext& e = s.e;
    int r = R_DONE, tier = 4;
    if (e.m + e.n != 0) {
      int A[4], B[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) { A[j] = NEG; B[j] = NEG; }
      if (threadIdx.x == 0) A[0] = 0;  // S(0,0) = 0 at window position 0
      r = run_btier<ALPHA, 4, 8>(e, A, B, L, tab, P, S, tier);
    }
    if (r == R_ESC) {
      // band wider than 2,048 cells: restart on the device-memory tier
      handed_on = true;
      if (threadIdx.x == 0) {
        const int slot = atomicAdd(P.counters + C_DEV_TAIL, 1);
        P.dev_queue[slot] = item;
      }
    } else if (r == R_CAP) {
      res.status = S_BAND;
    } else {
      res.best = e.T; res.x = e.bx; res.y = e.by; res.cells = e.W;
      res.tier = 5;
    }
  }
  if (!handed_on && threadIdx.x == 0) P.items[item] = res;
}

// Persistent block-tier kernel: one extension per workgroup at a time,
// pulled from the queue the wave kernel (or the workgroup form) filled.
template <int ALPHA>
__global__ __launch_bounds__(BT_NT) void xd_block_kernel(Params P) {
  __shared__ BlockLds<ALPHA> L;
  __shared__ int tab[ALPHA == 1 ? TAB_WORDS : 1];
  if constexpr (ALPHA == 1) fill_tab(tab, P);
  const Src S = make_src(P);
  const int tail = P.counters[C_GEN_TAIL];  // final: set by earlier kernels
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const int h = tail > 0 ? atomicAdd(P.counters + C_GEN_HEAD, 1) : 0;
      L.item = h < tail ? P.gen_queue[h] : -1;
    }
    __syncthreads();
    const int item = uni(L.item);
    if (item < 0) break;
    run_bitem<ALPHA>(P, S, item, L, tab);
  }
}

// ------------------------------------------------------------------ general
// Device-memory tier for bands wider than the block tier's 2,048 cells:
// antidiagonals d, d-1, d-2 in three rings of GEN_CAP cells in device memory
// (cell x at x mod GEN_CAP), every cell of [lo_d, hi_d] computed by the
// GEN_THREADS threads of the block, reductions through LDS.

__device__ __forceinline__ int sym_at(const Params& P, const Src& S,
                                      int64_t pos) {
  if (P.alphabet == 0) {
    uint32_t wv = load_word(S, pos >> 4);
    return (int)((wv >> (2 * (pos & 15))) & 3u);
  }
  uint32_t wv = load_word(S, pos >> 2);
  return (int)((wv >> (8 * (pos & 3))) & 31u);
}

__global__ __launch_bounds__(GEN_THREADS) void xd_general_kernel(Params P) {
  __shared__ int s_max, s_x, s_L, s_U, s_item;
  __shared__ int tab[TABLE_DIM * TABLE_DIM];
  for (int i = threadIdx.x; i < TABLE_DIM * TABLE_DIM; i += blockDim.x)
    tab[i] = P.table[i];
  const Src S = make_src(P);
  int* ring[3];
  for (int r = 0; r < 3; ++r)
    ring[r] = P.gen_scratch + ((int64_t)blockIdx.x * 3 + r) * GEN_CAP;
  const int tid = threadIdx.x;
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      const int tail = P.counters[C_DEV_TAIL];  // final: set by earlier kernels
      const int h = tail > 0 ? atomicAdd(P.counters + C_DEV_HEAD, 1) : 0;
      s_item = h < tail ? P.dev_queue[h] : -1;
    }
    __syncthreads();
    const int item = s_item;
    if (item < 0) break;
    ItemSetup st = setup_item(P, item);
    Ext& e = st.e;
    ItemResult res;
    res.best = 0; res.x = 0; res.y = 0; res.cells = 1; res.status = st.status;
    res.tier = -1; res.pad = 0;
    // antidiagonal ranges: computed span [lo, hi] and finite range [L, U]
    int lo1 = 0, hi1 = 0, lo2 = 1, hi2 = 0;  // d-1 = 0 holds x = 0 only
    if (tid == 0) ring[0][0] = 0;
    int T = 0, bx = 0, by = 0;
    int64_t W = 1;
    int alive1 = 1, L1 = 0, U1 = 0, alive2 = 0, L2 = 0, U2 = 0;
    int r1 = 0, r2 = 2, r0 = 1;  // ring indices of d-1, d-2, d
    for (int d = 1; d <= e.m + e.n && (alive1 || alive2); ++d) {
      int lo = 0x7fffffff, hi = -0x7fffffff;
      if (alive1) { lo = min(lo, L1); hi = max(hi, U1 + 1); }
      if (alive2) { lo = min(lo, L2 + 1); hi = max(hi, U2 + 1); }
      lo = max(lo, max(0, d - e.n));
      hi = min(hi, min(e.m, d));
      const int thr = max(T - P.X - P.gap * d, THR_FLOOR);
      __syncthreads();
      if (tid == 0) { s_max = NEG; s_x = 0x7fffffff; s_L = 0x7fffffff; s_U = -1; }
      __syncthreads();
      if (hi >= lo) {
        W += hi - lo + 1;
        if ((P.band_cap > 0 && hi - lo + 1 > P.band_cap) ||
            hi - lo + 1 > GEN_CAP) {
          res.status = S_BAND;
          break;
        }
      }
      const int* R1 = ring[r1];
      const int* R2 = ring[r2];
      int* R0 = ring[r0];
      int tmax = NEG, tL = 0x7fffffff, tU = -1;
      for (int x = lo + tid; x <= hi; x += GEN_THREADS) {
        const int y = d - x;
        int v = NEG;
        if (x >= 1 && x - 1 >= lo1 && x - 1 <= hi1)
          v = max(v, R1[(x - 1) & (GEN_CAP - 1)]);
        if (y >= 1 && x >= lo1 && x <= hi1)
          v = max(v, R1[x & (GEN_CAP - 1)]);
        if (x >= 1 && y >= 1 && x - 1 >= lo2 && x - 1 <= hi2) {
          const int ca = sym_at(P, S, e.a_start + (int64_t)e.a_dir * (x - 1));
          const int cb = sym_at(P, S, e.b_start + (int64_t)e.b_dir * (y - 1));
          int sv;
          if (P.alphabet == 0) sv = ca == cb ? P.mat_s : P.mis_s;
          else sv = tab[ca * TABLE_DIM + cb];
          v = max(v, R2[(x - 1) & (GEN_CAP - 1)] + sv);
        }
        if (v < thr) v = NEG;
        R0[x & (GEN_CAP - 1)] = v;
        if (v != NEG) {
          tL = min(tL, x);
          tU = max(tU, x);
          if (v > tmax) tmax = v;  // x ascending: first x kept on ties
        }
      }
      atomicMax(&s_max, tmax);
      atomicMin(&s_L, tL);
      atomicMax(&s_U, tU);
      __syncthreads();
      const int gm = s_max;
      if (gm != NEG && gm > T - P.gap * d) {
        for (int x = lo + tid; x <= hi; x += GEN_THREADS)
          if (R0[x & (GEN_CAP - 1)] == gm) atomicMin(&s_x, x);
      }
      __syncthreads();
      if (gm != NEG && gm > T - P.gap * d) {
        T = gm + P.gap * d;
        bx = s_x;
        by = d - bx;
      }
      alive2 = alive1; L2 = L1; U2 = U1;
      alive1 = s_U >= 0; L1 = s_L; U1 = s_U;
      lo2 = lo1; hi2 = hi1; lo1 = lo; hi1 = hi;
      const int rt = r2; r2 = r1; r1 = r0; r0 = rt;
    }
    if (res.status == S_OK) {
      res.best = T; res.x = bx; res.y = by; res.cells = W;
      res.tier = 6;
    } else if (res.status == S_BAND) {
      res.best = 0; res.x = 0; res.y = 0; res.cells = 0;
    }
    if (tid == 0) P.items[item] = res;
  }
}

// ------------------------------------------------------------------ misc
// Zero the counters once, when they are allocated (a kernel on the batch's
// stream); every batch's combine kernel leaves them zero for the next one.
__global__ void xd_reset_kernel(int32_t* counters) {
  for (int i = threadIdx.x; i < C_COUNT; i += blockDim.x) counters[i] = 0;
}

// Symbol check for byte-coded sequences, restricted to the sequences that
// seeds reference: state[s] = 0 unreferenced, 1 referenced, 2 referenced
// and holding a code >= asize.
__global__ void xd_clear_bytes_kernel(uint8_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void xd_mark_kernel(const int32_t* seeds, int32_t n_seeds,
                               int32_t n_seqs, uint8_t* state) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_seeds) return;
  const int q = seeds[5 * (int64_t)i], t = seeds[5 * (int64_t)i + 1];
  if (q >= 0 && q < n_seqs) state[q] = 1;
  if (t >= 0 && t < n_seqs) state[t] = 1;
}

// Bytes of the 32-bit word w at or above asize (asize <= 32): one 0x80 per
// such byte.  (b & 0x7F) + 0x80 - asize reaches 0x80 exactly when the low
// seven bits are >= asize and cannot carry into the next byte; b's own top
// bit covers codes of 128 and more.
__device__ __forceinline__ uint32_t bytes_at_least(uint32_t w, uint32_t k) {
  return (((w & 0x7F7F7F7Fu) + k) | w) & 0x80808080u;
}
// 0x80 in bytes lo .. hi-1 of a word (0 <= lo, hi <= 4).
__device__ __forceinline__ uint32_t byte_span_mask(int lo, int hi) {
  if (hi <= lo) return 0u;
  return (0xFFFFFFFFu >> (8 * (4 - hi))) & (0xFFFFFFFFu << (8 * lo)) &
         0x80808080u;
}

__global__ void xd_validate_kernel(const uint8_t* seqs, const int64_t* offsets,
                                   int32_t n_seqs, int32_t asize,
                                   uint8_t* state) {
  // four sequences per wave, 16 lanes each; a group reads its sequence in
  // 16-byte pieces, 256 bytes per round (the stream is read in whole words,
  // as the extension kernels read it, so the last piece may hold bytes of
  // the next sequence or past the stream end: they are masked); every byte
  // is tested against the alphabet on the whole word at once
  const int lane = lane_id();
  const int g = lane >> 4, gl = lane & 15;
  const int wpb = blockDim.x >> 6;
  const int64_t wave = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * wpb;
  const uint32_t* words = (const uint32_t*)seqs;
  const uint4* quads = (const uint4*)seqs;
  const int64_t tw = (offsets[n_seqs] + 3) >> 2;  // words of the stream
  const bool al16 = ((uintptr_t)seqs & 15) == 0;
  const uint32_t k = (uint32_t)(0x80 - asize) * 0x01010101u;
  for (int64_t s0 = wave * 4; s0 < n_seqs; s0 += nwaves * 4) {
    const int64_t s = s0 + g;
    uint32_t found = 0;
    if (s < n_seqs && state[s] == 1) {
      const int64_t a = offsets[s], b = offsets[s + 1];
      if (b > a) {
        const int64_t qend = (b - 1) >> 4;
        for (int64_t qi = (a >> 4) + gl; qi <= qend; qi += 16) {
          uint32_t v[4];
          if (al16 && 4 * qi + 3 < tw) {
            const uint4 q = quads[qi];
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              v[i] = 4 * qi + i < tw ? words[4 * qi + i] : 0u;
          }
          const int64_t pb = qi * 16;  // byte position of v[0]'s first byte
          const bool whole = pb >= a && pb + 16 <= b;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            uint32_t bad = bytes_at_least(v[i], k);
            if (!whole) {
              const int64_t wb = pb + 4 * i;
              const int lo = (int)(a > wb ? (a - wb < 4 ? a - wb : 4) : 0);
              const int hi = (int)(b > wb ? (b - wb < 4 ? b - wb : 4) : 0);
              bad &= byte_span_mask(lo, hi);
            }
            found |= bad;
          }
        }
      }
    }
    const uint64_t any = ballot(found != 0);
    if (gl == 0 && s < n_seqs && ((any >> (16 * g)) & 0xFFFFull))
      state[s] = 2;
  }
}

// Longest-first order.  The cost of an extension is m + n, the length of
// its antidiagonal chain (its latency; the paper's batcher uses the
// quadratic m*n, an area bound).  Extensions are bucketed on a log scale
// (8 buckets per power of two) and scattered longest bucket first: a
// counting sort without device-wide memsets, so it can be captured in a
// graph.  Order inside a bucket is arbitrary (results do not depend on it).
__device__ __forceinline__ int cost_bucket(const int32_t* seeds,
                                           const int64_t* offsets,
                                           int32_t n_seqs, int i) {
  const int seed = i >> 1, right = i & 1;
  const int* sd = seeds + 5 * (int64_t)seed;
  const int q = sd[0], t = sd[1], qp = sd[2], tp = sd[3], k = sd[4];
  uint32_t key = 0;
  if (q >= 0 && q < n_seqs && t >= 0 && t < n_seqs) {
    const int64_t lq = offsets[q + 1] - offsets[q];
    const int64_t lt = offsets[t + 1] - offsets[t];
    int64_t c = right ? (lq - qp - k) + (lt - tp - k) : (int64_t)qp + tp;
    c = c < 0 ? 0 : (c > 0x7fffffff ? 0x7fffffff : c);
    key = (uint32_t)c;
  }
  int f = 0;
  if (key >= 8) {
    const int e = 31 - __builtin_clz(key);
    f = e * 8 + (int)((key >> (e - 3)) & 7u);
  } else {
    f = (int)key;
  }
  return NBUCKET - 1 - min(f, NBUCKET - 1);  // longest first
}

__global__ void xd_hist_kernel(const int32_t* seeds, const int64_t* offsets,
                               int32_t n_seqs, int32_t n_items,
                               int32_t* counters) {
  __shared__ int h[NBUCKET];
  for (int b = threadIdx.x; b < NBUCKET; b += blockDim.x) h[b] = 0;
  __syncthreads();
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items;
       i += gridDim.x * blockDim.x)
    atomicAdd(&h[cost_bucket(seeds, offsets, n_seqs, i)], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < NBUCKET; b += blockDim.x)
    if (h[b]) atomicAdd(counters + C_HIST + b, h[b]);
}

__global__ void xd_scan_kernel(int32_t* counters) {
  // single block of NBUCKET threads: exclusive prefix sum into the cursors
  __shared__ int v[NBUCKET];
  const int b = threadIdx.x;
  v[b] = counters[C_HIST + b];
  __syncthreads();
  for (int off = 1; off < NBUCKET; off <<= 1) {
    const int add = b >= off ? v[b - off] : 0;
    __syncthreads();
    v[b] += add;
    __syncthreads();
  }
  counters[C_CURSOR + b] = v[b] - counters[C_HIST + b];
}

// Items of one block claim their slots bucket by bucket: one device atomic
// per (block, bucket) instead of one per item.
__global__ __launch_bounds__(1024) void xd_scatter_kernel(const int32_t* seeds, const int64_t* offsets,
                                  int32_t n_seqs, int32_t n_items,
                                  int32_t* counters, int32_t* order) {
  __shared__ int h[NBUCKET];
  __shared__ int first[NBUCKET];
  for (int b = threadIdx.x; b < NBUCKET; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0, rank = 0;
  if (i < n_items) {
    b = cost_bucket(seeds, offsets, n_seqs, i);
    rank = atomicAdd(&h[b], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < NBUCKET; c += blockDim.x)
    first[c] = h[c] ? atomicAdd(counters + C_CURSOR + c, h[c]) : 0;
  __syncthreads();
  if (i < n_items) order[first[b] + rank] = i;
}

// Score of a seed: the sum of sim over its k symbol pairs, read a word of
// codes at a time from each sequence (16 DNA or 4 byte codes per word; the
// pieces of two stream words are joined with one funnel shift).
template <int ALPHA>
__device__ __forceinline__ int seed_score(const Params& P, const Src& S,
                                          int64_t pa, int64_t pb, int k) {
  constexpr int PER = ALPHA == 0 ? 16 : 4, BITS = ALPHA == 0 ? 2 : 8;
  constexpr uint32_t MASK = ALPHA == 0 ? 3u : 31u;
  auto piece = [&](int64_t pos) {  // PER codes from pos, lowest code lowest
    const int64_t w = pos / PER;
    const uint32_t sh = (uint32_t)(pos - w * PER) * BITS;
    return funnel(load_word(S, w + 1), load_word(S, w), sh);
  };
  int sc = 0;
  for (int u = 0; u < k; u += PER) {
    const uint32_t wa = piece(pa + u), wb = piece(pb + u);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (u + j < k) {
        const int ca = (int)((wa >> (BITS * j)) & MASK);
        const int cb = (int)((wb >> (BITS * j)) & MASK);
        if constexpr (ALPHA == 0) sc += ca == cb ? P.mat_s : P.mis_s;
        else sc += P.table[ca * TABLE_DIM + cb];
      }
    }
  }
  return sc + 2 * P.gap * k;  // (the table holds sim - 2 gap)
}

// Seed level: score = left + seed score + right and positions (Sec. 4.1.1).
// It is the last kernel of every batch, so it also finishes the batch's
// bookkeeping: block 0 zeroes the queue and ordering counters for the next
// batch (no kernel of this batch uses them any more), which saves a reset
// launch, and every block stores the tier counts of its seeds' extensions
// (read from their results: ballots per wave, LDS per block) in its own
// slots, with no atomic on device memory.
__global__ __launch_bounds__(256) void xd_combine_kernel(Params P, void* out_v) {
  __shared__ int hist[N_TIERS];
  if (threadIdx.x < N_TIERS) hist[threadIdx.x] = 0;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < C_PART; i += blockDim.x) P.counters[i] = 0;
  __syncthreads();
  struct Out {
    int32_t score, left, right, seed_score;
    int32_t q_begin, q_end, t_begin, t_end;
    int64_t cells;
    int32_t status, reserved;
  };
  Out* out = (Out*)out_v;
  int cnt[N_TIERS] = {};  // this wave's counts (wave-uniform)
  // (the loop bound is uniform over the block, so every lane meets the
  // ballots)
  for (int s0 = blockIdx.x * blockDim.x; s0 < P.n_seeds;
       s0 += gridDim.x * blockDim.x) {
    const int s = s0 + (int)threadIdx.x;
    int tl = -1, tr = -1;
    if (s < P.n_seeds) {
      const ItemResult L = P.items[2 * (int64_t)s];
      const ItemResult R = P.items[2 * (int64_t)s + 1];
      tl = L.tier;
      tr = R.tier;
      Out o = {};
      int st = L.status != S_OK ? L.status : R.status;
      if (st == S_OK) {
        const int* sd = P.seeds + 5 * (int64_t)s;
        const int q = sd[0], t = sd[1], qp = sd[2], tp = sd[3], k = sd[4];
        const int64_t oq = P.offsets[q], ot = P.offsets[t];
        const Src S = make_src(P);
        const int seed =
            P.alphabet == 0 ? seed_score<0>(P, S, oq + qp, ot + tp, k)
                            : seed_score<1>(P, S, oq + qp, ot + tp, k);
        o.left = L.best; o.right = R.best; o.seed_score = seed;
        o.score = L.best + seed + R.best;
        o.q_begin = qp - L.x; o.t_begin = tp - L.y;
        o.q_end = qp + k + R.x; o.t_end = tp + k + R.y;
        o.cells = L.cells + R.cells;
      }
      o.status = st;
      out[s] = o;
    }
#pragma unroll
    for (int t = 0; t < N_TIERS; ++t)
      cnt[t] += __builtin_popcountll(ballot(tl == t)) +
                __builtin_popcountll(ballot(tr == t));
  }
  if (lane_id() == 0)
#pragma unroll
    for (int t = 0; t < N_TIERS; ++t)
      if (cnt[t]) atomicAdd(&hist[t], cnt[t]);
  __syncthreads();
  if (threadIdx.x < N_TIERS)
    P.counters[C_PART + N_TIERS * blockIdx.x + threadIdx.x] = hist[threadIdx.x];
}

template __global__ void xd_wave_kernel<0, 8>(Params);
template __global__ void xd_wave_kernel<1, 8>(Params);
template __global__ void xd_rows_kernel<0, 2>(Params);
template __global__ void xd_rows_kernel<1, 2>(Params);
template __global__ void xd_rows_kernel<0, 4>(Params);
template __global__ void xd_rows_kernel<1, 4>(Params);
template __global__ void xd_block_kernel<0>(Params);
template __global__ void xd_block_kernel<1>(Params);
template __global__ void xd_dual_kernel<0>(Params);
template __global__ void xd_dual_kernel<1>(Params);

}  // namespace xd

// ==================================================================== host
// Launch wrappers used by the C ABI (xdrop_host.cpp).
namespace xd {

// Fixed scratch of the allocation-free entry point: counters, queues, result
// slots and device-memory tier rings of one batch.  Every GPU the library
// runs on holds one copy until the process ends.
static __device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

// Its device address on `device` (the current device), looked up once per
// device; host code passes this address, never the array's name.
hipError_t noalloc_scratch(int device, void** out) {
  static std::mutex mu;
  static void* addr[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

__global__ void xd_fill_queue_kernel(const int32_t* order, int32_t n,
                                     int32_t* queue, int32_t* counters,
                                     int32_t tail_slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) queue[i] = order ? order[i] : i;
  if (i == 0) counters[tail_slot] = n;
}

hipError_t launch_reset(int32_t* counters, hipStream_t s) {
  hipLaunchKernelGGL(xd_reset_kernel, dim3(1), dim3(256), 0, s, counters);
  return hipGetLastError();
}

hipError_t launch_validate(const uint8_t* seqs, const int64_t* offsets,
                           int32_t n_seqs, const int32_t* seeds,
                           int32_t n_seeds, int32_t asize, uint8_t* state,
                           int grid, hipStream_t s) {
  if (n_seqs <= 0) return hipSuccess;
  hipLaunchKernelGGL(xd_clear_bytes_kernel,
                     dim3(std::min((n_seqs + 255) / 256, 1024)), dim3(256), 0,
                     s, state, (int64_t)n_seqs);
  if (n_seeds > 0)
    hipLaunchKernelGGL(xd_mark_kernel, dim3((n_seeds + 255) / 256), dim3(256),
                       0, s, seeds, n_seeds, n_seqs, state);
  hipLaunchKernelGGL(xd_validate_kernel, dim3(grid), dim3(256), 0, s, seqs,
                     offsets, n_seqs, asize, state);
  return hipGetLastError();
}

hipError_t launch_order(const int32_t* seeds, const int64_t* offsets,
                        int32_t n_seqs, int32_t n_items, int32_t* counters,
                        int32_t* order, int num_cu, hipStream_t s) {
  const int grid = std::min((n_items + 255) / 256, num_cu * 4);
  hipLaunchKernelGGL(xd_hist_kernel, dim3(std::max(grid, 1)), dim3(256), 0, s,
                     seeds, offsets, n_seqs, n_items, counters);
  hipLaunchKernelGGL(xd_scan_kernel, dim3(1), dim3(NBUCKET), 0, s, counters);
  // (blocks of 1024 items: a quarter of the contended cursor atomics)
  hipLaunchKernelGGL(xd_scatter_kernel, dim3((n_items + 1023) / 1024),
                     dim3(1024), 0, s, seeds, offsets, n_seqs, n_items,
                     counters, order);
  return hipGetLastError();
}

hipError_t launch_fill_queue(const int32_t* order, int32_t n, int32_t* queue,
                             int32_t* counters, int32_t tail_slot,
                             hipStream_t s) {
  hipLaunchKernelGGL(xd_fill_queue_kernel, dim3((n + 255) / 256 + 1),
                     dim3(256), 0, s, order, n, queue, counters, tail_slot);
  return hipGetLastError();
}

hipError_t launch_wave(const Params& P, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (P.alphabet == 0)
    hipLaunchKernelGGL((xd_wave_kernel<0, 8>), dim3(grid), dim3(WAVE * WPB),
                       0, s, P);
  else
    hipLaunchKernelGGL((xd_wave_kernel<1, 8>), dim3(grid), dim3(WAVE * WPB),
                       0, s, P);
  return hipGetLastError();
}

hipError_t launch_rows(const Params& P, int rows, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  const dim3 g(grid), b(WAVE * WPB);
  if (rows == 2) {
    if (P.alphabet == 0) hipLaunchKernelGGL((xd_rows_kernel<0, 2>), g, b, 0, s, P);
    else hipLaunchKernelGGL((xd_rows_kernel<1, 2>), g, b, 0, s, P);
  } else {
    if (P.alphabet == 0) hipLaunchKernelGGL((xd_rows_kernel<0, 4>), g, b, 0, s, P);
    else hipLaunchKernelGGL((xd_rows_kernel<1, 4>), g, b, 0, s, P);
  }
  return hipGetLastError();
}

int rows_blocks_per_cu(int alphabet, int rows) {
  int nb = 0;
  hipError_t e;
  if (rows == 2)
    e = alphabet == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb, xd_rows_kernel<0, 2>, WAVE * WPB, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb, xd_rows_kernel<1, 2>, WAVE * WPB, 0);
  else
    e = alphabet == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb, xd_rows_kernel<0, 4>, WAVE * WPB, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb, xd_rows_kernel<1, 4>, WAVE * WPB, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

hipError_t launch_dual(const Params& P, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (P.alphabet == 0)
    hipLaunchKernelGGL((xd_dual_kernel<0>), dim3(grid), dim3(WAVE * WPB), 0,
                       s, P);
  else
    hipLaunchKernelGGL((xd_dual_kernel<1>), dim3(grid), dim3(WAVE * WPB), 0,
                       s, P);
  return hipGetLastError();
}

int dual_blocks_per_cu(int alphabet) {
  int nb = 0;
  hipError_t e =
      alphabet == 0
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, xd_dual_kernel<0>, WAVE * WPB, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, xd_dual_kernel<1>, WAVE * WPB, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

bool dual_exact(const Params& P) {
  return (int64_t)P.X + (int64_t)DUAL_SPAN * P.max_abs <= 30000;
}

hipError_t launch_block(const Params& P, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (P.alphabet == 0)
    hipLaunchKernelGGL((xd_block_kernel<0>), dim3(grid), dim3(BT_NT), 0, s, P);
  else
    hipLaunchKernelGGL((xd_block_kernel<1>), dim3(grid), dim3(BT_NT), 0, s, P);
  return hipGetLastError();
}

int block_blocks_per_cu(int alphabet) {
  int nb = 0;
  hipError_t e =
      alphabet == 0
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, xd_block_kernel<0>, BT_NT, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, xd_block_kernel<1>, BT_NT, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

hipError_t launch_general(const Params& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL(xd_general_kernel, dim3(grid), dim3(GEN_THREADS), 0, s,
                     P);
  return hipGetLastError();
}

hipError_t launch_combine(const Params& P, void* out, hipStream_t s) {
  hipLaunchKernelGGL(xd_combine_kernel, dim3(combine_blocks(P.n_seeds)),
                     dim3(256), 0, s, P, out);
  return hipGetLastError();
}

int wave_blocks_per_cu(int alphabet) {
  int nb = 0;
  hipError_t e =
      alphabet == 0
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, xd_wave_kernel<0, 8>, WAVE * WPB, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, xd_wave_kernel<1, 8>, WAVE * WPB, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

}  // namespace xd
