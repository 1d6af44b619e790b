// Internal definitions shared by the host side and the HIP kernels of the
// X-Drop library (not part of the public ABI).
#pragma once
#include <stdint.h>

namespace xd {

// -infinity sentinel.  Stored values live in the frame V = S - gap * d (see
// the kernels); every finite V satisfies |V| <= 2^28 (checked per extension),
// so NEG plus any score entry stays far below every finite value and below
// the lowest prune threshold THR_FLOOR.
constexpr int32_t NEG = -(1 << 30);
constexpr int32_t THR_FLOOR = -(1 << 29);
constexpr int64_t VALUE_LIMIT = int64_t(1) << 28;
constexpr int32_t X_CLAMP = 1 << 30;  // X >= 2^30 acts as infinity
constexpr int32_t MAX_ENTRY = 1024;   // |matrix entry|, |gap| bound
// Finite range [L, U] of an antidiagonal with no finite cell: L > U, and the
// pair drops out of every min(L..) / max(U..) of band bounds.
constexpr int32_t DEAD_L = 1 << 30;
constexpr int32_t DEAD_U = -(1 << 30);

constexpr int WAVE = 64;
constexpr int WPB = 4;                // waves per block of the wave kernels
constexpr int TABLE_DIM = 32;         // substitution table is 32 x 32
constexpr int GEN_THREADS = 256;      // device-memory tier block size
constexpr int GEN_CAP = 1 << 16;      // device-memory tier band capacity

// Per-extension result written by the extension kernels.
struct ItemResult {
  int32_t best, x, y, status;
  int64_t cells;
  int32_t tier;  // tier that finished the extension (N_TIERS order)
  int32_t pad;
};

// Kernel flags.
enum : int32_t {
  F_PLAIN = 1,      // one wave per extension, no queue
  F_ORDERED = 2,    // items[] holds the processing order
  F_ESC = 4,        // items come from esc_queue (handed on by a row or 16-bit kernel)
};

// Per-seed / per-item status values (mirror the public enum).
enum : int32_t {
  S_OK = 0,
  S_RANGE = -2,
  S_SYMBOL = -6,
  S_BAND = -7,
};

// Launch parameters of one batch (kernel argument, < 4 KiB).
struct Params {
  const uint32_t* seqs;      // packed stream as 32-bit words
  const int64_t* offsets;    // n_seqs + 1
  const int32_t* seeds;      // 5 int32 per seed
  ItemResult* items;         // 2 * n_seeds
  const int32_t* order;      // processing order (F_ORDERED) or null
  int32_t* counters;         // queue heads and tier statistics
  const uint8_t* seq_bad;    // per-sequence check (BYTE): 2 = bad symbol
  int32_t* gen_queue;        // items handed to the block tier
  int32_t* dev_queue;        // items handed to the device-memory tier
  int32_t* esc_queue;        // items handed on by the row and 16-bit kernels
  int32_t* gen_scratch;      // device-memory tier rings
  int32_t n_seqs;
  int32_t n_seeds;
  int32_t n_items;
  int32_t flags;
  int32_t alphabet;          // 0 = DNA2, 1 = BYTE
  int32_t tile;              // starting cells per lane
  int32_t chunk;             // items per queue claim
  int32_t band_cap;          // 0 = none
  int32_t gap;
  int32_t X;                 // clamped to X_CLAMP
  int32_t mat_s, mis_s;      // DNA: match - 2 gap, mismatch - 2 gap
  int32_t max_abs;           // max |entry| + 2 |gap|  (value bound per d)
  int32_t gen_slots;         // concurrent device-memory tier workgroups
  int16_t table[TABLE_DIM * TABLE_DIM];  // BYTE: sim - 2 gap, row = query
};

// Extensions finished per tier, in this order: 1, 2, 4, 8 cells per lane
// (wave kernel), two rows per wave (pair form), block tier, device-memory
// tier, two-extension 16-bit kernel, four rows per wave.  Each result
// records its tier; the combine kernel counts them per block (no
// device-wide atomic per extension).
constexpr int N_TIERS = 9;
// Combine blocks of a batch (at most, so that the per-block tier counts fit
// in the counter block).
constexpr int MAX_COMBINE_BLOCKS = 2048;
inline int combine_blocks(int n_seeds) {
  const int b = (n_seeds + 255) / 256;
  return b < 1 ? 1 : b > MAX_COMBINE_BLOCKS ? MAX_COMBINE_BLOCKS : b;
}

// Counter layout (int32 slots).
enum {
  C_HEAD = 0,       // main queue head
  C_GEN_TAIL = 1,   // block tier queue tail
  C_GEN_HEAD = 2,   // block tier queue head
  C_ESC_TAIL = 3,   // hand-on queue tail (row and 16-bit kernels)
  C_ESC_HEAD = 4,   // its head (wave kernel)
  C_PAIR_HEAD = 5,  // row and 16-bit kernels: queue head
  C_DEV_TAIL = 6,   // device-memory tier queue tail
  C_DEV_HEAD = 7,   // its head
  C_HIST = 8,       // longest-first ordering: bucket sizes
  C_CURSOR = C_HIST + 256,  // bucket write cursors
  // the last batch's tier counts, N_TIERS per combine block (block b at
  // C_PART + N_TIERS * b); the host sums them when asked
  C_PART = C_CURSOR + 256,
  C_COUNT = C_PART + N_TIERS * MAX_COMBINE_BLOCKS
};
constexpr int NBUCKET = 256;

}  // namespace xd

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace xd {
constexpr size_t NOALLOC_BYTES = (size_t)16 << 20;
hipError_t noalloc_scratch(int device, void** out);
hipError_t launch_reset(int32_t* counters, hipStream_t s);
hipError_t launch_validate(const uint8_t* seqs, const int64_t* offsets,
                           int32_t n_seqs, const int32_t* seeds,
                           int32_t n_seeds, int32_t asize, uint8_t* state,
                           int grid, hipStream_t s);
hipError_t launch_order(const int32_t* seeds, const int64_t* offsets,
                        int32_t n_seqs, int32_t n_items, int32_t* counters,
                        int32_t* order, int num_cu, hipStream_t s);
hipError_t launch_fill_queue(const int32_t* order, int32_t n, int32_t* queue,
                             int32_t* counters, int32_t tail_slot,
                             hipStream_t s);
hipError_t launch_wave(const Params& P, int grid, hipStream_t s);
hipError_t launch_rows(const Params& P, int rows, int grid, hipStream_t s);
int rows_blocks_per_cu(int alphabet, int rows);
hipError_t launch_dual(const Params& P, int grid, hipStream_t s);
int dual_blocks_per_cu(int alphabet);
bool dual_exact(const Params& P);  // 16-bit relative scores exact here
hipError_t launch_block(const Params& P, int grid, hipStream_t s);
int block_blocks_per_cu(int alphabet);
hipError_t launch_general(const Params& P, int grid, hipStream_t s);
hipError_t launch_combine(const Params& P, void* out, hipStream_t s);
int wave_blocks_per_cu(int alphabet);
}  // namespace xd
