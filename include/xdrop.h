/*
 * xdrop.h -- C ABI of the MI355X (gfx950) batched X-Drop seed-extension
 * library.
 *
 * Operation (paper, Sec. 2.2 recurrence and X-Drop rule; Sec. 3 and
 * Algorithm 1, memory-restricted antidiagonal sweep; Sec. 4.1.1 seed records
 * and left/right extension split):
 *
 *   For each seed (q, t, q_pos, t_pos, k) two extensions are run:
 *     left  over the reversed prefixes  q[0:q_pos]      and t[0:t_pos],
 *     right over the suffixes           q[q_pos+k:]     and t[t_pos+k:].
 *   An extension E(a, b) fills cells (x, y) by antidiagonals d = x + y,
 *     S(0,0) = 0,
 *     S(x,y) = max{ S(x-1,y-1) + sim(a[x-1], b[y-1]), S(x-1,y) + gap,
 *                   S(x,y-1) + gap }   over predecessors inside the matrix,
 *   and sets a cell to -infinity when it is below T - X, where T is the best
 *   score of all earlier antidiagonals (strict '<').  The band of each
 *   antidiagonal is the span reachable from the finite cells of the two
 *   previous antidiagonals; the sweep stops when both hold no finite cell.
 *   Result: best score T, the first cell reaching it (antidiagonal order,
 *   lowest query offset on ties), and the live-span cell count.
 *   score = left + seed_score + right, seed_score = sum of sim over the seed.
 *
 * All arithmetic is int32 and integer-only; results are bit-exact and do not
 * depend on batch composition, order, variant, tile width or chunk size.
 *
 * Ownership: the caller owns every buffer passed in; the library keeps no
 * pointer after the enqueued work completes.  A context owns its device
 * workspace.  Threading: one host thread per context at a time.
 * Errors: every function returns an xdrop_status; argument errors are
 * detected on the host before any launch and leave outputs untouched;
 * data-dependent errors (seed out of range, symbol outside the alphabet,
 * score range, band cap) are reported per seed in xdrop_result.status while
 * the other seeds are still computed.
 */
#ifndef XDROP_H
#define XDROP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    XDROP_OK = 0,
    XDROP_E_INVALID = -1,  /* bad argument (host-detected, nothing launched) */
    XDROP_E_RANGE = -2,    /* per seed: seed outside its sequences, or the
                              int32 score range could be exceeded */
    XDROP_E_NOMEM = -3,    /* device or host allocation failed */
    XDROP_E_DEVICE = -4,   /* HIP runtime error; sticky on the context */
    XDROP_E_BUDGET = -5,   /* serving: request can never fit the budget */
    XDROP_E_SYMBOL = -6,   /* per seed: a code >= alphabet_size */
    XDROP_BAND_OVERFLOW = -7, /* per seed: band wider than opts->band_cap,
                                 or than 65536 cells (device-memory tier) */
    XDROP_E_SCRATCH = -8,  /* batch larger than the fixed scratch of
                              xdrop_extend_batch_noalloc */
    XDROP_PENDING = 1      /* serving: request not finished yet */
} xdrop_status;

/* Sequence encodings. */
enum {
    XDROP_DNA2 = 0, /* 2 bits per code, 16 codes per little-endian 32-bit
                       word, code i of the stream at bits 2*(i%16) of word
                       i/16; A=0 C=1 G=2 T=3 */
    XDROP_BYTE = 1  /* one code per byte, code < alphabet_size (<= 32) */
};

/* Scoring scheme (host struct, copied at the call). */
typedef struct {
    int32_t alphabet;      /* XDROP_DNA2 or XDROP_BYTE */
    int32_t alphabet_size; /* 4 for XDROP_DNA2; 1..32 for XDROP_BYTE */
    int32_t match;         /* used iff matrix == NULL */
    int32_t mismatch;      /* used iff matrix == NULL */
    const int32_t *matrix; /* host, alphabet_size^2, row = query code,
                              column = target code; |entry| <= 1024 */
    int32_t gap;           /* linear gap, added per gap symbol; -1024..0 */
    int32_t X;             /* X-Drop threshold, >= 0 (INT32_MAX allowed) */
} xdrop_scoring;

/* Seed record (device array, 20 bytes each). The seed aligns q[q_pos, q_pos+k)
 * against t[t_pos, t_pos+k); q and t index the offsets table. */
typedef struct {
    int32_t q, t;
    int32_t q_pos, t_pos, k;
} xdrop_seed;

/* Per-seed result (device array, 48 bytes each). Positions are half-open
 * intervals on q and t after extension. */
typedef struct {
    int32_t score, left, right, seed_score;
    int32_t q_begin, q_end, t_begin, t_end;
    int64_t cells;  /* live-span cells of both extensions */
    int32_t status; /* XDROP_OK or a per-seed error */
    int32_t reserved;
} xdrop_result;

/* Launch options (host struct; NULL = defaults). */
enum {
    XDROP_VARIANT_AUTO = 0,      /* choose per batch: the tuned table, else
                                    PLAIN when the whole batch fits in one
                                    wave of the persistent grid (every
                                    extension starts at once), else WAVE;
                                    PAIR runs as WAVE when a band cap is set */
    XDROP_VARIANT_WAVE = 1,      /* one wavefront per extension */
    XDROP_VARIANT_WORKGROUP = 2, /* one 4-wave workgroup per extension
                                    (window of 1,024..2,048 cells over the
                                    registers of the four waves) */
    XDROP_VARIANT_PLAIN = 3,     /* one wave per extension, one launch wave per
                                    extension, no queue: the baseline form */
    XDROP_VARIANT_PAIR = 4,      /* two extensions per wavefront (32-cell
                                    windows, one cell per lane); extensions
                                    whose band outgrows 32 cells restart on
                                    the wave kernel.  Ignores band_cap (runs
                                    as WAVE when a cap is set) */
    XDROP_VARIANT_DUAL16 = 5,    /* two extensions per wavefront, one in each
                                    16-bit half of every register (64-cell
                                    windows, packed 16-bit integer
                                    arithmetic on relative scores, paper
                                    Sec. 4.1.4's change of ALU type); used
                                    only where X + 40 * (max |entry| +
                                    2 |gap|) <= 30,000 keeps every relative
                                    score within 16 bits, else it runs as
                                    WAVE (int32).  Extensions whose band
                                    fills 60 lanes restart on the wave
                                    kernel.  Ignores band_cap (runs as WAVE
                                    when a cap is set).  Results are
                                    bit-exact as on every form */
    XDROP_VARIANT_ROWS16 = 6     /* four extensions per wavefront (16-cell
                                    windows, one cell per lane, rows of 16
                                    lanes); extensions whose band outgrows
                                    16 cells restart on the wave kernel.
                                    Suits narrow bands (small X).  Ignores
                                    band_cap (runs as WAVE when a cap is
                                    set) */
};
typedef struct {
    int32_t variant;      /* XDROP_VARIANT_* */
    int32_t tile;         /* starting cells per lane: 1, 2, 4 or 8 (band
                             tile 64..512 cells; wider bands widen the tile
                             and then move to the workgroup tier);
                             0 = automatic */
    int32_t chunk;        /* extensions claimed per queue access, 1..64;
                             0 = automatic */
    int32_t band_cap;     /* > 0: seeds whose band exceeds it get
                             XDROP_BAND_OVERFLOW; 0 = no cap */
    int32_t order;        /* 0: longest-first (by m+n) queue order;
                             1: input order */
    int32_t waves_per_cu; /* persistent grid size; 0 = automatic */
    int32_t reserved[2];
} xdrop_options;

typedef struct xdrop_ctx xdrop_ctx;

/* Context options (host struct; NULL = defaults). */
typedef struct {
    int32_t device_tier_slots; /* extensions with bands wider than 2,048
                                  cells that run at once on the
                                  device-memory tier (each holds 768 KiB of
                                  rings); 0 = 32 */
    int32_t reserved[7];
} xdrop_ctx_opts;

/* Create a context on HIP device `device` (the device is made current).
 * *out receives the handle.  A context owns the device workspace of its
 * batches, which every batch reuses: batches on one context must run one
 * after another -- enqueue them on one stream, or order the streams (an
 * event wait, or a synchronisation) between batches on different streams. */
int xdrop_ctx_create(int device, const xdrop_ctx_opts *opts, xdrop_ctx **out);
int xdrop_ctx_destroy(xdrop_ctx *ctx);

/* Extend every seed of a batch.
 *   d_seqs    device, packed sequence stream (encoding = scoring->alphabet);
 *             readable up to the end of the 32-bit word that holds symbol
 *             d_offsets[n_seqs] - 1 (the library never reads further)
 *   d_offsets device, n_seqs+1 int64 symbol offsets; sequence s is symbols
 *             [d_offsets[s], d_offsets[s+1]) of the stream (no alignment
 *             requirement)
 *   d_seeds   device, n_seeds records
 *   d_results device, n_seeds records, written by the enqueued work
 *   stream    hipStream_t (as void*), NULL = default stream
 * Enqueues the work and returns; results are valid after the stream
 * synchronises.  Inputs must stay alive until then.  n_seeds == 0 is a no-op.
 * Returns XDROP_E_INVALID on bad arguments (nothing is launched),
 * XDROP_E_NOMEM / XDROP_E_DEVICE on runtime failures. */
int xdrop_extend_batch(xdrop_ctx *ctx, const uint8_t *d_seqs,
                       const int64_t *d_offsets, int32_t n_seqs,
                       const xdrop_seed *d_seeds, int32_t n_seeds,
                       const xdrop_scoring *scoring,
                       const xdrop_options *opts, xdrop_result *d_results,
                       void *stream);

/* Allocation-free variant of xdrop_extend_batch, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and per-seed
 * statuses as xdrop_extend_batch; it calls no hipMalloc/hipFree and creates
 * no events (phase timing is off for it).  Its counters, queues, result slots
 * and device-memory tier rings live in one fixed 16 MiB device array per GPU
 * (held until the process ends), so a batch may hold at most
 * XDROP_NOALLOC_MAX_SEEDS seeds over at most XDROP_NOALLOC_MAX_SEQS
 * sequences (else XDROP_E_SCRATCH, nothing launched), and at most 4
 * extensions with bands wider than 2,048 cells run at once.  Every call on a
 * GPU shares that array: calls that overlap on one GPU (other streams, other
 * contexts or threads) race and must be ordered by the caller.  Each call
 * clears the counters it needs before use. */
#define XDROP_NOALLOC_MAX_SEEDS 65536
#define XDROP_NOALLOC_MAX_SEQS 1048576
int xdrop_extend_batch_noalloc(xdrop_ctx *ctx, const uint8_t *d_seqs,
                               const int64_t *d_offsets, int32_t n_seqs,
                               const xdrop_seed *d_seeds, int32_t n_seeds,
                               const xdrop_scoring *scoring,
                               const xdrop_options *opts,
                               xdrop_result *d_results, void *stream);

/* Autotune the launch parameters (paper Sec. 4.2: batching extensions of
 * uneven lengths; here the launch form, the starting tile and the queue
 * chunk) on a sample batch: same arguments as xdrop_extend_batch, d_results
 * is scratch.  Every candidate variant / tile / chunk is timed on `stream`
 * (median of three runs after a warm run); the fastest is stored in the
 * context for batches of the same key -- alphabet, X class (X < 24, < 100,
 * >= 100: a stand-in for the band width) and batch size class (seeds
 * < 2,048, < 32,768, < 524,288, more) -- and, if cache_path is not NULL,
 * appended to that JSON-lines file with the device architecture, the
 * sample's mean extension length and the time of the plain form.
 * *best_out (optional) receives the chosen options.  Synchronises `stream`.
 * Results of later batches do not depend on the choice (bit-exact). */
int xdrop_autotune(xdrop_ctx *ctx, const uint8_t *d_seqs,
                   const int64_t *d_offsets, int32_t n_seqs,
                   const xdrop_seed *d_seeds, int32_t n_seeds,
                   const xdrop_scoring *scoring, xdrop_result *d_results,
                   void *stream, const char *cache_path,
                   xdrop_options *best_out);

/* Load tuned options from a JSON-lines cache written by xdrop_autotune:
 * entries whose "arch" is this device's architecture and that hold every
 * key (alphabet, x_class, size_class, variant, tile, chunk, waves_per_cu);
 * a later entry of the same key replaces an earlier one.  XDROP_E_INVALID
 * if the file cannot be read or holds no usable entry. */
int xdrop_load_tuning(xdrop_ctx *ctx, const char *cache_path);

/* The options a batch of n_seeds seeds with this scoring would run with
 * (caller's options over the tuned entry of its key over the defaults, with
 * the automatic form and chunk resolved); nothing is launched. */
int xdrop_resolve_options(xdrop_ctx *ctx, const xdrop_scoring *scoring,
                          int32_t n_seeds, const xdrop_options *opts,
                          xdrop_options *out);

/* Capture the launch sequence of one batch shape into a HIP graph and replay
 * it: identical to xdrop_extend_batch, but the launches are recorded once per
 * (pointers, sizes, scoring, options) and replayed afterwards. */
int xdrop_extend_batch_graph(xdrop_ctx *ctx, const uint8_t *d_seqs,
                             const int64_t *d_offsets, int32_t n_seqs,
                             const xdrop_seed *d_seeds, int32_t n_seeds,
                             const xdrop_scoring *scoring,
                             const xdrop_options *opts,
                             xdrop_result *d_results, void *stream);

/* Phase timing: with timing on, every batch records HIP events on its stream
 * around its launch phases (no host synchronisation).  xdrop_last_timing
 * waits for the last recorded batch, writes to ms[0..n) the durations summed
 * over all batches recorded since timing was switched on or last read --
 * (0) counters, symbol check and longest-first ordering, (1) the first
 * extension kernel (the row kernel for XDROP_VARIANT_PAIR and
 * XDROP_VARIANT_ROWS16, the 16-bit kernel for XDROP_VARIANT_DUAL16, else the
 * wave kernel of 1..8 cells per lane), (2) the wave kernel on the extensions
 * the first kernel handed on (0 for the other variants), (3) the workgroup tier,
 * (4) the seed-level combine -- sets *batches (optional) to their number,
 * and starts a new record.  Returns XDROP_E_INVALID if none was recorded. */
int xdrop_ctx_set_timing(xdrop_ctx *ctx, int32_t on);
int xdrop_last_timing(xdrop_ctx *ctx, float *ms, int32_t n,
                      int32_t *batches);

/* Statistics of the last batch on this context (after stream sync):
 * counts of extensions finished at each tile width: counts[0..3] = 1, 2, 4,
 * 8 cells per lane (wave kernel), counts[4] = two-row (pair) kernel, counts[5] =
 * workgroup (block) tier, bands of 513..2,048 cells, counts[6] =
 * device-memory tier, wider bands, counts[7] = two-extension 16-bit
 * kernel, counts[8] = four-row kernel (XDROP_VARIANT_ROWS16). */
int xdrop_last_stats(xdrop_ctx *ctx, int64_t *counts, int32_t n_counts);

/* ---------------------------------------------------------------- serving
 * Continuous batching: requests (host sequences + seeds + scoring) are
 * admitted against a device-memory budget, copied into a resident pool, and
 * their extensions are fed to a device queue that the worker keeps draining;
 * requests that arrive while others run are admitted as memory frees up.
 */
typedef struct xdrop_server xdrop_server;

typedef struct {
    const uint8_t *seqs;     /* host, packed stream as for xdrop_extend_batch
                                (ignored when seq_set != 0) */
    const int64_t *offsets;  /* host, n_seqs+1 (ignored when seq_set != 0) */
    int32_t n_seqs;
    const xdrop_seed *seeds; /* host; q and t index the request's sequences,
                                or those of the set seq_set */
    int32_t n_seeds;
    xdrop_scoring scoring;
    uint64_t seq_set;        /* 0: the request's own sequences; else a set
                                from xdrop_server_put_sequences (same
                                encoding as scoring.alphabet), shared with
                                other requests and not copied again */
} xdrop_request;

typedef struct {
    int32_t max_inflight;   /* requests admitted to run at once; 0 = 256 */
    int32_t streams;        /* micro-batches in flight at once; 0 = 4 */
    int32_t arena_mib;      /* sequence arena in MiB; 0 = everything the
                               budget leaves after the per-stream staging and
                               workspace (40 MiB per stream) */
    int32_t staging_mib;    /* pinned host staging of sequences not yet on
                               the device (host memory, outside the budget);
                               0 = 64 */
    int32_t reserved[4];
} xdrop_server_opts;

/* Counters of a server since its creation. */
typedef struct {
    int64_t requests_submitted, requests_done;
    int64_t batches_launched;
    int64_t batches_in_flight;      /* micro-batches on the device now */
    int64_t max_batches_in_flight;  /* most at once so far */
    int64_t admitted_while_busy;    /* requests admitted while a micro-batch
                                       of other requests was running */
    int64_t h2d_bytes;              /* sequence bytes copied to the device */
    int64_t reused_bytes;           /* bytes of the sequences that requests
                                       seeded against resident sets used
                                       without copying them */
    int64_t reserved[8];
} xdrop_server_counters;

/* hbm_budget_bytes bounds all device memory of the server: the sequence
 * arena plus 40 MiB per stream.  XDROP_E_BUDGET if that does not fit. */
int xdrop_server_create(int device, size_t hbm_budget_bytes,
                        const xdrop_server_opts *opts, xdrop_server **out);
/* Copies the request (its sequences into pinned staging, from where the
 * worker moves them to the device asynchronously); returns XDROP_E_BUDGET if
 * it can never fit, XDROP_E_INVALID for an unknown or released seq_set. */
int xdrop_server_submit(xdrop_server *srv, const xdrop_request *req,
                        uint64_t *ticket);
/* Register sequences that many requests will seed against (paper Sec.
 * 4.1.1 and Sec. 4.3: sequences kept apart from the seed tuples and shared
 * between comparisons): copied once, resident until released and no
 * request uses them.  *set_id receives the id for xdrop_request.seq_set.
 * XDROP_E_BUDGET if the set can never fit the arena or holds more than
 * 131,071 sequences. */
int xdrop_server_put_sequences(xdrop_server *srv, const uint8_t *seqs,
                               const int64_t *offsets, int32_t n_seqs,
                               int32_t alphabet, uint64_t *set_id);
/* No new request may use the set; its memory is freed when the requests
 * that use it are done. */
int xdrop_server_release_sequences(xdrop_server *srv, uint64_t set_id);
int xdrop_server_stats(xdrop_server *srv, xdrop_server_counters *out);
/* XDROP_PENDING or XDROP_OK (then host_out holds n_seeds results and the
 * ticket is released). */
int xdrop_server_poll(xdrop_server *srv, uint64_t ticket,
                      xdrop_result *host_out);
/* Block until done or timeout_ns passes (< 0: no limit). */
int xdrop_server_wait(xdrop_server *srv, uint64_t ticket,
                      xdrop_result *host_out, int64_t timeout_ns);
int xdrop_server_destroy(xdrop_server *srv);

const char *xdrop_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* XDROP_H */
