/* hda.h -- out-of-band-metadata allocators for memory the allocator never
 * reads, replayed on an AMD Instinct MI355X (gfx950).
 *
 * The allocators are those of "Host-Based Allocators for Device Memory"
 * (Bell, Kumar, Gill): first fit, next fit, best fit (Sec. II-A, Sec. IV,
 * Alg. 1-3) and segregated fit (Sec. II-B, Sec. V-A, Alg. 4-5).  The managed
 * arena is virtual: the library hands out byte offsets into [0, arena_bytes)
 * and never reads, writes or backs that range (Sec. I: large arenas come from
 * the driver, fine-grained allocation happens elsewhere, and the allocator
 * cannot read the memory it manages).  A caller that owns real memory adds its
 * base pointer to the offsets.
 *
 * Conventions shared by every entry point
 *  - Sizes and offsets are bytes (int64).  A request of `size` bytes is
 *    normalised to s = max(align, roundup(size, align)); a block is always
 *    taken from the low end of the chosen free block (Alg. 1, Alg. 4).
 *  - Allocation failure is the value -1 (HDA_FAIL), never an error.
 *  - Every error leaves the heap's state unchanged.
 *  - Pointers documented as "device" must be device-accessible memory
 *    (hipMalloc / torch CUDA tensors) that stays alive until the stream
 *    work that uses them has completed; the library never frees them.
 *  - Functions taking a `stream` enqueue work on that hipStream_t (NULL = the
 *    null stream) and return without waiting, unless stated otherwise.
 */
#ifndef HDA_H
#define HDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Algorithms (per heap). */
enum {
  HDA_FIRST_FIT = 0, /* lowest-address free block with size >= s (Sec. II-A) */
  HDA_NEXT_FIT = 1,  /* first fit resumed at a rover (Sec. II-A, Sec. IV)    */
  HDA_BEST_FIT = 2,  /* smallest block >= s, lowest address on ties (Alg. 3) */
  HDA_SEG_FIT = 3,   /* power-of-two classes + bitmap, LIFO lists (Alg. 4-5) */
  HDA_TLSF = 4,      /* two-level segregated fit (Sec. V-B): each power of two
                        split into 32 linear sub-classes; a request is rounded
                        up to the next sub-class bound and served from the
                        first non-empty class at or above it (two-level
                        bitmap lookup); lists as in segregated fit          */
  HDA_BITMAP = 5     /* bitmask allocator (Sec. III-B): one flag per granule;
                        an allocation takes the first run of free granules
                        found scanning from the rover (the end of the last
                        allocation), else from granule 0.  Replayed only by
                        hda_bitmap_replay; its state lists the free runs and
                        the rover as for next fit                           */
};

/* Status codes. */
enum {
  HDA_OK = 0,
  HDA_FAIL = -1,      /* allocation: nothing fits (a result, not an error)   */
  HDA_E_INVAL = -2,   /* bad argument (see each function)                    */
  HDA_E_BADFREE = -3, /* free of an offset that is not a live block's start
                          (partial free: that lies in no live block)         */
  HDA_E_NOMETA = -4,  /* per-heap metadata capacity exhausted                */
  HDA_E_DEVICE = -5,  /* a HIP runtime call failed                           */
  HDA_E_BUSY = -6,    /* resource in use (service running, budget held)      */
  HDA_E_RANGE = -7    /* an output buffer is too small                       */
};

/* ------------------------------------------------------------------------ */
/* Device memory the library keeps for itself.                              */
/* ------------------------------------------------------------------------ */

/* The library's own device buffers -- call-by-call heap metadata and result
 * buffers, the service's heap pool, the autotuner's trial batch -- are
 * obtained from `alloc` and returned to `release`, each called with `ctx`
 * (for instance the caller's caching allocator); with none installed (both
 * NULL, the default) hipMalloc / hipFree are used.  `alloc` returns device
 * memory of at least `bytes` bytes, 256-byte aligned, or NULL (the library
 * call then fails with HDA_E_DEVICE); the library never touches a buffer
 * after releasing it and releases it only once its own work on it has
 * completed.  Callbacks run on the thread that made the library call.
 * HDA_E_INVAL if exactly one of the two is NULL; HDA_E_BUSY while buffers
 * from the allocator installed before are still held (release them first:
 * destroy heaps, stop the service).  Batch buffers and workspaces of the
 * replay calls are always the caller's. */
typedef void *(*hda_dev_alloc_fn)(size_t bytes, void *ctx);
typedef void (*hda_dev_free_fn)(void *ptr, void *ctx);
int hda_set_device_allocator(hda_dev_alloc_fn alloc, hda_dev_free_fn release, void *ctx);

/* ------------------------------------------------------------------------ */
/* Batched replay (many independent heaps, one persistent launch).          */
/* ------------------------------------------------------------------------ */

/* Request encoding, one int64 per request, heap h owning
 * req[req_off[h] .. req_off[h+1]):
 *   req >= 0 : allocate req bytes;           result = byte offset, or -1.
 *   req <  0 : free one live block: with u = ~req, r = u mod 2^32 is a
 *              uniform 32-bit draw and the victim is live[(r * L) >> 32],
 *              where live[] lists the heap's live blocks (a successful
 *              allocation appends its block; a whole free moves the last
 *              entry into the freed slot) and L is their number.  The cut
 *              c = u >> 32 (< 2^31) asks for a partial deallocation (Sec.
 *              II-A, Alg. 2; first, next and best fit): the victim's first
 *              floor(c * granules / 2^31) granules stay live and the rest is
 *              freed; 0 granules kept is a whole free.  Segregated fit
 *              ignores c (Alg. 5 frees whole blocks).  result = the byte
 *              offset of the freed part, or -1 when no block is live (the
 *              request then does nothing).
 * A request that would exceed the heap's metadata capacity yields
 * HDA_E_NOMETA as its result and changes nothing.
 *
 * Canonical state of a heap, int64 words (all addresses/sizes in bytes):
 *   n_free, (addr, size) x n_free in address order,
 *   n_live, (addr, size) x n_live in live[] order,
 *   rover (next fit: the byte address the next search resumes at) or -1,
 *   class bitmap (segregated fit: bit k <=> class k list non-empty; TLSF:
 *     bit fl <=> one of the lists of level fl non-empty) or 0,
 *   segregated fit: for each class k = 0..63 (sizes in [2^k, 2^(k+1))):
 *     len_k, then the block addresses from list head to tail;
 *   TLSF: the same for each class c = fl * 32 + sl = 0..2047, which holds
 *     sizes b with floor(log2 b) = fl and (b >> (fl - 5)) - 32 = sl
 *     ((b << (5 - fl)) - 32 below 32 bytes).
 * A heap with n_req requests needs at most 4 + 4 * (n_req + 1) words, plus
 * 64 + n_req + 1 for segregated fit and 2048 + n_req + 1 for TLSF.
 */
/* Where each heap's tables live.  Default (lean) path: the first
 * 64*reg_free free-table entries are held in vector registers (reg_free = 1,
 * 2 or 4; 0 = 2); the rest of the free table and the whole live table share
 * one LDS pool per heap of lds_free * 16 + lds_live * 8 bytes (defaults 128
 * and 1024: 10 KiB), free entries from its start and live entries from its
 * end.  A heap whose tables outgrow the pool before reaching meta_free /
 * meta_live moves them, mid-trace, to the general path in its device-memory
 * slot of the workspace and continues there; results do not depend on the
 * tuning.  reg_free = -1 selects the general path for every heap: no
 * registers, lds_free free and lds_live live entries in LDS (defaults 64 and
 * 1024), the rest in device memory (workspace).  reg_live must be 0 or -1
 * (the live table is never held in registers).  0 = default for every
 * field; -1 = none of that storage.  Any other value is E_INVAL. */
typedef struct hda_tuning {
  int32_t heaps_per_group; /* waves (= heaps in flight) per workgroup (1..16)  */
  int32_t reg_free;        /* free-table 64-entry chunks in registers          */
  int32_t reg_live;        /* live-table 64-entry chunks in registers          */
  int32_t lds_free;        /* free-table entries in LDS per heap (mult. of 64) */
  int32_t lds_live;        /* live-table entries in LDS per heap (mult. of 64) */
  int32_t groups;          /* persistent workgroups (0 = fill the device)      */
  int32_t heavy_heaps;     /* the first heavy_heaps heaps of the order are
                              replayed by the ordered core in a launch of
                              their own beside the others' (0 = none)          */
  int32_t heavy_kib;       /* LDS pool per ordered-core heap, KiB (16 up to the
                              device's LDS per workgroup; 0 = 64)             */
} hda_tuning;

typedef struct hda_batch_desc {
  int64_t n_heaps;          /* H >= 0                                          */
  const int64_t *arena;     /* device [H]: arena bytes (> 0, multiple of align) */
  const int64_t *align;     /* device [H]: alignment bytes (power of two)       */
  const int32_t *algo;      /* device [H]: HDA_FIRST_FIT .. HDA_TLSF            */
  const int64_t *req_off;   /* device [H+1]: CSR offsets into req/res           */
  const int64_t *req;       /* device [req_off[H]]: encoded requests (non-null,
                               also when req_off[H] == 0)                       */
  int64_t *res;             /* device [req_off[H]]: results (written; non-null) */
  const int32_t *order;     /* device [H] or NULL: heap processing order
                               (a permutation; NULL = 0..H-1)                   */
  int64_t *state;           /* device or NULL: canonical states (written)       */
  const int64_t *state_off; /* device [H+1]: heap h's state slot is
                               state[state_off[h] .. state_off[h+1])            */
  int64_t *state_len;       /* device [H]: words of heap h's state (written;
                               set even when the slot is too small)             */
  int32_t *status;          /* device [H]: HDA_OK or the heap's first error
                               (E_INVAL bad heap params, E_NOMETA capacity,
                               E_RANGE state slot too small)                    */
  int64_t meta_free;        /* free-table capacity per heap (entries)           */
  int64_t meta_live;        /* live-table capacity per heap (entries)           */
  void *workspace;          /* device scratch of hda_replay_workspace() bytes   */
  size_t workspace_bytes;
  hda_tuning tuning;
} hda_batch_desc;

/* Bitmask-allocator replay (Sec. III-B): every heap of `d` must be
 * HDA_BITMAP with arena / align <= max_granules (< 2^32); other heaps get
 * HDA_E_INVAL as status and as every result.  One wavefront per heap keeps
 * one flag per granule and a summary per 4,096 granules (free runs at the
 * bottom, at the top, longest), and searches 64 words of flags or 64
 * summaries per step.  Requests, results, states and statuses as for
 * hda_replay (partial frees included; the live table holds meta_live
 * entries, HDA_E_NOMETA past it; meta_free is not used).  The workspace
 * holds each wave's flags, summaries and live table, about
 * max_granules / 8 + 8 * meta_live bytes per wave for up to 4,096 waves:
 * hda_bitmap_workspace(d, max_granules) bytes (0 on invalid arguments).
 * Asynchronous on `stream`; HDA_E_RANGE if the workspace is too small. */
size_t hda_bitmap_workspace(const hda_batch_desc *d, uint64_t max_granules);
int hda_bitmap_replay(const hda_batch_desc *d, uint64_t max_granules, void *stream);

/* Bytes of device scratch hda_replay needs for `d` (reads only n_heaps,
 * meta_free, meta_live and tuning).  Returns 0 on invalid arguments. */
size_t hda_replay_workspace(const hda_batch_desc *d);

/* hda_replay for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid allocation):
 * the same replay, but the scratch it needs lives in a device array of
 * HDA_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; d->workspace and d->workspace_bytes are ignored.
 * Nothing is allocated or freed (no hipMalloc / hipFree, no allocator
 * callback).  HDA_E_RANGE when hda_replay_workspace(d) exceeds
 * HDA_STATIC_SCRATCH_BYTES (fewer heaps per call, smaller meta_free /
 * meta_live, or fewer persistent groups bring it down); HDA_E_INVAL /
 * HDA_E_DEVICE as for hda_replay.  Every call on one GPU uses that GPU's one
 * array, which keeps the last call's contents: calls whose work overlaps on
 * one GPU (on different streams, or from different threads) race and must
 * not be made; calls in sequence on one stream are fine.  Asynchronous on
 * `stream`; the caller's buffers in `d` as for hda_replay. */
#define HDA_STATIC_SCRATCH_BYTES (64u << 20)
int hda_replay_static(const hda_batch_desc *d, void *stream);

/* Resolve the tuning actually used for `d` (autotuned defaults filled in). */
int hda_replay_resolve(const hda_batch_desc *d, hda_tuning *out);

/* Enqueue the replay of every heap of `d` on `stream` as one persistent
 * kernel launch.  Heaps are pulled from a device queue in `order`; each heap
 * is replayed in request order by one wavefront, so results are identical to
 * sequential in-order replay of each heap whatever the tuning.
 * Returns HDA_E_INVAL for null or inconsistent descriptor fields,
 * HDA_E_RANGE if workspace_bytes is too small, HDA_E_DEVICE on launch
 * failure; per-heap problems are reported through `status`. */
int hda_replay(const hda_batch_desc *d, void *stream);

/* The per-heap-launch baseline: the same kernel body launched once per heap
 * (H launches of one wavefront each, in `order`, on `stream`). */
int hda_replay_per_heap(const hda_batch_desc *d, void *stream);

/* Autotuner.  Picks heaps_per_group and the LDS residency (lds_free,
 * lds_live) of the default path for `d` by timing candidate tunings, with HIP
 * events on `stream`, on a private copy of the batch's longest heaps (which
 * set the makespan): up to sample_heaps of them (0 = as many as the device
 * holds at once), each trace cut to its first 65,536 requests, at most 16 M
 * requests in all.  Candidates: 1, 2, 4, 8 or 16 heaps per workgroup x
 * (lds_free, lds_live) = (64, 512), (128, 1024), (256, 2048), (512, 4096),
 * those that fit the device's LDS; then, with the fastest of those, 0, 16,
 * 64 or 128 heaps (the longest) on the ordered core (heavy_heaps, 64 KiB
 * pools), timed on the 128 longest heaps with traces cut to 1 M requests
 * (not tried when meta_free exceeds the 4,096 free blocks that core holds).
 * A later call on a batch of the same shape on the same device (heap count,
 * capacities, sample_heaps, reg_free, and every heap's trace length, arena,
 * alignment and algorithm) returns the earlier choice without timing.  The
 * fastest is written to *out; put it
 * into d->tuning (and size the workspace for it) before the replay.  The
 * caller's buffers are only read.  Temporary device memory is allocated and
 * freed here.  Synchronous.  HDA_E_INVAL for an invalid descriptor,
 * HDA_E_DEVICE on a HIP failure. */
int hda_replay_autotune(const hda_batch_desc *d, int32_t sample_heaps, void *stream,
                        hda_tuning *out);

/* One hda_replay call on `d` recorded as a hipGraph (the classify kernel and
 * the replay kernel, captured on a private stream),
 * for callers that replay the same descriptor buffers repeatedly: each
 * hda_graph_launch re-runs the whole replay from the heaps' initial state on
 * `stream`, exactly as hda_replay would.  The descriptor's buffers must stay
 * valid and in place while the graph exists; the graph records no memset.
 * Library-owned; release with hda_graph_destroy.  Capture is synchronous.
 * HDA_E_INVAL / HDA_E_RANGE as for hda_replay, HDA_E_DEVICE on a HIP
 * failure. */
typedef struct hda_graph hda_graph; /* opaque, library-owned */
int hda_replay_capture(const hda_batch_desc *d, hda_graph **out);
int hda_graph_launch(hda_graph *g, void *stream);
int hda_graph_destroy(hda_graph *g);

/* ------------------------------------------------------------------------ */
/* Single heaps driven call by call (Alg. 6 init; Alg. 1-5 per call).       */
/* ------------------------------------------------------------------------ */

typedef struct hda_heap hda_heap; /* opaque, library-owned */

/* Create a heap over a virtual arena of arena_bytes (Alg. 6: one free block
 * [0, arena_bytes)).  Metadata lives in device memory the library obtains
 * from the installed device allocator (hda_set_device_allocator): meta_cap
 * bounds both the free-table and the live-table entries (0 = 4096).  Calls
 * on heaps of one device run on one library stream of that device.
 * HDA_E_INVAL: align not a power of two, arena_bytes == 0 or not a multiple
 * of align, arena_bytes / align >= 2^32, unknown algo, out == NULL.
 * HDA_E_NOMETA: the metadata budget (hda_set_meta_budget) is exhausted.
 * Synchronous. */
int hda_heap_create(uint64_t arena_bytes, uint64_t align, int algo,
                    uint32_t meta_cap, hda_heap **out);

/* Release a heap and return its metadata to the budget.  Synchronous. */
int hda_heap_destroy(hda_heap *h);

/* Allocate `size` bytes: returns the byte offset, -1 when nothing fits, or
 * HDA_E_NOMETA / HDA_E_DEVICE / HDA_E_INVAL (h == NULL).  Synchronous: one
 * kernel launch on the library's stream. */
int64_t hda_alloc(hda_heap *h, uint64_t size);

/* Free the block starting at `offset`; neighbours that are free are merged
 * (Alg. 2, Alg. 5).  HDA_E_BADFREE if `offset` is not the start of a live
 * block.  Synchronous. */
int hda_free(hda_heap *h, int64_t offset);

/* Partial deallocation (Sec. II-A, Alg. 2): free from `offset` to the end of
 * the live block holding it.  The block keeps [start, offset) live; at the
 * block's start this is hda_free.  HDA_E_BADFREE, state unchanged, if
 * `offset` is not a multiple of the alignment or lies in no live block, and,
 * for segregated fit (which frees whole keyed blocks, Alg. 5), if it is not
 * a block's start.  HDA_E_NOMETA if the freed tail needs a table entry past
 * the capacity.  Synchronous. */
int hda_free_partial(hda_heap *h, int64_t offset);

/* Copy the heap's canonical state (format above) into host buffer `buf` of
 * `cap` words; *len receives the words needed.  HDA_E_RANGE if cap < *len.
 * Synchronous. */
int hda_heap_state(const hda_heap *h, int64_t *buf, size_t cap, size_t *len);

/* Resume a heap from a canonical state (the format above, as written by
 * hda_heap_state or by a replay's state dump) of a heap with the same arena,
 * alignment and algorithm: the free blocks, the live blocks in live-table
 * order, the next-fit rover and the class lists in head-to-tail order all
 * become this heap's (Alg. 6 initialises a heap from one block; this
 * initialises it from any reachable state).  `buf` is a host buffer of `len`
 * words.  HDA_E_INVAL, heap unchanged, when the state is malformed or not a
 * state of this heap: words missing or left over, free blocks not in
 * ascending address order, blocks that are unaligned, empty, overlapping or
 * do not tile [0, arena), two adjacent free blocks, a rover outside
 * [0, arena] or unaligned (next fit) or not -1 (the others), a bitmap that
 * does not match the lists, a free block in no list, in the wrong list or in
 * two (segregated fit, TLSF), lists or a bitmap on the other algorithms.
 * HDA_E_NOMETA, heap unchanged, when the blocks exceed the heap's metadata
 * capacity.  Synchronous. */
int hda_heap_load(hda_heap *h, const int64_t *buf, size_t len);

/* Metadata budget (bytes of device memory all live heaps may hold);
 * 0 = unlimited (the default).  Returns the bytes currently held. */
int64_t hda_set_meta_budget(int64_t bytes);

/* ------------------------------------------------------------------------ */
/* Serving: a device-resident allocator service with continuous batching.   */
/* ------------------------------------------------------------------------ */

/* A persistent kernel keeps every admitted heap's state in device memory
 * and serves alloc/free requests that clients submit while it runs.  Heap
 * slot s is served by wave s % waves, which applies that heap's requests in
 * submission (FIFO) order; requests of different heaps run in parallel on
 * different waves, and a request submitted while others are on the GPU is
 * picked up by its wave as soon as the wave reaches it -- there is no batch
 * boundary.  Requests travel through per-wave rings in pinned host memory
 * (submission and completion); the kernel exits when hda_serve_stop raises
 * its stop flag or after max_seconds, whichever comes first.  Each heap runs
 * the same allocator code as hda_alloc / hda_free (Alg. 1-5). */
typedef struct hda_server hda_server;

typedef struct hda_serve_config {
  int32_t waves;          /* service wavefronts; 0 = 2 per CU               */
  int32_t max_heaps;      /* heap slots in the device pool (> 0)            */
  int32_t slot_free;      /* free-table capacity per heap; 0 = 512          */
  int32_t slot_live;      /* live-table capacity per heap; 0 = 512          */
  int32_t ring_entries;   /* ring size per wave, power of two; 0 = 1024     */
  int32_t reserved;
  int64_t meta_budget;    /* bytes of heap metadata admitted at once;
                             0 = every slot                                 */
  double max_seconds;     /* watchdog on the kernel; 0 = 600                */
} hda_serve_config;

enum { HDA_OP_ALLOC = 1, HDA_OP_FREE = 2 };

/* Start the service on the current device (allocates the pool and rings,
 * launches the kernel on a library stream).  HDA_E_INVAL for bad config. */
int hda_serve_start(const hda_serve_config *cfg, hda_server **out);

/* Admit a heap (Alg. 6 init on its wave; asynchronous).  *heap receives its
 * slot id.  HDA_E_NOMETA when the metadata budget or the slots are used up
 * (close a heap and retry); HDA_E_INVAL for bad arena/align/algo as in
 * hda_heap_create. */
int hda_serve_open(hda_server *s, uint64_t arena_bytes, uint64_t align, int algo,
                   int32_t *heap);

/* Submit one request: op = HDA_OP_ALLOC with arg = size in bytes, or
 * HDA_OP_FREE with arg = byte offset.  *ticket identifies the result.
 * Blocks only while the heap's ring is full.  The result is the offset / -1
 * / HDA_E_NOMETA for an allocation and HDA_OK / HDA_E_BADFREE for a free. */
int hda_serve_submit(hda_server *s, int32_t heap, int op, int64_t arg, uint64_t *ticket);

/* Non-blocking: *done = 1 and *result set once the ticket has completed.
 * HDA_E_RANGE if the ticket is older than the ring keeps. */
int hda_serve_poll(hda_server *s, uint64_t ticket, int64_t *result, int *done);

/* Blocking form of hda_serve_poll; HDA_E_BUSY after 30 s without the
 * completion (for instance once the service has stopped). */
int hda_serve_wait(hda_server *s, uint64_t ticket, int64_t *result);

/* Release a heap: waits for its queued requests, frees its slot and returns
 * its metadata to the budget. */
int hda_serve_close(hda_server *s, int32_t heap);

/* Stop the kernel (drains nothing further), wait for it, free everything. */
int hda_serve_stop(hda_server *s);

/* Open-loop load: `clients` clients, each owning one heap, issue requests at
 * Poisson arrival times of total rate `rate` per second (each arrival picks a
 * client uniformly).  A client whose earliest-expiring live block has expired
 * frees it, otherwise it allocates: with probability p_pow2 a size 2^k,
 * k uniform in [pow2_lo, pow2_hi], else log-uniform in [size_lo, size_hi]
 * bytes; a successful allocation lives ceil(Exp(lifetime_mean)) of that
 * client's requests.  A client has at most one request in flight; arrivals
 * meanwhile wait in its queue (their wait counts in their latency).
 * Latency = completion seen by the host - arrival time. */
typedef struct hda_load_config {
  int32_t clients;
  int32_t algo;
  int32_t threads;        /* host threads driving clients; 0 = 4            */
  int32_t log_clients;    /* first clients whose requests/results are logged */
  int64_t log_cap;        /* entries per logged client                      */
  int64_t *log;           /* host [log_clients * log_cap * 3]: row 0 is
                             (0, arena, align), then (op, arg, result) per
                             completed request in the client's order          */
  int64_t *log_len;       /* host [log_clients]                             */
  uint64_t arena_lo, arena_hi, align;   /* per-client arena: log-uniform   */
  double rate;            /* arrivals per second                            */
  double warmup_s, measure_s;
  double p_pow2;
  int32_t pow2_lo, pow2_hi;
  uint64_t size_lo, size_hi;
  double lifetime_mean;
  uint64_t seed;
  int32_t close_heaps;    /* 1: close every client heap at the end          */
  int32_t session_len;    /* 0: every client holds one heap for the whole
                             run (all admitted before it starts; a refused
                             admission ends the call with its error).  n > 0:
                             clients work in sessions of n requests -- a
                             session opens a fresh heap of the client's arena
                             when the metadata budget admits it (until then
                             the client's arrivals wait, and their wait counts
                             in their latency) and closes it after its n-th
                             request, returning its budget; a logged client's
                             log then has a (0, arena, align) row at the start
                             of each session                                */
} hda_load_config;

typedef struct hda_load_report {
  int64_t issued, completed, measured;  /* requests; measured = in window  */
  int64_t alloc_ok, alloc_fail, frees, errors;
  double window_s;                      /* measured window length           */
  double throughput;                    /* completions per second in window */
  double p50_us, p90_us, p99_us, p999_us, max_us, mean_us;
  /* components of the measured latencies (p50 and p99 of each): waiting on
   * the host before submission (the client's earlier request still in
   * flight, or the load thread behind), queueing on the device (seen in the
   * ring -> picked up by its wave), service on the device (picked up ->
   * done), and the rest (ring transit both ways and harvesting) */
  double host_p50_us, host_p99_us, queue_p50_us, queue_p99_us;
  double service_p50_us, service_p99_us, transit_p50_us, transit_p99_us;
  int64_t sessions;         /* sessions ended (heaps closed) during the run  */
  int64_t admission_waits;  /* times a client with requests waited for
                               admission                                     */
  int64_t max_open;         /* most heaps open at once                       */
  int64_t slot_bytes;       /* metadata bytes one open heap holds             */
} hda_load_report;

int hda_serve_load(hda_server *s, const hda_load_config *cfg, hda_load_report *rep);

/* Bytes of device metadata one admitted heap holds under `cfg` (the unit of
 * the metadata budget), or HDA_E_INVAL. */
int64_t hda_serve_slot_bytes(const hda_serve_config *cfg);

/* Static description of an error code. */
const char *hda_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* HDA_H */
