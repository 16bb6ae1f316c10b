/*
 * convhull.h -- C ABI of the MI355X (gfx950) convex-hull library.
 *
 * The library computes, on the GPU, the heaphull-style filter and a device
 * hull pass described by A. Keith, H. Ferrada, C. A. Navarro, "Accelerating
 * the Convex Hull Computation with a Parallel GPU Algorithm" (arXiv 2209.12310):
 *   - Alg. 1 (heaphull): n points P[1..n] in, the hull CH[1..h] out in
 *     counter-clockwise order.
 *   - Alg. 2 (GPUfilter) and Sec. III: the extreme points (four axis extremes,
 *     then the four points closest in Manhattan distance to the corners of
 *     their box) form an octagon; a point survives when it lies outside it.
 *   - Sec. I, stage 1: a point on a side of the octagon that is not one of
 *     its vertices is discarded.
 *
 * Conventions shared by every entry point:
 *   - Points are interleaved float32 pairs (x0, y0, x1, y1, ...), at least
 *     8-byte aligned. Every coordinate must equal k * 2^-20 for an integer k
 *     in [0, 2^20) (the value -0.0 counts as 0). Anything else (NaN, inf,
 *     outside [0,1), off the grid) is a domain error. On this grid every
 *     orientation test is exact, so results are bit-for-bit reproducible.
 *   - Indices are 0-based uint32 (the paper's arrays are 1-based).
 *   - The hull lists the strict vertices (collinear boundary points are not
 *     vertices) counter-clockwise, starting at the lexicographic minimum
 *     (smallest x, then smallest y). Duplicated coordinates are reported by
 *     their smallest index. A single distinct point gives h = 1; a collinear
 *     set gives its two end points, lexicographic minimum first; n = 0 gives
 *     h = 0.
 *   - Pointers named d_* are device memory, h_* host memory. All buffers are
 *     owned by the caller. The library allocates no device memory on any call
 *     after ch_ctx_create; scratch memory is the caller's workspace d_ws of at
 *     least the size the matching *_workspace_bytes function returns.
 *   - A workspace passed to a context must not be written by the caller while
 *     that context uses it; the library keeps its own counters there in a
 *     consistent state from one call to the next.
 *   - stream is a hipStream_t (NULL = the legacy default stream).
 *   - A ch_ctx is used by one host thread at a time.
 */
#ifndef CONVHULL_H
#define CONVHULL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CH_OK = 0,
  CH_E_INVALID_ARG = 1, /* bad pointer, size, alignment or workspace size   */
  CH_E_DOMAIN = 2,      /* a coordinate is off the 2^-20 grid in [0,1)     */
  CH_E_CAPACITY = 3,    /* output buffer too small; required size reported */
  CH_E_NOMEM = 4,       /* host or device allocation failed (create only)  */
  CH_E_DEVICE = 5,      /* a HIP runtime call failed                       */
  CH_E_BUSY = 6,        /* admission refused: budget or queue full         */
  CH_E_TIMEOUT = 7,     /* a wait ran out of time                          */
  CH_E_CANCELLED = 8,   /* the request was cancelled                       */
  CH_E_SHUTDOWN = 9,    /* the server stopped before the request finished  */
  CH_E_NOT_FOUND = 10   /* unknown ticket                                  */
} ch_status;

/* Count value ch_filter writes when the input has a domain error. */
#define CH_COUNT_DOMAIN_ERROR 0xFFFFFFFFu
/* Largest point count of one set (indices and counts stay below 2^31). */
#define CH_MAX_POINTS 0x7FFFFFFFu

typedef struct ch_ctx ch_ctx;

/* The octagon of Sec. III in slot order E, NE, N, NW, W, SW, S, SE:
 * grid coordinates (kx = x * 2^20) and the smallest index holding each
 * vertex. Ties in an extreme are broken towards the counter-clockwise end of
 * the supporting side (E: larger y, N: smaller x, W: smaller y, S: larger x,
 * NE/SE: larger y, NW/SW: smaller y). */
typedef struct {
  int32_t kx[8];
  int32_t ky[8];
  uint32_t idx[8];
} ch_octagon;

/* Create a context bound to HIP device `hip_device`. tune_cache_path (may be
 * NULL) names a text file of batch tuning results (see ch_tune_batch); it is
 * read here if it exists. Allocates pinned host staging memory and nothing
 * on the device. Environment variables read here (tests and measurement;
 * none changes a result): CH_REDUCE_BLOCKS, CH_FILTER_BLOCKS,
 * CH_FUSED_BLOCKS, CH_NARROW_BLOCKS (grid sizes of the streaming passes),
 * CH_HULL_WAIT=stream (wait for ch_hull's stream instead of watching the
 * result block), CH_LARGE_DIRECT (survivors from which ch_hull goes
 * straight to the large-hull path), CH_SECOND_POLY=0 (no second polygon in
 * ch_hull).
 * Errors: CH_E_INVALID_ARG (out is NULL), CH_E_DEVICE, CH_E_NOMEM. */
ch_status ch_ctx_create(int hip_device, const char* tune_cache_path, ch_ctx** out);
/* Destroy a context (NULL is ignored). Waits for nothing: the caller must
 * have synchronised the streams it used. */
void ch_ctx_destroy(ch_ctx* ctx);
/* Static text for a status code. */
const char* ch_status_string(ch_status s);
/* Detail text of the last error on this context (never NULL). */
const char* ch_last_error(const ch_ctx* ctx);

/* Device workspace bytes needed by ch_filter / ch_hull for n points. */
size_t ch_filter_workspace_bytes(uint32_t n);
size_t ch_hull_workspace_bytes(uint32_t n);

/*
 * ch_filter -- the filtering stage (Alg. 2 with Sec. III's extremes).
 * Asynchronous: enqueues its kernels on `stream` and returns.
 *   d_xy        n points (see conventions).
 *   d_survivors capacity n; receives the surviving indices in ascending order.
 *   d_count     one uint32: the number of survivors, or
 *               CH_COUNT_DOMAIN_ERROR when the input has a domain error (the
 *               other outputs are then unspecified).
 *   d_label     optional (NULL to skip), n bytes: 0 for a discarded point, else
 *               1 + floor(i/2) for the first octagon edge i (from slot i to
 *               slot i+1) the point lies strictly outside of, or for a vertex
 *               outside no edge 1 + floor(k/2) with k its first slot. (The
 *               paper's findQueue rule is not given; this one is ours.)
 *   d_oct       optional (NULL to skip): the octagon.
 *   d_ws        workspace of ws_bytes >= ch_filter_workspace_bytes(n).
 * Returns CH_OK once enqueued; CH_E_INVALID_ARG for NULL required pointers,
 * n > CH_MAX_POINTS, a misaligned d_xy or a small workspace; CH_E_DEVICE when
 * a launch fails. n = 0 writes a zero count.
 */
ch_status ch_filter(ch_ctx* ctx, const float* d_xy, uint32_t n, uint32_t* d_survivors,
                    uint32_t* d_count, uint8_t* d_label, ch_octagon* d_oct, void* d_ws,
                    size_t ws_bytes, void* stream);

/*
 * ch_filter_noalloc -- ch_filter for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same kernels and outputs as ch_filter, with no
 * workspace argument. Its scratch is a fixed library-owned device array of
 * ch_filter_noalloc_scratch_bytes() bytes per device (the ch_filter workspace
 * for CH_FILTER_NOALLOC_MAX_POINTS points), loaded with the library and held
 * until the process ends. Nothing is allocated or freed on the call path.
 *   Arguments as ch_filter (d_xy, d_survivors, d_count, d_label, d_oct,
 *   stream; caller-owned device buffers).
 * Returns CH_E_INVALID_ARG for n > CH_FILTER_NOALLOC_MAX_POINTS (and as
 * ch_filter), CH_E_DEVICE as ch_filter. Every call on one device shares that
 * device's scratch: calls that overlap on one device (concurrent streams,
 * several host threads or contexts) race and must be serialised by the
 * caller; calls in one stream are ordered and safe.
 */
#define CH_FILTER_NOALLOC_MAX_POINTS (1u << 22)
size_t ch_filter_noalloc_scratch_bytes(void);
ch_status ch_filter_noalloc(ch_ctx* ctx, const float* d_xy, uint32_t n, uint32_t* d_survivors,
                            uint32_t* d_count, uint8_t* d_label, ch_octagon* d_oct, void* stream);

/*
 * ch_hull -- the whole path of Alg. 1: filter, then the hull of the survivors
 * on the device. Synchronous with respect to `stream`: returns after the hull
 * is in host memory.
 *   h_hull_idx  host buffer of `cap` entries for the hull indices.
 *   h_out       receives h.
 * Errors: CH_E_DOMAIN (outputs untouched), CH_E_CAPACITY (*h_out = required
 * h, h_hull_idx untouched), CH_E_INVALID_ARG, CH_E_DEVICE.
 */
ch_status ch_hull(ch_ctx* ctx, const float* d_xy, uint32_t n, uint32_t* h_hull_idx, uint32_t cap,
                  uint32_t* h_out, void* d_ws, size_t ws_bytes, void* stream);

/* What the last successful ch_hull on this context did: n; the candidate
 * records of the refined filter's single read (0 when it was not used: below
 * 131072 points, or no usable sample polygon); the records left after the
 * octagon test (the hull pass's input); the tile-hull rounds; whether the
 * large-hull path ran; h; and how the single read ran: bit 0 set when it
 * used the sample polygon, bit 1 when its inner region was the octagon (else
 * the disc), bit 2 when it streamed on its whole grid (many points outside
 * the inner region) rather than one workgroup per CU; 0 without a single
 * read; and the records left by the second polygon, built from the
 * survivors when one workgroup could not take them all (0 when it did not
 * run; then the rounds and the large-hull path start from those). Not in
 * the paper: a refinement of Alg. 1's filter stage, exact like it.
 * Diagnostics only. */
typedef struct {
  uint32_t n;
  uint32_t candidates;
  uint32_t survivors;
  uint32_t rounds;
  uint32_t large_path;
  uint32_t h;
  uint32_t single_read;
  uint32_t refined;
} ch_hull_info;
ch_status ch_last_hull_info(const ch_ctx* ctx, ch_hull_info* out);

/*
 * The extreme search of Alg. 1/2 (findExtremes) comes in two forms:
 *   CH_EXTREMES_TWO_KERNELS  as Sec. III runs it on the GPU: one reduction for
 *                            the four axis extremes, then a second one for the
 *                            point of least Manhattan distance to each corner
 *                            of the box they span (it needs the first result);
 *                            the points are read twice.
 *   CH_EXTREMES_FUSED        all eight in one read: for a point inside that box
 *                            the Manhattan distance to a corner is a constant
 *                            minus +-x +-y, so no second pass is needed.
 * Both give the same octagon (with the tie-breaks of ch_octagon).
 */
#define CH_EXTREMES_FUSED 0
#define CH_EXTREMES_TWO_KERNELS 1

/* Device workspace bytes needed by ch_gpufilter / ch_hull_queues for n points. */
size_t ch_gpufilter_workspace_bytes(uint32_t n);
size_t ch_hull_queues_workspace_bytes(uint32_t n);

/*
 * ch_gpufilter -- Alg. 2 (GPUfilter): findExtremes (extremes_mode), then the
 * queue label of every point, the array Q the paper copies back to the host
 * to build its four queues (Sec. III). Asynchronous like ch_filter.
 *   d_label   n bytes: 0 for a discarded point, else its queue 1..4 (the rule
 *             of ch_filter's d_label).
 *   d_oct     optional (NULL to skip): the octagon.
 *   d_count   optional (NULL to skip): the number of surviving points, or
 *             CH_COUNT_DOMAIN_ERROR (the labels are then unspecified).
 *   d_ws      workspace of ws_bytes >= ch_gpufilter_workspace_bytes(n).
 * Errors as ch_filter; CH_E_INVALID_ARG also for an unknown extremes_mode.
 */
ch_status ch_gpufilter(ch_ctx* ctx, const float* d_xy, uint32_t n, int extremes_mode,
                       uint8_t* d_label, ch_octagon* d_oct, uint32_t* d_count, void* d_ws,
                       size_t ws_bytes, void* stream);

/*
 * ch_hull_queues -- Alg. 1 stage by stage, all on the device: (1) findExtremes
 * (extremes_mode) and the octagon; (2) the octagon filter with the label
 * array of Alg. 2, and the four queues Q_1..Q_4 built from it (each in
 * ascending index order); (3) a partial order per queue: its points bucketed
 * by grid column (only the top point of a column can lie on the upper arcs
 * fed by Q_1 and Q_2, only the bottom one on the lower arcs of Q_3 and Q_4);
 * (4) the hull of each queue -- the counter-clockwise arc between its two
 * axis extremes (Q_1: E to N, Q_2: N to W, Q_3: W to S, Q_4: S to E) -- and
 * their union. Synchronous like ch_hull, with the same result and errors.
 *   h_qcount  optional (NULL to skip): 4 uint32, the queue sizes n_1..n_4.
 *   d_ws      workspace of ws_bytes >= ch_hull_queues_workspace_bytes(n).
 */
ch_status ch_hull_queues(ch_ctx* ctx, const float* d_xy, uint32_t n, int extremes_mode,
                         uint32_t* h_hull_idx, uint32_t cap, uint32_t* h_out, uint32_t* h_qcount,
                         void* d_ws, size_t ws_bytes, void* stream);

/* Count value ch_hull_batch writes for every set when the offsets are not
 * non-decreasing from 0 to total_points (a set with a domain error gets
 * CH_COUNT_DOMAIN_ERROR, above). Every other set gets its hull, whatever its
 * size or shape. */
#define CH_COUNT_INVALID 0xFFFFFFFDu

/* Device workspace bytes needed by ch_hull_batch. */
size_t ch_hull_batch_workspace_bytes(uint32_t nsets, uint64_t total_points);

/*
 * ch_hull_batch -- Alg. 1 for many independent point sets at once.
 * Asynchronous: enqueues a fixed sequence of kernels on `stream` (no host
 * synchronisation, so the call can be captured in a HIP graph) and returns.
 *   d_xy          all points, set after set, 16-byte aligned.
 *   d_off         nsets + 1 uint64 offsets: set s is points [d_off[s],
 *                 d_off[s+1]); d_off[0] = 0, d_off[nsets] = total_points.
 *   total_points  below 2^32.
 *   d_hull_idx    capacity total_points: the hull of set s, as indices local
 *                 to the set (0 = its first point), starts at d_hull_idx[d_off[s]].
 *   d_hull_count  nsets uint32: h of each set, or a CH_COUNT_* code.
 *   d_ws          workspace of ch_hull_batch_workspace_bytes(nsets, total).
 * Returns CH_OK once enqueued; CH_E_INVALID_ARG / CH_E_DEVICE as ch_filter.
 * Each set's hull follows the conventions of ch_hull exactly.
 */
ch_status ch_hull_batch(ch_ctx* ctx, const float* d_xy, const uint64_t* d_off, uint32_t nsets,
                        uint64_t total_points, uint32_t* d_hull_idx, uint32_t* d_hull_count,
                        void* d_ws, size_t ws_bytes, void* stream);

/*
 * Batch-mode launch parameters (not in the paper; they change speed, never
 * results). tile_points: points per pass tile of a set (power of two, 4096 ..
 * 65536); pass_blocks / hull_blocks: workgroups of the persistent filter
 * grid and of the per-set hull kernels (1 .. 65535); sample_min: sets of at
 * least this many points (and at least 2048) get a refined filter polygon
 * from a sample of their points (0xFFFFFFFF: none).
 */
typedef struct {
  uint32_t tile_points;
  uint32_t pass_blocks;
  uint32_t hull_blocks;
  uint32_t sample_min;
} ch_batch_params;

/* The parameters ch_hull_batch would use for nsets sets of total_points
 * points: those set with ch_batch_params_set, else the tuned entry (this
 * context's tuning or the tune cache) nearest in log2 of both sizes, else
 * the defaults. */
ch_status ch_batch_params_get(const ch_ctx* ctx, uint32_t nsets, uint64_t total_points,
                              ch_batch_params* out);
/* Fix the parameters for every later call (NULL: back to tuned/defaults).
 * CH_E_INVALID_ARG when out of range. */
ch_status ch_batch_params_set(ch_ctx* ctx, const ch_batch_params* p);

/*
 * ch_tune_batch -- autotuner: runs ch_hull_batch on the given batch with
 * candidate parameters (coordinate descent over tile size, pass grid, hull
 * grid and sample threshold, median of three timed runs each), keeps the
 * fastest for batches of this shape (log2 of nsets and total_points), and,
 * when the context was created with a tune_cache_path, rewrites that file
 * with this device's entries (ch_ctx_create loads it). Synchronous; the
 * arguments are those of ch_hull_batch, whose outputs hold the batch's
 * result on return. best_out may be NULL.
 */
ch_status ch_tune_batch(ch_ctx* ctx, const float* d_xy, const uint64_t* d_off, uint32_t nsets,
                        uint64_t total_points, uint32_t* d_hull_idx, uint32_t* d_hull_count,
                        void* d_ws, size_t ws_bytes, void* stream, ch_batch_params* best_out);

/*
 * Serving: a request is one point set in host memory; the server copies it to
 * the device, solves it with other pending requests in one ch_hull_batch call
 * (continuous batching over several streams) and hands the hull back. Not in
 * the paper, which solves one set per call (Alg. 1); every request's hull
 * follows the conventions of ch_hull exactly.
 *
 * Device memory: the caller's arena of arena_bytes, split evenly into one
 * slot per stream. A slot holds one batch at a time: its points (8 B each),
 * offsets, hull indices, counts and workspace. A request is admitted to a
 * batch only when the batch still fits its slot, so the arena size is the
 * admission budget and the server never allocates device memory.
 */
typedef struct {
  void* d_arena;             /* device memory, 256-byte aligned, owned by the caller */
  size_t arena_bytes;        /* admission budget (the whole arena)                   */
  uint32_t max_inflight;     /* requests submitted and not yet collected by          */
                             /* ch_serve_wait; 0 means 65536                         */
  int n_streams;             /* worker streams and arena slots, 1..16; 0 means 4     */
  uint64_t max_batch_points; /* points a batch of several requests holds at most    */
                             /* (a larger request runs alone); 0 means no cap       */
                             /* beyond what a slot holds                            */
} ch_serve_config;

typedef struct ch_server ch_server;

/* Largest request (points) a server with this configuration admits, or 0
 * when the configuration is invalid. */
uint64_t ch_serve_max_request_points(const ch_serve_config* cfg);

/* Start a server on the context's device: one worker thread, stream and
 * library context per slot, plus pinned host staging (allocated here).
 * `ctx` is only read (device) and may be used or destroyed afterwards.
 * Errors: CH_E_INVALID_ARG (NULL pointers, misaligned or too small arena,
 * n_streams out of range), CH_E_NOMEM, CH_E_DEVICE. */
ch_status ch_serve_start(ch_ctx* ctx, const ch_serve_config* cfg, ch_server** out);

/* Queue one request: n points at h_xy (host memory; pinned memory is copied
 * by DMA directly, pageable memory through the HIP runtime). The buffer stays
 * owned by the caller and must stay unchanged until ch_serve_wait has returned
 * a final status for the ticket. Thread-safe.
 * Errors: CH_E_BUSY (max_inflight requests outstanding: retry after a wait),
 * CH_E_INVALID_ARG (NULL pointers, or n above ch_serve_max_request_points),
 * CH_E_SHUTDOWN (stop has begun). */
ch_status ch_serve_submit(ch_server* srv, const float* h_xy, uint32_t n, uint64_t* ticket);

/* Wait for a ticket. timeout_us < 0 waits without limit, 0 polls.
 * On CH_OK the hull (h_out entries, local indices) is in hull_idx and the
 * ticket is released. t_ns (nullable) receives steady-clock nanoseconds
 * (CLOCK_MONOTONIC) of arrival (submit), admission (batch start) and
 * completion. Thread-safe; one waiter per ticket.
 * Final statuses (ticket released): CH_OK, CH_E_DOMAIN (the set has a domain
 * error), CH_E_SHUTDOWN (stopped before admission), CH_E_DEVICE.
 * Non-final (ticket kept): CH_E_TIMEOUT; CH_E_CAPACITY (*h_out = h, hull_idx
 * untouched: call again with a larger buffer). CH_E_NOT_FOUND: unknown or
 * already released ticket. */
ch_status ch_serve_wait(ch_server* srv, uint64_t ticket, int64_t timeout_us, uint32_t* hull_idx,
                        uint32_t cap, uint32_t* h_out, uint64_t* t_ns);

/* Counters since start: completed requests, batches run, requests per
 * second over the span from the first arrival to the last completion, and
 * the 50th / 99th percentile of completion - arrival in microseconds over all
 * completed requests. Any output pointer may be NULL. Thread-safe. */
ch_status ch_serve_stats(ch_server* srv, uint64_t* completed, uint64_t* batches,
                         double* hulls_per_s, double* p50_us, double* p99_us);

/* Stop: refuse new submissions, finish every admitted batch, resolve queued
 * requests that were never admitted with CH_E_SHUTDOWN, wake blocked waiters
 * (they return their ticket's final status), then free the server. No call on
 * `srv` may start once stop has been called. */
ch_status ch_serve_stop(ch_server* srv);

/* Per-kernel timing with HIP events recorded on the launch stream around each
 * kernel. While enabled, every ch_* call synchronises its stream before
 * returning. ch_profile_read fills up to cap records and returns the number
 * of kernels seen in *n_out. */
typedef struct {
  const char* name;   /* static string */
  uint64_t launches;
  double total_ms;
} ch_kernel_stat;
ch_status ch_profile_enable(ch_ctx* ctx, int on);
ch_status ch_profile_reset(ch_ctx* ctx);
ch_status ch_profile_read(ch_ctx* ctx, ch_kernel_stat* out, int cap, int* n_out);

/* Diagnostic, not part of the method: reads the first `bytes` (a multiple of
 * 16) of the device buffer d_buf once, as a plain non-temporal stream of
 * 16-byte loads on `blocks` workgroups (0: two per CU), and returns without
 * waiting (enqueued on `stream`). Timing it gives the read bandwidth the
 * device reaches, the reference for the hull path's roofline fraction.
 * d_buf must be 16-byte aligned and caller-owned. Errors: CH_E_INVALID_ARG
 * (null context or buffer, bytes not a multiple of 16), CH_E_DEVICE. */
ch_status ch_diag_read_stream(ch_ctx* ctx, const void* d_buf, size_t bytes, uint32_t blocks,
                              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CONVHULL_H */
