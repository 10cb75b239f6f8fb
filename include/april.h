/*
 * april.h -- C ABI of the MI355X APRIL intermediate filter.
 *
 * APRIL (Georgiadis, Tzirita Zacharatou, Mamoulis, "Raster Interval Object
 * Approximations for Spatial Intersection Joins") approximates every polygon
 * by two sorted lists of Hilbert-ordered cell intervals on one global
 * 2^N x 2^N grid: the A-list (every cell the polygon touches) and the F-list
 * (every cell it fully covers) (Sec. 4.1).  For a candidate pair (r, s) left
 * by an MBR filter, three merge-joins decide (Sec. 4.2, Alg. 2):
 *   A(r) x A(s) empty                        -> true negative (APRIL_TN)
 *   A(r) x F(s) or F(r) x A(s) non-empty     -> true hit      (APRIL_TH)
 *   otherwise                                -> indecisive    (APRIL_INDECISIVE)
 *
 * Conventions
 *   - Coordinates are float64 multiples of 2^-30 ("the lattice"); the grid
 *     origin is a lattice point and the cell side an integer number of
 *     lattice units, so all geometry is decided exactly in integers.
 *   - Cell (i, j) is the closed square [x0 + i w, x0 + (i+1) w] x
 *     [y0 + j w, y0 + (j+1) w]; a cell is in the A-list iff the closed cell
 *     meets the closed polygon, in the F-list iff it lies inside it.  (The
 *     paper defines the classes by covered fraction, 0 / partial / 100 %;
 *     closed sets make touching polygons share a cell, so true negatives and
 *     true hits stay exact for polygons that only touch.)
 *   - Intervals are half-open [start, end) of Hilbert positions, uint32.
 *   - Pointers named d_* are device (HBM) pointers; all others are host.
 *   - Every call returns APRIL_OK (0), APRIL_PENDING (1) or a negative error
 *     code; april_last_error() gives a message for the calling thread.
 *   - hip_stream is a hipStream_t passed as void* (NULL = default stream).
 */
#ifndef APRIL_H
#define APRIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility push(default)
#endif

/* ---------------------------------------------------------------- codes */
#define APRIL_OK 0
#define APRIL_PENDING 1
#define APRIL_E_INVALID -1   /* bad argument, bad polygon, pair index out of range */
#define APRIL_E_GRID -2      /* grid not exact, polygon outside the guarded grid,
                                lists from different grids */
#define APRIL_E_NOMEM -3     /* host or device allocation failed / over budget */
#define APRIL_E_HIP -4       /* a HIP runtime call failed */
#define APRIL_E_CORRUPT -5   /* lists not sorted/disjoint (validation) */
#define APRIL_E_NODEV -6     /* no usable gfx950 device */
#define APRIL_E_IO -7        /* a file could not be opened, read or written */

/* verdicts (Sec. 4.2) */
#define APRIL_TN 0
#define APRIL_TH 1
#define APRIL_INDECISIVE 2
#define APRIL_BAD_PAIR 255   /* pair index out of range; not counted */

/* ----------------------------------------------------------------- grid */
/*
 * The global 2^order x 2^order grid over the square data space
 * [x0, x0 + side] x [y0, y0 + side] (Sec. 3.1).  order <= 16 so that
 * Hilbert positions fit in uint32 (Sec. 3.2, "Practical considerations").
 * side * 2^30 must be divisible by 2^order; x0, y0 must be lattice points.
 * Polygons must keep clear of the outermost ring of cells (every vertex
 * strictly between x0 + w and x0 + side - w, likewise in y), so the last
 * Hilbert cell is never used and every interval end fits in uint32.
 */
typedef struct {
    double x0, y0, side;
    uint32_t order;
    uint32_t flags;   /* 0, or APRIL_GRID_PARTITIONED in the descriptor of a
                         partitioned collection (set by the library) */
} april_grid_t;

#define APRIL_GRID_PARTITIONED 1u

/* ---------------------------------------------------------------- lists */
/* A- and F-lists of one collection, resident on the host or on a device. */
typedef struct april_lists april_lists_t;

typedef struct {
    uint64_t n_objects;
    uint64_t n_a;          /* total A intervals */
    uint64_t n_f;          /* total F intervals */
    uint64_t device_bytes; /* bytes held in HBM (0 for host lists) */
    int32_t on_device;     /* device ordinal, or -1 for host lists */
    uint32_t codec;        /* APRIL_CODEC_* of the device copy */
} april_lists_info_t;

#define APRIL_STRICT 1u    /* april_build_lists: reject non-lattice coordinates
                              instead of rounding them to the lattice */

/*
 * Build the A- and F-lists of n_polys simple polygons (Sec. 4.1; built by
 * one-step intervalization, Sec. 6.2, Alg. 3).
 *   xy       interleaved float64 vertices (x, y), counter-clockwise or not,
 *            no closing duplicate; polygon k owns xy[2*vtx_off[k] .. 2*vtx_off[k+1])
 *   vtx_off  n_polys + 1 offsets; every polygon needs >= 3 vertices
 *   flags    0 or APRIL_STRICT
 *   out      receives host-resident lists; free with april_lists_free
 * Runs on the host, multi-threaded.  Errors: APRIL_E_INVALID (n_polys == 0,
 * < 3 vertices, non-lattice coordinate under APRIL_STRICT), APRIL_E_GRID
 * (a vertex in the outer cell ring or outside the grid), APRIL_E_NOMEM.
 */
int april_build_lists(const april_grid_t *grid, const double *xy, const uint64_t *vtx_off,
                      uint64_t n_polys, uint32_t flags, april_lists_t **out);

/*
 * The same lists built on the current GPU (Sec. 6: edge traversal, Hilbert
 * ids, one-step intervalization), for the whole collection at once; the
 * result is identical, bit for bit, to april_lists_to_device(
 * april_build_lists(...), APRIL_CODEC_RAW).
 *   grid, xy, vtx_off, n_polys, flags  as for april_build_lists
 *   hip_stream  the stream the work runs on; the call returns when the lists
 *               are complete (it synchronizes the stream twice, to size the
 *               output) and frees its stream-ordered scratch
 *   out         receives device-resident raw lists; free with april_lists_free
 * Errors: as april_build_lists (the first failing polygon is reported), and
 * APRIL_E_INVALID for n_polys >= 2^31, APRIL_E_HIP, APRIL_E_NODEV.
 */
int april_build_lists_gpu(const april_grid_t *grid, const double *xy, const uint64_t *vtx_off,
                          uint64_t n_polys, uint32_t flags, void *hip_stream, april_lists_t **out);

/*
 * Partitioning (Sec. 5.2): the data space is split into disjoint partitions,
 * each with its own grid (of order <= 16) over its raster area; an object
 * that meets several partitions has one instance per partition.  This builds
 * one collection of instances: polygon k is rasterized on grids[grid_of[k]].
 * The collection's descriptor is grids[0] with APRIL_GRID_PARTITIONED set,
 * and the filter accepts R and S only if they were built on the same set of
 * grids; the caller pairs only instances of the same partition.
 */
int april_build_lists_partitioned(const april_grid_t *grids, uint32_t n_grids, const uint32_t *grid_of,
                                  const double *xy, const uint64_t *vtx_off, uint64_t n_polys,
                                  uint32_t flags, april_lists_t **out);

/*
 * Wrap caller-made lists (host arrays, copied) as host lists on `grid`.
 * off_a/off_f: n_objects + 1 offsets; start/end: SoA uint32 endpoints.
 * Lists must be what APRIL lists are: sorted, disjoint, non-empty intervals
 * (start < end <= next start), and every F interval inside one A interval
 * (a Full cell is a cell of the object, Sec. 4.1).  The batched schedule
 * relies on the last property.  With validate != 0 all of this is checked
 * and APRIL_E_CORRUPT returned on a violation.
 */
int april_lists_from_arrays(const april_grid_t *grid, uint64_t n_objects,
                            const uint64_t *off_a, const uint32_t *start_a, const uint32_t *end_a,
                            const uint64_t *off_f, const uint32_t *start_f, const uint32_t *end_f,
                            int validate, april_lists_t **out);

int april_lists_info(const april_lists_t *lists, april_lists_info_t *info);

/* Copy host lists out (arrays sized from april_lists_info). */
int april_lists_export(const april_lists_t *lists, uint64_t *off_a, uint32_t *start_a,
                       uint32_t *end_a, uint64_t *off_f, uint32_t *start_f, uint32_t *end_f);

#define APRIL_CODEC_RAW 0u    /* SoA uint32 start[] / end[] + uint64 CSR offsets */
#define APRIL_CODEC_VBYTE 1u  /* delta + VByte byte streams (Sec. 5.1): per list the
                                 sequence s_0 < e_0 < s_1 < ... stored as varint(s_0),
                                 then varint(gap - 1) for every later value; 7 bits per
                                 byte, low first, high bit = more bytes follow; plus a
                                 block entry every 64 intervals (absolute first start
                                 and byte offset) so decoding can begin mid-list.  The
                                 kernels decode while joining. */

/*
 * Upload host lists to the current HIP device in the layout the kernels
 * read (Sec. 4.1: per object a sorted interval sequence; here split into
 * SoA start[] and end[] arrays plus CSR offsets, or compressed with
 * APRIL_CODEC_VBYTE).  Allocates device memory owned by *out.  RAW copies are
 * asynchronous on hip_stream (the host lists must stay alive until the
 * stream has passed the copy); VBYTE encodes on the host and returns after
 * the copy.  Free with april_lists_free.
 */
int april_lists_to_device(const april_lists_t *host, uint32_t codec, void *hip_stream,
                          april_lists_t **out);

void april_lists_free(april_lists_t *lists);

/*
 * Copy device lists back to new host lists, decoding compressed ones on the
 * device (the decoder the filter kernels use).  Synchronous on hip_stream.
 */
int april_lists_download(const april_lists_t *device_lists, void *hip_stream, april_lists_t **out);

/*
 * List files: the approximations are precomputed once and stored (Sec. 4.1,
 * Sec. 6), then reloaded.  A file holds one collection of host lists: a
 * versioned 88-byte header (magic "APRILLST", version 1, the grid, the
 * partition key of a partitioned collection, the counts), the six raw arrays
 * of april_lists_export in that order (little-endian), and a SHA-256
 * (FIPS 180-4) of every byte before it.  The raw form only: compress at
 * upload (april_lists_to_device with APRIL_CODEC_VBYTE).
 *
 * april_lists_save writes `path` through `path`.tmp and a rename, so a
 * reader never sees a partial file (two saves to one path at once race).
 * Host lists only (download device lists first): APRIL_E_INVALID; a file
 * that cannot be created or written: APRIL_E_IO.
 *
 * april_lists_load reads a file into new host lists (free with
 * april_lists_free).  A missing or unreadable file gives APRIL_E_IO; a file
 * whose header, size or digest does not match, or whose grid is not exact,
 * gives APRIL_E_CORRUPT.  With validate != 0 the lists are also checked as
 * april_lists_from_arrays does (sorted, disjoint, F inside A), else only
 * the offsets are (enough for every access to stay in bounds).
 */
int april_lists_save(const april_lists_t *lists, const char *path);
int april_lists_load(const char *path, int validate, april_lists_t **out);

/* ---------------------------------------------------------------- filter */
#define APRIL_SCHED_PLAIN 0u    /* one wavefront per candidate pair */
#define APRIL_SCHED_BATCHED 1u  /* length-binned persistent schedule */

#define APRIL_VALIDATE 1u       /* check indices first; synchronous; APRIL_E_INVALID */
#define APRIL_WAVE_TIMES 4u      /* batched schedule on raw lists, caller workspace: five uint64 at
                                    byte APRIL_WAVE_TIMES_OFFSET of the workspace receive, in
                                    ticks of the device's real-time clock, the call's start, the
                                    earliest and latest wavefront end of its wave kernel, and the
                                    earliest and latest wavefront end of its workgroup-bin kernel
                                    (~0 and 0 when it does not run); a
                                    kernel's latest end - earliest end is its tail */
#define APRIL_WAVE_TIMES_OFFSET 24448u
#define APRIL_WS_DECODE_CACHE 2u /* compressed lists: the workspace also holds the decode
                                    cache (april_filter_workspace_size counts it when this
                                    flag is set), so the call allocates nothing */

typedef struct {
    uint32_t schedule;     /* APRIL_SCHED_* */
    uint32_t flags;        /* APRIL_VALIDATE | APRIL_WS_DECODE_CACHE | APRIL_WAVE_TIMES */
    uint32_t waves;        /* resident wavefronts (0 = library default) */
    uint32_t tile;         /* batched: intervals per list kept in LDS per wavefront:
                              128, 256 or 512 (0 = 256 when the two collections' A-lists
                              average at most 256 intervals, else 512; compressed lists:
                              256, 512, 1024, 0 = 512) */
    uint32_t chunk;        /* batched: streamed intervals per lane per step: 1, 2 or 4 (0 = 2);
                              compressed lists: decoding windows (up to 130 intervals each) in
                              the first tile of each join, 1 to 4, capped at the tile (0 = 1) */
    uint32_t thread_max;   /* batched: pairs whose four lists all have at most this many
                              intervals run one lane per pair (0 = 8) */
    uint32_t search_min;   /* batched: streamed lists longer than this are first narrowed
                              to the resident list's Hilbert range by a 64-ary search
                              (0 = 512; compressed lists: 64) */
    uint32_t wg_min;       /* batched, raw lists: the workgroup bin.  Pairs in which both
                              objects have a list of at least `tile` intervals and the
                              shorter object's longer list holds at least wg_min run on a
                              whole workgroup, whose four wavefronts share one tile four
                              times as long and split the other object's stream; a binning
                              pass queues them first (0 = 4096; 0xFFFFFFFF = never; no
                              binning pass either when a collection uploaded from host lists
                              has no object that long) */
    void *d_workspace;     /* device scratch of april_filter_workspace_size() bytes
                              (work counters; count sums), or NULL to let the library
                              allocate it (stream-ordered) when it needs it; pass one to
                              capture a batched call in a hipGraph */
    uint64_t workspace_bytes;
} april_filter_opts_t;

/*
 * Device scratch a filter call may use: the batched schedule's work
 * counters and, for any schedule, the slots that sum d_counts (16 KiB,
 * whatever n_pairs and the schedule); with APRIL_WS_DECODE_CACHE in
 * opts->flags, plus the compressed filter's decode cache on the current
 * device.
 */
int april_filter_workspace_size(uint64_t n_pairs, const april_filter_opts_t *opts, uint64_t *bytes);

/*
 * The intermediate filter (Sec. 4.2, Alg. 2) on n_pairs candidate pairs.
 *
 * Schedules (the verdicts are identical):
 *   APRIL_SCHED_PLAIN    one wavefront per pair; the three joins run as
 *                        merge paths over LDS tiles of both lists.
 *   APRIL_SCHED_BATCHED  pairs are binned by list length.  A binning
 *                        pass queues the pairs of two long objects (see
 *                        wg_min), and a persistent kernel joins each on the
 *                        four wavefronts of a workgroup.  Then one
 *                        persistent kernel takes the other pairs in input
 *                        order (each XCD its own range first): one
 *                        wavefront per pair keeps one object's lists in LDS
 *                        (reused while consecutive pairs share the object;
 *                        cut into key-range pieces when neither fits) and
 *                        streams the other's in coalesced chunks; pairs
 *                        whose lists are all very short run one lane per
 *                        pair.  Launches only kernels when a workspace is
 *                        passed, so it can be captured in a hipGraph.
 *                        Compressed lists (APRIL_CODEC_VBYTE) run one
 *                        wavefront per pair decoding as it joins, with a
 *                        decode cache (64 KiB per wavefront, 512 MiB on 256
 *                        CUs) that keeps R objects of up to 4,096 intervals
 *                        per list decoded while consecutive pairs share
 *                        them.  With APRIL_WS_DECODE_CACHE the cache is the
 *                        workspace's tail; else the call takes it from the
 *                        stream (stream-ordered), and when that allocation is
 *                        refused every pair decodes both objects (the
 *                        verdicts are the same).
 *   R, S        device-resident lists on the same grid (else APRIL_E_GRID)
 *   d_r, d_s    device uint32[n_pairs]: pair p is (R object d_r[p], S object d_s[p])
 *   d_verdict   device uint8[n_pairs]: APRIL_TN / APRIL_TH / APRIL_INDECISIVE,
 *               APRIL_BAD_PAIR for an out-of-range index
 *   d_counts    uint64[3] (TN, TH, INDECISIVE totals) or NULL; overwritten,
 *               not accumulated, by three plain stores of the call's last
 *               kernel, so it may be device memory or pinned host memory
 *               (hipHostMalloc) that the host reads once the stream passes
 *               the call
 *   opts        NULL = plain schedule, library defaults
 * Asynchronous on hip_stream; inputs are borrowed until the stream passes
 * the call.  Every verdict is a pure function of the pair's four lists, so
 * pair order and duplicates do not matter.  With APRIL_VALIDATE the call
 * synchronizes and returns APRIL_E_INVALID if any index is out of range.
 */
int april_filter_pairs(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                       const uint32_t *d_s, uint64_t n_pairs, uint8_t *d_verdict,
                       uint64_t *d_counts, const april_filter_opts_t *opts, void *hip_stream);

/*
 * april_filter_pairs for callers that cannot allocate device memory: code
 * being captured into a HIP graph, tight serving loops, harnesses that
 * forbid allocation.  Same arguments, verdicts and counts as
 * april_filter_pairs, but it allocates nothing: its scratch (work counters,
 * count slots, the batched schedule's workgroup queues) is a static device
 * array of the library, 4 MiB + 64 KiB per device plus a 256-byte flag word,
 * held from the device's first library call until the process ends.  The
 * device's address of that array is looked up once per device
 * (hipGetSymbolAddress) at that first call.
 *   opts        as for april_filter_pairs, except: d_workspace must be NULL
 *               and workspace_bytes 0, APRIL_WS_DECODE_CACHE is refused
 *   R, S        raw lists only (compressed lists need a decode cache)
 * Every call on one device shares the array and leaves its contents behind;
 * each call clears what it needs before its kernels read it (with a kernel,
 * not a memset).  Two calls that overlap in time on one device (two streams,
 * or two host threads) race on the array: serialize them.  Errors: those of
 * april_filter_pairs, and APRIL_E_INVALID for a workspace, compressed lists,
 * or a call whose scratch would exceed the static array.
 */
int april_filter_pairs_static(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                              const uint32_t *d_s, uint64_t n_pairs, uint8_t *d_verdict,
                              uint64_t *d_counts, const april_filter_opts_t *opts, void *hip_stream);

/*
 * Data movement of Alg. 2 itself, per pair: the bytes the sequential
 * AA -> AF -> FA merge-joins with early exit must read and write.
 * d_bytes[p] (device uint64[n_pairs]) = 8 (the pair's two uint32 ids)
 *   + 16 per list whose CSR bounds Alg. 2 reads (two uint64 offsets)
 *   + 8 per distinct interval it reads (two uint32 endpoints), or, for
 *     compressed lists (Sec. 5.1), the bytes of each list's prefix that
 *     decoding those intervals consumes (Alg. 2 reads every list from its
 *     start, so no block-index entry)
 *   + 1 (the verdict); 0 for an out-of-range pair.
 * Summed over a batch this is the "algorithmic bytes" of the filter.
 * Computed on the device, one lane per pair; asynchronous on hip_stream.
 */
int april_alg2_bytes(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                     const uint32_t *d_s, uint64_t n_pairs, uint64_t *d_bytes, void *hip_stream);

/* -------------------------------------------------------------- mbr join */
/*
 * Candidate pairs of the MBR filter step (Sec. 2): every (r, s) whose closed
 * bounding rectangles intersect.  Boxes are host float64 [n][4] =
 * (xmin, ymin, xmax, ymax).  Pairs are written to the host arrays r_out,
 * s_out of `capacity` entries, grouped by r, the r objects in the Z-order of
 * their MBR centres and s ascending within each r -- pairs close in the
 * output are close in space, which lets the filter reuse cached lists;
 * *n_out receives the count.  If
 * capacity is too small nothing is written, *n_out holds the required count
 * and APRIL_E_NOMEM is returned.  Host, multi-threaded.
 */
int april_mbr_join(const double *boxes_r, uint64_t n_r, const double *boxes_s, uint64_t n_s,
                   uint32_t *r_out, uint32_t *s_out, uint64_t capacity, uint64_t *n_out);

/* ------------------------------------------------------------- serving */
/*
 * Served selection queries (Sec. 4.3.1): query polygons arrive one by one;
 * each is answered against a device-resident collection S -- the S objects
 * whose MBRs meet the query's MBR, each with its verdict.  Requests are
 * batched continuously: the query's lists are built on host threads, ready
 * requests are packed into the next free slot (a batch with its own stream
 * and device buffers) as long as the slot's memory holds their lists and an
 * upper bound of their candidate pairs, and several slots run on the device
 * at once.  A request that alone exceeds a slot's capacity fails with
 * APRIL_E_NOMEM.
 */
typedef struct april_server april_server_t;

typedef struct {
    uint32_t mbr_grid;      /* cells per side of the uniform MBR index of S (0 = 1024) */
    uint32_t slots;         /* batches in flight at once, one stream each (0 = 3) */
    uint64_t mem_budget;    /* device bytes for all slots' buffers (0 = 2 GiB) */
    uint32_t max_batch;     /* queries per batch at most (0 = 8192) */
    uint32_t host_threads;  /* query-list builder threads (0 = host cores - 2) */
    uint32_t gpu_build_cells;   /* a query whose edges span about this many grid cells
                                   or more has its lists built on the GPU
                                   (april_build_lists_gpu; one thread builds all such
                                   queries waiting at once in one call), the others on
                                   the host (0 = 2^18, 0xFFFFFFFF = never) */
    uint32_t reserved;      /* must be 0 */
    april_filter_opts_t filter;   /* batched-filter tuning (schedule/workspace ignored) */
} april_serve_opts_t;

typedef struct {
    int32_t status;          /* APRIL_OK, APRIL_PENDING, or the request's error code */
    uint32_t reserved;
    uint64_t n_pairs;        /* S objects whose MBR meets the query's MBR */
    const uint32_t *s_ids;   /* host, ascending; valid until april_serve_release */
    const uint8_t *verdict;  /* host; verdict[k] belongs to s_ids[k] */
    uint64_t counts[3];      /* TN, TH, INDECISIVE */
    double t_submit, t_built, t_done;   /* steady-clock seconds: submitted, lists
                                           built, result ready */
} april_result_t;

typedef struct {
    uint32_t slots, slots_busy;
    uint64_t queued, ready;  /* requests waiting for a builder / for a slot */
    uint64_t cap_pairs, cap_intervals, cap_queries;   /* per slot */
} april_serve_stats_t;

/*
 * S_dev: device lists of S (borrowed: must outlive the server); s_boxes:
 * host float64 [n][4] MBRs of S, copied.  Allocates the MBR index and every
 * slot's buffers up front (no device allocation afterwards) and starts the
 * builder and dispatcher threads.
 */
int april_serve_create(const april_lists_t *S_dev, const double *s_boxes,
                       const april_serve_opts_t *opts, april_server_t **out);

/* Queue a query polygon (xy copied; >= 3 vertices, on S's grid).  Returns at once. */
int april_serve_submit(april_server_t *server, const double *xy, uint64_t n_vertices,
                       uint64_t *ticket);

/* APRIL_PENDING (1) until the result is ready, then APRIL_OK with *out filled. */
int april_serve_poll(april_server_t *server, uint64_t ticket, april_result_t *out);

/* Like poll, waiting up to timeout_s seconds. */
int april_serve_wait(april_server_t *server, uint64_t ticket, double timeout_s, april_result_t *out);

/* Drop a finished request and its result buffers. */
int april_serve_release(april_server_t *server, uint64_t ticket);

/* Forget a request; one already on the device is dropped when its batch ends. */
int april_serve_cancel(april_server_t *server, uint64_t ticket);

int april_serve_stats(april_server_t *server, april_serve_stats_t *stats);

/* Finish batches in flight, stop the threads, free everything. */
void april_serve_destroy(april_server_t *server);

/* ------------------------------------------------------ query variants */
/* Sec. 4.3.2-4.3.3 and 5.3: the filter with another predicate, another data
 * type, or lists of two grid orders.  One wavefront per pair; the same
 * verdict codes (APRIL_TN / APRIL_TH / APRIL_INDECISIVE, APRIL_BAD_PAIR for
 * an index out of range) and count layout as april_filter_pairs; device
 * pointers, asynchronous on `hip_stream` (a 16 KiB stream-ordered scratch
 * when d_counts is given).  Lists must be device-resident and raw. */

/*
 * Within join (Sec. 4.3.2): is R[d_r[p]] within S[d_s[p]]?  AA-join first:
 * no overlap -> APRIL_TN (disjoint); then every A(r) interval inside one
 * F(s) interval -> APRIL_TH (r lies inside s); else APRIL_INDECISIVE.  No
 * FA-join (it could only show that s is within r).
 * Errors: APRIL_E_INVALID, APRIL_E_GRID (different grids), APRIL_E_HIP.
 */
int april_filter_within(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                        const uint32_t *d_s, uint64_t n_pairs, uint8_t *d_verdict, uint64_t *d_counts,
                        void *hip_stream);

/* Linestring approximations (Sec. 4.3.3): per linestring, the sorted ids of
 * the cells whose closed square one of its segments meets (a linestring has
 * only Partial cells, and its cells seldom form runs, so ids, not intervals). */
typedef struct april_cells april_cells_t;

/*
 * Build the cell lists of n_lines linestrings on `grid` (host, multi-threaded).
 *   xy, vtx_off  as for april_build_lists, but open chains of >= 2 vertices
 *                (no closing segment)
 *   flags        0 or APRIL_STRICT
 * Errors: APRIL_E_INVALID (NULL, n_lines == 0, < 2 vertices, non-lattice
 * under APRIL_STRICT), APRIL_E_GRID (a vertex in the outer cell ring or out
 * of the grid), APRIL_E_NOMEM.
 */
int april_build_cells(const april_grid_t *grid, const double *xy, const uint64_t *vtx_off,
                      uint64_t n_lines, uint32_t flags, april_cells_t **out);

/* Upload host cells; free both with april_cells_free.  The device copy holds
 * each list as maximal runs of consecutive ids, [start, end), which the
 * polygon-linestring join streams like an A-list (a run meets an interval
 * exactly when one of its cells does).  Device cells cannot be exported. */
int april_cells_to_device(const april_cells_t *host, void *hip_stream, april_cells_t **out);
/* Counts of linestrings and of cell ids. */
int april_cells_info(const april_cells_t *cells, uint64_t *n_lines, uint64_t *n_ids);
/* Host cells into caller arrays: off[n_lines+1], ids[n_ids]. */
int april_cells_export(const april_cells_t *cells, uint64_t *off, uint32_t *ids);
void april_cells_free(april_cells_t *cells);

/*
 * Polygon-linestring join (Sec. 4.3.3): for pair p, polygon P[d_p[p]] and
 * linestring L[d_l[p]], Alg. 2's joins with the cell ids as intervals
 * [c, c+1): A(p) against them, no overlap -> APRIL_TN; F(p) against them,
 * an overlap -> APRIL_TH (the linestring meets a cell inside the polygon);
 * else APRIL_INDECISIVE.
 * Errors: APRIL_E_INVALID, APRIL_E_GRID (different grids), APRIL_E_HIP.
 */
int april_filter_linestrings(const april_lists_t *P, const april_cells_t *L, const uint32_t *d_p,
                             const uint32_t *d_l, uint64_t n_pairs, uint8_t *d_verdict, uint64_t *d_counts,
                             void *hip_stream);

/*
 * Alg. 2 across grid orders (Sec. 5.3): R and S built on grids with the
 * same origin and side and orders NR, NS.  With NR != NS, the finer side's
 * A-intervals are mapped to the coarser grid, a' = [a_start >> n,
 * (a_end - 1) >> n] with n = 2 |NR - NS| (taken half-open), and only two
 * joins run: mapped A against the coarse A-list (no overlap -> APRIL_TN),
 * mapped A against the coarse F-list (an overlap -> APRIL_TH); else
 * APRIL_INDECISIVE.  With NR == NS this is april_filter_pairs' verdict.
 * Errors: APRIL_E_INVALID, APRIL_E_GRID (different data spaces or
 * partitioned collections), APRIL_E_HIP.
 */
int april_filter_mixed(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                       const uint32_t *d_s, uint64_t n_pairs, uint8_t *d_verdict, uint64_t *d_counts,
                       void *hip_stream);

/* ---------------------------------------------------------- refinement */
/* The step after the filter (Sec. 2): the pairs it leaves indecisive are
 * decided by an exact intersection test of the two polygons. */
typedef struct april_polys april_polys_t;

/*
 * Upload n_polys polygons to the current device as exact lattice
 * coordinates (multiples of 2^-30, int64), with their MBRs.
 *   xy, vtx_off  as for april_build_lists (>= 3 vertices per polygon, no
 *                closing duplicate); coordinates below 2^32 in magnitude
 *   flags        0 (round to the nearest lattice point) or APRIL_STRICT
 *                (a non-lattice coordinate is an error)
 * The copy runs on `hip_stream` and is complete on return (the call
 * synchronizes the stream); free with april_polys_free after the work that
 * reads the collection is done.
 * Errors: APRIL_E_INVALID (NULL, n_polys == 0, < 3 vertices, non-lattice
 * under APRIL_STRICT, coordinate out of range), APRIL_E_NOMEM, APRIL_E_HIP.
 */
int april_polys_to_device(const double *xy, const uint64_t *vtx_off, uint64_t n_polys, uint32_t flags,
                          void *hip_stream, april_polys_t **out);

void april_polys_free(april_polys_t *polys);

/*
 * Exact refinement: d_out[i] = 1 if polygons R[d_r[i]] and S[d_s[i]] share
 * at least one point (closed sets: boundary contact counts), 0 if not.
 * The test: some edge of one meets some edge of the other (exact, in
 * integers), or else one polygon's first vertex lies inside the other.
 *   d_verdict  optional (NULL = test every pair): the filter's verdicts for
 *              the same pairs; APRIL_TN gives 0 and APRIL_TH
 *              gives 1 without geometry, APRIL_INDECISIVE pairs are tested
 *   d_counts   optional device uint64[2]: pairs that intersect, pairs
 *              tested exactly (overwritten)
 * A pair with an id out of range gets APRIL_BAD_PAIR.  Device pointers,
 * asynchronous on `hip_stream` (a 16 KiB stream-ordered scratch holds the
 * work counters and the count sums).
 * Errors: APRIL_E_INVALID (NULL collections or out array with n_pairs > 0,
 * n_pairs >= 2^32, collections on another device), APRIL_E_NOMEM (scratch),
 * APRIL_E_HIP.
 */
int april_refine_pairs(const april_polys_t *R, const april_polys_t *S, const uint32_t *d_r,
                       const uint32_t *d_s, uint64_t n_pairs, const uint8_t *d_verdict, uint8_t *d_out,
                       unsigned long long *d_counts, void *hip_stream);

/* ---------------------------------------------------------------- misc */
typedef struct {
    int32_t device;
    int32_t compute_units;
    int32_t wavefront_size;
    int32_t reserved;
    uint64_t hbm_bytes;
    char arch[64];
    char name[128];
} april_device_info_t;

int april_device_info(april_device_info_t *info);

/* Message of the calling thread's last error ("" if none). */
const char *april_last_error(void);

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif

#endif /* APRIL_H */
