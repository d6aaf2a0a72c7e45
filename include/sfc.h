/*
 * sfc.h -- C ABI of libsfc, exact distance reporting on MI355X (gfx950) by
 * sorting points along a space-filling curve.
 *
 * Method: "Simpler is Faster: Practical Distance Reporting by Sorting Along a
 * Space-Filling Curve" (arXiv 2508.19891).
 *   - Problem (Sec. 2, Problem Statement): store a point set P; for a query
 *     (q, delta) report every p in P with |p - q| <= delta (closed ball).
 *   - Construction (Sec. 2.1, "Storing P twice"; Alg. 2; Def. 3): compute a
 *     64-bit curve key per point (Z-order by bit interleaving, or Hilbert),
 *     sort (key, id) pairs, keep the sorted keys beside the sorted points.
 *   - Query (Alg. 1 with cells(Q) and the Observation): the bounding square of
 *     the ball is covered by at most four quadtree cells of side in [s, 2s);
 *     each cell is one contiguous key interval, located by search in the
 *     sorted keys and scanned with the exact distance test.
 *   - Dynamic setting (Sec. 2.1, "Dynamic implementation"): insertions and
 *     deletions of points.
 *
 * Conventions shared by every entry point
 *   - Coordinates are IEEE binary64 in [0,1)^2, stored interleaved
 *     (x0, y0, x1, y1, ...).  Each axis maps to the 32-bit grid cell
 *     floor(v * 2^32).
 *   - The distance test is evaluated in binary64, round-to-nearest-even, with
 *     no fused multiply-add, in this order:
 *        dx = px-qx; dy = py-qy; t = dx*dx; u = dy*dy; s = t+u; r2 = d*d;
 *        report iff s <= r2.
 *   - Point ids are uint32: the index of the point in the build input, then
 *     consecutive ids for inserted points.  At most 2^32 - 1 points.
 *   - Pointers named "device" must be device memory of the current HIP device
 *     (hipMalloc / torch CUDA tensors); "host" pointers are host memory.  The
 *     caller owns every buffer it passes; the index owns its own arrays.
 *   - All work is ordered on the stream given in sfc_options.  Calls that
 *     return a count to the host synchronise that stream before returning.
 *   - Out-parameters are written only when the call returns SFC_OK, unless an
 *     entry point says otherwise.  No C++ exception crosses this interface.
 *   - A handle must not be used by two calls at once.  Distinct handles are
 *     independent.
 */
#ifndef SFC_H_
#define SFC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfc_index sfc_index; /* opaque; owns its device arrays */

typedef enum {
  SFC_OK = 0,
  SFC_ERR_INVALID = -1,  /* NULL pointer, size out of range, bad option, or a
                            query with delta < 0 or a non-finite value */
  SFC_ERR_DOMAIN = -2,   /* a point coordinate outside [0,1) (or NaN) */
  SFC_ERR_NOMEM = -3,    /* a device allocation failed; state unchanged */
  SFC_ERR_CAPACITY = -4, /* output buffer too small; see sfc_query_batch */
  SFC_ERR_DEVICE = -5,   /* a HIP runtime error */
  SFC_ERR_UNSUPPORTED = -6,
  SFC_ERR_SCRATCH = -7   /* the batch needs more than the fixed scratch of
                            sfc_query_batch_static */
} sfc_status;

/* SFC_CURVE_MORTON3: points in [0,1)^3 (x, y, z interleaved, three doubles
   per point and per query) keyed by the d = 3 Morton code (Sec. 1 and
   Sec. 2.1: the Z-order method generalises to R^d): 21 bits per axis, a
   63-bit key, at most 8 cube ranges per query.  With it: binary search or
   the static search tree, with or without refinement (a crowded cube is
   split once into at most four runs of its children that meet the box); no
   early termination, learned index, point sets, updates or range inspection
   (SFC_ERR_UNSUPPORTED). */
enum { SFC_CURVE_MORTON = 0, SFC_CURVE_HILBERT = 1, SFC_CURVE_MORTON3 = 2 };
/* The search that turns a key interval into an index range (all three give
   the same ranges: std::lower_bound / std::upper_bound over the keys):
   binary search; the learned index; the static search tree of Sec. 2.1
   "Storing P twice" (a B+-tree over the keys whose lowest layer is the key
   array and whose upper layers hold the first key of every 16-key line of
   the layer below: about n/15 extra keys, one line read per layer, rebuilt
   after inserts and compactions). */
enum { SFC_SEARCH_BINARY = 0, SFC_SEARCH_LEARNED = 1, SFC_SEARCH_STREE = 2 };
/* The exact test of a query (q, delta): SFC_METRIC_L2 reports the points of
   the closed Euclidean ball of radius delta (Sec. 2, Problem Statement);
   SFC_METRIC_LINF those of the closed axis-parallel square window of half
   side delta (the queries of the experiments, Sec. 4, whose window side is
   2 * delta).  Both use the same cells(Q): the window is the ball's
   bounding square. */
enum { SFC_METRIC_L2 = 0, SFC_METRIC_LINF = 1 };

typedef struct {
  int curve;    /* SFC_CURVE_MORTON (Alg. 2) or SFC_CURVE_HILBERT */
  int search;   /* SFC_SEARCH_BINARY; SFC_SEARCH_LEARNED fits the learned
                   index at build time (binary search stays the fallback);
                   SFC_SEARCH_STREE builds the static search tree */
  int refine;   /* 0: scan the at most four cells of cells(Q) whole (Alg. 1);
                   1: split a crowded cell once and scan only its children
                   that meet the query box.  Same reported ids, same order. */
  int learn_steps; /* training steps of the learned router when search is
                      SFC_SEARCH_LEARNED; 0 = its quantile initialisation
                      only; < 0 = the default (256) */
  void* stream; /* hipStream_t, NULL = the null stream */
  /* Device memory hooks; alloc == NULL uses the library's caching pool over
     hipMalloc.  alloc returns NULL on failure.  release(NULL, ctx) is never
     called. */
  void* (*alloc)(size_t bytes, void* ctx);
  void (*release)(void* ptr, void* ctx);
  void* alloc_ctx;
  int early_term; /* 1: keep an occupancy bit for every quadtree node down to
                     depth 12 (Sec. 2.2 "Early termination"; 2.8 MB) and skip
                     the cells of cells(Q) that hold no point; rebuilt after
                     inserts and compactions (an erase leaves a bit set, which
                     only costs a search).  Same results.  Not with point sets. */
  int metric;     /* SFC_METRIC_L2 (default) or SFC_METRIC_LINF, for every
                     query entry point; sfc_set_metric changes it */
} sfc_options;

/* Fills *opt with Morton curve, binary search, no refinement, default
   training steps, null stream, the pool, no early termination, the
   Euclidean metric. */
void sfc_default_options(sfc_options* opt);

/* Human-readable name of a status code (static string). */
const char* sfc_status_string(sfc_status s);

/*
 * Build the index of n points (Sec. 2.1; Alg. 2; Def. 3).
 *   xy      device, 2*n doubles, interleaved, each in [0,1).
 *   n       number of points, 0 <= n <= 2^32 - 1.
 *   opt     options (curve, search, stream, allocator); NULL = defaults.
 *   out     host; receives the new handle on SFC_OK.
 * Keys: each coordinate is quantised to floor(v * 2^32); Morton puts x's
 * bit i at key bit 2i and y's at 2i+1; Hilbert follows the four-state
 * Hilbert order starting at (0,0) and ending at (2^32-1, 0), most significant
 * level first.  The points are then sorted by (key, id): ties keep input
 * order.  Errors: SFC_ERR_INVALID (NULL xy with n > 0, NULL out, bad option),
 * SFC_ERR_DOMAIN (a coordinate outside [0,1)), SFC_ERR_NOMEM, SFC_ERR_DEVICE.
 * On error nothing is allocated and *out is not written.  Synchronises the
 * stream.
 */
sfc_status sfc_build(const double* xy, uint64_t n, const sfc_options* opt,
                     sfc_index** out);

/*
 * Batched distance queries (Alg. 1; Problem Statement).
 *   q         device, 2*m doubles (qx, qy interleaved); q may lie anywhere.
 *   delta     device, m doubles, each finite and >= 0.
 *   m         number of queries.
 *   offsets   device, m+1 uint64: CSR row starts; offsets[m] = total.
 *   ids       device, ids_cap uint32: the reported point ids.  Within a query
 *             they come in curve order (ascending key, ties by id).
 *   ids_cap   capacity of ids in elements.
 *   total_out host; receives the number of reported ids.
 * If total > ids_cap the call returns SFC_ERR_CAPACITY after writing offsets
 * and *total_out.  When the batch has at most 2^25 candidate rows (64
 * candidates each; every batch in practice) the ids buffer is left untouched
 * and the batch's test results are kept: sfc_query_retry then writes the ids
 * into a large enough buffer without rerunning the searches and the test.
 * Larger batches write the first ids_cap ids and must be rerun.  A query with
 * delta < 0 or a non-finite value makes the call return SFC_ERR_INVALID with
 * offsets and ids unspecified.  Synchronises the stream.
 */
sfc_status sfc_query_batch(sfc_index* h, const double* q, const double* delta,
                           uint64_t m, uint64_t* offsets, uint32_t* ids,
                           uint64_t ids_cap, uint64_t* total_out);

/*
 * sfc_query_batch without allocating: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results (offsets and
 * ids bit for bit), errors and stream behaviour as sfc_query_batch, with
 * these differences:
 *   - its scratch is a fixed 64 MiB array inside the library, one per device
 *     (held until the process ends); a batch whose query scratch (about 260
 *     bytes per query) and compaction scratch (about 32 bytes per row of 64
 *     candidates, e.g. 2^16 queries with 10^6 rows) exceed it returns
 *     SFC_ERR_SCRATCH (offsets and ids unspecified);
 *   - it calls no allocator (no hipMalloc, hipHostMalloc or pool request):
 *     an index whose candidates must read the points in key order and whose
 *     points are not gathered yet (cell filter off, before the first
 *     sfc_query_batch) returns SFC_ERR_UNSUPPORTED;
 *   - on SFC_ERR_CAPACITY offsets and *total_out are written, but the batch
 *     is not kept for sfc_query_retry (rerun it with a larger ids buffer);
 *   - every call on a device shares that device's scratch, which keeps the
 *     last call's contents: two calls that overlap on one device (other
 *     threads, other streams) race and give unspecified results.
 * Point sets and query epochs are not taken (plain batches only).
 */
sfc_status sfc_query_batch_static(sfc_index* h, const double* q, const double* delta,
                                  uint64_t m, uint64_t* offsets, uint32_t* ids,
                                  uint64_t ids_cap, uint64_t* total_out);

/*
 * Updates (the paper's dynamic variant: Section 2, implementation details,
 * "Dynamic implementation", there a B-tree multimap of (key, point) pairs;
 * measured in the dynamic synthetic experiments of Section 3).  The stored
 * run stays one sorted array: an insert sorts its batch like sfc_build and
 * merges the two sorted runs; an erase marks the entry with a tombstone;
 * tombstones are dropped by a compaction.  Not available for indexes built
 * with sfc_build_sets (SFC_ERR_UNSUPPORTED).
 *
 * Epochs.  A built index is at epoch 0; every sfc_insert and sfc_erase with
 * k > 0 advances the epoch by one.  An entry inserted at epoch i and erased
 * at epoch r (r = infinity while live) is visible at epochs e with
 * i <= e < r.  sfc_query_batch answers at the current epoch;
 * sfc_query_epochs answers query j at qepoch[j], any epoch in
 * [oldest, current].  By default oldest follows the current epoch (only the
 * latest state is queryable); after sfc_hold_epochs(h, 1) older epochs stay
 * queryable until the caller calls sfc_retire(h, e) (oldest = e).
 * Compaction drops the tombstones with r <= oldest; it runs by itself when
 * they reach a tenth of the stored entries, or on sfc_compact.
 * The learned index, when fitted, has its leaves refitted (router kept)
 * after every merge and compaction.  Each update synchronises the stream and
 * makes every recorded graph of h stale (sfc_graph_launch then returns
 * SFC_ERR_INVALID); the arrays of sfc_index_view move.
 *
 * sfc_insert: k points (device, 2*k doubles, in [0,1)) get the ids
 *   next_id .. next_id + k - 1 in input order (next_id: see
 *   sfc_update_info; it starts at n); ids_out (device, k uint32, or NULL)
 *   receives them.  SFC_ERR_DOMAIN leaves h unchanged.  Ids are never
 *   reused; at most 2^32 - 2 ids over the life of h.
 * sfc_erase: ids (device, k uint32); unknown, already erased and repeated
 *   ids are skipped; *erased_out (host, or NULL) = entries erased.
 * sfc_query_epochs: as sfc_query_batch, with qepoch (device, m uint32);
 *   an epoch outside [oldest, current] gives SFC_ERR_INVALID.
 * sfc_hold_epochs: hold = 1 keeps older epochs queryable; hold = 0 retires
 *   every epoch before the current one.
 * sfc_retire: epochs below `epoch` (<= current) are no longer queried.
 */
sfc_status sfc_insert(sfc_index* h, const double* xy, uint64_t k, uint32_t* ids_out);
/* Inserts `runs` consecutive batches (1 <= runs <= 65536) with one sort and
   one merge, with the same result as sfc_insert on each batch in order:
   run_off (host, runs + 1 offsets into xy, run_off[0] = 0, non-decreasing)
   delimits them; xy (device, run_off[runs] points, interleaved) holds them;
   run r's points get the ids that follow the previous runs' and are
   inserted at epoch e + 1 + r (e the current epoch), and the epoch advances
   by `runs`, an empty run included.  ids_out as sfc_insert.  SFC_ERR_DOMAIN
   leaves h unchanged. */
sfc_status sfc_insert_runs(sfc_index* h, const double* xy, const uint64_t* run_off, uint32_t runs,
                           uint32_t* ids_out);
sfc_status sfc_erase(sfc_index* h, const uint32_t* ids, uint64_t k, uint64_t* erased_out);
sfc_status sfc_query_epochs(sfc_index* h, const double* q, const double* delta,
                            const uint32_t* qepoch, uint64_t m, uint64_t* offsets,
                            uint32_t* ids, uint64_t ids_cap, uint64_t* total_out);
sfc_status sfc_hold_epochs(sfc_index* h, int hold);
sfc_status sfc_retire(sfc_index* h, uint32_t epoch);
sfc_status sfc_compact(sfc_index* h);
typedef struct {
  uint32_t epoch;       /* current epoch */
  uint32_t oldest;      /* oldest queryable epoch */
  uint32_t next_id;     /* id of the next inserted point */
  uint32_t hold;        /* sfc_hold_epochs state */
  uint64_t stored;      /* entries in the sorted run (sfc_size) */
  uint64_t live;        /* stored entries without a tombstone */
  uint64_t dead;        /* stored entries with a tombstone */
  uint64_t droppable;   /* tombstones the next compaction drops */
  uint64_t merges;      /* inserts merged */
  uint64_t compactions; /* compactions run */
} sfc_update_info;
sfc_status sfc_update_info_get(const sfc_index* h, sfc_update_info* out);

/*
 * A query batch queued on h's stream without waiting for it (for serving
 * loops that admit more work while a batch runs).  q, delta, qepoch (NULL:
 * the current epoch), offsets and ids as in sfc_query_epochs; the candidate
 * rows are bounded by max_rows as in sfc_graph_query.  When the stream
 * reaches the end of the batch, *flags (device uint32) holds its status bits:
 * 0 = complete; 2 = an invalid query or epoch; 16 = more rows than max_rows
 * (offsets and ids unspecified; rerun with a larger bound); 8 = internal
 * error.  offsets[m] is the total; ids beyond ids_cap are not written (compare
 * the total with ids_cap).  The caller keeps every buffer alive until then.
 * Batches and updates issued later on h are ordered after it (same stream).
 * SFC_ERR_UNSUPPORTED for indexes of point sets.
 */
sfc_status sfc_query_async(sfc_index* h, const double* q, const double* delta,
                           const uint32_t* qepoch, uint64_t m, uint64_t max_rows,
                           uint64_t* offsets, uint32_t* ids, uint64_t ids_cap, uint32_t* flags);

/*
 * Query batches that run side by side (the serving setting of Sec. 2.1
 * "Dynamic implementation", queries interleaved with updates): a batch on a
 * stream of the caller's choosing, with its scratch in caller memory, so
 * that several batches over one index are on the device at once.
 *
 * sfc_query_scratch_size: *bytes (host) = the scratch one batch of m
 *   queries with at most max_rows candidate rows needs (about 260 bytes per
 *   query and 32 per row).
 * sfc_query_async_on: as sfc_query_async (same q, delta, qepoch, m,
 *   max_rows, offsets, ids, ids_cap, flags and results), queued on `stream`
 *   (hipStream_t) after the work already queued on the handle's stream,
 *   with scratch (device, 256-byte aligned, scratch_bytes >= the size
 *   above) owned by the call until `stream` has passed the batch.  Batches
 *   on different streams with different scratch run concurrently.  The
 *   batch only reads the index: every later call that rewrites or frees the
 *   index's arrays (inserts, erases, compactions, fits, recorded
 *   constructions, sfc_free) first makes the handle's stream wait for it, on
 *   the device.  Errors: SFC_ERR_INVALID (arguments, scratch too small or
 *   misaligned), SFC_ERR_UNSUPPORTED (point sets), SFC_ERR_NOMEM (the first
 *   query of an index whose points were not yet gathered in key order).
 */
sfc_status sfc_query_scratch_size(const sfc_index* h, uint64_t m, uint64_t max_rows,
                                  uint64_t* bytes);
sfc_status sfc_query_async_on(sfc_index* h, void* stream, void* scratch, uint64_t scratch_bytes,
                              const double* q, const double* delta, const uint32_t* qepoch,
                              uint64_t m, uint64_t max_rows, uint64_t* offsets, uint32_t* ids,
                              uint64_t ids_cap, uint32_t* flags);

/*
 * Write pass of the last sfc_query_batch / sfc_query_sets / sfc_query_epochs
 * call on h that returned SFC_ERR_CAPACITY with its test results kept:
 * offsets (device, m+1) and ids (device, ids_cap) as in that call.  Valid
 * until the next call that queries or updates h; SFC_ERR_UNSUPPORTED if no
 * such batch is kept, SFC_ERR_CAPACITY (with *total_out) if ids_cap is still
 * too small.  The query inputs are not read again.  Synchronises the stream.
 */
sfc_status sfc_query_retry(sfc_index* h, uint64_t* offsets, uint32_t* ids, uint64_t ids_cap,
                           uint64_t* total_out);

/*
 * Many independent point sets in one index (batched instances).  Set s owns
 * the input points xy[set_off[s] .. set_off[s+1]) (set_off: host, n_sets + 1
 * non-decreasing offsets, set_off[0] = 0, 1 <= n_sets <= 65536).  The
 * construction runs every set in the same kernels: the key passes of the
 * radix sort are followed by stable passes over the set index, so the sorted
 * arrays hold the sets one after another, each in (key, id) order at its own
 * input positions.  Ids are input positions, as in sfc_build.  Binary search
 * only (another search or early_term -> SFC_ERR_UNSUPPORTED).  Errors as
 * sfc_build.
 */
sfc_status sfc_build_sets(const double* xy, const uint64_t* set_off, uint32_t n_sets,
                          const sfc_options* opt, sfc_index** out);
/* Queries over an index built by sfc_build_sets: query j is answered within
   set qset[j] (device, m uint32); a set index >= n_sets is an invalid query.
   Output and errors as sfc_query_batch. */
sfc_status sfc_query_sets(sfc_index* h, const double* q, const double* delta,
                          const uint32_t* qset, uint64_t m, uint64_t* offsets, uint32_t* ids,
                          uint64_t ids_cap, uint64_t* total_out);

/*
 * Graphs: one construction or one query batch recorded once (HIP graph) and
 * replayed by a single launch.  Every size that depends on the data lives in
 * device memory, so no step synchronises with the host inside the graph.
 *
 * sfc_graph_build: replaying rebuilds h in place (keys, ids, points; the
 *   learned model is not refitted) from the current contents of xy (device,
 *   same n and sets as h was built with).  sfc_graph_wait reports
 *   SFC_ERR_DOMAIN for a coordinate outside [0,1).
 * sfc_graph_query: one batch of m >= 1 queries over fixed buffers (q, delta,
 *   qset or NULL, offsets, ids as in sfc_query_batch / sfc_query_sets).
 *   max_rows bounds the candidate rows (64 candidates each, at most 2^40;
 *   the graph's scratch covers one chunk of at most 2^25 rows, so it stays
 *   under 1 GB however large the bound);
 *   a batch with more rows makes sfc_graph_wait return SFC_ERR_CAPACITY
 *   (offsets and ids then unspecified; build a graph with a larger bound).
 *   An output larger than ids_cap returns SFC_ERR_CAPACITY with *total_out
 *   set.  The graph reads h's arrays at replay time; it must not outlive h.
 * sfc_graph_launch enqueues one replay on h's stream; sfc_graph_wait waits
 *   for it and checks its flags.  A graph holds its own scratch, so two graphs
 *   of one handle may be launched on the handle's stream one after another,
 *   not concurrently.
 */
typedef struct sfc_graph sfc_graph;
sfc_status sfc_graph_build(sfc_index* h, const double* xy, sfc_graph** out);
sfc_status sfc_graph_query(sfc_index* h, const double* q, const double* delta,
                           const uint32_t* qset, uint64_t m, uint64_t max_rows,
                           uint64_t* offsets, uint32_t* ids, uint64_t ids_cap,
                           sfc_graph** out);
sfc_status sfc_graph_launch(sfc_graph* g);
sfc_status sfc_graph_wait(sfc_graph* g, uint64_t* total_out);
void sfc_graph_free(sfc_graph* g);   /* NULL-safe; waits for h's stream */

/*
 * Autotuner.  Times the launch shapes of a kernel on the caller's data with
 * HIP events and records the fastest for the size bucket (floor(log2)) of
 * that data; later calls of this process with sizes in the same bucket use
 * it.  Results are identical for every shape.
 * sfc_autotune_build: keys of a radix tile per 256 (8, 12, 16, 20, 24; 3
 *   timed builds each; ms[5], *best = the chosen count).  set_off/n_sets as in
 *   sfc_build_sets, or NULL/0.
 * sfc_autotune_query: row groups of the exact-test kernel (5 shapes, 3 timed
 *   batches each; ms[5], *best = the chosen shape index), for the bucket of
 *   the batch's candidate rows; buffers as in sfc_query_batch (qset may be
 *   NULL).  best and ms may be NULL.  Synchronises the stream.
 */
sfc_status sfc_autotune_build(const double* xy, uint64_t n, const uint64_t* set_off,
                              uint32_t n_sets, const sfc_options* opt, int* best, double* ms);
sfc_status sfc_autotune_query(sfc_index* h, const double* q, const double* delta,
                              const uint32_t* qset, uint64_t m, uint64_t* offsets,
                              uint32_t* ids, uint64_t ids_cap, int* best, double* ms);

/* Pins a launch shape for the size bucket (floor(log2)) of `size`, as the
 * autotuner records one: what = SFC_TUNE_SORT_ITEMS (keys of a radix tile per
 * 256: 8, 12, 16, 20 or 24; size = points of the build) or
 * SFC_TUNE_TEST_SHAPE (the exact-test kernel's row groups, 0..4; size = the
 * batch's candidate rows); value -1 removes the pin, so that the default
 * applies again.  Results are identical for every shape.  SFC_ERR_INVALID
 * for another `what` or value. */
#define SFC_TUNE_SORT_ITEMS 0
#define SFC_TUNE_TEST_SHAPE 1
sfc_status sfc_tune_pin(int what, uint64_t size, int value);

/* Number of points currently reported by queries (live points). */
uint64_t sfc_size(const sfc_index* h);

/*
 * Read-only view of the sorted construction (for inspection and tests).
 *   keys  device, n uint64 curve keys, ascending.
 *   ids   device, n uint32 point ids in the same order.
 *   xy    device, 2*n doubles, the points in the same order.
 * The pointers stay valid until the next call that modifies the handle.
 */
sfc_status sfc_index_view(const sfc_index* h, const uint64_t** keys,
                          const uint32_t** ids, const double** xy,
                          uint64_t* n);

/* Copies the sorted construction into caller buffers (device memory, sized
   as in sfc_index_view; any pointer may be NULL).  Stream-ordered; waits for
   the copies before returning. */
sfc_status sfc_index_copy(const sfc_index* h, uint64_t* keys, uint32_t* ids, double* xy);

/*
 * Curve keys only (the first step of the construction), no sort.
 *   xy device 2*n doubles; keys device n uint64; curve as in sfc_options.
 * Errors: SFC_ERR_INVALID, SFC_ERR_DOMAIN, SFC_ERR_DEVICE.  Synchronises the
 * stream.
 */
sfc_status sfc_keys(const double* xy, uint64_t n, int curve, void* stream,
                    uint64_t* keys);

/*
 * Key ranges and index ranges of queries (cells(Q) and the binary searches of
 * Alg. 1), four slots per query.  Slot r < nranges[j] of query j holds the
 * r-th merged key interval [key_lo, key_hi] (inclusive, ascending) and its
 * index range [begin, end) in the sorted keys.  Unused slots hold zeros.
 *   q, delta        device, as in sfc_query_batch.
 *   key_lo, key_hi  device, 4*m uint64.
 *   begin, end      device, 4*m uint64.
 *   nranges         device, m uint32 (0 when the box misses [0,1)^2).
 * Errors: SFC_ERR_INVALID for a bad query.  Synchronises the stream.
 */
sfc_status sfc_query_ranges(sfc_index* h, const double* q, const double* delta,
                            uint64_t m, uint64_t* key_lo, uint64_t* key_hi,
                            uint64_t* begin, uint64_t* end, uint32_t* nranges);

/* Counters of the last sfc_query_batch on h. */
typedef struct {
  uint64_t queries;
  uint64_t rows;        /* candidate rows: each non-empty range contributes
                           ceil(length / 64); a recorded query batch of the
                           same queries needs max_rows >= this */
  uint64_t candidates;  /* points scanned (sum of index range lengths) */
  uint64_t reported;    /* ids reported */
  uint64_t pruned;      /* cells skipped by early termination */
} sfc_query_stats;
sfc_status sfc_last_query_stats(const sfc_index* h, sfc_query_stats* out);
/* The early-termination bitmap (device out, at least 699051 uint32 words):
   bit (4^k - 1)/3 + p is set when a stored key has top 2k bits p (k = 0..12).
   SFC_ERR_UNSUPPORTED when the index was built without it. */
sfc_status sfc_occupancy_copy(const sfc_index* h, uint32_t* out, uint64_t words);

/*
 * Learned index (an addition to the paper's method; binary search stays the
 * reference and the fallback).  The router is a network 1 -> 32 -> 32 -> 1
 * of clipped ramp units (min(max(w x + b, 0), 1)) with non-negative weights,
 * evaluated in FP32 with fused multiply-adds in a fixed order; its input is
 * the key's top 24 bits / 2^24 and its output, times 4096, picks one of 4096
 * leaves.  Non-negative weights make the router monotone in the key, so each
 * leaf holds a contiguous range keys[S..E) of the sorted keys.  A leaf is cut
 * into pieces of 256 keys; the last piece whose first key is below the query
 * key brackets the lower bound, and the piece predicts it by linear
 * interpolation (FP64) with the exact range [elo, ehi] of (lower bound -
 * prediction) over every query key that can reach it.  A lower bound
 * searches that window, is checked against its neighbours, and falls back to
 * a full binary search if the check fails, so results equal plain binary
 * search for any model.  The pieces of all leaves tile the sorted keys in
 * key order, so a query takes the last piece whose first key is below its
 * key, found through a table of how many pieces start below each 20-bit
 * key prefix (the router itself, and its exact tabulation, serve the fit);
 * each piece's window covers every key up to the next piece's first key.
 * The router is trained on the GPU (Adam, mean squared error to rank/n over
 * 2^16 evenly spaced sorted keys, batches of 128), starting from ramps
 * placed at the sample quantiles.
 */
typedef struct {
  int fitted;                 /* 0 until a model exists */
  uint32_t steps;             /* training steps used */
  float loss_init, loss_final;/* sample MSE before / after training */
  uint32_t leaves, leaves_nonempty, max_leaf;
  double mean_window;         /* last-mile window, averaged over the keys */
  uint32_t max_window;
  uint64_t endpoints_last;    /* learned lower bounds in the last batch */
  uint64_t fallbacks_last;    /* of which fell back to binary search */
  uint32_t pieces;            /* pieces over all leaves */
  double search_steps;        /* ceil(log2(pieces of the leaf + 1)) + ceil(log2(window
                                 + 1)), averaged over the keys: the search steps of a
                                 lower bound after routing (binary search takes
                                 about log2(n)) */
} sfc_learned_info;

/* Selects the search for later queries; SFC_SEARCH_LEARNED fits the model
   first if there is none (n >= 2), SFC_SEARCH_STREE builds the tree if it
   is not built.  SFC_ERR_UNSUPPORTED for a search other than binary on an
   index of point sets.  Synchronises the stream. */
sfc_status sfc_set_search(sfc_index* h, int search);
/* Selects the exact test (SFC_METRIC_L2 or SFC_METRIC_LINF) of later query
   batches, sfc_graph_query recordings included; a recorded graph keeps the
   metric it was recorded with, and sfc_query_retry completes its batch with
   the metric that batch was tested with.  SFC_ERR_INVALID for another
   value.  No device work. */
sfc_status sfc_set_metric(sfc_index* h, int metric);
/* The index keeps the grid cell of every stored point beside its
   coordinates (8 bytes per point).  With on = 1 (the default) the exact test
   decides a candidate from its cell when the whole cell lies inside or
   outside the query by a relative margin of 2^-40, far beyond the test's
   rounding, and reads the coordinates only for the rest: the same results
   as the test on every candidate (on = 0), from about half the memory
   traffic.  An index drops its cells at its first insert or erase (its
   queries then test every candidate exactly).  SFC_ERR_INVALID for another
   value.  No device work. */
sfc_status sfc_set_cell_filter(sfc_index* h, int on);
/* Copies the grid cells of the sorted points (device, count >= sfc_size
   words): x | y << 32 per point, or x | y << 21 | z << 42 in three
   dimensions (x, y, z the cell coordinates, floor(v * 2^32) or
   floor(v * 2^21)).  SFC_ERR_UNSUPPORTED once the index dropped them (after
   its first update).  Synchronises the stream. */
sfc_status sfc_cells_copy(const sfc_index* h, uint64_t* out, uint64_t count);
/* (Re)fits the learned index with the given training steps (< 0: the
   handle's default).  SFC_ERR_UNSUPPORTED for n < 2. */
sfc_status sfc_learned_fit(sfc_index* h, int steps);
sfc_status sfc_learned_info_get(const sfc_index* h, sfc_learned_info* out);
/* Router parameters (1153 floats, host): w1[32], b1[32], W2[32][32] (row =
   output unit), b2[32], w3[32], b3.  SFC_ERR_UNSUPPORTED before a fit. */
sfc_status sfc_learned_params(const sfc_index* h, float* params);
/* Test hook for the compaction's chunking: candidate rows are tested and
   written in chunks of up to 2^19 tiles of 64 rows (2^25 rows); this sets the
   chunk to `tiles` tiles for every later call and graph recording in the
   process (0 or more than 2^19 restores 2^19), so that the multi-chunk path
   can be checked on small inputs.  Results do not depend on it. */
sfc_status sfc_debug_chunk_tiles(uint64_t tiles);
/* Test hook of the construction's sort (process-wide).  force_plain 1: every
   build uses the plain eight-pass radix sort; 0: builds without point sets
   first order the keys by their top 32 bits and sort chunks of equal top
   bits in LDS, falling back to the plain sort when a run of equal top bits
   is too long (results are the same either way); negative: unchanged.
   *last_fallback (may be null) receives 1 if the last build fell back. */
sfc_status sfc_debug_sort_path(int force_plain, int* last_fallback);
/* Leaf of each key (device keys[count]) by evaluating the router network
   (direct) and through the tabulation the queries use (table); both device
   uint32[count].  For checking that the two agree.  SFC_ERR_UNSUPPORTED
   before a fit. */
sfc_status sfc_learned_route(sfc_index* h, const uint64_t* keys, uint64_t count,
                             uint32_t* direct, uint32_t* table);
/* Test hook for the fallback path: sets every piece's window to the single
   predicted position, so that most learned lower bounds fail verification
   and fall back to binary search.  Results stay exact. */
sfc_status sfc_learned_shrink_windows(sfc_index* h);
/* Gradient (host, 1153 floats) and loss of the mean squared error of one
   batch of count <= 128 samples (host x[count], t[count]) at the given
   parameters (host), computed by the trainer's own GPU code.  For checking
   the training kernels; synchronous, uses the null stream. */
sfc_status sfc_learned_grad(const float* params, const float* x, const float* t,
                            uint32_t count, float* grad, float* loss);

/* Frees the handle and its device memory (NULL-safe).  Waits for the
   handle's stream first. */
void sfc_free(sfc_index* h);

/*
 * Kernel timing.  While enabled, every kernel launch of the library is
 * bracketed by two HIP events recorded on the stream it is launched on.
 * sfc_profile_read synchronises those events and returns, per kernel name,
 * the number of launches and the summed duration in milliseconds.
 *   names   host, array of max pointers to static strings (may be NULL).
 *   launches, ms  host arrays of max entries (may be NULL).
 * Returns the number of distinct kernels seen (which may exceed max).
 */
void sfc_profile_enable(int on);
/* Restricts the timing to the launches of one kernel (name as reported by
   sfc_profile_read; host string, copied), so that the others run without
   events between them; NULL or "" times every kernel again. */
void sfc_profile_only(const char* name);
void sfc_profile_reset(void);
int sfc_profile_read(const char** names, uint64_t* launches, double* ms,
                     int max);

/* Releases the cached device blocks of the library's allocation pool. */
void sfc_pool_trim(void);

#ifdef __cplusplus
}
#endif

#endif /* SFC_H_ */
