// Internal host-side interfaces between the translation units of libsfc.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "learned.h"
#include "stree.h"

namespace sfc {

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Occupancy bitmap of the quadtree nodes of depths 0..kOccDepth (early
// termination): depth k starts at bit (4^k - 1) / 3, node p of depth k (the
// top 2k key bits) at that offset + p.
constexpr int kOccDepth = 12;
__host__ __device__ constexpr uint64_t occ_level_offset(int k) {
  return ((1ull << (2 * k)) - 1) / 3;
}
constexpr uint64_t kOccBits = occ_level_offset(kOccDepth + 1);
constexpr uint64_t kOccWords = (kOccBits + 31) / 32;

// Launch shapes chosen by the autotuner, per size bucket (floor(log2 size)).
// tuned(op, size) returns -1 when the bucket has no entry.
enum TuneOp { kTuneSortItems = 0, kTuneTestShape = 1 };
int tuned(TuneOp op, uint64_t size);
void set_tuned(TuneOp op, uint64_t size, int value);

// Fill kernel (used instead of hipMemsetAsync so that every step of a batch
// can be recorded into a HIP graph).
hipError_t fill_u64(uint64_t* p, uint64_t value, uint64_t count, hipStream_t s);
hipError_t fill_u32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t s);

// ---- construction (build.hip) ----
size_t build_scratch_bytes(uint64_t n);
// Run condition of a kernel sequence recorded beside an alternative one (a
// recorded graph cannot branch on the host): with word != null each of its
// kernels returns at once unless the kErrOversized bit of *word is set
// (when_set) or clear (!when_set).
struct SortGuard {
  const uint32_t* word = nullptr;
  bool when_set = true;
};
// Keys of n points (err: device word, kErrDomain is or-ed in); counts, if
// not null, receives the first digit's counts per sort tile.
hipError_t launch_keys(const double* xy, uint64_t n, int curve, uint64_t* keys, uint32_t* err,
                       uint32_t* counts, hipStream_t s, double* xy_copy = nullptr,
                       int count_shift = 0, SortGuard guard = SortGuard{});
// xy_out (may be null): the points in sorted order.  cells_out (may be
// null): the grid cells of the sorted points (pack_cell2 / pack_cell3),
// decoded from the keys (or taken from the points when they are gathered).
// xy_copy (may be null): a copy of the input points in input order.
hipError_t sort_build(const double* xy, uint64_t n, int curve, uint64_t* keys_out,
                      uint32_t* ids_out, double* xy_out, void* scratch, uint32_t* err,
                      hipStream_t s, const uint64_t* set_off = nullptr, uint32_t n_sets = 0,
                      uint64_t* cells_out = nullptr, double* xy_copy = nullptr,
                      SortGuard guard = {});
// sort_build without point sets or xy_out, by four radix passes over the
// top 32 key bits and an LDS sort of each chunk of whole runs of equal top
// bits (same results).  A run too long for a chunk raises kErrOversized in
// *err, and the arrays are then unspecified: run sort_build instead.  Same
// scratch as sort_build.
hipError_t sort_build_chunked(const double* xy, uint64_t n, int curve, uint64_t* keys_out,
                              uint32_t* ids_out, void* scratch, uint32_t* err, hipStream_t s,
                              uint64_t* cells_out, double* xy_copy);
// sort_build_chunked with point sets (set_off and n_sets as in sort_build;
// none: the chunked sort alone): the chunked sort of all points by key, then
// stable passes over the set index (so that the order is by set, key, id, as
// sort_build's).  A run too
// long for a chunk raises kErrOversized and the set passes do nothing; with
// fallback the plain sort_build (with the sets) then runs on the device,
// its kernels recorded after these and doing nothing unless the bit is set.
// xy_out (may be null): the points in sorted order.  No host
// synchronisation: the whole sequence can be recorded into a graph.  Same
// scratch as sort_build.
hipError_t sort_build_sets_chunked(const double* xy, uint64_t n, int curve, uint64_t* keys_out,
                                   uint32_t* ids_out, double* xy_out, void* scratch, uint32_t* err,
                                   hipStream_t s, const uint64_t* set_off, uint32_t n_sets,
                                   uint64_t* cells_out, double* xy_copy, bool fallback);
// out[i] = xy[ids[i]] for points of dim (2 or 3) doubles.
hipError_t gather_sorted(const uint32_t* ids, const double* xy, double* out, uint64_t n, int dim,
                         hipStream_t s);
// Order of a batch of m queries (centres clamped into the square) by the
// top 16 bits of their curve keys, stable: perm[i] = the i-th query in that
// order.  scratch holds order_scratch_bytes(m); err: device error word.
size_t order_scratch_bytes(uint64_t m);
hipError_t order_queries(const double* q, uint64_t m, int curve, uint32_t* perm, void* scratch,
                         uint32_t* err, hipStream_t s);
// Early-termination occupancy bitmap (kOccWords words) of n sorted keys.
hipError_t build_occupancy(const uint64_t* keys, uint64_t n, uint32_t* occ, hipStream_t s);

// ---- device-wide scan (scan.hip) ----
// out[i] = carry + sum(in[0..i)), out[count] = carry + sum(in); carry_in is a
// device word or null (zero).  partial holds scan_scratch_bytes(count).
size_t scan_scratch_bytes(uint64_t count);
hipError_t scan_excl(const uint32_t* in, uint64_t* out, uint64_t count, const uint64_t* carry_in,
                     uint64_t* partial, hipStream_t s);

// ---- queries (query.hip) ----
struct QueryScratch {
  uint32_t* slot_begin;   // per query slot: first sorted index of its range
  uint32_t* slot_count;   // per query slot: its number of candidates
  uint32_t* slot_rows;    // per query slot: rows of 64 candidates
  uint64_t* row_off;      // per query: its first row (+ the total at [m])
  uint64_t* scan_tmp;     // scan partials
  uint32_t* counters;     // [2] error word; u64 at [4]: candidates, [6]: learned
                          // endpoints, [8]: learned fallbacks
  int ss;                 // log2 of the slots per query (2: method's ranges, 3: refined)
  uint64_t* pairs;        // dense (query, cell) work list: 4 * query + cell
  void* qfilt;            // per query: its grid cell and the cell filter's limits (32 B)
  uint32_t* perm;         // queries in curve order (the search's lane order)
  uint32_t* qrows;        // per query: the rows of its slots
  void* order_scratch;    // order_scratch_bytes(m)
};
constexpr uint64_t kCompactTileRows = 64;           // rows of 64 candidates per tile
constexpr uint64_t kCompactChunkTiles = 1ull << 19; // tiles per launch
// Tiles per chunk in effect (kCompactChunkTiles unless a test lowered it).
uint64_t compact_chunk_tiles();
void set_compact_chunk_tiles(uint64_t tiles);
// Query scratch for m queries of up to `slots` slots each (8: the plane,
// either layout, and three dimensions unrefined; 32: three dimensions
// refined).
size_t query_scratch_bytes(uint64_t m, uint32_t slots = 8);
void query_scratch_carve(void* base, uint64_t m, QueryScratch* qs, uint32_t slots = 8);
size_t compact_scratch_bytes(uint64_t total_rows);

// Ranges and searches per query slot, then the scan of candidate counts into
// segment offsets; optionally records the ranges (dbg_* may be null).  ball:
// the Euclidean metric (the refinement may then also drop sub-cells outside
// the disc).
// lview non-null: searches go through the learned index; else sview
// non-null: through the static search tree (both only without point sets).
// occ non-null: cells whose occupancy bit is clear are skipped (early
// termination; not applied when the ranges are recorded for inspection).
// qset/set_off non-null: query j searches only set qset[j] (positions
// [set_off[s], set_off[s+1]) of the sorted arrays).
hipError_t launch_ranges(const double* q, const double* delta, uint64_t m, const uint64_t* keys,
                         uint64_t n, int curve, bool refine, uint32_t refine_min, bool ball,
                         const LearnedView* lview, const StreeView* sview, const uint32_t* occ,
                         const uint32_t* qset, const uint64_t* set_off, uint32_t n_sets,
                         QueryScratch& qs, uint64_t* dbg_lo, uint64_t* dbg_hi, uint64_t* dbg_b,
                         uint64_t* dbg_e, uint32_t* dbg_nr, hipStream_t s);
// Three dimensions (points and queries of three doubles, d = 3 Morton keys):
// the at most 8 cube ranges of every query and their searches (binary, or the
// static search tree when sview is non-null; refine: crowded cubes split once
// into at most four runs of children, 32 slots per query), then the scan, as
// launch_ranges.
hipError_t launch_ranges3(const double* q, const double* delta, uint64_t m, const uint64_t* keys,
                          uint64_t n, bool refine, uint32_t refine_min, const StreeView* sview,
                          QueryScratch& qs, hipStream_t s);
// Test-and-compact over the candidate rows.  device_sized = false: max_rows
// is the exact row count (known on the host), processed in chunks.
// device_sized = true: max_rows is a capacity, the count is read on the
// device (a plan for graph capture); more rows raise kErrOverflow.  cscratch
// holds compact_scratch_bytes(max_rows).  window: the square-window test
// (half side delta) instead of the Euclidean ball.  dim: 2, or 3 for points
// and queries of three doubles.  cells (may be null): the grid cells of the
// sorted points (pack_cell2 / pack_cell3); with them most candidates are
// decided from their cell and only the undecided ones read their coordinates,
// from pts (the sorted points) when not null, else from pts_in (input order)
// through their ids.  Without cells pts must not be null.  coarse: whether
// some radius of the batch lies above the cell filter's shift limit (the
// flag that launch_ranges sets in the counters: 1, 0 when the caller read
// it, -1 when not; with 0 the test pass takes its shortest form).
struct EpochView;
hipError_t launch_compact(const double* q, const double* delta, uint64_t m, const double* pts,
                          const double* pts_in, const uint64_t* cells, const uint32_t* ids,
                          uint64_t npts, const QueryScratch& qs,
                          uint64_t max_rows, bool device_sized, void* cscratch,
                          uint64_t* offsets, uint32_t* out_ids, uint64_t cap, bool window,
                          int dim, hipStream_t s,
                          const EpochView* ev = nullptr, bool write_only = false,
                          int coarse = -1);
// Whether a batch of total_rows rows (host-sized) is compacted in one chunk:
// then an output larger than the capacity leaves the ids untouched, and the
// write pass can be rerun alone (write_only) for a larger buffer.
bool compact_single_chunk(uint64_t total_rows);
// Scan with the element count in device memory (count_dev <= max_count).
hipError_t scan_excl_dev(const uint32_t* in, uint64_t* out, const uint32_t* count_dev,
                         uint64_t max_count, const uint64_t* carry_in, uint64_t* partial,
                         hipStream_t s);

// ---- updates (update.hip) ----
constexpr uint32_t kLiveEpoch = 0xFFFFFFFFu;   // era of an entry not erased
// The stored run: sorted (key, id) with the points and the epochs at which
// each entry was inserted (ins) and erased (era).
struct Run {
  uint64_t* keys = nullptr;
  uint32_t* ids = nullptr;
  double* xy = nullptr;
  uint32_t* ins = nullptr;
  uint32_t* era = nullptr;
  uint64_t* cells = nullptr;   // grid cells of the points (pack_cell2) if kept (may be null)
};
// Which stored entries a query sees: those with ins <= e < era, e = the
// query's epoch (qepoch[j], or `epoch` when qepoch is null).  ins == null:
// every entry is visible.
struct EpochView {
  const uint32_t* ins = nullptr;
  const uint32_t* era = nullptr;
  const uint32_t* qepoch = nullptr;
  uint32_t epoch = 0;
};
// Merges the stored run (n entries) with a sorted batch (k entries, local
// ids bids) into `out` (n + k entries).  The batch's entries are inserted at
// `epoch`; with run_off (device, runs + 1 offsets of local ids, run_off[0] =
// 0), those of run r at epoch + r.
hipError_t merge_runs(const Run& stored, uint64_t n, const uint64_t* bkeys, const uint32_t* bids,
                      const double* bxy, uint64_t k, uint32_t id_base, uint32_t epoch,
                      const Run& out, uint64_t* key_of, hipStream_t s,
                      const uint64_t* run_off = nullptr, uint32_t runs = 0);
hipError_t record_keys(const uint64_t* keys, const uint32_t* ids, uint64_t n, uint64_t* key_of,
                       hipStream_t s);
hipError_t erase_entries(const uint32_t* del, uint64_t k, uint32_t next_id, const uint64_t* key_of,
                         const Run& stored, uint64_t n, uint32_t epoch,
                         unsigned long long* erased, hipStream_t s);
// Drops the entries with era <= oldest; *kept_total points at the device
// word that receives the number kept.
size_t compact_entries_scratch(uint64_t n);
hipError_t compact_entries(const Run& stored, uint64_t n, uint32_t oldest, const Run& out,
                           void* scratch, uint64_t** kept_total, hipStream_t s);
hipError_t fill_iota(uint32_t* out, uint64_t k, uint32_t first, hipStream_t s);
// Raises kErrInvalidQuery in *err for an epoch outside [oldest, epoch].
hipError_t validate_epochs(const uint32_t* qe, uint64_t m, uint32_t oldest, uint32_t epoch,
                           uint32_t* err, hipStream_t s);

// ---- learned index (learned.hip) ----
size_t learned_scratch_bytes();
// Device arrays of a learned index sized for n keys (learned_model_bytes(n)
// bytes, carved by learned_carve).
size_t learned_model_bytes(uint64_t n);
uint32_t learned_max_pieces(uint64_t n);
LearnedArrays learned_carve(void* base, uint64_t n);
// Trains the router (steps Adam steps, 0 = quantile initialisation only) on
// samples of the sorted keys, tabulates it, then fits the leaves' pieces.
// params: kParams floats; losses: 2 floats (sample loss before / after).
hipError_t learned_fit(const uint64_t* keys, uint64_t n, uint32_t steps, float lr, float* params,
                       const LearnedArrays& a, void* scratch, float* losses, hipStream_t s);
// Refits the leaves' pieces for changed keys with the router kept (after an
// update); a must have been carved for at least n keys.
hipError_t learned_refit_leaves(const uint64_t* keys, uint64_t n, const LearnedArrays& a,
                                hipStream_t s);
// Leaf of each key by evaluating the router and through its tabulation.
hipError_t learned_route_both(const float* params, const LearnedArrays& a, const uint64_t* keys,
                              uint64_t count, uint32_t* direct, uint32_t* table, hipStream_t s);
// Gradient of one batch (cnt <= 128 samples) with the trainer's own code.
hipError_t learned_grad(const float* params, const float* xs, const float* ts, int cnt,
                        float* grad, float* loss, hipStream_t s);

}  // namespace sfc
