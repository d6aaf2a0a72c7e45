// C ABI of libsfc: handle management, device memory, kernel timing, and the
// host-side sequencing of the construction and query kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "internal.h"
#include "learned.h"
#include "sfc.h"

// Test switches of the construction's sort (process-wide): always the plain
// radix sort, and whether the last build fell back to it.
static std::atomic<bool> g_force_plain_sort{false};
// Most batches one sfc_insert_runs call takes.
constexpr uint32_t kMaxInsertRuns = 1u << 16;
static std::atomic<int> g_last_sort_fallback{0};

// ---- caching device allocator -----------------------------------------------

namespace sfc {
namespace {

// Blocks are kept per device and rounded size; a released block is reused by
// the next request of the same rounded size.  Every call of the library
// synchronises its stream before it returns a block, so reuse never overlaps
// work in flight.
struct Pool {
  std::mutex mu;
  std::map<std::pair<int, size_t>, std::vector<void*>> free_blocks;
  std::map<void*, std::pair<int, size_t>> live;
};
Pool& pool() {
  static Pool* p = new Pool();
  return *p;
}

size_t round_size(size_t b) {
  const size_t g = b <= (1u << 20) ? 256 : (size_t)2 << 20;
  return (b + g - 1) / g * g;
}

}  // namespace

void* Allocator::get(size_t bytes) const {
  if (bytes == 0) bytes = 256;
  if (alloc) return alloc(bytes, ctx);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  const size_t r = round_size(bytes);
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> g(P.mu);
    auto it = P.free_blocks.find({dev, r});
    if (it != P.free_blocks.end() && !it->second.empty()) {
      void* ptr = it->second.back();
      it->second.pop_back();
      P.live[ptr] = {dev, r};
      return ptr;
    }
  }
  void* ptr = nullptr;
  if (hipMalloc(&ptr, r) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> g(P.mu);
  P.live[ptr] = {dev, r};
  return ptr;
}

void Allocator::put(void* ptr) const {
  if (!ptr) return;
  if (release) {
    release(ptr, ctx);
    return;
  }
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  auto it = P.live.find(ptr);
  if (it == P.live.end()) return;
  P.free_blocks[it->second].push_back(ptr);
  P.live.erase(it);
}

// ---- kernel timing ----------------------------------------------------------

namespace {
struct ProfState {
  std::mutex mu;
  bool on = false;
  std::string only;   // non-empty: time only the launches of this kernel
  struct Pending {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> spare;
  std::map<std::string, std::pair<uint64_t, double>> acc;
  std::vector<std::string> order;
};
ProfState& prof() {
  static ProfState* p = new ProfState();
  return *p;
}
hipEvent_t take_event(ProfState& P) {
  if (!P.spare.empty()) {
    hipEvent_t e = P.spare.back();
    P.spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

std::atomic<int> g_capturing{0};   // no timing events inside graph capture

ProfScope::ProfScope(const char* n, hipStream_t s) : name(n), stream(s) {
  ProfState& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  if (!P.on || g_capturing.load() > 0) return;
  if (!P.only.empty() && P.only != n) return;
  hipEvent_t e = take_event(P);
  if (e && hipEventRecord(e, s) == hipSuccess) ev0 = e;
}

ProfScope::~ProfScope() {
  if (!ev0) return;
  ProfState& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  hipEvent_t e = take_event(P);
  if (e && hipEventRecord(e, stream) == hipSuccess) {
    P.pending.push_back({name, (hipEvent_t)ev0, e});
  } else {
    P.spare.push_back((hipEvent_t)ev0);
  }
}

namespace {
void prof_drain(ProfState& P) {
  for (auto& pe : P.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(pe.b) == hipSuccess &&
        hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
      auto it = P.acc.find(pe.name);
      if (it == P.acc.end()) {
        P.order.push_back(pe.name);
        P.acc[pe.name] = {1, (double)ms};
      } else {
        it->second.first += 1;
        it->second.second += ms;
      }
    }
    P.spare.push_back(pe.a);
    P.spare.push_back(pe.b);
  }
  P.pending.clear();
}
}  // namespace

namespace {
std::mutex g_tune_mu;
std::map<std::pair<int, int>, int> g_tune;   // (op, size bucket) -> choice
int bucket(uint64_t size) { return size ? 63 - __builtin_clzll(size) : 0; }
}  // namespace

int tuned(TuneOp op, uint64_t size) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find({(int)op, bucket(size)});
  return it == g_tune.end() ? -1 : it->second;
}

void set_tuned(TuneOp op, uint64_t size, int value) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[{(int)op, bucket(size)}] = value;
}

uint64_t* pinned_scratch() {
  static thread_local uint64_t* p = nullptr;
  if (!p) {
    if (hipHostMalloc((void**)&p, 4096, hipHostMallocDefault) != hipSuccess) p = nullptr;
  }
  return p;
}

}  // namespace sfc

// ---- the handle --------------------------------------------------------------

struct sfc_index {
  int curve = SFC_CURVE_MORTON;
  int search = SFC_SEARCH_BINARY;
  int refine = 0;
  int metric = SFC_METRIC_L2;   // exact test of the query batches
  uint32_t refine_min = 64;   // a cell with more points is refined (measured best of 8 to 128)
  hipStream_t stream = nullptr;
  sfc::Allocator alloc;
  uint64_t n = 0;
  uint64_t* keys = nullptr;
  uint32_t* ids = nullptr;
  double* xy = nullptr;        // points in sorted order: gathered when first needed
  double* xy_in = nullptr;     // points in input order (until the sorted copy exists)
  void* ws = nullptr;          // query scratch (grow-only)
  size_t ws_bytes = 0;
  void* cws = nullptr;         // compaction scratch (grow-only)
  size_t cws_bytes = 0;
  sfc_query_stats last{};
  // learned index
  float* lparams = nullptr;        // device, sfc::kParams
  void* lmodel = nullptr;          // device: tabulated router, leaves and pieces
  uint64_t lmodel_n = 0;           // keys lmodel is sized for
  bool lstats_stale = false;       // leaf statistics not yet read back after a refit
  sfc::LearnedArrays larr{};       // carved from lmodel
  sfc_learned_info linfo{};
  int learn_steps = 256;
  // point sets (sfc_build_sets)
  uint32_t n_sets = 0;
  uint64_t* set_off = nullptr;     // device, n_sets + 1
  // grid cells of the sorted points (decide most candidates without reading
  // their coordinates); kept in step with xy
  uint64_t* cells = nullptr;
  bool cell_filter = true;
  // static search tree: layers above the keys (built while search is STREE)
  void* stree = nullptr;
  size_t stree_bytes = 0;
  bool stree_ready = false;
  // early termination: occupancy bits of the quadtree nodes (null: off)
  uint32_t* occ = nullptr;
  uint64_t last_pruned = 0;
  int last_coarse = -1;   // the last batch's ranges: some radius past the cell shift limit
  // updates (sfc_insert / sfc_erase); ins == null until the first update
  uint32_t* ins = nullptr;         // device, insert epoch per stored entry
  uint32_t* era = nullptr;         // device, erase epoch per stored entry
  uint64_t cap = 0;                // entries allocated in keys/ids/xy/ins/era
  sfc::Run spare{};                // the other half of the merge ping-pong
  uint64_t spare_cap = 0;
  uint64_t* key_of = nullptr;      // device, key of every id handed out
  uint64_t key_of_cap = 0;
  uint64_t* upd_word = nullptr;    // device, counters of the update kernels
  uint32_t next_id = 0;
  uint32_t epoch = 0, oldest = 0, max_ins = 0;
  int hold = 0;
  uint64_t dead = 0;               // stored entries with a tombstone
  std::vector<std::pair<uint32_t, uint64_t>> tombs;   // (erase epoch, entries), not dropped
  uint64_t generation = 0;         // bumped by every update; recorded graphs check it
  // A batch that returned SFC_ERR_CAPACITY from a single compaction chunk:
  // its masks and offsets are still in ws/cws, so the same call with a
  // larger ids buffer reruns only the write pass.
  struct Pending {
    bool valid = false;
    uint64_t m = 0, rows = 0, total = 0, generation = 0;
    sfc::QueryScratch qs{};
  } pending;
  uint64_t merges = 0, compactions = 0;
  // Query batches running on other streams (sfc_query_async_on) read the
  // arrays above: the event recorded after each, until something that
  // rewrites or frees the arrays has made the handle's stream wait for it.
  std::vector<hipEvent_t> readers;
  std::vector<hipEvent_t> idle_events;   // recorded-and-waited events for reuse
};

namespace {

using sfc::align256;

sfc_status from_hip(hipError_t e) {
  if (e == hipSuccess) return SFC_OK;
  if (e == hipErrorOutOfMemory) return SFC_ERR_NOMEM;
  return SFC_ERR_DEVICE;
}

#define SFC_TRY(expr)                              \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) {                        \
      (void)hipGetLastError();                     \
      return from_hip(_e);                         \
    }                                              \
  } while (0)

// An event for ordering work across streams (no timing).
hipError_t take_sync_event(sfc_index* h, hipEvent_t* out) {
  if (!h->idle_events.empty()) {
    *out = h->idle_events.back();
    h->idle_events.pop_back();
    return hipSuccess;
  }
  return hipEventCreateWithFlags(out, hipEventDisableTiming);
}

// Makes the handle's stream wait for every query batch still reading the
// index on another stream (no host wait).  Called by everything that
// rewrites or frees the index's arrays, before it does.
hipError_t wait_readers(sfc_index* h) {
  for (hipEvent_t e : h->readers) {
    const hipError_t r = hipStreamWaitEvent(h->stream, e, 0);
    if (r != hipSuccess) return r;
    h->idle_events.push_back(e);
  }
  h->readers.clear();
  return hipSuccess;
}

bool valid_options(const sfc_options& o) {
  if (o.curve != SFC_CURVE_MORTON && o.curve != SFC_CURVE_HILBERT &&
      o.curve != SFC_CURVE_MORTON3)
    return false;
  if (o.search != SFC_SEARCH_BINARY && o.search != SFC_SEARCH_LEARNED &&
      o.search != SFC_SEARCH_STREE)
    return false;
  if (o.refine != 0 && o.refine != 1) return false;
  if (o.early_term != 0 && o.early_term != 1) return false;
  if (o.metric != SFC_METRIC_L2 && o.metric != SFC_METRIC_LINF) return false;
  if ((o.alloc == nullptr) != (o.release == nullptr)) return false;
  return true;
}

// Reads `count` uint64 words from device memory after the stream's work.
hipError_t read_words(const void* dev, uint64_t* host, size_t count, hipStream_t s) {
  uint64_t* pin = sfc::pinned_scratch();
  if (!pin || count > 512) return hipErrorInvalidValue;
  hipError_t e = hipMemcpyAsync(pin, dev, count * 8, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  std::memcpy(host, pin, count * 8);
  return hipSuccess;
}

sfc_status grow(sfc_index* h, void** buf, size_t* have, size_t bytes) {
  if (*have >= bytes) return SFC_OK;
  if (*buf) {
    (void)hipStreamSynchronize(h->stream);
    h->alloc.put(*buf);
    *buf = nullptr;
    *have = 0;
  }
  *buf = h->alloc.get(bytes);
  if (!*buf) return SFC_ERR_NOMEM;
  *have = bytes;
  return SFC_OK;
}

sfc_status ensure_ws(sfc_index* h, size_t bytes) { return grow(h, &h->ws, &h->ws_bytes, bytes); }

void release_arrays(sfc_index* h) {
  h->alloc.put(h->keys);
  h->alloc.put(h->ids);
  h->alloc.put(h->xy);
  h->alloc.put(h->xy_in);
  h->xy_in = nullptr;
  h->alloc.put(h->ws);
  h->alloc.put(h->cws);
  h->cws = nullptr;
  h->cws_bytes = 0;
  h->alloc.put(h->lparams);
  h->alloc.put(h->lmodel);
  h->alloc.put(h->set_off);
  h->set_off = nullptr;
  h->alloc.put(h->ins);
  h->alloc.put(h->era);
  h->alloc.put(h->spare.keys);
  h->alloc.put(h->spare.ids);
  h->alloc.put(h->spare.xy);
  h->alloc.put(h->spare.ins);
  h->alloc.put(h->spare.era);
  h->alloc.put(h->spare.cells);
  h->alloc.put(h->key_of);
  h->alloc.put(h->upd_word);
  h->alloc.put(h->occ);
  h->occ = nullptr;
  h->alloc.put(h->stree);
  h->stree = nullptr;
  h->alloc.put(h->cells);
  h->cells = nullptr;
  h->stree_bytes = 0;
  h->stree_ready = false;
  h->ins = h->era = nullptr;
  h->spare = sfc::Run{};
  h->spare_cap = 0;
  h->key_of = nullptr;
  h->key_of_cap = 0;
  h->upd_word = nullptr;
  h->lparams = nullptr;
  h->lmodel = nullptr;
  h->lmodel_n = 0;
  h->larr = sfc::LearnedArrays{};
  h->linfo = sfc_learned_info{};
  h->keys = nullptr;
  h->ids = nullptr;
  h->xy = nullptr;
  h->ws = nullptr;
  h->ws_bytes = 0;
}

// The static search tree's layers above the current keys, (re)built on the
// handle's stream; the buffer grows first when the keys outgrew it.
sfc_status stree_refresh(sfc_index* h) {
  SFC_TRY(wait_readers(h));
  const size_t need = sfc::stree_bytes(h->n);
  if (need > h->stree_bytes) {
    // room for a quarter more keys, so that a stream of inserts rarely grows it
    const size_t room = sfc::stree_bytes(h->n + h->n / 4);
    SFC_TRY(hipStreamSynchronize(h->stream));   // the old layers may still be read
    h->alloc.put(h->stree);
    h->stree = h->alloc.get(room);
    h->stree_bytes = h->stree ? room : 0;
    h->stree_ready = false;
    if (!h->stree) return SFC_ERR_NOMEM;
  }
  SFC_TRY(sfc::stree_build(sfc::stree_view(h->keys, h->n, h->stree), h->stream));
  h->stree_ready = true;
  return SFC_OK;
}

// Grows the layer buffer to hold the layers of n keys; the current layers
// are rebuilt into the new buffer, so the tree stays usable.
sfc_status stree_reserve(sfc_index* h, uint64_t n) {
  const size_t need = sfc::stree_bytes(n);
  if (need <= h->stree_bytes) return SFC_OK;
  SFC_TRY(wait_readers(h));   // the old layers are released below
  const size_t room = sfc::stree_bytes(n + n / 4);
  void* buf = h->alloc.get(room);
  if (!buf) return SFC_ERR_NOMEM;
  hipError_t e = hipSuccess;
  if (h->stree_ready) {
    e = sfc::stree_build(sfc::stree_view(h->keys, h->n, buf), h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    h->alloc.put(buf);
    return from_hip(e);
  }
  h->alloc.put(h->stree);
  h->stree = buf;
  h->stree_bytes = room;
  return SFC_OK;
}

bool stree_on(const sfc_index* h) { return h->search == SFC_SEARCH_STREE && h->stree_ready; }

// The cells the test may decide candidates from (null: every candidate takes
// the exact test).
const uint64_t* test_cells(const sfc_index* h) { return h->cell_filter ? h->cells : nullptr; }


// Coordinates per point and per query.
int dim_of(const sfc_index* h) { return h->curve == SFC_CURVE_MORTON3 ? 3 : 2; }

// The points in sorted order, gathered from the input-order copy the first
// time something needs them (a view of them, updates, a test without cells);
// the input-order copy is released then.
sfc_status ensure_sorted_xy(sfc_index* h) {
  if (h->xy || h->n == 0) return SFC_OK;
  SFC_TRY(wait_readers(h));   // the input-order copy is released below
  double* xy = (double*)h->alloc.get(h->n * 8 * dim_of(h));
  if (!xy) return SFC_ERR_NOMEM;
  hipError_t e = sfc::gather_sorted(h->ids, h->xy_in, xy, h->n, dim_of(h), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    h->alloc.put(xy);
    return from_hip(e);
  }
  h->xy = xy;
  h->alloc.put(h->xy_in);
  h->xy_in = nullptr;
  return SFC_OK;
}

// What the test pass of a query batch reads: without cells it tests every
// candidate on the sorted points.
sfc_status points_for_test(sfc_index* h) {
  return test_cells(h) ? SFC_OK : ensure_sorted_xy(h);
}

// Query slots per query the scratch must hold (three dimensions refined:
// four runs for each of eight cubes).
uint32_t slots_of(const sfc_index* h) { return dim_of(h) == 3 && h->refine ? 32 : 8; }

// Runs ranges + searches + scan; on SFC_OK *total_rows holds the number of
// candidate rows and *total_cand the number of candidates.
// The same into query scratch at ws (query_scratch_bytes(m, slots_of(h))
// bytes), reading the counts back through rb (host, 8 words).
sfc_status run_ranges_into(sfc_index* h, void* ws, uint64_t* rb, const double* q,
                           const double* delta, const uint32_t* qset, uint64_t m,
                           sfc::QueryScratch* qs, uint64_t* total_rows, uint64_t* total_cand,
                           uint64_t* dbg_lo, uint64_t* dbg_hi, uint64_t* dbg_b, uint64_t* dbg_e,
                           uint32_t* dbg_nr, const uint32_t* qepoch);

sfc_status run_ranges(sfc_index* h, const double* q, const double* delta, const uint32_t* qset,
                      uint64_t m, sfc::QueryScratch* qs, uint64_t* total_rows, uint64_t* total_cand,
                      uint64_t* dbg_lo, uint64_t* dbg_hi, uint64_t* dbg_b, uint64_t* dbg_e,
                      uint32_t* dbg_nr, const uint32_t* qepoch = nullptr) {
  h->pending.valid = false;   // the scratch is about to be reused
  sfc_status st = ensure_ws(h, sfc::query_scratch_bytes(m, slots_of(h)));
  if (st != SFC_OK) return st;
  uint64_t* pin = sfc::pinned_scratch();
  if (!pin) return SFC_ERR_NOMEM;
  return run_ranges_into(h, h->ws, pin, q, delta, qset, m, qs, total_rows, total_cand, dbg_lo,
                         dbg_hi, dbg_b, dbg_e, dbg_nr, qepoch);
}

sfc_status run_ranges_into(sfc_index* h, void* ws, uint64_t* rb, const double* q,
                           const double* delta, const uint32_t* qset, uint64_t m,
                           sfc::QueryScratch* qs, uint64_t* total_rows, uint64_t* total_cand,
                           uint64_t* dbg_lo, uint64_t* dbg_hi, uint64_t* dbg_b, uint64_t* dbg_e,
                           uint32_t* dbg_nr, const uint32_t* qepoch) {
  sfc::query_scratch_carve(ws, m, qs, slots_of(h));
  const bool learned = h->search == SFC_SEARCH_LEARNED && h->linfo.fitted && !qset;
  const sfc::LearnedView lv = h->larr.view();
  const sfc::StreeView sv = sfc::stree_view(h->keys, h->n, h->stree);
  if (dim_of(h) == 3)
    SFC_TRY(sfc::launch_ranges3(q, delta, m, h->keys, h->n, h->refine != 0, h->refine_min,
                                stree_on(h) ? &sv : nullptr, *qs,
                                h->stream));
  else
    SFC_TRY(sfc::launch_ranges(q, delta, m, h->keys, h->n, h->curve, h->refine != 0,
                               h->refine_min, h->metric == SFC_METRIC_L2,
                               learned ? &lv : nullptr,
                               stree_on(h) ? &sv : nullptr, h->occ, qset,
                               qset ? h->set_off : nullptr, h->n_sets, *qs, dbg_lo, dbg_hi, dbg_b,
                               dbg_e, dbg_nr, h->stream));
  if (qepoch)
    SFC_TRY(sfc::validate_epochs(qepoch, m, h->oldest, h->epoch, qs->counters + 2, h->stream));
  uint64_t* pin = rb;
  SFC_TRY(hipMemcpyAsync(pin, qs->row_off + m, 8, hipMemcpyDeviceToHost, h->stream));
  SFC_TRY(hipMemcpyAsync(pin + 1, qs->counters, 56, hipMemcpyDeviceToHost, h->stream));
  SFC_TRY(hipStreamSynchronize(h->stream));
  const uint32_t err = ((const uint32_t*)(pin + 1))[2];
  if (err & sfc::kErrInvalidQuery) return SFC_ERR_INVALID;
  if (err & (sfc::kErrLookback | sfc::kErrInternal)) return SFC_ERR_DEVICE;
  *total_rows = pin[0];
  *total_cand = pin[3];   // counters[4..5]
  h->linfo.endpoints_last = learned ? pin[4] : 0;
  h->linfo.fallbacks_last = learned ? pin[5] : 0;
  h->last_pruned = pin[6];   // counters[10..11]
  h->last_coarse = (pin[7] >> 32) != 0 ? 1 : 0;   // counters[13]: radii past the shift limit
  return SFC_OK;
}

// Size and window statistics of the fitted leaves and pieces (read back).
hipError_t leaf_stats(sfc_index* h) {
  const sfc::LearnedArrays& a = h->larr;
  std::vector<uint2> lp(sfc::kLeaves + 1);
  hipError_t e = hipMemcpyAsync(lp.data(), a.lp, lp.size() * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return e;
  std::vector<uint32_t> lb(sfc::kLeaves + 1), po(sfc::kLeaves + 1);
  for (int l = 0; l <= sfc::kLeaves; ++l) {
    lb[l] = lp[l].x;
    po[l] = lp[l].y;
  }
  const uint32_t np = po[sfc::kLeaves] < a.max_pieces ? po[sfc::kLeaves] : a.max_pieces;
  std::vector<sfc::PieceRec> pr(np);
  if (np) {
    e = hipMemcpyAsync(pr.data(), a.pr, np * sizeof(sfc::PieceRec), hipMemcpyDeviceToHost,
                       h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
  }
  sfc_learned_info& I = h->linfo;
  I.leaves = sfc::kLeaves;
  I.leaves_nonempty = 0;
  I.max_leaf = 0;
  I.max_window = 0;
  I.pieces = np;
  double wsum = 0.0, ssum = 0.0;
  for (int l = 0; l < sfc::kLeaves; ++l) {
    const uint32_t size = lb[l + 1] > lb[l] ? lb[l + 1] - lb[l] : 0;
    if (size == 0) continue;
    ++I.leaves_nonempty;
    if (size > I.max_leaf) I.max_leaf = size;
    const uint32_t f = po[l + 1] - po[l];
    const double piece_steps = std::ceil(std::log2((double)f + 1.0));
    for (uint32_t j = po[l]; j < po[l + 1] && j < np; ++j) {
      const uint32_t keys_j = std::min<uint32_t>(sfc::kPiece, size - (j - po[l]) * sfc::kPiece);
      const uint32_t win = (uint32_t)(pr[j].ehi - pr[j].elo + 1);
      if (win > I.max_window) I.max_window = win;
      wsum += (double)keys_j * win;
      ssum += (double)keys_j * (piece_steps + std::ceil(std::log2((double)win + 1.0)));
    }
  }
  I.mean_window = h->n ? wsum / (double)h->n : 0.0;
  I.search_steps = h->n ? ssum / (double)h->n : 0.0;
  return hipSuccess;
}

// The model buffer holds the arrays for at least n keys; a larger buffer
// keeps the router's tabulation (its first part).
sfc_status ensure_lmodel(sfc_index* h, uint64_t n) {
  if (h->lmodel && h->lmodel_n >= n) return SFC_OK;
  const uint64_t cap = n + n / 4;
  void* buf = h->alloc.get(sfc::learned_model_bytes(cap));
  if (!buf) return SFC_ERR_NOMEM;
  sfc::LearnedArrays a = sfc::learned_carve(buf, cap);
  if (h->lmodel) {
    hipError_t e = hipMemcpyAsync(a.xb, h->larr.xb, (sfc::kLeaves + 1) * 4,
                                  hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(a.rt, h->larr.rt, (sfc::kRouteSlots + 1) * 4, hipMemcpyDeviceToDevice,
                         h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      h->alloc.put(buf);
      return from_hip(e);
    }
    h->alloc.put(h->lmodel);
  }
  h->lmodel = buf;
  h->lmodel_n = cap;
  h->larr = a;
  return SFC_OK;
}

sfc_status fit_learned(sfc_index* h, int steps) {
  if (h->n < 2) return SFC_ERR_UNSUPPORTED;
  SFC_TRY(wait_readers(h));
  if (steps < 0) steps = h->learn_steps;
  if (!h->lparams) h->lparams = (float*)h->alloc.get(sfc::kParams * sizeof(float));
  if (!h->lparams) return SFC_ERR_NOMEM;
  sfc_status st = ensure_lmodel(h, h->n);
  if (st != SFC_OK) return st;
  void* scratch = h->alloc.get(sfc::learned_scratch_bytes());
  if (!scratch) return SFC_ERR_NOMEM;
  float* losses = (float*)((char*)scratch + sfc::learned_scratch_bytes() - 256);
  h->linfo.fitted = 0;
  hipError_t e = sfc::learned_fit(h->keys, h->n, (uint32_t)steps, 1e-3f, h->lparams, h->larr,
                                  scratch, losses, h->stream);
  float lh[2] = {0.f, 0.f};
  if (e == hipSuccess) e = hipMemcpyAsync(lh, losses, 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  h->alloc.put(scratch);
  if (e == hipSuccess) e = leaf_stats(h);
  h->lstats_stale = false;
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return from_hip(e);
  }
  sfc_learned_info& I = h->linfo;
  I.fitted = 1;
  I.steps = (uint32_t)steps;
  I.loss_init = lh[0];
  I.loss_final = lh[1];
  return SFC_OK;
}

// Refits the pieces of a fitted learned index after the keys changed (the
// router is kept); with fewer than two keys the index falls back to binary
// search until the next fit.
sfc_status refit_leaves(sfc_index* h) {
  if (!h->linfo.fitted) return SFC_OK;
  SFC_TRY(wait_readers(h));
  if (h->n < 2) {
    h->linfo.fitted = 0;
    return SFC_OK;
  }
  sfc_status st = ensure_lmodel(h, h->n);
  if (st != SFC_OK) {
    h->linfo.fitted = 0;
    return st;
  }
  // The statistics are read back when asked for (sfc_learned_info_get), so
  // that an update does not wait for a copy of every piece.
  hipError_t e = sfc::learned_refit_leaves(h->keys, h->n, h->larr, h->stream);
  h->lstats_stale = true;
  if (e != hipSuccess) {
    (void)hipGetLastError();
    h->linfo.fitted = 0;
    return from_hip(e);
  }
  return SFC_OK;
}

}  // namespace

extern "C" {

void sfc_default_options(sfc_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->curve = SFC_CURVE_MORTON;
  opt->search = SFC_SEARCH_BINARY;
  opt->learn_steps = -1;
  opt->early_term = 0;
  opt->metric = SFC_METRIC_L2;
}

const char* sfc_status_string(sfc_status s) {
  switch (s) {
    case SFC_OK: return "ok";
    case SFC_ERR_INVALID: return "invalid argument";
    case SFC_ERR_DOMAIN: return "point coordinate outside [0,1)";
    case SFC_ERR_NOMEM: return "out of device memory";
    case SFC_ERR_CAPACITY: return "output buffer too small";
    case SFC_ERR_DEVICE: return "HIP device error";
    case SFC_ERR_SCRATCH: return "batch needs more than the library's static scratch";
    case SFC_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

sfc_status sfc_keys(const double* xy, uint64_t n, int curve, void* stream, uint64_t* keys) {
  if ((n > 0 && (!xy || !keys)) || n > 0xFFFFFFFFull) return SFC_ERR_INVALID;
  if (curve != SFC_CURVE_MORTON && curve != SFC_CURVE_HILBERT && curve != SFC_CURVE_MORTON3)
    return SFC_ERR_INVALID;
  if (n == 0) return SFC_OK;
  hipStream_t s = (hipStream_t)stream;
  sfc::Allocator a;
  void* tmp = a.get(256);
  if (!tmp) return SFC_ERR_NOMEM;
  uint32_t* err = (uint32_t*)tmp;
  sfc_status st = SFC_OK;
  hipError_t e = sfc::fill_u32(err, 0, 1, s);
  if (e == hipSuccess) e = sfc::launch_keys(xy, n, curve, keys, err, nullptr, s);
  uint64_t w = 0;
  if (e == hipSuccess) e = read_words(err, &w, 1, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    st = from_hip(e);
  } else if ((uint32_t)w & sfc::kErrDomain) {
    st = SFC_ERR_DOMAIN;
  }
  a.put(tmp);
  return st;
}

}  // extern "C"

namespace {
sfc_status build_impl(const double* xy, uint64_t n, const uint64_t* set_off_host, uint32_t n_sets,
                      const sfc_options* opt, sfc_index** out) {
  sfc_options o;
  sfc_default_options(&o);
  if (opt) o = *opt;
  if (!out || (n > 0 && !xy) || n > 0xFFFFFFFFull || !valid_options(o)) return SFC_ERR_INVALID;
  if (o.curve == SFC_CURVE_MORTON3 &&
      (o.search == SFC_SEARCH_LEARNED || o.early_term || set_off_host))
    return SFC_ERR_UNSUPPORTED;
  sfc_index* h = new (std::nothrow) sfc_index();
  if (!h) return SFC_ERR_NOMEM;
  h->curve = o.curve;
  h->search = o.search;
  h->refine = o.refine;
  h->metric = o.metric;
  if (o.learn_steps >= 0) h->learn_steps = o.learn_steps;
  if (const char* env = std::getenv("SFC_REFINE_MIN")) h->refine_min = (uint32_t)std::atoi(env);
  h->stream = (hipStream_t)o.stream;
  h->alloc.alloc = o.alloc;
  h->alloc.release = o.release;
  h->alloc.ctx = o.alloc_ctx;
  h->n = n;
  h->cap = n;
  h->next_id = (uint32_t)n;
  if (set_off_host) {
    h->n_sets = n_sets;
    h->set_off = (uint64_t*)h->alloc.get((n_sets + 1) * 8);
    if (!h->set_off) {
      delete h;
      return SFC_ERR_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(h->set_off, set_off_host, (n_sets + 1) * 8,
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      release_arrays(h);
      delete h;
      return from_hip(e);
    }
  }
  if (n > 0) {
    h->keys = (uint64_t*)h->alloc.get(n * 8);
    h->ids = (uint32_t*)h->alloc.get(n * 4);
    h->xy_in = (double*)h->alloc.get(n * 8 * dim_of(h));
    h->cells = (uint64_t*)h->alloc.get(n * 8);
    const size_t sb = sfc::build_scratch_bytes(n) + 256;
    void* scratch = h->alloc.get(sb);
    if (!h->keys || !h->ids || !h->xy_in || !h->cells || !scratch) {
      h->alloc.put(scratch);
      release_arrays(h);
      delete h;
      return SFC_ERR_NOMEM;
    }
    uint32_t* err = (uint32_t*)((char*)scratch + sb - 256);
    hipError_t e = sfc::fill_u32(err, 0, 1, h->stream);
    // The chunked sort runs first (with point sets, followed by the passes
    // over the set index); a run of equal top key bits too long for it is
    // reported in the error word (read here anyway), and the plain sort then
    // builds the arrays again.
    const bool chunked = !g_force_plain_sort;
    if (e == hipSuccess)
      e = !chunked ? sfc::sort_build(xy, n, h->curve, h->keys, h->ids, nullptr, scratch, err,
                                     h->stream, h->set_off, h->n_sets, h->cells, h->xy_in)
          : h->set_off
              ? sfc::sort_build_sets_chunked(xy, n, h->curve, h->keys, h->ids, nullptr, scratch,
                                             err, h->stream, h->set_off, h->n_sets, h->cells,
                                             h->xy_in, false)
              : sfc::sort_build_chunked(xy, n, h->curve, h->keys, h->ids, scratch, err, h->stream,
                                        h->cells, h->xy_in);
    uint64_t w = 0;
    if (e == hipSuccess) e = read_words(err, &w, 1, h->stream);
    g_last_sort_fallback = 0;
    if (e == hipSuccess && chunked && ((uint32_t)w & sfc::kErrOversized) &&
        !((uint32_t)w & sfc::kErrDomain)) {
      g_last_sort_fallback = 1;
      e = sfc::fill_u32(err, 0, 1, h->stream);
      if (e == hipSuccess)
        e = sfc::sort_build(xy, n, h->curve, h->keys, h->ids, nullptr, scratch, err, h->stream,
                            h->set_off, h->n_sets, h->cells, h->xy_in);
      if (e == hipSuccess) e = read_words(err, &w, 1, h->stream);
    }
    h->alloc.put(scratch);
    sfc_status st = SFC_OK;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      st = from_hip(e);
    } else if ((uint32_t)w & sfc::kErrDomain) {
      st = SFC_ERR_DOMAIN;
    } else if ((uint32_t)w & (sfc::kErrLookback | sfc::kErrInternal)) {
      st = SFC_ERR_DEVICE;
    }
    if (st != SFC_OK) {
      (void)hipStreamSynchronize(h->stream);
      release_arrays(h);
      delete h;
      return st;
    }
  }
  if (o.early_term) {
    h->occ = (uint32_t*)h->alloc.get(sfc::kOccWords * 4);
    hipError_t e = h->occ ? sfc::build_occupancy(h->keys, h->n, h->occ, h->stream)
                          : hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      release_arrays(h);
      delete h;
      return from_hip(e);
    }
  }
  if (h->search == SFC_SEARCH_STREE) {
    sfc_status st = stree_refresh(h);
    if (st == SFC_OK) st = from_hip(hipStreamSynchronize(h->stream));
    if (st != SFC_OK) {
      release_arrays(h);
      delete h;
      return st;
    }
  }
  if (h->search == SFC_SEARCH_LEARNED && n >= 2 && !set_off_host) {
    sfc_status st = fit_learned(h, -1);
    if (st != SFC_OK) {
      release_arrays(h);
      delete h;
      return st;
    }
  }
  *out = h;
  return SFC_OK;
}

}  // namespace

extern "C" {

sfc_status sfc_build(const double* xy, uint64_t n, const sfc_options* opt, sfc_index** out) {
  return build_impl(xy, n, nullptr, 0, opt, out);
}

sfc_status sfc_build_sets(const double* xy, const uint64_t* set_off, uint32_t n_sets,
                          const sfc_options* opt, sfc_index** out) {
  if (!set_off || n_sets < 1 || n_sets > 65536 || set_off[0] != 0) return SFC_ERR_INVALID;
  for (uint32_t i = 0; i < n_sets; ++i)
    if (set_off[i + 1] < set_off[i]) return SFC_ERR_INVALID;
  if (opt && (opt->search != SFC_SEARCH_BINARY || opt->early_term)) return SFC_ERR_UNSUPPORTED;
  return build_impl(xy, set_off[n_sets], set_off, n_sets, opt, out);
}

}  // extern "C"

namespace {
// The entries a query of h sees: all stored ones unless updates left
// tombstones or entries newer than the oldest queryable epoch.
bool epoch_view(const sfc_index* h, const uint32_t* qepoch, sfc::EpochView* ev) {
  if (!h->ins || (h->dead == 0 && h->max_ins <= h->oldest)) return false;
  ev->ins = h->ins;
  ev->era = h->era;
  ev->qepoch = qepoch;
  ev->epoch = h->epoch;
  return true;
}

sfc_status query_impl(sfc_index* h, const double* q, const double* delta, const uint32_t* qset,
                      uint64_t m, uint64_t* offsets, uint32_t* ids, uint64_t ids_cap,
                      uint64_t* total_out, const uint32_t* qepoch = nullptr) {
  if (!h || !offsets || !total_out || (m > 0 && (!q || !delta)) || (ids_cap > 0 && !ids))
    return SFC_ERR_INVALID;
  if (m > (1ull << 36)) return SFC_ERR_INVALID;
  {
    sfc_status st = points_for_test(h);
    if (st != SFC_OK) return st;
  }
  sfc::QueryScratch qs{};
  uint64_t total_rows = 0, total_cand = 0;
  sfc::EpochView ev;
  const bool filtered = epoch_view(h, qepoch, &ev);
  h->pending.valid = false;
  if (m > 0) {
    sfc_status st = run_ranges(h, q, delta, qset, m, &qs, &total_rows, &total_cand, nullptr,
                               nullptr, nullptr, nullptr, nullptr, qepoch);
    if (st != SFC_OK) return st;
  } else {
    sfc_status st = ensure_ws(h, sfc::query_scratch_bytes(0));
    if (st != SFC_OK) return st;
    sfc::query_scratch_carve(h->ws, 0, &qs);
  }
  {
    sfc_status st = grow(h, &h->cws, &h->cws_bytes, sfc::compact_scratch_bytes(total_rows));
    if (st != SFC_OK) return st;
  }
  SFC_TRY(sfc::launch_compact(q, delta, m, h->xy, h->xy_in, test_cells(h), h->ids, h->n, qs,
                              total_rows, false, h->cws, offsets, ids, ids_cap,
                              h->metric == SFC_METRIC_LINF, dim_of(h), h->stream,
                              filtered ? &ev : nullptr, false, m > 0 ? h->last_coarse : 0));
  uint64_t total = 0;
  SFC_TRY(read_words(offsets + m, &total, 1, h->stream));
  if (m > 0) {
    uint64_t cw[2];
    SFC_TRY(read_words(qs.counters, cw, 2, h->stream));
    if (((const uint32_t*)cw)[2] & (sfc::kErrLookback | sfc::kErrInternal)) return SFC_ERR_DEVICE;
  }
  h->last.queries = m;
  h->last.candidates = total_cand;
  h->last.reported = total;
  h->last.rows = total_rows;
  h->last.pruned = m > 0 ? h->last_pruned : 0;
  *total_out = total;
  if (total > ids_cap && m > 0 && sfc::compact_single_chunk(total_rows)) {
    sfc_index::Pending& p = h->pending;
    p.valid = true;
    p.m = m;
    p.rows = total_rows;
    p.total = total;
    p.generation = h->generation;
    p.qs = qs;
  }
  return total > ids_cap ? SFC_ERR_CAPACITY : SFC_OK;
}

}  // namespace

extern "C" {

sfc_status sfc_query_batch(sfc_index* h, const double* q, const double* delta, uint64_t m,
                           uint64_t* offsets, uint32_t* ids, uint64_t ids_cap,
                           uint64_t* total_out) {
  return query_impl(h, q, delta, nullptr, m, offsets, ids, ids_cap, total_out);
}

sfc_status sfc_query_async(sfc_index* h, const double* q, const double* delta,
                           const uint32_t* qepoch, uint64_t m, uint64_t max_rows,
                           uint64_t* offsets, uint32_t* ids, uint64_t ids_cap, uint32_t* flags) {
  if (!h || !offsets || !flags || m == 0 || !q || !delta || (ids_cap > 0 && !ids))
    return SFC_ERR_INVALID;
  if (m > (1ull << 36) || max_rows == 0 || max_rows > (1ull << 40)) return SFC_ERR_INVALID;
  if (h->n_sets) return SFC_ERR_UNSUPPORTED;
  h->pending.valid = false;
  // Growing a scratch buffer waits for the work queued on it first.
  sfc_status st = points_for_test(h);
  if (st == SFC_OK) st = ensure_ws(h, sfc::query_scratch_bytes(m, slots_of(h)));
  if (st == SFC_OK) st = grow(h, &h->cws, &h->cws_bytes, sfc::compact_scratch_bytes(max_rows));
  if (st != SFC_OK) return st;
  sfc::QueryScratch qs{};
  sfc::query_scratch_carve(h->ws, m, &qs, slots_of(h));
  const bool learned = h->search == SFC_SEARCH_LEARNED && h->linfo.fitted;
  const sfc::LearnedView lv = h->larr.view();
  const sfc::StreeView sv = sfc::stree_view(h->keys, h->n, h->stree);
  sfc::EpochView ev;
  const bool filtered = epoch_view(h, qepoch, &ev);
  if (dim_of(h) == 3)
    SFC_TRY(sfc::launch_ranges3(q, delta, m, h->keys, h->n, h->refine != 0, h->refine_min,
                                stree_on(h) ? &sv : nullptr, qs,
                                h->stream));
  else
    SFC_TRY(sfc::launch_ranges(q, delta, m, h->keys, h->n, h->curve, h->refine != 0,
                               h->refine_min, h->metric == SFC_METRIC_L2,
                               learned ? &lv : nullptr,
                               stree_on(h) ? &sv : nullptr, h->occ, nullptr, nullptr, 0, qs,
                               nullptr, nullptr, nullptr, nullptr, nullptr, h->stream));
  if (qepoch)
    SFC_TRY(sfc::validate_epochs(qepoch, m, h->oldest, h->epoch, qs.counters + 2, h->stream));
  SFC_TRY(sfc::launch_compact(q, delta, m, h->xy, h->xy_in, test_cells(h), h->ids, h->n, qs,
                              max_rows, true, h->cws, offsets, ids, ids_cap,
                              h->metric == SFC_METRIC_LINF, dim_of(h), h->stream,
                              filtered ? &ev : nullptr));
  SFC_TRY(hipMemcpyAsync(flags, qs.counters + 2, 4, hipMemcpyDeviceToDevice, h->stream));
  return SFC_OK;
}

sfc_status sfc_query_scratch_size(const sfc_index* h, uint64_t m, uint64_t max_rows,
                                  uint64_t* bytes) {
  if (!h || !bytes || m == 0 || m > (1ull << 36) || max_rows == 0 || max_rows > (1ull << 40))
    return SFC_ERR_INVALID;
  *bytes = align256(sfc::query_scratch_bytes(m, slots_of(h))) + sfc::compact_scratch_bytes(max_rows);
  return SFC_OK;
}

sfc_status sfc_query_async_on(sfc_index* h, void* stream, void* scratch, uint64_t scratch_bytes,
                              const double* q, const double* delta, const uint32_t* qepoch,
                              uint64_t m, uint64_t max_rows, uint64_t* offsets, uint32_t* ids,
                              uint64_t ids_cap, uint32_t* flags) {
  if (!h || !offsets || !flags || !scratch || m == 0 || !q || !delta || (ids_cap > 0 && !ids))
    return SFC_ERR_INVALID;
  if (m > (1ull << 36) || max_rows == 0 || max_rows > (1ull << 40)) return SFC_ERR_INVALID;
  if (((uintptr_t)scratch & 255) != 0) return SFC_ERR_INVALID;
  if (h->n_sets) return SFC_ERR_UNSUPPORTED;
  const size_t qbytes = align256(sfc::query_scratch_bytes(m, slots_of(h)));
  if (scratch_bytes < qbytes + sfc::compact_scratch_bytes(max_rows)) return SFC_ERR_INVALID;
  sfc_status st = points_for_test(h);   // a first gather of the points, on h's stream
  if (st != SFC_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // After the work already queued on the handle's stream (an update's last
  // kernels).
  hipEvent_t ready = nullptr, done = nullptr;
  SFC_TRY(take_sync_event(h, &ready));
  h->idle_events.push_back(ready);   // reusable once the wait below is queued
  SFC_TRY(hipEventRecord(ready, h->stream));
  SFC_TRY(hipStreamWaitEvent(s, ready, 0));
  SFC_TRY(take_sync_event(h, &done));
  sfc::QueryScratch qs{};
  sfc::query_scratch_carve(scratch, m, &qs, slots_of(h));
  const bool learned = h->search == SFC_SEARCH_LEARNED && h->linfo.fitted;
  const sfc::LearnedView lv = h->larr.view();
  const sfc::StreeView sv = sfc::stree_view(h->keys, h->n, h->stree);
  sfc::EpochView ev;
  const bool filtered = epoch_view(h, qepoch, &ev);
  hipError_t e =
      dim_of(h) == 3
          ? sfc::launch_ranges3(q, delta, m, h->keys, h->n, h->refine != 0, h->refine_min,
                                stree_on(h) ? &sv : nullptr, qs, s)
          : sfc::launch_ranges(q, delta, m, h->keys, h->n, h->curve, h->refine != 0,
                               h->refine_min, h->metric == SFC_METRIC_L2,
                               learned ? &lv : nullptr, stree_on(h) ? &sv : nullptr, h->occ,
                               nullptr, nullptr, 0, qs, nullptr, nullptr, nullptr, nullptr,
                               nullptr, s);
  if (e == hipSuccess && qepoch)
    e = sfc::validate_epochs(qepoch, m, h->oldest, h->epoch, qs.counters + 2, s);
  if (e == hipSuccess)
    e = sfc::launch_compact(q, delta, m, h->xy, h->xy_in, test_cells(h), h->ids, h->n, qs,
                            max_rows, true, (char*)scratch + qbytes, offsets, ids, ids_cap,
                            h->metric == SFC_METRIC_LINF, dim_of(h), s, filtered ? &ev : nullptr);
  if (e == hipSuccess) e = hipMemcpyAsync(flags, qs.counters + 2, 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(done, s);
  if (e != hipSuccess) {
    h->idle_events.push_back(done);
    (void)hipGetLastError();
    return from_hip(e);
  }
  // Later writers of the index wait for this batch (finished batches are
  // dropped from the list first).
  for (size_t i = 0; i < h->readers.size();) {
    if (hipEventQuery(h->readers[i]) == hipSuccess) {
      h->idle_events.push_back(h->readers[i]);
      h->readers[i] = h->readers.back();
      h->readers.pop_back();
    } else {
      ++i;
    }
  }
  (void)hipGetLastError();   // hipEventQuery's not-ready status
  h->readers.push_back(done);
  return SFC_OK;
}

sfc_status sfc_query_retry(sfc_index* h, uint64_t* offsets, uint32_t* ids, uint64_t ids_cap,
                           uint64_t* total_out) {
  if (!h || !offsets || !total_out || (ids_cap > 0 && !ids)) return SFC_ERR_INVALID;
  const sfc_index::Pending p = h->pending;
  if (!p.valid || p.generation != h->generation) return SFC_ERR_UNSUPPORTED;
  if (ids_cap < p.total) {
    *total_out = p.total;
    return SFC_ERR_CAPACITY;
  }
  h->pending.valid = false;
  SFC_TRY(sfc::launch_compact(nullptr, nullptr, p.m, h->xy, h->xy_in, nullptr, h->ids, h->n,
                              p.qs, p.rows, false, h->cws, offsets, ids, ids_cap, false, dim_of(h),
                              h->stream, nullptr, true));
  uint64_t total = 0;
  SFC_TRY(read_words(offsets + p.m, &total, 1, h->stream));
  if (total != p.total) return SFC_ERR_DEVICE;
  h->last.reported = total;
  *total_out = total;
  return SFC_OK;
}

}  // extern "C"

// ---- query batches in the library's static scratch --------------------------

namespace {

// The scratch of sfc_query_batch_static: a fixed array in the library's code
// object, one copy per device, held until the process ends.  Host code must
// not pass the array's name to a kernel or a copy (in host code it names a
// host-side stand-in): its device address comes from hipGetSymbolAddress,
// taken once per device with that device current.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch.
sfc_status static_scratch(void** out) {
  int dev = 0;
  SFC_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SFC_ERR_DEVICE;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    SFC_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return SFC_ERR_DEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SFC_OK;
}

}  // namespace

extern "C" {

sfc_status sfc_query_batch_static(sfc_index* h, const double* q, const double* delta, uint64_t m,
                                  uint64_t* offsets, uint32_t* ids, uint64_t ids_cap,
                                  uint64_t* total_out) {
  if (!h || !offsets || !total_out || (m > 0 && (!q || !delta)) || (ids_cap > 0 && !ids))
    return SFC_ERR_INVALID;
  if (m > (1ull << 36)) return SFC_ERR_INVALID;
  // The test pass reads the cells, or the points in key order: gathering
  // those would allocate.
  if (!test_cells(h) && !h->xy && h->n > 0) return SFC_ERR_UNSUPPORTED;
  const size_t qbytes = align256(sfc::query_scratch_bytes(m, slots_of(h)));
  if (qbytes > kStaticScratchBytes) return SFC_ERR_SCRATCH;
  void* base = nullptr;
  {
    sfc_status st = static_scratch(&base);
    if (st != SFC_OK) return st;
  }
  h->pending.valid = false;   // the handle's kept batch is not this one
  sfc::QueryScratch qs{};
  uint64_t total_rows = 0, total_cand = 0;
  if (m > 0) {
    uint64_t rb[8];
    sfc_status st = run_ranges_into(h, base, rb, q, delta, nullptr, m, &qs, &total_rows,
                                    &total_cand, nullptr, nullptr, nullptr, nullptr, nullptr,
                                    nullptr);
    if (st != SFC_OK) return st;
  } else {
    sfc::query_scratch_carve(base, 0, &qs, slots_of(h));
  }
  if (qbytes + sfc::compact_scratch_bytes(total_rows) > kStaticScratchBytes)
    return SFC_ERR_SCRATCH;
  sfc::EpochView ev;
  const bool filtered = epoch_view(h, nullptr, &ev);
  SFC_TRY(sfc::launch_compact(q, delta, m, h->xy, h->xy_in, test_cells(h), h->ids, h->n, qs,
                              total_rows, false, (char*)base + qbytes, offsets, ids, ids_cap,
                              h->metric == SFC_METRIC_LINF, dim_of(h), h->stream,
                              filtered ? &ev : nullptr, false, m > 0 ? h->last_coarse : 0));
  uint64_t tail[3] = {0, 0, 0};   // the total, then the error word's doubleword
  SFC_TRY(hipMemcpyAsync(&tail[0], offsets + m, 8, hipMemcpyDeviceToHost, h->stream));
  if (m > 0)
    SFC_TRY(hipMemcpyAsync(&tail[1], qs.counters, 16, hipMemcpyDeviceToHost, h->stream));
  SFC_TRY(hipStreamSynchronize(h->stream));
  if (m > 0 && (((const uint32_t*)&tail[1])[2] & (sfc::kErrLookback | sfc::kErrInternal)))
    return SFC_ERR_DEVICE;
  const uint64_t total = tail[0];
  h->last.queries = m;
  h->last.candidates = total_cand;
  h->last.reported = total;
  h->last.rows = total_rows;
  h->last.pruned = m > 0 ? h->last_pruned : 0;
  *total_out = total;
  return total > ids_cap ? SFC_ERR_CAPACITY : SFC_OK;
}

sfc_status sfc_query_epochs(sfc_index* h, const double* q, const double* delta,
                            const uint32_t* qepoch, uint64_t m, uint64_t* offsets, uint32_t* ids,
                            uint64_t ids_cap, uint64_t* total_out) {
  if (!h || (m > 0 && !qepoch)) return SFC_ERR_INVALID;
  return query_impl(h, q, delta, nullptr, m, offsets, ids, ids_cap, total_out, qepoch);
}

sfc_status sfc_query_sets(sfc_index* h, const double* q, const double* delta,
                          const uint32_t* qset, uint64_t m, uint64_t* offsets, uint32_t* ids,
                          uint64_t ids_cap, uint64_t* total_out) {
  if (!h || (m > 0 && !qset) || h->n_sets == 0) return SFC_ERR_INVALID;
  return query_impl(h, q, delta, qset, m, offsets, ids, ids_cap, total_out);
}

sfc_status sfc_query_ranges(sfc_index* h, const double* q, const double* delta, uint64_t m,
                            uint64_t* key_lo, uint64_t* key_hi, uint64_t* begin, uint64_t* end,
                            uint32_t* nranges) {
  if (!h || (m > 0 && (!q || !delta || !key_lo || !key_hi || !begin || !end || !nranges)))
    return SFC_ERR_INVALID;
  if (dim_of(h) == 3) return SFC_ERR_UNSUPPORTED;   // eight ranges per query, not four
  if (m == 0) return SFC_OK;
  sfc::QueryScratch qs{};
  uint64_t total_rows = 0, total_cand = 0;
  return run_ranges(h, q, delta, nullptr, m, &qs, &total_rows, &total_cand, key_lo, key_hi, begin,
                    end, nranges);
}

uint64_t sfc_size(const sfc_index* h) { return h ? h->n : 0; }

sfc_status sfc_index_view(const sfc_index* h, const uint64_t** keys, const uint32_t** ids,
                          const double** xy, uint64_t* n) {
  if (!h) return SFC_ERR_INVALID;
  if (xy) {
    // Filling the sorted copy on first use does not change what the index holds.
    sfc_status st = ensure_sorted_xy(const_cast<sfc_index*>(h));
    if (st != SFC_OK) return st;
  }
  if (keys) *keys = h->keys;
  if (ids) *ids = h->ids;
  if (xy) *xy = h->xy;
  if (n) *n = h->n;
  return SFC_OK;
}

sfc_status sfc_index_copy(const sfc_index* h, uint64_t* keys, uint32_t* ids, double* xy) {
  if (!h) return SFC_ERR_INVALID;
  if (h->n == 0) return SFC_OK;
  if (keys) SFC_TRY(hipMemcpyAsync(keys, h->keys, h->n * 8, hipMemcpyDeviceToDevice, h->stream));
  if (ids) SFC_TRY(hipMemcpyAsync(ids, h->ids, h->n * 4, hipMemcpyDeviceToDevice, h->stream));
  if (xy && h->xy)
    SFC_TRY(hipMemcpyAsync(xy, h->xy, h->n * 8 * dim_of(h), hipMemcpyDeviceToDevice, h->stream));
  else if (xy)
    SFC_TRY(sfc::gather_sorted(h->ids, h->xy_in, xy, h->n, dim_of(h), h->stream));
  SFC_TRY(hipStreamSynchronize(h->stream));
  return SFC_OK;
}

sfc_status sfc_cells_copy(const sfc_index* h, uint64_t* out, uint64_t count) {
  if (!h || (count > 0 && !out) || count < h->n) return SFC_ERR_INVALID;
  if (!h->cells) return SFC_ERR_UNSUPPORTED;
  if (h->n == 0) return SFC_OK;
  SFC_TRY(hipMemcpyAsync(out, h->cells, h->n * 8, hipMemcpyDeviceToDevice, h->stream));
  SFC_TRY(hipStreamSynchronize(h->stream));
  return SFC_OK;
}

sfc_status sfc_occupancy_copy(const sfc_index* h, uint32_t* out, uint64_t words) {
  if (!h || (words > 0 && !out)) return SFC_ERR_INVALID;
  if (!h->occ) return SFC_ERR_UNSUPPORTED;
  if (words < sfc::kOccWords) return SFC_ERR_CAPACITY;
  SFC_TRY(hipMemcpyAsync(out, h->occ, sfc::kOccWords * 4, hipMemcpyDeviceToDevice, h->stream));
  SFC_TRY(hipStreamSynchronize(h->stream));
  return SFC_OK;
}

sfc_status sfc_last_query_stats(const sfc_index* h, sfc_query_stats* out) {
  if (!h || !out) return SFC_ERR_INVALID;
  *out = h->last;
  return SFC_OK;
}

sfc_status sfc_set_search(sfc_index* h, int search) {
  if (!h || (search != SFC_SEARCH_BINARY && search != SFC_SEARCH_LEARNED &&
             search != SFC_SEARCH_STREE))
    return SFC_ERR_INVALID;
  if (h->n_sets && search != SFC_SEARCH_BINARY) return SFC_ERR_UNSUPPORTED;
  if (dim_of(h) == 3 && search == SFC_SEARCH_LEARNED) return SFC_ERR_UNSUPPORTED;
  if (search == SFC_SEARCH_LEARNED && !h->linfo.fitted && h->n >= 2) {
    sfc_status st = fit_learned(h, -1);
    if (st != SFC_OK) return st;
  }
  if (search == SFC_SEARCH_STREE && !h->stree_ready) {
    sfc_status st = stree_refresh(h);
    if (st != SFC_OK) return st;
  }
  h->search = search;
  return SFC_OK;
}

sfc_status sfc_set_cell_filter(sfc_index* h, int on) {
  if (!h || (on != 0 && on != 1)) return SFC_ERR_INVALID;
  h->cell_filter = on != 0;
  return SFC_OK;
}

sfc_status sfc_set_metric(sfc_index* h, int metric) {
  if (!h || (metric != SFC_METRIC_L2 && metric != SFC_METRIC_LINF)) return SFC_ERR_INVALID;
  h->metric = metric;
  return SFC_OK;
}

sfc_status sfc_learned_fit(sfc_index* h, int steps) {
  if (!h) return SFC_ERR_INVALID;
  return fit_learned(h, steps);
}

sfc_status sfc_debug_sort_path(int force_plain, int* last_fallback) {
  if (force_plain >= 0) g_force_plain_sort = force_plain != 0;
  if (last_fallback) *last_fallback = g_last_sort_fallback;
  return SFC_OK;
}

sfc_status sfc_debug_chunk_tiles(uint64_t tiles) {
  sfc::set_compact_chunk_tiles(tiles);
  return SFC_OK;
}

sfc_status sfc_learned_shrink_windows(sfc_index* h) {
  if (!h) return SFC_ERR_INVALID;
  if (!h->linfo.fitted) return SFC_ERR_UNSUPPORTED;
  SFC_TRY(wait_readers(h));
  if (h->lstats_stale) {
    SFC_TRY(leaf_stats(h));
    h->lstats_stale = false;
  }
  const uint32_t np = h->linfo.pieces;
  std::vector<sfc::PieceRec> pr(np);
  if (np == 0) return SFC_OK;
  SFC_TRY(hipMemcpyAsync(pr.data(), h->larr.pr, np * sizeof(sfc::PieceRec),
                         hipMemcpyDeviceToHost, h->stream));
  SFC_TRY(hipStreamSynchronize(h->stream));
  for (sfc::PieceRec& r : pr) r.elo = r.ehi = 0;
  SFC_TRY(hipMemcpyAsync(h->larr.pr, pr.data(), np * sizeof(sfc::PieceRec),
                         hipMemcpyHostToDevice, h->stream));
  SFC_TRY(hipStreamSynchronize(h->stream));
  return SFC_OK;
}

sfc_status sfc_learned_route(sfc_index* h, const uint64_t* keys, uint64_t count,
                             uint32_t* direct, uint32_t* table) {
  if (!h || (count > 0 && (!keys || !direct || !table))) return SFC_ERR_INVALID;
  if (!h->linfo.fitted) return SFC_ERR_UNSUPPORTED;
  SFC_TRY(sfc::learned_route_both(h->lparams, h->larr, keys, count, direct, table, h->stream));
  SFC_TRY(hipStreamSynchronize(h->stream));
  return SFC_OK;
}

sfc_status sfc_learned_info_get(const sfc_index* h, sfc_learned_info* out) {
  if (!h || !out) return SFC_ERR_INVALID;
  if (h->linfo.fitted && h->lstats_stale) {
    // Reading the statistics back changes no observable state of the index.
    sfc_index* m = const_cast<sfc_index*>(h);
    SFC_TRY(leaf_stats(m));
    m->lstats_stale = false;
  }
  *out = h->linfo;
  return SFC_OK;
}

sfc_status sfc_learned_params(const sfc_index* h, float* params) {
  if (!h || !params) return SFC_ERR_INVALID;
  if (!h->linfo.fitted) return SFC_ERR_UNSUPPORTED;
  SFC_TRY(hipMemcpyAsync(params, h->lparams, sfc::kParams * sizeof(float), hipMemcpyDeviceToHost,
                         h->stream));
  SFC_TRY(hipStreamSynchronize(h->stream));
  return SFC_OK;
}

sfc_status sfc_learned_grad(const float* params, const float* x, const float* t, uint32_t count,
                            float* grad, float* loss) {
  if (!params || !x || !t || !grad || !loss || count < 1 || count > 128) return SFC_ERR_INVALID;
  sfc::Allocator a;
  const size_t pb = sfc::align256(sfc::kParams * 4);
  char* d = (char*)a.get(2 * pb + 2 * 512 + 256);
  if (!d) return SFC_ERR_NOMEM;
  float* dp = (float*)d;
  float* dg = (float*)(d + pb);
  float* dx = (float*)(d + 2 * pb);
  float* dt = (float*)(d + 2 * pb + 512);
  float* dl = (float*)(d + 2 * pb + 1024);
  hipError_t e = hipMemcpy(dp, params, sfc::kParams * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dx, x, count * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dt, t, count * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = sfc::learned_grad(dp, dx, dt, (int)count, dg, dl, nullptr);
  if (e == hipSuccess) e = hipMemcpy(grad, dg, sfc::kParams * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(loss, dl, 4, hipMemcpyDeviceToHost);
  a.put(d);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return from_hip(e);
  }
  return SFC_OK;
}

}  // extern "C"

struct sfc_graph {
  sfc_index* h = nullptr;
  int kind = 0;                 // 0: construction, 1: query batch
  hipStream_t cap = nullptr;    // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* scratch = nullptr;      // construction scratch, or query scratch
  void* cscratch = nullptr;     // compaction scratch (queries)
  uint32_t* err = nullptr;      // construction error word
  sfc::QueryScratch qs{};
  uint64_t m = 0, max_rows = 0, cap_ids = 0;
  uint64_t* offsets = nullptr;
  uint64_t generation = 0;      // h's generation at recording
};

namespace {

void graph_release(sfc_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  if (g->h) {
    g->h->alloc.put(g->scratch);
    g->h->alloc.put(g->cscratch);
  }
  delete g;
}

// Records fn(stream) into g's graph and instantiates it.
template <typename F>
sfc_status graph_capture(sfc_graph* g, F fn) {
  SFC_TRY(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
  SFC_TRY(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
  sfc::g_capturing.fetch_add(1);
  hipError_t e = fn(g->cap);
  sfc::g_capturing.fetch_sub(1);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(g->cap, &graph);
  if (e == hipSuccess) e = e2;
  g->graph = graph;
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return from_hip(e);
  }
  return SFC_OK;
}

}  // namespace

extern "C" {

sfc_status sfc_graph_build(sfc_index* h, const double* xy, sfc_graph** out) {
  if (!h || !out || (h->n > 0 && !xy)) return SFC_ERR_INVALID;
  if (h->n == 0 || h->ins) return SFC_ERR_UNSUPPORTED;
  sfc_graph* g = new (std::nothrow) sfc_graph();
  if (!g) return SFC_ERR_NOMEM;
  g->h = h;
  g->kind = 0;
  g->generation = h->generation;
  const size_t sb = sfc::build_scratch_bytes(h->n) + 256;
  g->scratch = h->alloc.get(sb);
  if (!g->scratch) {
    graph_release(g);
    return SFC_ERR_NOMEM;
  }
  g->err = (uint32_t*)((char*)g->scratch + sb - 256);
  sfc_status st = graph_capture(g, [&](hipStream_t s) {
    hipError_t e = sfc::fill_u32(g->err, 0, 1, s);
    // The chunked sort with the plain one recorded behind it, which runs (on
    // the device) only when a run was too long for the chunks.
    if (e == hipSuccess)
      e = g_force_plain_sort
              ? sfc::sort_build(xy, h->n, h->curve, h->keys, h->ids, h->xy, g->scratch, g->err,
                                s, h->set_off, h->n_sets, h->cells, h->xy_in)
              : sfc::sort_build_sets_chunked(xy, h->n, h->curve, h->keys, h->ids, h->xy,
                                             g->scratch, g->err, s, h->set_off, h->n_sets,
                                             h->cells, h->xy_in, true);
    if (e == hipSuccess && h->occ) e = sfc::build_occupancy(h->keys, h->n, h->occ, s);
    if (e == hipSuccess && h->stree_ready)
      e = sfc::stree_build(sfc::stree_view(h->keys, h->n, h->stree), s);
    return e;
  });
  if (st != SFC_OK) {
    graph_release(g);
    return st;
  }
  *out = g;
  return SFC_OK;
}

sfc_status sfc_graph_query(sfc_index* h, const double* q, const double* delta,
                           const uint32_t* qset, uint64_t m, uint64_t max_rows, uint64_t* offsets,
                           uint32_t* ids, uint64_t ids_cap, sfc_graph** out) {
  if (!h || !out || !offsets || m == 0 || !q || !delta || (ids_cap > 0 && !ids)) return SFC_ERR_INVALID;
  if (qset && h->n_sets == 0) return SFC_ERR_INVALID;
  if (max_rows == 0 || max_rows > (1ull << 40)) return SFC_ERR_INVALID;
  {
    sfc_status st = points_for_test(h);
    if (st != SFC_OK) return st;
  }
  sfc_graph* g = new (std::nothrow) sfc_graph();
  if (!g) return SFC_ERR_NOMEM;
  g->h = h;
  g->kind = 1;
  g->generation = h->generation;
  g->m = m;
  g->max_rows = max_rows;
  g->cap_ids = ids_cap;
  g->offsets = offsets;
  g->scratch = h->alloc.get(sfc::query_scratch_bytes(m, slots_of(h)));
  g->cscratch = h->alloc.get(sfc::compact_scratch_bytes(max_rows));
  if (!g->scratch || !g->cscratch) {
    graph_release(g);
    return SFC_ERR_NOMEM;
  }
  sfc::query_scratch_carve(g->scratch, m, &g->qs, slots_of(h));
  const bool learned = h->search == SFC_SEARCH_LEARNED && h->linfo.fitted && !qset;
  const sfc::LearnedView lv = h->larr.view();
  const sfc::StreeView sv = sfc::stree_view(h->keys, h->n, h->stree);
  sfc::EpochView ev;
  const bool filtered = epoch_view(h, nullptr, &ev);
  sfc_status st = graph_capture(g, [&](hipStream_t s) {
    hipError_t e =
        dim_of(h) == 3
            ? sfc::launch_ranges3(q, delta, m, h->keys, h->n, h->refine != 0, h->refine_min,
                                stree_on(h) ? &sv : nullptr, g->qs,
                                  s)
            : sfc::launch_ranges(q, delta, m, h->keys, h->n, h->curve, h->refine != 0,
                                 h->refine_min, h->metric == SFC_METRIC_L2,
                                 learned ? &lv : nullptr,
                                 stree_on(h) ? &sv : nullptr, h->occ, qset,
                                 qset ? h->set_off : nullptr, h->n_sets, g->qs, nullptr, nullptr,
                                 nullptr, nullptr, nullptr, s);
    if (e == hipSuccess)
      e = sfc::launch_compact(q, delta, m, h->xy, h->xy_in, test_cells(h), h->ids, h->n,
                              g->qs, max_rows, true, g->cscratch, offsets, ids, ids_cap,
                              h->metric == SFC_METRIC_LINF, dim_of(h), s,
                              filtered ? &ev : nullptr);
    return e;
  });
  if (st != SFC_OK) {
    graph_release(g);
    return st;
  }
  *out = g;
  return SFC_OK;
}

sfc_status sfc_graph_launch(sfc_graph* g) {
  if (!g || !g->exec) return SFC_ERR_INVALID;
  if (g->generation != g->h->generation) return SFC_ERR_INVALID;   // recorded before an update
  if (g->kind == 0) SFC_TRY(wait_readers(g->h));
  SFC_TRY(hipGraphLaunch(g->exec, g->h->stream));
  return SFC_OK;
}

sfc_status sfc_graph_wait(sfc_graph* g, uint64_t* total_out) {
  if (!g) return SFC_ERR_INVALID;
  sfc_index* h = g->h;
  if (g->kind == 0) {
    uint64_t w = 0;
    SFC_TRY(read_words(g->err, &w, 1, h->stream));
    if ((uint32_t)w & sfc::kErrDomain) return SFC_ERR_DOMAIN;
    if ((uint32_t)w & (sfc::kErrLookback | sfc::kErrInternal)) return SFC_ERR_DEVICE;
    return SFC_OK;
  }
  uint64_t cw[2];
  uint64_t total = 0;
  SFC_TRY(read_words(g->qs.counters, cw, 2, h->stream));
  SFC_TRY(read_words(g->offsets + g->m, &total, 1, h->stream));
  const uint32_t err = ((const uint32_t*)cw)[2];
  if (err & sfc::kErrInvalidQuery) return SFC_ERR_INVALID;
  if (err & (sfc::kErrLookback | sfc::kErrInternal)) return SFC_ERR_DEVICE;
  if (err & sfc::kErrOverflow) return SFC_ERR_CAPACITY;   // more candidate rows than max_rows
  if (total_out) *total_out = total;
  return total > g->cap_ids ? SFC_ERR_CAPACITY : SFC_OK;
}

void sfc_graph_free(sfc_graph* g) {
  if (g && g->h) (void)hipStreamSynchronize(g->h->stream);
  graph_release(g);
}

}  // extern "C"

namespace {
// Mean milliseconds of fn() over reps launches after one warm-up, timed with
// HIP events on stream s.
template <typename F>
sfc_status time_ms(hipStream_t s, int reps, F fn, double* ms) {
  sfc_status st = fn();
  if (st != SFC_OK && st != SFC_ERR_CAPACITY) return st;
  hipEvent_t a, b;
  SFC_TRY(hipEventCreate(&a));
  SFC_TRY(hipEventCreate(&b));
  SFC_TRY(hipEventRecord(a, s));
  for (int i = 0; i < reps; ++i) {
    st = fn();
    if (st != SFC_OK && st != SFC_ERR_CAPACITY) break;
  }
  SFC_TRY(hipEventRecord(b, s));
  SFC_TRY(hipEventSynchronize(b));
  float t = 0.f;
  SFC_TRY(hipEventElapsedTime(&t, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = t / reps;
  return st == SFC_ERR_CAPACITY ? SFC_OK : st;
}
}  // namespace

extern "C" {

sfc_status sfc_autotune_build(const double* xy, uint64_t n, const uint64_t* set_off,
                              uint32_t n_sets, const sfc_options* opt, int* best, double* ms) {
  if (n == 0 || !xy) return SFC_ERR_INVALID;
  static const int kItems[5] = {8, 12, 16, 20, 24};
  sfc_options o;
  sfc_default_options(&o);
  if (opt) o = *opt;
  o.search = SFC_SEARCH_BINARY;
  double t[5] = {0, 0, 0, 0, 0};
  int pick = 16;
  double tb = 1e30;
  for (int v = 0; v < 5; ++v) {
    sfc::set_tuned(sfc::kTuneSortItems, n, kItems[v]);
    sfc_status st = time_ms((hipStream_t)o.stream, 3, [&] {
      sfc_index* h = nullptr;
      sfc_status r = set_off ? sfc_build_sets(xy, set_off, n_sets, &o, &h) : sfc_build(xy, n, &o, &h);
      sfc_free(h);
      return r;
    }, &t[v]);
    if (st != SFC_OK) return st;
    if (t[v] < tb) {
      tb = t[v];
      pick = kItems[v];
    }
  }
  sfc::set_tuned(sfc::kTuneSortItems, n, pick);
  if (best) *best = pick;
  if (ms) for (int v = 0; v < 5; ++v) ms[v] = t[v];
  return SFC_OK;
}

sfc_status sfc_autotune_query(sfc_index* h, const double* q, const double* delta,
                              const uint32_t* qset, uint64_t m, uint64_t* offsets, uint32_t* ids,
                              uint64_t ids_cap, int* best, double* ms) {
  if (!h || m == 0) return SFC_ERR_INVALID;
  uint64_t total = 0;
  sfc_status st = query_impl(h, q, delta, qset, m, offsets, ids, ids_cap, &total);
  if (st != SFC_OK && st != SFC_ERR_CAPACITY) return st;
  // The test kernel's shape is chosen per bucket of the batch's candidate rows.
  sfc::QueryScratch qs{};
  uint64_t rows = 0, cand = 0;
  st = run_ranges(h, q, delta, qset, m, &qs, &rows, &cand, nullptr, nullptr, nullptr, nullptr,
                  nullptr);
  if (st != SFC_OK) return st;
  double t[5] = {0, 0, 0, 0, 0};
  int pick = 0;
  double tb = 1e30;
  for (int v = 0; v < 5; ++v) {
    sfc::set_tuned(sfc::kTuneTestShape, rows, v);
    st = time_ms(h->stream, 3, [&] {
      uint64_t tot = 0;
      return query_impl(h, q, delta, qset, m, offsets, ids, ids_cap, &tot);
    }, &t[v]);
    if (st != SFC_OK) return st;
    if (t[v] < tb) {
      tb = t[v];
      pick = v;
    }
  }
  sfc::set_tuned(sfc::kTuneTestShape, rows, pick);
  if (best) *best = pick;
  if (ms) for (int v = 0; v < 5; ++v) ms[v] = t[v];
  return SFC_OK;
}

sfc_status sfc_tune_pin(int what, uint64_t size, int value) {
  if (what == SFC_TUNE_SORT_ITEMS) {
    if (value != -1 && value != 8 && value != 12 && value != 16 && value != 20 && value != 24)
      return SFC_ERR_INVALID;
    sfc::set_tuned(sfc::kTuneSortItems, size, value);
    return SFC_OK;
  }
  if (what == SFC_TUNE_TEST_SHAPE) {
    if (value < -1 || value > 4) return SFC_ERR_INVALID;
    sfc::set_tuned(sfc::kTuneTestShape, size, value);
    return SFC_OK;
  }
  return SFC_ERR_INVALID;
}

void sfc_free(sfc_index* h) {
  if (!h) return;
  (void)wait_readers(h);
  (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->idle_events) (void)hipEventDestroy(e);
  release_arrays(h);
  delete h;
}

void sfc_profile_enable(int on) {
  sfc::ProfState& P = sfc::prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.on = on != 0;
}

void sfc_profile_only(const char* name) {
  sfc::ProfState& P = sfc::prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.only = name ? name : "";
}

void sfc_profile_reset(void) {
  sfc::ProfState& P = sfc::prof();
  std::lock_guard<std::mutex> g(P.mu);
  sfc::prof_drain(P);
  P.acc.clear();
  P.order.clear();
}

int sfc_profile_read(const char** names, uint64_t* launches, double* ms, int max) {
  sfc::ProfState& P = sfc::prof();
  std::lock_guard<std::mutex> g(P.mu);
  sfc::prof_drain(P);
  int i = 0;
  for (const std::string& k : P.order) {
    if (i < max) {
      const auto& v = P.acc[k];
      // The key strings live in the map for the life of the process.
      if (names) names[i] = P.acc.find(k)->first.c_str();
      if (launches) launches[i] = v.first;
      if (ms) ms[i] = v.second;
    }
    ++i;
  }
  return i;
}

void sfc_pool_trim(void) {
  sfc::Pool& P = sfc::pool();
  std::lock_guard<std::mutex> g(P.mu);
  for (auto& kv : P.free_blocks)
    for (void* p : kv.second) (void)hipFree(p);
  P.free_blocks.clear();
}

}  // extern "C"

// ---- updates ---------------------------------------------------------------

namespace {

// Allocates the epoch arrays (everything stored so far: inserted at epoch 0,
// live) and the id -> key table, before the first update.
sfc_status ensure_dynamic(sfc_index* h) {
  if (h->ins) return SFC_OK;
  {
    sfc_status st = ensure_sorted_xy(h);   // merges move the sorted points
    if (st != SFC_OK) return st;
  }
  const uint64_t c = h->cap ? h->cap : 1;
  const uint64_t kc = h->next_id > 1024 ? h->next_id : 1024;
  uint32_t* ins = (uint32_t*)h->alloc.get(c * 4);
  uint32_t* era = (uint32_t*)h->alloc.get(c * 4);
  uint64_t* key_of = (uint64_t*)h->alloc.get(kc * 8);
  uint64_t* word = (uint64_t*)h->alloc.get(256);
  if (!ins || !era || !key_of || !word) {
    h->alloc.put(ins);
    h->alloc.put(era);
    h->alloc.put(key_of);
    h->alloc.put(word);
    return SFC_ERR_NOMEM;
  }
  hipError_t e = sfc::fill_u32(ins, 0, c, h->stream);
  if (e == hipSuccess) e = sfc::fill_u32(era, sfc::kLiveEpoch, c, h->stream);
  if (e == hipSuccess) e = sfc::record_keys(h->keys, h->ids, h->n, key_of, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    h->alloc.put(ins);
    h->alloc.put(era);
    h->alloc.put(key_of);
    h->alloc.put(word);
    return from_hip(e);
  }
  h->ins = ins;
  h->era = era;
  h->key_of = key_of;
  h->key_of_cap = kc;
  h->upd_word = word;
  // An index that takes updates drops the grid cells: every merge and
  // compaction rewrites the whole run, and carrying the cells would add a
  // fifth of its traffic; its queries test every candidate exactly.
  h->alloc.put(h->cells);
  h->cells = nullptr;
  return SFC_OK;
}

// The spare run holds at least `need` entries (grown by a quarter beyond).
sfc_status ensure_spare(sfc_index* h, uint64_t need) {
  if (need == 0) need = 1;
  if (h->spare_cap >= need) return SFC_OK;
  sfc::Run& r = h->spare;
  h->alloc.put(r.keys);
  h->alloc.put(r.ids);
  h->alloc.put(r.xy);
  h->alloc.put(r.ins);
  h->alloc.put(r.era);
  h->alloc.put(r.cells);
  r = sfc::Run{};
  h->spare_cap = 0;
  const uint64_t c = need + need / 4;
  r.keys = (uint64_t*)h->alloc.get(c * 8);
  r.ids = (uint32_t*)h->alloc.get(c * 4);
  r.xy = (double*)h->alloc.get(c * 16);
  r.ins = (uint32_t*)h->alloc.get(c * 4);
  r.era = (uint32_t*)h->alloc.get(c * 4);
  if (!r.keys || !r.ids || !r.xy || !r.ins || !r.era) {
    h->alloc.put(r.keys);
    h->alloc.put(r.ids);
    h->alloc.put(r.xy);
    h->alloc.put(r.ins);
    h->alloc.put(r.era);
    h->alloc.put(r.cells);
    r = sfc::Run{};
    return SFC_ERR_NOMEM;
  }
  h->spare_cap = c;
  return SFC_OK;
}

// The id -> key table covers ids [0, need).
sfc_status ensure_key_of(sfc_index* h, uint64_t need) {
  if (h->key_of_cap >= need) return SFC_OK;
  uint64_t c = h->key_of_cap * 2;
  if (c < need) c = need;
  uint64_t* t = (uint64_t*)h->alloc.get(c * 8);
  if (!t) return SFC_ERR_NOMEM;
  hipError_t e = hipMemcpyAsync(t, h->key_of, (uint64_t)h->next_id * 8, hipMemcpyDeviceToDevice,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    h->alloc.put(t);
    return from_hip(e);
  }
  h->alloc.put(h->key_of);
  h->key_of = t;
  h->key_of_cap = c;
  return SFC_OK;
}

sfc::Run current_run(const sfc_index* h) {
  sfc::Run r;
  r.keys = h->keys;
  r.ids = h->ids;
  r.xy = h->xy;
  r.ins = h->ins;
  r.era = h->era;
  r.cells = h->cells;
  return r;
}

void swap_runs(sfc_index* h) {
  std::swap(h->keys, h->spare.keys);
  std::swap(h->ids, h->spare.ids);
  std::swap(h->xy, h->spare.xy);
  std::swap(h->ins, h->spare.ins);
  std::swap(h->era, h->spare.era);
  std::swap(h->cells, h->spare.cells);
  std::swap(h->cap, h->spare_cap);
}

uint64_t droppable(const sfc_index* h) {
  uint64_t d = 0;
  for (const auto& t : h->tombs)
    if (t.first <= h->oldest) d += t.second;
  return d;
}

// Drops every tombstone no queryable epoch sees (era <= oldest).
sfc_status compact_now(sfc_index* h) {
  const uint64_t drop = droppable(h);
  if (drop == 0) return SFC_OK;
  SFC_TRY(wait_readers(h));
  const uint64_t keep = h->n - drop;
  // Room for every stored entry: the device's count decides what is written.
  sfc_status st = ensure_spare(h, h->n);
  if (st != SFC_OK) return st;
  void* scratch = h->alloc.get(sfc::compact_entries_scratch(h->n));
  if (!scratch) return SFC_ERR_NOMEM;
  uint64_t* kept_dev = nullptr;
  uint64_t kept = 0;
  hipError_t e = sfc::compact_entries(current_run(h), h->n, h->oldest, h->spare, scratch,
                                      &kept_dev, h->stream);
  if (e == hipSuccess) e = read_words(kept_dev, &kept, 1, h->stream);
  h->alloc.put(scratch);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return from_hip(e);
  }
  if (kept != keep) return SFC_ERR_DEVICE;   // the host's tombstone count disagrees
  swap_runs(h);
  h->n = keep;
  h->dead -= drop;
  if (h->occ) SFC_TRY(sfc::build_occupancy(h->keys, h->n, h->occ, h->stream));
  if (h->stree_ready) {
    sfc_status st2 = stree_refresh(h);
    if (st2 != SFC_OK) return st2;
  }

  std::vector<std::pair<uint32_t, uint64_t>> rest;
  for (const auto& t : h->tombs)
    if (t.first > h->oldest) rest.push_back(t);
  h->tombs.swap(rest);
  ++h->generation;
  ++h->compactions;
  return refit_leaves(h);
}

// Compacts once the droppable tombstones reach a tenth of the stored entries.
// A compaction that finds no memory is put off to a later update: the
// tombstones stay (queries skip them), so nothing the caller sees changes.
sfc_status maybe_compact(sfc_index* h) {
  const uint64_t d = droppable(h);
  if (d > 0 && d * 10 >= h->n) {
    const sfc_status st = compact_now(h);
    return st == SFC_ERR_NOMEM ? SFC_OK : st;
  }
  return SFC_OK;
}

}  // namespace

extern "C" {

namespace {

// Inserts `runs` consecutive batches of xy (host offsets run_off, runs + 1
// of them) as one sort and one merge; run r's points are inserted at epoch
// h->epoch + 1 + r, and the index's epoch advances by `runs`.
sfc_status insert_impl(sfc_index* h, const double* xy, uint64_t k, const uint64_t* run_off,
                       uint32_t runs, uint32_t* ids_out) {
  if (k == 0 && runs <= 1) return SFC_OK;
  if ((uint64_t)h->next_id + k > 0xFFFFFFFEull) return SFC_ERR_INVALID;
  if ((uint64_t)h->epoch + runs >= 0xFFFFFFFEull) return SFC_ERR_UNSUPPORTED;
  if (k == 0) {   // runs of no points: the epochs still advance
    h->epoch += runs;
    if (!h->hold) h->oldest = h->epoch;
    return SFC_OK;
  }
  SFC_TRY(wait_readers(h));
  sfc_status st = ensure_dynamic(h);
  if (st == SFC_OK) st = ensure_key_of(h, (uint64_t)h->next_id + k);
  if (st == SFC_OK) st = ensure_spare(h, h->n + k);
  // The learned leaves and the search tree of n + k keys get their memory
  // now, so that nothing after the merge allocates: a failed allocation
  // leaves the index as it was.
  if (st == SFC_OK && h->linfo.fitted) st = ensure_lmodel(h, h->n + k);
  if (st == SFC_OK && h->stree_ready) st = stree_reserve(h, h->n + k);
  if (st != SFC_OK) return st;
  const size_t sb = sfc::build_scratch_bytes(k) + 256;
  const size_t rb = runs > 1 ? align256((runs + 1) * 8) : 0;
  char* batch =
      (char*)h->alloc.get(align256(k * 8) + align256(k * 4) + align256(k * 16) + sb + rb);
  if (!batch) return SFC_ERR_NOMEM;
  uint64_t* bkeys = (uint64_t*)batch;
  uint32_t* bids = (uint32_t*)(batch + align256(k * 8));
  double* bxy = (double*)(batch + align256(k * 8) + align256(k * 4));
  void* scratch = batch + align256(k * 8) + align256(k * 4) + align256(k * 16);
  uint32_t* err = (uint32_t*)((char*)scratch + sb - 256);
  uint64_t* roff = runs > 1 ? (uint64_t*)((char*)scratch + sb) : nullptr;
  const uint32_t ep = h->epoch + 1;
  // Sort the batch, merge it into the spare run; the swap happens only when
  // the batch's coordinates were all in the domain.
  hipError_t e = sfc::fill_u32(err, 0, 1, h->stream);
  if (e == hipSuccess && roff)
    e = hipMemcpyAsync(roff, run_off, (runs + 1) * 8, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = sfc::sort_build(xy, k, h->curve, bkeys, bids, bxy, scratch, err, h->stream);
  if (e == hipSuccess)
    e = sfc::merge_runs(current_run(h), h->n, bkeys, bids, bxy, k, h->next_id, ep, h->spare,
                        h->key_of, h->stream, roff, runs > 1 ? runs : 0);
  if (e == hipSuccess && ids_out) e = sfc::fill_iota(ids_out, k, h->next_id, h->stream);
  uint64_t w = 0;
  if (e == hipSuccess) e = read_words(err, &w, 1, h->stream);
  h->alloc.put(batch);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return from_hip(e);
  }
  if ((uint32_t)w & sfc::kErrDomain) return SFC_ERR_DOMAIN;
  if ((uint32_t)w & (sfc::kErrLookback | sfc::kErrInternal)) return SFC_ERR_DEVICE;
  swap_runs(h);
  h->n += k;
  h->next_id += (uint32_t)k;
  h->epoch = ep + (runs > 1 ? runs - 1 : 0);
  h->max_ins = h->epoch;
  if (h->occ) SFC_TRY(sfc::build_occupancy(h->keys, h->n, h->occ, h->stream));
  if (h->stree_ready) {
    st = stree_refresh(h);
    if (st != SFC_OK) return st;
  }
  if (!h->hold) h->oldest = h->epoch;
  ++h->generation;
  ++h->merges;
  const uint64_t compactions = h->compactions;
  st = maybe_compact(h);   // a compaction refits the learned leaves itself
  if (st == SFC_OK && h->compactions == compactions) st = refit_leaves(h);
  return st;
}

}  // namespace

sfc_status sfc_insert(sfc_index* h, const double* xy, uint64_t k, uint32_t* ids_out) {
  if (!h || (k > 0 && !xy)) return SFC_ERR_INVALID;
  if (h->n_sets || dim_of(h) == 3) return SFC_ERR_UNSUPPORTED;
  if (k == 0) return SFC_OK;
  const uint64_t off[2] = {0, k};
  return insert_impl(h, xy, k, off, 1, ids_out);
}

sfc_status sfc_insert_runs(sfc_index* h, const double* xy, const uint64_t* run_off, uint32_t runs,
                           uint32_t* ids_out) {
  if (!h || !run_off || runs == 0 || runs > kMaxInsertRuns || run_off[0] != 0)
    return SFC_ERR_INVALID;
  for (uint32_t r = 0; r < runs; ++r)
    if (run_off[r + 1] < run_off[r]) return SFC_ERR_INVALID;
  const uint64_t k = run_off[runs];
  if (k > 0 && !xy) return SFC_ERR_INVALID;
  if (h->n_sets || dim_of(h) == 3) return SFC_ERR_UNSUPPORTED;
  return insert_impl(h, xy, k, run_off, runs, ids_out);
}

sfc_status sfc_erase(sfc_index* h, const uint32_t* ids, uint64_t k, uint64_t* erased_out) {
  if (!h || (k > 0 && !ids)) return SFC_ERR_INVALID;
  if (h->n_sets || dim_of(h) == 3) return SFC_ERR_UNSUPPORTED;
  if (k == 0) {
    if (erased_out) *erased_out = 0;
    return SFC_OK;
  }
  if (h->epoch >= 0xFFFFFFFEu) return SFC_ERR_UNSUPPORTED;
  SFC_TRY(wait_readers(h));
  sfc_status st = ensure_dynamic(h);
  if (st != SFC_OK) return st;
  const uint32_t ep = h->epoch + 1;
  uint64_t cnt = 0;
  hipError_t e = sfc::fill_u64(h->upd_word, 0, 1, h->stream);
  if (e == hipSuccess)
    e = sfc::erase_entries(ids, k, h->next_id, h->key_of, current_run(h), h->n, ep,
                           (unsigned long long*)h->upd_word, h->stream);
  if (e == hipSuccess) e = read_words(h->upd_word, &cnt, 1, h->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return from_hip(e);
  }
  h->epoch = ep;
  if (cnt) {
    h->tombs.emplace_back(ep, cnt);
    h->dead += cnt;
  }
  if (!h->hold) h->oldest = ep;
  ++h->generation;
  if (erased_out) *erased_out = cnt;
  return maybe_compact(h);
}

sfc_status sfc_hold_epochs(sfc_index* h, int hold) {
  if (!h || (hold != 0 && hold != 1)) return SFC_ERR_INVALID;
  h->hold = hold;
  if (!hold && h->oldest != h->epoch) {
    h->oldest = h->epoch;
    return maybe_compact(h);
  }
  return SFC_OK;
}

sfc_status sfc_retire(sfc_index* h, uint32_t epoch) {
  if (!h || epoch > h->epoch) return SFC_ERR_INVALID;
  if (epoch <= h->oldest) return SFC_OK;
  h->oldest = epoch;
  return maybe_compact(h);
}

sfc_status sfc_compact(sfc_index* h) {
  if (!h) return SFC_ERR_INVALID;
  return compact_now(h);
}

sfc_status sfc_update_info_get(const sfc_index* h, sfc_update_info* out) {
  if (!h || !out) return SFC_ERR_INVALID;
  out->epoch = h->epoch;
  out->oldest = h->oldest;
  out->next_id = h->next_id;
  out->hold = (uint32_t)h->hold;
  out->stored = h->n;
  out->dead = h->dead;
  out->live = h->n - h->dead;
  out->droppable = droppable(h);
  out->merges = h->merges;
  out->compactions = h->compactions;
  return SFC_OK;
}

}  // extern "C"
