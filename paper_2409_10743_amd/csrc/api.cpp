// C ABI and host-side pipeline of the DBSCAN library (FDBSCAN path).
//
// One call enqueues the whole path on the caller's stream and waits once at
// the end for a 4-byte status word:
//   prep -> scene bounds -> Morton codes (+ digit histograms) -> radix sort
//   -> sorted leaves -> Apetrei build (Karras order, ropes) -> [counting, minPts > 2]
//   -> pair traversal + union-find -> labels
// All scratch comes from the context's arena (one device allocation, grown
// on demand, reused by later calls), so a warmed context allocates nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dbscan_mi355x.h"
#include "pipeline.hpp"

using namespace dbx;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(DBSCAN_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// One timing slot per kernel launch of a run (a slot a run skips reads 0).
enum Phase {
  PH_PREP, PH_BOUNDS, PH_MORTON, PH_SORT0, PH_GATHER = PH_SORT0 + SORT_PASSES, PH_CELLS,
  PH_BUILD_FRAME, PH_BUILD_LEVELS, PH_COUNT, PH_PAIRS, PH_FINAL_ROOTS,
  PH_FINAL_LABELS, NPHASES
};
// "morton" is the point codes (FDBSCAN) or the cell codes (DenseBox);
// "cells" (DenseBox only) covers run heads, scans, cell stats, primitives.
const char* const kPhaseNames[NPHASES] = {
    "prep",  "bounds",  "morton",      "sort0",        "sort1",  "sort2",
    "sort3", "sort4",   "sort5",       "sort6",        "sort7",  "gather",
    "cells", "build_frame", "build_levels", "count", "pairs", "final_roots",
    "final_labels"};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of every buffer of a job inside the arena.
struct Layout {
  size_t keys_a, keys_b, vals_a, vals_b, leaf, nodes, parent, minlab, flag, bestcore, deg,
      pending;
  // DenseBox only (0 otherwise)
  size_t cid, cell_start, cell_lo, cell_hi, cell_minorig, cell_dense, prim_count,
      prim_start, prims, pkey, scan1, scan2, scan_ctr, ncells, nprims;
  size_t set_e2, set_mp, set_th, grid;  // the one-set table of a plain DenseBox call
  uint32_t pending_entries;
  size_t zero;        // start of the region zeroed by k_prep
  size_t hist, tile_ctr, status, count, walkq, ncore, sort_status;
  size_t zero_words;  // 32-bit words from `zero`
  size_t bounds, drop, root;
  size_t total;
};

Layout make_layout(uint32_t n, bool need_bestcore, bool densebox = false) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(std::max<size_t>(bytes, 4));
    return at;
  };
  L.keys_a = take(size_t(n) * 8);
  L.keys_b = take(size_t(n) * 8);  // after the sort: the build's exchange slots
  L.vals_a = take(size_t(n) * 4);
  L.vals_b = take(size_t(n) * 4);
  L.leaf = take((size_t(n) + 1) * 16);  // + one padding record read by the walks
  L.nodes = take(size_t(n > 1 ? n - 1 : 1) * sizeof(Node));
  L.parent = take(size_t(n) * 4);
  L.minlab = need_bestcore ? take(size_t(n) * 4) : 0;  // border points' label minima
  L.flag = take(size_t(n));
  L.bestcore = need_bestcore ? take(size_t(n) * 8) : 0;
  L.deg = need_bestcore ? take(size_t(n) * 4) : 0;  // pair counts (DBSCAN_FLAG_PAIR_COUNT)
  L.pending_entries = uint32_t(build_pending_entries(n));
  L.pending = take(size_t(L.pending_entries) * 16);
  if (densebox) {
    L.cid = take(size_t(n) * 4);
    L.cell_start = take((size_t(n) + 1) * 4);
    L.cell_lo = take(size_t(n) * 16);
    L.cell_hi = take(size_t(n) * 16);
    L.cell_minorig = take(size_t(n) * 8);
    L.cell_dense = take(size_t(n));
    L.prim_count = take(size_t(n) * 4);
    L.prim_start = take(size_t(n) * 4);
    L.prims = take(size_t(n) * sizeof(Node));
    L.pkey = take(size_t(n) * 8);
    L.set_e2 = take(4);
    L.set_mp = take(4);
    L.set_th = take(4);
    L.grid = take(sizeof(MortonGrid));
  }
  L.bounds = take(8 * 4);
  L.drop = take(4);
  L.root = take(4);
  // zeroed region: hist | tile counters | status word | pair count | walk
  // queues | (DenseBox scans) | the first sort pass's look-back words
  L.zero = o;
  L.hist = take(SORT_PASSES * RADIX * 4);
  L.tile_ctr = take(SORT_PASSES * 4);
  L.status = take(4);
  L.count = take(4 * 8);  // pairs, internal-node visits, descents, leaf tests
  L.walkq = take(4 * 8 * 4);  // chunk counters of up to four persistent walks
  L.ncore = take(4);          // core points (counting by pair traversal)
  if (densebox) {
    L.scan_ctr = take(8);
    L.ncells = take(8);  // ncells and nprims side by side: read back together
    L.nprims = L.ncells + 4;
    L.scan1 = take(scan_status_words(n) * 4);
    L.scan2 = take(scan_status_words(n) * 4);
  }
  L.sort_status = take(sort_status_words(n) * 4);
  // zeroed up to the first sort pass's look-back words (each pass clears
  // the next pass's)
  L.zero_words = (L.sort_status - L.zero) / 4 + sort_first_status_words(n);
  L.total = o;
  return L;
}

}  // namespace

struct dbscan_ctx {
  int device = 0;
  uint64_t budget = 0;
  hipStream_t stream = nullptr;  // the context's own stream: where a NULL stream argument goes
  char* arena = nullptr;
  size_t cap = 0;
  uint32_t* host_status = nullptr;  // pinned
  char* stage = nullptr;            // pinned staging for per-set parameters
  size_t stage_cap = 0;
  hipEvent_t ev[NPHASES + 1] = {};
  float times[NPHASES] = {};
  int ntimes = 0;
  bool recorded[NPHASES + 1] = {};
  int sort_passes = SORT_PASSES;  // sort passes the last clustering call ran
  int sort_items = 0;             // keys per sort thread of the current call (0: default)
  // captured call sequences (DBSCAN_FLAG_GRAPH), replayed while the key
  // matches; the oldest is replaced
  struct Graph {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
  };
  Graph graphs[4];
  uint64_t graph_clock = 0;
  // DBSCAN_ALGO_AUTO: the density probe's device buffer and the last pick
  char* probe = nullptr;
  size_t probe_cap = 0;
  std::vector<uint64_t> auto_key;
  int32_t auto_algo = DBSCAN_ALGO_FDBSCAN;
  bool auto_pair_count = false;
  // dbscan_mst: the Borůvka rounds' device buffer
  char* mst = nullptr;
  size_t mst_cap = 0;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// The stream a call runs on: the caller's, or the context's own for NULL.
hipStream_t stream_of(const dbscan_ctx* c, void* stream) {
  return stream ? reinterpret_cast<hipStream_t>(stream) : c->stream;
}

int ensure_arena(dbscan_ctx* c, size_t bytes) {
  if (c->budget && bytes > c->budget)
    return fail(DBSCAN_ETOOBIG, "job needs " + std::to_string(bytes) +
                                    " bytes of scratch, budget is " + std::to_string(c->budget));
  if (bytes <= c->cap) return DBSCAN_OK;
  if (c->arena) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(c->arena));
    c->arena = nullptr;
    c->cap = 0;
  }
  size_t want = bytes + bytes / 8;  // headroom so slightly larger jobs reuse it
  if (c->budget && want > c->budget) want = bytes;
  if (hipMalloc(&c->arena, want) != hipSuccess) {
    (void)hipGetLastError();
    c->arena = nullptr;
    return fail(DBSCAN_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  c->cap = want;
  return DBSCAN_OK;
}

int check_args(const void* pts, int64_t n, float eps, int32_t min_pts, const void* out) {
  if (n < 0) return fail(DBSCAN_EINVAL, "n < 0");
  if (n > int64_t(SORT_MAX_N)) return fail(DBSCAN_EINVAL, "n must be below 2^30");
  if (n > 0 && (pts == nullptr || out == nullptr)) return fail(DBSCAN_EINVAL, "null pointer");
  if (!(eps >= 0.0f) || std::isinf(eps)) return fail(DBSCAN_EINVAL, "eps must be finite and >= 0");
  volatile float e2 = eps * eps;
  if (std::isinf(e2)) return fail(DBSCAN_EINVAL, "eps*eps overflows binary32");
  if (min_pts < 1) return fail(DBSCAN_EINVAL, "min_pts must be >= 1");
  return DBSCAN_OK;
}

int check_opts(const dbscan_options& o, int32_t min_pts) {
  if (o.algorithm < DBSCAN_ALGO_AUTO || o.algorithm > DBSCAN_ALGO_DENSEBOX)
    return fail(DBSCAN_EINVAL, "unknown algorithm");
  if (o.dense_threshold != 0 && o.dense_threshold < min_pts)
    return fail(DBSCAN_EINVAL, "dense_threshold below min_pts");
  if (o.block_size != 0 && (o.block_size < 64 || o.block_size > 1024 || o.block_size % 64))
    return fail(DBSCAN_EINVAL, "block_size must be a multiple of 64 in [64, 1024]");
  if (o.sort_tile != 0 && o.sort_tile != 2048 && o.sort_tile != 3072 && o.sort_tile != 4096)
    return fail(DBSCAN_EINVAL, "sort_tile must be 0, 2048, 3072 or 4096");
  return DBSCAN_OK;
}

template <class T>
T* at(dbscan_ctx* c, size_t off) {
  return reinterpret_cast<T*>(c->arena + off);
}

// Everything up to and including the ropes: the BVH over the sorted points.
struct Index {
  Layout L;
  uint64_t* keys;
  uint32_t* bounds;
  uint32_t* drop;  // device word: the low code bits the keys cleared
  uint32_t* perm;
  float4* leaf;
  Node* nodes;
  int32_t* root;
  uint32_t* status;
};

// ev[0] is recorded before the first kernel, ev[k + 1] right after phase
// k's kernels; a phase's time runs from the previous recorded event, and a
// phase that records nothing reads 0.
void start_timing(dbscan_ctx* c, bool timing, hipStream_t s) {
  for (auto& r : c->recorded) r = false;
  if (!timing) return;
  (void)hipEventRecord(c->ev[0], s);
  c->recorded[0] = true;
}
void mark(dbscan_ctx* c, bool timing, int phase, hipStream_t s) {
  if (!timing) return;
  (void)hipEventRecord(c->ev[phase + 1], s);
  c->recorded[phase + 1] = true;
}
struct SortMarks {
  dbscan_ctx* c;
  hipStream_t s;
};
void sort_mark(void* arg, int pass) {
  auto* m = static_cast<SortMarks*>(arg);
  mark(m->c, true, PH_SORT0 + pass, m->s);
}
void build_mark(void* arg, int level) {  // level 1 = the frame kernel
  auto* m = static_cast<SortMarks*>(arg);
  if (level == 1) mark(m->c, true, PH_BUILD_FRAME, m->s);
}

// labels (or null): set to -1 here, by the build's first level; so is deg
// to 0 (or null).
int build_index(dbscan_ctx* c, const float* pts, uint32_t n, bool need_bestcore, bool timing,
                hipStream_t s, Index* out, float code_eps, int32_t* labels, uint32_t* deg) {
  Layout L = make_layout(n, need_bestcore);
  int st = ensure_arena(c, L.total);
  if (st != DBSCAN_OK) return st;
  out->L = L;
  uint64_t* ka = at<uint64_t>(c, L.keys_a);
  uint64_t* kb = at<uint64_t>(c, L.keys_b);
  uint32_t* va = at<uint32_t>(c, L.vals_a);
  uint32_t* vb = at<uint32_t>(c, L.vals_b);
  uint32_t* bounds = at<uint32_t>(c, L.bounds);
  uint32_t* status = at<uint32_t>(c, L.status);
  SortScratch sc{at<uint32_t>(c, L.hist), at<uint32_t>(c, L.tile_ctr),
                 at<uint32_t>(c, L.sort_status), status};

  start_timing(c, timing, s);
  launch_prep(at<uint32_t>(c, L.zero), L.zero_words, bounds, at<int4>(c, L.pending),
              L.pending_entries, s);
  mark(c, timing, PH_PREP, s);
  launch_bounds(pts, n, bounds, status, s);
  mark(c, timing, PH_BOUNDS, s);
  // codes as fine as eps needs (decided on the device: no host round trip)
  uint32_t* drop = at<uint32_t>(c, L.drop);
  launch_morton(pts, n, bounds, code_eps, ka, kb, drop, sc.hist, s);
  mark(c, timing, PH_MORTON, s);
  SortMarks sm{c, s};
  launch_radix_sort_dropped(ka, kb, va, vb, n, drop, sc, s, timing ? sort_mark : nullptr, &sm,
                            c->sort_items);
  // the sort moved 32-bit halves of the codes and leaves none: the build's
  // first level recomputes the codes into ka (where the sort ended)
  uint64_t* keys = ka;
  uint32_t* perm = va;
  // the other key buffer is free now: the build's scratch
  int32_t* other = reinterpret_cast<int32_t*>(kb);
  // the build's first level gathers the leaves and sets up the union-find
  launch_build_coded(keys, bounds, drop, pts, perm, at<float4>(c, L.leaf),
                     at<int32_t>(c, L.parent), need_bestcore ? at<int32_t>(c, L.minlab) : nullptr,
                     at<uint8_t>(c, L.flag),
                     need_bestcore ? at<unsigned long long>(c, L.bestcore) : nullptr, labels, deg,
                     n, at<Node>(c, L.nodes), other, at<int32_t>(c, L.root),
                     at<int4>(c, L.pending), status, s, timing ? build_mark : nullptr, &sm);
  mark(c, timing, PH_BUILD_LEVELS, s);
  out->keys = keys;
  out->bounds = bounds;
  out->drop = drop;
  out->perm = perm;
  out->leaf = at<float4>(c, L.leaf);
  out->nodes = at<Node>(c, L.nodes);
  out->root = at<int32_t>(c, L.root);
  out->status = status;
  HIP_TRY(hipGetLastError());
  return DBSCAN_OK;
}

// Wait for the stream and turn the device status word into a status code.
// dev_drop (may be null): the code bits the sort dropped, read back for
// dbscan_sort_passes.
int finish(dbscan_ctx* c, const uint32_t* dev_status, bool timing, hipStream_t s,
           const uint32_t* dev_drop = nullptr) {
  HIP_TRY(hipMemcpyAsync(c->host_status, dev_status, 4, hipMemcpyDeviceToHost, s));
  if (dev_drop) HIP_TRY(hipMemcpyAsync(c->host_status + 1, dev_drop, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  c->sort_passes = dev_drop ? SORT_PASSES - int(c->host_status[1] / 8) : SORT_PASSES;
  HIP_TRY(hipGetLastError());
  if (timing) {
    int prev = 0;
    for (int k = 0; k < NPHASES; ++k) {
      float ms = 0.f;
      if (c->recorded[k + 1]) {
        if (hipEventElapsedTime(&ms, c->ev[prev], c->ev[k + 1]) != hipSuccess) ms = 0.f;
        prev = k + 1;
      }
      c->times[k] = ms;
    }
    c->ntimes = NPHASES;
    (void)hipGetLastError();
  }
  uint32_t w = *c->host_status;
  if (w & STATUS_NONFINITE) return fail(DBSCAN_ENONFINITE, "non-finite coordinate");
  if (w & STATUS_SORT_STALL) return fail(DBSCAN_EDEVICE, "a sort look-back wait hit its bound");
  if (w & STATUS_TREE) return fail(DBSCAN_EDEVICE, "malformed tree detected on the device");
  return DBSCAN_OK;
}

// Enqueue a call's kernels with `enqueue(s)`: directly, or (graph) as a HIP
// graph captured on first use and replayed while `key` (every host value
// the enqueued work depends on) matches.  Nothing inside `enqueue` may
// allocate, synchronise or record timing events when graph is set; clears
// go through kernels, not hipMemsetAsync.  A stream that cannot be
// captured (the null stream) runs the work directly.
template <class F>
int run_enqueued(dbscan_ctx* c, hipStream_t s, bool graph, const std::vector<uint64_t>& key,
                 F&& enqueue) {
  if (!graph || s == nullptr) return enqueue(s);
  dbscan_ctx::Graph* g = nullptr;
  for (auto& e : c->graphs)
    if (e.exec && e.key == key) g = &e;
  if (!g) {
    dbscan_ctx::Graph* slot = &c->graphs[0];
    for (auto& e : c->graphs)
      if (!e.exec || e.used < slot->used) slot = &e;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int st = enqueue(s);
    hipGraph_t captured = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &captured);
    if (st != DBSCAN_OK || e != hipSuccess) {
      if (captured) (void)hipGraphDestroy(captured);
      (void)hipGetLastError();
      return st != DBSCAN_OK ? st : fail(DBSCAN_EDEVICE, "graph capture failed");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, captured, nullptr, nullptr, 0);
    (void)hipGraphDestroy(captured);
    if (ie != hipSuccess) return fail(DBSCAN_EDEVICE, "graph instantiation failed");
    if (slot->exec) (void)hipGraphExecDestroy(slot->exec);
    slot->exec = exec;
    slot->key = key;
    g = slot;
  }
  g->used = ++c->graph_clock;
  HIP_TRY(hipGraphLaunch(g->exec, s));
  return DBSCAN_OK;
}

// Host values a plain call's enqueued work depends on.
uint64_t bits_of(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

int run_fdbscan(dbscan_ctx* c, const float* pts, uint32_t n, float eps, int32_t min_pts,
                int32_t* labels, hipStream_t s, const dbscan_options& o) {
  const bool graph = (o.flags & DBSCAN_FLAG_GRAPH) != 0;
  const bool timing = !graph && (o.flags & DBSCAN_FLAG_TIMING) != 0;
  const int block = o.block_size ? o.block_size : 256;
  const float e2 = eps * eps;
  const bool core_mode = min_pts > 2;
  const bool pair_count = core_mode && (o.flags & DBSCAN_FLAG_PAIR_COUNT) != 0;
  const Layout L = make_layout(n, core_mode);
  int st = ensure_arena(c, L.total);  // before any capture
  if (st != DBSCAN_OK) return st;
  const std::vector<uint64_t> key = {1,
                                     reinterpret_cast<uint64_t>(pts),
                                     reinterpret_cast<uint64_t>(labels),
                                     reinterpret_cast<uint64_t>(c->arena),
                                     n,
                                     bits_of(eps),
                                     uint64_t(uint32_t(min_pts)),
                                     uint64_t(block),
                                     uint64_t(pair_count),
                                     uint64_t(c->sort_items)};
  st = run_enqueued(c, s, graph, key, [&](hipStream_t gs) {
    Index ix;
    uint32_t* deg = pair_count ? at<uint32_t>(c, L.deg) : nullptr;
    int r = build_index(c, pts, n, core_mode, timing, gs, &ix, eps, labels, deg);
    if (r != DBSCAN_OK) return r;
    uint8_t* flag = at<uint8_t>(c, L.flag);
    int32_t* parent = at<int32_t>(c, L.parent);
    unsigned long long* bestcore =
        core_mode ? at<unsigned long long>(c, L.bestcore) : nullptr;
    uint32_t* ncore = pair_count ? at<uint32_t>(c, L.ncore) : nullptr;
    if (pair_count)
      launch_count_pairs(ix.nodes, ix.leaf, ix.keys, ix.bounds, ix.drop, n, e2, min_pts,
                         deg, flag, ncore, ix.status, block, gs);
    else if (core_mode)
      launch_count(ix.nodes, ix.leaf, ix.keys, ix.bounds, ix.drop, n, ix.root, e2,
                   min_pts, flag, ix.status, block, gs);
    mark(c, timing, PH_COUNT, gs);
    // with the counts of the pair traversal at hand, points whose counting
    // walk found no pair (most of a sparse field, and the last point of
    // every pair) start no main-phase walk, and with no core point at all
    // no walk starts
    if (core_mode)
      launch_pairs_core(ix.nodes, ix.leaf, ix.keys, ix.bounds, ix.drop, n, e2, flag,
                        ix.perm, parent, bestcore, pair_count ? deg : nullptr, ncore,
                        ix.status, block, gs);
    else
      launch_pairs_fof(ix.nodes, ix.leaf, ix.keys, ix.bounds, ix.drop, n, e2, ix.perm,
                       parent, flag, ix.status, block, gs);
    mark(c, timing, PH_PAIRS, gs);
    int32_t* minlab = core_mode ? at<int32_t>(c, L.minlab) : nullptr;
    launch_final(n, min_pts, flag, bestcore, ix.perm, parent, minlab, labels, gs);
    mark(c, timing, PH_FINAL_LABELS, gs);
    HIP_TRY(hipGetLastError());
    return int(DBSCAN_OK);
  });
  if (st != DBSCAN_OK) return st;
  return finish(c, at<uint32_t>(c, L.status), timing, s, at<uint32_t>(c, L.drop));
}

// DenseBox from the (unsorted) cell keys in keys_a, their digit counts in
// hist and the set table on: sort, cells, primitives, build, walks, labels.
// Nothing is read back: the call can be captured as a graph.
// d_off: the sets' offsets (batched calls; labels set-local), else null
// and min_pts is the plain call's.
// pair_count: core flags by pair traversal (DBSCAN_FLAG_PAIR_COUNT) instead
// of the counting walk from each set's root.
int densebox_from_keys(dbscan_ctx* c, const Layout& L, const float* pts, uint32_t n,
                       DbSets S, bool any_core, const int64_t* d_off, int32_t min_pts,
                       int32_t* labels, int block, bool timing, hipStream_t s,
                       bool pair_count) {
  uint64_t* ka = at<uint64_t>(c, L.keys_a);
  uint64_t* kb = at<uint64_t>(c, L.keys_b);
  uint32_t* va = at<uint32_t>(c, L.vals_a);
  uint32_t* vb = at<uint32_t>(c, L.vals_b);
  uint32_t* status = at<uint32_t>(c, L.status);
  SortScratch sc{at<uint32_t>(c, L.hist), at<uint32_t>(c, L.tile_ctr),
                 at<uint32_t>(c, L.sort_status), status};
  float4* spts = at<float4>(c, L.leaf);  // points in cell order
  int32_t* parent = at<int32_t>(c, L.parent);
  uint8_t* flag = at<uint8_t>(c, L.flag);
  int32_t* minlab = any_core ? at<int32_t>(c, L.minlab) : nullptr;
  unsigned long long* bestcore = any_core ? at<unsigned long long>(c, L.bestcore) : nullptr;

  SortMarks sm{c, s};
  const bool in_a = launch_radix_sort(ka, kb, va, vb, n, 0, true, sc, s,
                                      timing ? sort_mark : nullptr, &sm, c->sort_items);
  const uint64_t* keys = in_a ? ka : kb;
  const uint32_t* perm = in_a ? va : vb;
  int32_t* other = reinterpret_cast<int32_t*>(in_a ? kb : ka);
  // the other value buffer is free after the sort: the pair counts
  uint32_t* deg = any_core && pair_count ? (in_a ? vb : va) : nullptr;
  launch_gather(pts, perm, n, spts, parent, minlab, flag, bestcore, labels, s);
  mark(c, timing, PH_GATHER, s);

  uint32_t* scan_ctr = at<uint32_t>(c, L.scan_ctr);
  uint32_t* ncells = at<uint32_t>(c, L.ncells);
  uint32_t* nprims = at<uint32_t>(c, L.nprims);
  uint32_t* cell_start = at<uint32_t>(c, L.cell_start);
  uint32_t* cid = at<uint32_t>(c, L.cid);
  launch_cells(keys, n, cid, ncells, cell_start, at<uint32_t>(c, L.scan1), scan_ctr, status, s);
  unsigned long long* cell_minorig = at<unsigned long long>(c, L.cell_minorig);
  float4* cell_lo = at<float4>(c, L.cell_lo);
  float4* cell_hi = at<float4>(c, L.cell_hi);
  uint8_t* cell_dense = at<uint8_t>(c, L.cell_dense);
  uint32_t* prim_count = at<uint32_t>(c, L.prim_count);
  uint32_t* prim_start = at<uint32_t>(c, L.prim_start);
  launch_cell_stats(spts, perm, keys, n, ncells, cell_start, S, cell_lo, cell_hi, cell_minorig,
                    cell_dense, prim_count, s);
  launch_scan(prim_count, prim_start, n, nprims, at<uint32_t>(c, L.scan2), scan_ctr + 1, status,
              s);
  // the primitive count (at most n) stays on the device: the build and the
  // walks read it there, launched for n
  Node* prims = at<Node>(c, L.prims);
  uint64_t* pkey = at<uint64_t>(c, L.pkey);
  launch_make_prims(spts, keys, n, cid, cell_start, prim_start, cell_dense, cell_lo, cell_hi,
                    cell_minorig, prims, pkey, parent, flag, deg, s);
  mark(c, timing, PH_CELLS, s);

  Node* nodes = at<Node>(c, L.nodes);
  launch_build_boxes(pkey, S.shift, prims, n, nprims, nodes, other, const_cast<int32_t*>(S.root),
                     at<int4>(c, L.pending), status, s);
  mark(c, timing, PH_BUILD_LEVELS, s);
  const DbTables T{spts, cell_start, perm, cell_minorig, cell_lo, cell_hi, parent, flag,
                   bestcore};
  uint32_t* walkq = at<uint32_t>(c, L.walkq);
  if (any_core && deg)
    launch_count_pairs_db(nodes, prims, pkey, n, nprims, S, T, deg, walkq, status, block, s);
  else if (any_core)
    launch_count_db(nodes, prims, pkey, n, nprims, S, T, walkq, status, block, s);
  mark(c, timing, PH_COUNT, s);
  launch_pairs_db(nodes, prims, pkey, n, nprims, S, T, walkq + 8, status, block, s);
  mark(c, timing, PH_PAIRS, s);
  if (d_off) {
    launch_final_sets(n, keys, S.shift, S.minpts, d_off, flag, bestcore, perm, parent, minlab,
                      labels, s);
    mark(c, timing, PH_FINAL_LABELS, s);
  } else {
    launch_final(n, min_pts, flag, bestcore, perm, parent, minlab, labels, s);
    mark(c, timing, PH_FINAL_LABELS, s);
  }
  return DBSCAN_OK;
}

// side of a DenseBox cell: eps / sqrt(3), shrunk a little so rounding rarely
// makes a full cell's diagonal exceed eps (the dense test on the actual box
// decides); its inverse, infinite for eps = 0
float inv_cell_side(float eps) {
  const double h = double(eps) / std::sqrt(3.0) * (1.0 - 1e-4);
  return h > 0 ? float(1.0 / h) : INFINITY;
}

int run_densebox(dbscan_ctx* c, const float* pts, uint32_t n, float eps, int32_t min_pts,
                 int32_t* labels, hipStream_t s, const dbscan_options& o) {
  const bool graph = (o.flags & DBSCAN_FLAG_GRAPH) != 0;
  const bool timing = !graph && (o.flags & DBSCAN_FLAG_TIMING) != 0;
  const int block = o.block_size ? o.block_size : 256;
  const bool core_mode = min_pts > 2;
  const bool pair_count = core_mode && (o.flags & DBSCAN_FLAG_PAIR_COUNT) != 0;
  const int32_t thresh = o.dense_threshold ? o.dense_threshold : min_pts;

  Layout L = make_layout(n, core_mode, true);
  int st = ensure_arena(c, L.total);  // before any capture
  if (st != DBSCAN_OK) return st;
  uint32_t* bounds = at<uint32_t>(c, L.bounds);
  uint32_t* status = at<uint32_t>(c, L.status);
  MortonGrid* grid = at<MortonGrid>(c, L.grid);
  const DbSets S{at<float>(c, L.set_e2), at<int32_t>(c, L.set_mp), at<int32_t>(c, L.set_th),
                 grid, at<int32_t>(c, L.root), 64};
  const std::vector<uint64_t> key = {3,
                                     reinterpret_cast<uint64_t>(pts),
                                     reinterpret_cast<uint64_t>(labels),
                                     reinterpret_cast<uint64_t>(c->arena),
                                     n,
                                     bits_of(eps),
                                     uint64_t(uint32_t(min_pts)),
                                     uint64_t(uint32_t(thresh)),
                                     uint64_t(block),
                                     uint64_t(c->sort_items),
                                     uint64_t(pair_count)};
  st = run_enqueued(c, s, graph, key, [&](hipStream_t gs) {
    start_timing(c, timing, gs);
    launch_prep(at<uint32_t>(c, L.zero), L.zero_words, bounds, at<int4>(c, L.pending),
                L.pending_entries, gs);
    launch_one_set(eps * eps, min_pts, thresh, const_cast<float*>(S.e2),
                   const_cast<int32_t*>(S.minpts), const_cast<int32_t*>(S.thresh), gs);
    mark(c, timing, PH_PREP, gs);
    launch_bounds(pts, n, bounds, status, gs);
    mark(c, timing, PH_BOUNDS, gs);
    launch_cell_keys(pts, n, bounds, inv_cell_side(eps), at<uint64_t>(c, L.keys_a),
                     at<uint32_t>(c, L.hist), grid, gs);
    mark(c, timing, PH_MORTON, gs);
    int r = densebox_from_keys(c, L, pts, n, S, core_mode, nullptr, min_pts, labels, block,
                               timing, gs, pair_count);
    if (r != DBSCAN_OK) return r;
    HIP_TRY(hipGetLastError());
    return int(DBSCAN_OK);
  });
  if (st != DBSCAN_OK) return st;
  return finish(c, status, timing, s);
}

// Pinned host staging of at least `bytes` (per-set parameters on their way
// to the device).
int ensure_stage(dbscan_ctx* c, size_t bytes, hipStream_t s) {
  if (c->stage_cap >= bytes) return DBSCAN_OK;
  HIP_TRY(hipStreamSynchronize(s));  // the old staging buffer may still be read
  if (c->stage) (void)hipHostFree(c->stage);
  c->stage = nullptr;
  c->stage_cap = 0;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->stage), bytes) != hipSuccess)
    return fail(DBSCAN_ENOMEM, "hipHostMalloc of the per-set staging buffer failed");
  c->stage_cap = bytes;
  return DBSCAN_OK;
}

// Byte offsets of a batched call's per-set arrays, after the job's buffers:
// offsets, e2, minPts, dense threshold, inverse cell side, roots, grids.
struct SetLayout {
  size_t off, e2, mp, th, ih, root, grid, total;
};
SetLayout make_set_layout(const Layout& L, uint32_t num_sets) {
  SetLayout S{};
  S.off = align_up(L.total);
  S.e2 = S.off + align_up((size_t(num_sets) + 1) * 8);
  S.mp = S.e2 + align_up(size_t(num_sets) * 4);
  S.th = S.mp + align_up(size_t(num_sets) * 4);
  S.ih = S.th + align_up(size_t(num_sets) * 4);
  S.root = S.ih + align_up(size_t(num_sets) * 4);
  S.grid = S.root + align_up(size_t(num_sets) * 4);
  S.total = S.grid + align_up(size_t(num_sets) * sizeof(MortonGrid));
  return S;
}

// Many independent sets in one pass (keys tagged with the set id).
int run_batched(dbscan_ctx* c, const float* pts, const int64_t* h_off, uint32_t num_sets,
                const float* h_eps, const int32_t* h_minpts, int32_t* labels, hipStream_t s,
                const dbscan_options& o) {
  const bool db = o.algorithm == DBSCAN_ALGO_DENSEBOX;
  const bool graph = (o.flags & DBSCAN_FLAG_GRAPH) != 0;
  const bool timing = !graph && (o.flags & DBSCAN_FLAG_TIMING) != 0;
  const int block = o.block_size ? o.block_size : 256;
  const uint32_t n = uint32_t(h_off[num_sets]);
  int set_bits = 1;
  while ((1u << set_bits) < num_sets) ++set_bits;
  const int bits = std::min(MORTON_BITS, (63 - set_bits) / 3);
  const int set_shift = 3 * bits;
  bool any_core = false;
  for (uint32_t k = 0; k < num_sets; ++k) any_core |= h_minpts[k] > 2;
  // core flags by pair traversal: DenseBox only (batched FDBSCAN counts by walks)
  const bool pair_count = db && any_core && (o.flags & DBSCAN_FLAG_PAIR_COUNT) != 0;

  Layout L = make_layout(n, any_core, db);
  const SetLayout SL = make_set_layout(L, num_sets);
  const size_t off_b = SL.off, e2_b = SL.e2, mp_b = SL.mp, th_b = SL.th, ih_b = SL.ih,
               root_b = SL.root, grid_b = SL.grid;
  int st = ensure_arena(c, SL.total);
  if (st != DBSCAN_OK) return st;
  st = ensure_stage(c, (size_t(num_sets) + 1) * 8 + size_t(num_sets) * 16, s);
  if (st != DBSCAN_OK) return st;
  int64_t* s_off = reinterpret_cast<int64_t*>(c->stage);
  float* s_e2 = reinterpret_cast<float*>(s_off + num_sets + 1);
  int32_t* s_mp = reinterpret_cast<int32_t*>(s_e2 + num_sets);
  int32_t* s_th = s_mp + num_sets;
  float* s_ih = reinterpret_cast<float*>(s_th + num_sets);
  std::memcpy(s_off, h_off, (size_t(num_sets) + 1) * 8);
  for (uint32_t k = 0; k < num_sets; ++k) {
    s_e2[k] = h_eps[k] * h_eps[k];
    s_mp[k] = h_minpts[k];
    s_th[k] = o.dense_threshold ? o.dense_threshold : h_minpts[k];
    s_ih[k] = inv_cell_side(h_eps[k]);
  }
  int64_t* d_off = at<int64_t>(c, off_b);
  float* d_e2 = at<float>(c, e2_b);
  int32_t* d_mp = at<int32_t>(c, mp_b);
  int32_t* d_root = at<int32_t>(c, root_b);
  MortonGrid* d_grid = at<MortonGrid>(c, grid_b);
  uint32_t* status = at<uint32_t>(c, L.status);
  const std::vector<uint64_t> key = {db ? 4u : 2u,
                                     reinterpret_cast<uint64_t>(pts),
                                     reinterpret_cast<uint64_t>(labels),
                                     reinterpret_cast<uint64_t>(c->arena),
                                     reinterpret_cast<uint64_t>(c->stage),
                                     n,
                                     num_sets,
                                     uint64_t(any_core),
                                     uint64_t(block),
                                     uint64_t(c->sort_items),
                                     uint64_t(pair_count)};
  if (db) {
    int32_t* d_th = at<int32_t>(c, th_b);
    float* d_ih = at<float>(c, ih_b);
    st = run_enqueued(c, s, graph, key, [&](hipStream_t gs) {
      // per-set values come from the pinned staging buffer at each replay
      HIP_TRY(hipMemcpyAsync(d_off, s_off, (size_t(num_sets) + 1) * 8, hipMemcpyHostToDevice,
                             gs));
      HIP_TRY(hipMemcpyAsync(d_e2, s_e2, size_t(num_sets) * 4, hipMemcpyHostToDevice, gs));
      HIP_TRY(hipMemcpyAsync(d_mp, s_mp, size_t(num_sets) * 4, hipMemcpyHostToDevice, gs));
      HIP_TRY(hipMemcpyAsync(d_th, s_th, size_t(num_sets) * 4, hipMemcpyHostToDevice, gs));
      HIP_TRY(hipMemcpyAsync(d_ih, s_ih, size_t(num_sets) * 4, hipMemcpyHostToDevice, gs));
      start_timing(c, timing, gs);
      launch_prep(at<uint32_t>(c, L.zero), L.zero_words, at<uint32_t>(c, L.bounds),
                  at<int4>(c, L.pending), L.pending_entries, gs);
      mark(c, timing, PH_PREP, gs);
      launch_set_morton(pts, d_off, num_sets, bits, set_shift, d_ih, at<uint64_t>(c, L.keys_a),
                        at<uint32_t>(c, L.hist), d_root, d_grid, status, gs);
      mark(c, timing, PH_MORTON, gs);
      const DbSets S{d_e2, d_mp, d_th, d_grid, d_root, set_shift};
      int r = densebox_from_keys(c, L, pts, n, S, any_core, d_off, 0, labels, block, timing, gs,
                                 pair_count);
      if (r != DBSCAN_OK) return r;
      HIP_TRY(hipGetLastError());
      return int(DBSCAN_OK);
    });
    if (st != DBSCAN_OK) return st;
    return finish(c, status, timing, s);
  }
  st = run_enqueued(c, s, graph, key, [&](hipStream_t gs) {
    // the per-set parameters are read from the pinned staging buffer when
    // the copies run, so a replayed graph picks up this call's values
    HIP_TRY(hipMemcpyAsync(d_off, s_off, (size_t(num_sets) + 1) * 8, hipMemcpyHostToDevice, gs));
    HIP_TRY(hipMemcpyAsync(d_e2, s_e2, size_t(num_sets) * 4, hipMemcpyHostToDevice, gs));
    HIP_TRY(hipMemcpyAsync(d_mp, s_mp, size_t(num_sets) * 4, hipMemcpyHostToDevice, gs));

    uint64_t* ka = at<uint64_t>(c, L.keys_a);
    uint64_t* kb = at<uint64_t>(c, L.keys_b);
    uint32_t* va = at<uint32_t>(c, L.vals_a);
    uint32_t* vb = at<uint32_t>(c, L.vals_b);
    uint32_t* bounds = at<uint32_t>(c, L.bounds);
    SortScratch sc{at<uint32_t>(c, L.hist), at<uint32_t>(c, L.tile_ctr),
                   at<uint32_t>(c, L.sort_status), status};
    float4* leaf = at<float4>(c, L.leaf);
    int32_t* parent = at<int32_t>(c, L.parent);
    uint8_t* flag = at<uint8_t>(c, L.flag);
    int32_t* minlab = any_core ? at<int32_t>(c, L.minlab) : nullptr;
    unsigned long long* bestcore = any_core ? at<unsigned long long>(c, L.bestcore) : nullptr;

    start_timing(c, timing, gs);
    launch_prep(at<uint32_t>(c, L.zero), L.zero_words, bounds, at<int4>(c, L.pending),
              L.pending_entries, gs);
    mark(c, timing, PH_PREP, gs);
    mark(c, timing, PH_BOUNDS, gs);
    launch_set_morton(pts, d_off, num_sets, bits, set_shift, nullptr, ka, sc.hist, d_root, d_grid,
                      status, gs);
    mark(c, timing, PH_MORTON, gs);
    SortMarks sm{c, gs};
    const bool in_a = launch_radix_sort(ka, kb, va, vb, n, 0, true, sc, gs,
                                        timing ? sort_mark : nullptr, &sm, c->sort_items);
    const uint64_t* keys = in_a ? ka : kb;
    const uint32_t* perm = in_a ? va : vb;
    int32_t* other = reinterpret_cast<int32_t*>(in_a ? kb : ka);
    Node* nodes = at<Node>(c, L.nodes);
    launch_build(keys, set_shift, pts, perm, leaf, parent, minlab, flag, bestcore, labels,
                 nullptr, n, nodes, other, d_root, at<int4>(c, L.pending), status, gs,
                 timing ? build_mark : nullptr, &sm);
    mark(c, timing, PH_BUILD_LEVELS, gs);
    if (any_core)
      launch_count_sets(nodes, leaf, n, keys, set_shift, d_root, d_e2, d_mp, d_grid, flag,
                        at<uint32_t>(c, L.walkq), status, block, gs);
    mark(c, timing, PH_COUNT, gs);
    launch_pairs_sets(nodes, leaf, n, keys, set_shift, d_e2, d_mp, d_grid, perm, parent, flag,
                      bestcore, at<uint32_t>(c, L.walkq) + 8, status, block, gs);
    mark(c, timing, PH_PAIRS, gs);
    launch_final_sets(n, keys, set_shift, d_mp, d_off, flag, bestcore, perm, parent, minlab,
                      labels, gs);
    mark(c, timing, PH_FINAL_LABELS, gs);
    HIP_TRY(hipGetLastError());
    return int(DBSCAN_OK);
  });
  if (st != DBSCAN_OK) return st;
  return finish(c, status, timing, s);
}

std::mutex g_default_mu;
dbscan_ctx* g_default[64] = {};

int default_ctx(dbscan_ctx** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(DBSCAN_EDEVICE, "device id out of range");
  std::lock_guard<std::mutex> g(g_default_mu);
  if (!g_default[dev]) {
    int st = dbscan_ctx_create(dev, 0, &g_default[dev]);
    if (st != DBSCAN_OK) return st;
  }
  *out = g_default[dev];
  return DBSCAN_OK;
}

dbscan_options defaults() {
  dbscan_options o{};
  o.algorithm = DBSCAN_ALGO_AUTO;
  return o;
}

// ---- DBSCAN_ALGO_AUTO ------------------------------------------------------------
// DenseBox is chosen when points have, on average, at least this many
// eps-neighbours per unit of minPts (point-weighted over the sets).  On the
// 4,096 sub-halo sets (eps 0.05, minPts 5) the mean is about 35 and DenseBox
// takes half FDBSCAN's time; on the 2^24-point halo field (eps 0.2, minPts
// 2) it is 0.06 and FDBSCAN takes 0.6 of DenseBox's.
constexpr double AUTO_DENSE_FACTOR = 4.0;
// With FDBSCAN and minPts > 2, core points come from the pair traversal
// (DBSCAN_FLAG_PAIR_COUNT) when points have fewer eps-neighbours on average
// than minPts: the counting walk from the root then seldom stops early
// (the 2^24 field at minPts 5: 0.65 against 2.0 ms; the 2^27 field at
// minPts 10: 21 against 33 ms per call).
constexpr uint32_t PROBE_SAMPLES_ONE_SET = 4096;  // sample points of a plain call
constexpr uint32_t PROBE_SAMPLES_PER_SET = 256;   // and of each set of a batch

uint64_t mix(uint64_t h, uint64_t v) { return (h ^ v) * 0x100000001b3ull; }

// The algorithm AUTO stands for on this input: FDBSCAN or DenseBox, from the
// density probe (probe.hip); the pick is kept for calls with the same
// points, sizes, eps and minPts, so graph replays need no probe.
int resolve_auto(dbscan_ctx* c, const float* pts, const int64_t* h_off, uint32_t num_sets,
                 const float* h_eps, const int32_t* h_mp, hipStream_t s, int32_t* algo,
                 bool* pair_count) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (uint32_t k = 0; k < num_sets; ++k)
    h = mix(mix(mix(h, uint64_t(h_off[k + 1])), bits_of(h_eps[k])), uint64_t(uint32_t(h_mp[k])));
  const std::vector<uint64_t> key = {reinterpret_cast<uint64_t>(pts), num_sets, h};
  if (key == c->auto_key) {
    *algo = c->auto_algo;
    *pair_count = c->auto_pair_count;
    return DBSCAN_OK;
  }
  const size_t off_b = 0, e2_b = align_up((size_t(num_sets) + 1) * 8);
  const size_t out_b = e2_b + align_up(size_t(num_sets) * 4), total = out_b + 256;
  if (c->probe_cap < total) {
    if (c->probe) {
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipFree(c->probe));
    }
    c->probe = nullptr;
    c->probe_cap = 0;
    if (hipMalloc(&c->probe, total) != hipSuccess) {
      (void)hipGetLastError();
      return fail(DBSCAN_ENOMEM, "hipMalloc of the density probe's buffer failed");
    }
    c->probe_cap = total;
  }
  // the parameters go through the pinned staging buffer, laid out like the
  // device buffer: offsets, e2, the result
  int st = ensure_stage(c, total, s);
  if (st != DBSCAN_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));  // earlier work may still read the staging buffer
  int64_t* s_off = reinterpret_cast<int64_t*>(c->stage + off_b);
  float* s_e2 = reinterpret_cast<float*>(c->stage + e2_b);
  double* s_sum = reinterpret_cast<double*>(c->stage + out_b);
  double n = 0, mp = 0;
  for (uint32_t k = 0; k < num_sets; ++k) {
    s_e2[k] = h_eps[k] * h_eps[k];
    const double nk = double(h_off[k + 1] - h_off[k]);
    n += nk;
    mp += nk * double(h_mp[k]);
  }
  std::memcpy(s_off, h_off, (size_t(num_sets) + 1) * 8);
  *s_sum = 0.0;
  HIP_TRY(hipMemcpyAsync(c->probe, c->stage, total, hipMemcpyHostToDevice, s));
  launch_density_probe(pts, reinterpret_cast<const int64_t*>(c->probe + off_b),
                       reinterpret_cast<const float*>(c->probe + e2_b), num_sets,
                       num_sets == 1 ? PROBE_SAMPLES_ONE_SET : PROBE_SAMPLES_PER_SET,
                       reinterpret_cast<double*>(c->probe + out_b), s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(s_sum, c->probe + out_b, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double sum = *s_sum;
  const double mean = n > 0 ? sum / n : 0, mp_mean = n > 0 ? mp / n : 2;
  *algo = mean >= AUTO_DENSE_FACTOR * std::max(mp_mean, 2.0) ? DBSCAN_ALGO_DENSEBOX
                                                              : DBSCAN_ALGO_FDBSCAN;
  // DenseBox counts by pair traversal: what is dense is in dense cells,
  // which need no count, and the walk from each set's root dominates the
  // counting walk elsewhere (the 4,096 sub-halo sets: 33 against 25.6 ms)
  *pair_count = *algo == DBSCAN_ALGO_DENSEBOX || mean < mp_mean;
  c->auto_key = key;
  c->auto_algo = *algo;
  c->auto_pair_count = *pair_count;
  return DBSCAN_OK;
}

// ---- scratch of the entry point that allocates nothing -----------------------
// One fixed device array; the code object is loaded per GPU, so every GPU
// holds its own copy (at its own address) until the process ends.  Host
// code never uses the name `scratch` as an address: it is a host-side
// stand-in, and a kernel given it would fault.  Its device address comes
// from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoAllocBytes = size_t(DBSCAN_NOALLOC_SCRATCH_BYTES);
static_assert(kNoAllocBytes % 256 == 0, "scratch size");
__device__ __align__(256) char scratch[kNoAllocBytes];

struct NoAllocDevice {
  std::mutex mu;         // one call at a time on this device (the array is shared)
  char* ptr = nullptr;   // device address of `scratch` on this device
};
NoAllocDevice g_noalloc[64];

}  // namespace

// ---- autotuning -------------------------------------------------------------
namespace {
template <class Run>
int tune(dbscan_ctx* c, hipStream_t s, const std::vector<dbscan_options>& cands,
         dbscan_options* best, float* best_ms, Run run) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float bm = 0;
  int bi = -1, st = DBSCAN_OK;
  for (size_t k = 0; k < cands.size() && st == DBSCAN_OK; ++k) {
    st = run(cands[k]);  // warm: sizes the arena, loads the code
    float t = 1e30f;
    for (int r = 0; r < 2 && st == DBSCAN_OK; ++r) {
      (void)hipEventRecord(e0, s);
      st = run(cands[k]);
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      t = std::min(t, ms);
    }
    if (st == DBSCAN_OK && (bi < 0 || t < bm)) { bm = t; bi = int(k); }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DBSCAN_OK) return st;
  *best = cands[size_t(bi)];
  if (best_ms) *best_ms = bm;
  (void)c;
  return DBSCAN_OK;
}

// the second stage: the first stage's pick with each sort tile (the default
// first, so that a tie keeps it)
std::vector<dbscan_options> sort_tiles_of(const dbscan_options& best) {
  std::vector<dbscan_options> v;
  for (int t : {0, 3072, 2048}) {
    dbscan_options o = best;
    o.sort_tile = t;
    v.push_back(o);
  }
  return v;
}

std::vector<dbscan_options> candidates(int32_t algorithm, int32_t min_pts) {
  std::vector<dbscan_options> v;
  for (int bs : {64, 128, 256, 512}) {
    dbscan_options o{};
    o.algorithm = algorithm;
    o.block_size = bs;
    if (algorithm == DBSCAN_ALGO_DENSEBOX) {
      for (int f : {1, 2, 4}) {
        o.dense_threshold = min_pts * f;
        v.push_back(o);
      }
    } else {
      v.push_back(o);
      if (min_pts > 2) {  // core flags by pair traversal too
        o.flags = DBSCAN_FLAG_PAIR_COUNT;
        v.push_back(o);
      }
    }
  }
  return v;
}
}  // namespace

// ---- what the job server needs to know about a context ------------------------
namespace dbx {
// Device bytes a context holds (its arena).
uint64_t ctx_arena_bytes(const dbscan_ctx* c) { return c ? c->cap : 0; }
// Cap on the context's arena (0 = none): a grow takes 1/8 headroom only
// when that stays under it.
void ctx_set_budget(dbscan_ctx* c, uint64_t bytes) { c->budget = bytes; }
// Free the arena (and the graphs captured over it); the next call grows it
// again.
int ctx_release_arena(dbscan_ctx* c) {
  DeviceGuard g(c->device);
  if (c->stream) HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto& e : c->graphs) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    e = dbscan_ctx::Graph{};
  }
  if (c->arena) HIP_TRY(hipFree(c->arena));
  c->arena = nullptr;
  c->cap = 0;
  return DBSCAN_OK;
}
// Arena bytes of a batched FDBSCAN call over `sets` sets of `n` points in
// all (the per-set arrays included).
uint64_t batched_scratch_bytes(int64_t n, uint32_t sets, bool any_core) {
  if (n < 0 || n > int64_t(SORT_MAX_N)) return 0;
  return make_set_layout(make_layout(uint32_t(n), any_core, false), sets).total;
}
}  // namespace dbx

extern "C" {

int dbscan_ctx_create(int device, uint64_t hbm_budget_bytes, dbscan_ctx** out) {
  if (!out) return fail(DBSCAN_EINVAL, "null out pointer");
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(DBSCAN_EINVAL, "no such device");
  DeviceGuard g(device);
  dbscan_ctx* c = new dbscan_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host_status), 64) != hipSuccess) {
    delete c;
    return fail(DBSCAN_ENOMEM, "hipHostMalloc failed");
  }
  for (auto& e : c->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      dbscan_ctx_destroy(c);
      return fail(DBSCAN_EDEVICE, "hipEventCreate failed");
    }
  }
  // default flags: ordered with the null stream, so NULL-stream work the
  // caller enqueued before a call is finished when the call starts
  if (hipStreamCreate(&c->stream) != hipSuccess) {
    c->stream = nullptr;
    dbscan_ctx_destroy(c);
    return fail(DBSCAN_EDEVICE, "hipStreamCreate failed");
  }
  *out = c;
  return DBSCAN_OK;
}

int dbscan_ctx_destroy(dbscan_ctx* c) {
  if (!c) return DBSCAN_OK;
  DeviceGuard g(c->device);
  for (auto& e : c->graphs)
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (c->arena) (void)hipFree(c->arena);
  if (c->host_status) (void)hipHostFree(c->host_status);
  if (c->stage) (void)hipHostFree(c->stage);
  if (c->probe) (void)hipFree(c->probe);
  if (c->mst) (void)hipFree(c->mst);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return DBSCAN_OK;
}

uint64_t dbscan_scratch_bytes(int64_t n, int32_t min_pts, int32_t algorithm) {
  if (n < 0 || n > int64_t(SORT_MAX_N)) return 0;
  return make_layout(uint32_t(n), min_pts > 2, algorithm == DBSCAN_ALGO_DENSEBOX).total;
}

int dbscan_cluster_ex(dbscan_ctx* c, const float* points, int64_t n, float eps, int32_t min_pts,
                      int32_t* labels, void* stream, const dbscan_options* opts) {
  if (!c) return fail(DBSCAN_EINVAL, "null context");
  int st = check_args(points, n, eps, min_pts, labels);
  if (st != DBSCAN_OK) return st;
  dbscan_options o = opts ? *opts : defaults();
  st = check_opts(o, min_pts);
  if (st != DBSCAN_OK) return st;
  if (n == 0) return DBSCAN_OK;
  DeviceGuard g(c->device);
  c->sort_items = o.sort_tile / SORT_THREADS;
  if (!stream) o.flags &= ~DBSCAN_FLAG_GRAPH;  // graphs only on a stream the caller names
  if (o.algorithm == DBSCAN_ALGO_AUTO) {
    const int64_t off[2] = {0, n};
    bool pair_count = false;
    st = resolve_auto(c, points, off, 1, &eps, &min_pts, stream_of(c, stream), &o.algorithm,
                      &pair_count);
    if (st != DBSCAN_OK) return st;
    if (pair_count) o.flags |= DBSCAN_FLAG_PAIR_COUNT;
  }
  if (o.algorithm == DBSCAN_ALGO_DENSEBOX)
    return run_densebox(c, points, uint32_t(n), eps, min_pts, labels, stream_of(c, stream), o);
  return run_fdbscan(c, points, uint32_t(n), eps, min_pts, labels, stream_of(c, stream), o);
}

int dbscan_cluster_batched(dbscan_ctx* c, const float* points, const int64_t* offsets,
                           int32_t num_sets, const float* eps, const int32_t* min_pts,
                           int32_t* labels, void* stream, const dbscan_options* opts) {
  if (!c) return fail(DBSCAN_EINVAL, "null context");
  if (num_sets < 0 || num_sets > (1 << 20)) return fail(DBSCAN_EINVAL, "num_sets out of range");
  if (num_sets == 0) return DBSCAN_OK;
  if (!offsets || !eps || !min_pts) return fail(DBSCAN_EINVAL, "null pointer");
  if (offsets[0] != 0) return fail(DBSCAN_EINVAL, "offsets[0] must be 0");
  for (int32_t k = 0; k < num_sets; ++k)
    if (offsets[k + 1] < offsets[k]) return fail(DBSCAN_EINVAL, "offsets must not decrease");
  const int64_t n = offsets[num_sets];
  dbscan_options o = opts ? *opts : defaults();
  for (int32_t k = 0; k < num_sets; ++k) {
    int st = check_args(points, n, eps[k], min_pts[k], labels);
    if (st != DBSCAN_OK) return st;
    st = check_opts(o, min_pts[k]);
    if (st != DBSCAN_OK) return st;
  }
  if (n == 0) return DBSCAN_OK;
  DeviceGuard g(c->device);
  c->sort_items = o.sort_tile / SORT_THREADS;
  if (!stream) o.flags &= ~DBSCAN_FLAG_GRAPH;  // graphs only on a stream the caller names
  if (o.algorithm == DBSCAN_ALGO_AUTO) {
    bool pair_count = false;  // (used by DenseBox: batched FDBSCAN counts by walk)
    int st = resolve_auto(c, points, offsets, uint32_t(num_sets), eps, min_pts,
                          stream_of(c, stream), &o.algorithm, &pair_count);
    if (st != DBSCAN_OK) return st;
    if (pair_count) o.flags |= DBSCAN_FLAG_PAIR_COUNT;
  }
  return run_batched(c, points, offsets, uint32_t(num_sets), eps, min_pts, labels,
                     stream_of(c, stream), o);
}

int dbscan_cluster(const float* points, int64_t n, float eps, int32_t min_pts, int32_t* labels,
                   void* stream) {
  int st = check_args(points, n, eps, min_pts, labels);
  if (st != DBSCAN_OK || n == 0) return st;
  dbscan_ctx* c = nullptr;
  st = default_ctx(&c);
  if (st != DBSCAN_OK) return st;
  return dbscan_cluster_ex(c, points, n, eps, min_pts, labels, stream, nullptr);
}

int dbscan_cluster_host(const float* host_points, int64_t n, float eps, int32_t min_pts,
                        int32_t* host_labels) {
  int st = check_args(host_points, n, eps, min_pts, host_labels);
  if (st != DBSCAN_OK || n == 0) return st;
  float* dp = nullptr;
  int32_t* dl = nullptr;
  if (hipMalloc(&dp, size_t(n) * 12) != hipSuccess || hipMalloc(&dl, size_t(n) * 4) != hipSuccess) {
    (void)hipGetLastError();
    if (dp) (void)hipFree(dp);
    return fail(DBSCAN_ENOMEM, "hipMalloc of the host-call buffers failed");
  }
  st = DBSCAN_OK;
  if (hipMemcpy(dp, host_points, size_t(n) * 12, hipMemcpyHostToDevice) != hipSuccess)
    st = fail(DBSCAN_EDEVICE, "host-to-device copy failed");
  if (st == DBSCAN_OK) st = dbscan_cluster(dp, n, eps, min_pts, dl, nullptr);
  if (st == DBSCAN_OK &&
      hipMemcpy(host_labels, dl, size_t(n) * 4, hipMemcpyDeviceToHost) != hipSuccess)
    st = fail(DBSCAN_EDEVICE, "device-to-host copy failed");
  (void)hipFree(dp);
  (void)hipFree(dl);
  return st;
}

int dbscan_cluster_noalloc(const float* points, int64_t n, float eps, int32_t min_pts,
                           int32_t* labels, void* stream) {
  int st = check_args(points, n, eps, min_pts, labels);
  if (st != DBSCAN_OK) return st;
  if (n > int64_t(DBSCAN_NOALLOC_MAX_POINTS))
    return fail(DBSCAN_ETOOBIG, "n = " + std::to_string(n) +
                                    " exceeds the no-allocation entry point's maximum of " +
                                    std::to_string(DBSCAN_NOALLOC_MAX_POINTS) + " points");
  if (n == 0) return DBSCAN_OK;
  const Layout L = make_layout(uint32_t(n), min_pts > 2);
  if (L.total > kNoAllocBytes)  // the maximum is chosen so that this never happens
    return fail(DBSCAN_ETOOBIG, "job needs " + std::to_string(L.total) +
                                    " bytes of scratch, the fixed array holds " +
                                    std::to_string(kNoAllocBytes));
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(DBSCAN_EDEVICE, "device id out of range");
  NoAllocDevice& d = g_noalloc[dev];
  std::lock_guard<std::mutex> lock(d.mu);
  if (!d.ptr) {  // first call on this device, which is current
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return fail(DBSCAN_EDEVICE, std::string("hipGetSymbolAddress of the scratch array: ") +
                                      hipGetErrorString(e));
    }
    d.ptr = static_cast<char*>(p);
  }
  // A context on the stack over the fixed array: its budget is the array,
  // so the arena is never grown (nothing is freed or allocated), and the
  // status words come back to pageable memory on this stack.
  dbscan_ctx c;
  c.device = dev;
  c.budget = kNoAllocBytes;
  c.arena = d.ptr;
  c.cap = kNoAllocBytes;
  uint32_t host_words[16] = {};
  c.host_status = host_words;
  c.sort_items = 0;
  return run_fdbscan(&c, points, uint32_t(n), eps, min_pts, labels,
                     reinterpret_cast<hipStream_t>(stream), defaults());
}

int dbscan_phase_times(const dbscan_ctx* c, float* ms, int32_t max) {
  if (!c || !ms || max < 0) return 0;
  int k = std::min<int>(max, c->ntimes);
  for (int i = 0; i < k; ++i) ms[i] = c->times[i];
  return k;
}

int dbscan_sort_passes(const dbscan_ctx* c) { return c ? c->sort_passes : -1; }

const char* dbscan_phase_name(int32_t k) {
  return (k >= 0 && k < NPHASES) ? kPhaseNames[k] : nullptr;
}

int dbscan_morton_codes(dbscan_ctx* c, const float* points, int64_t n, uint64_t* codes,
                        void* stream) {
  if (!c) return fail(DBSCAN_EINVAL, "null context");
  int st = check_args(points, n, 0.0f, 1, codes);
  if (st != DBSCAN_OK || n == 0) return st;
  DeviceGuard g(c->device);
  hipStream_t s = stream_of(c, stream);
  Layout L = make_layout(uint32_t(n), false);
  st = ensure_arena(c, L.total);
  if (st != DBSCAN_OK) return st;
  uint32_t* bounds = at<uint32_t>(c, L.bounds);
  uint32_t* status = at<uint32_t>(c, L.status);
  launch_prep(at<uint32_t>(c, L.zero), L.zero_words, bounds, at<int4>(c, L.pending),
              L.pending_entries, s);
  launch_bounds(points, uint32_t(n), bounds, status, s);
  launch_morton(points, uint32_t(n), bounds, 0.0f, codes, codes, nullptr, at<uint32_t>(c, L.hist),
                s);
  HIP_TRY(hipGetLastError());
  return finish(c, status, false, s);
}

int dbscan_sort_pairs(dbscan_ctx* c, uint64_t* keys, uint32_t* vals, int64_t n, void* stream) {
  if (!c) return fail(DBSCAN_EINVAL, "null context");
  if (n < 0 || n > int64_t(SORT_MAX_N)) return fail(DBSCAN_EINVAL, "n out of range");
  if (n > 0 && (!keys || !vals)) return fail(DBSCAN_EINVAL, "null pointer");
  if (n == 0) return DBSCAN_OK;
  DeviceGuard g(c->device);
  hipStream_t s = stream_of(c, stream);
  Layout L = make_layout(uint32_t(n), false);
  int st = ensure_arena(c, L.total);
  if (st != DBSCAN_OK) return st;
  uint32_t* status = at<uint32_t>(c, L.status);
  SortScratch sc{at<uint32_t>(c, L.hist), at<uint32_t>(c, L.tile_ctr),
                 at<uint32_t>(c, L.sort_status), status};
  launch_prep(at<uint32_t>(c, L.zero), L.zero_words, at<uint32_t>(c, L.bounds),
              at<int4>(c, L.pending), L.pending_entries, s);
  launch_digit_histogram(keys, uint32_t(n), sc.hist, s);
  bool in_a = launch_radix_sort(keys, at<uint64_t>(c, L.keys_b), vals, at<uint32_t>(c, L.vals_b),
                                uint32_t(n), 0, false, sc, s);
  if (!in_a) {
    HIP_TRY(hipMemcpyAsync(keys, at<uint64_t>(c, L.keys_b), size_t(n) * 8,
                           hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(vals, at<uint32_t>(c, L.vals_b), size_t(n) * 4,
                           hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipGetLastError());
  return finish(c, status, false, s);
}

int dbscan_build_tree(dbscan_ctx* c, const float* points, int64_t n, uint32_t* perm, float* leaf,
                      float* nodes, int32_t* root, void* stream) {
  if (!c) return fail(DBSCAN_EINVAL, "null context");
  int st = check_args(points, n, 0.0f, 1, perm);
  if (st != DBSCAN_OK) return st;
  if (n > 0 && (!leaf || !root || (n > 1 && !nodes))) return fail(DBSCAN_EINVAL, "null pointer");
  if (n == 0) return DBSCAN_OK;
  DeviceGuard g(c->device);
  hipStream_t s = stream_of(c, stream);
  Index ix;
  c->sort_items = 0;  // the default sort tile
  st = build_index(c, points, uint32_t(n), false, false, s, &ix, 0.0f, nullptr, nullptr);
  if (st != DBSCAN_OK) return st;
  HIP_TRY(hipMemcpyAsync(perm, ix.perm, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(leaf, ix.leaf, size_t(n) * 16, hipMemcpyDeviceToDevice, s));
  if (n > 1)
    HIP_TRY(hipMemcpyAsync(nodes, ix.nodes, size_t(n - 1) * sizeof(Node),
                           hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(root, ix.root, 4, hipMemcpyDeviceToDevice, s));
  return finish(c, ix.status, false, s);
}

int dbscan_core_flags(dbscan_ctx* c, const float* points, int64_t n, float eps, int32_t min_pts,
                      uint8_t* core, void* stream) {
  if (!c) return fail(DBSCAN_EINVAL, "null context");
  int st = check_args(points, n, eps, min_pts, core);
  if (st != DBSCAN_OK || n == 0) return st;
  DeviceGuard g(c->device);
  hipStream_t s = stream_of(c, stream);
  Index ix;
  c->sort_items = 0;  // the default sort tile
  st = build_index(c, points, uint32_t(n), false, false, s, &ix, eps, nullptr, nullptr);
  if (st != DBSCAN_OK) return st;
  uint8_t* flag = at<uint8_t>(c, ix.L.flag);
  launch_count(ix.nodes, ix.leaf, ix.keys, ix.bounds, ix.drop, uint32_t(n), ix.root,
               eps * eps, min_pts, flag, ix.status, 256, s);
  launch_scatter_u8(flag, ix.perm, uint32_t(n), core, s);
  HIP_TRY(hipGetLastError());
  return finish(c, ix.status, false, s);
}

int dbscan_pair_count(dbscan_ctx* c, const float* points, int64_t n, float eps, int64_t* count,
                      void* stream) {
  int64_t st4[4];
  int st = dbscan_traversal_stats(c, points, n, eps, st4, stream);
  if (st == DBSCAN_OK && count) *count = st4[0];
  return st;
}

int dbscan_traversal_stats(dbscan_ctx* c, const float* points, int64_t n, float eps,
                           int64_t* out4, void* stream) {
  int64_t* count = out4;
  if (!c) return fail(DBSCAN_EINVAL, "null context");
  int st = check_args(points, n, eps, 1, count);
  if (st != DBSCAN_OK) return st;
  if (n == 0) { count[0] = count[1] = count[2] = count[3] = 0; return DBSCAN_OK; }
  DeviceGuard g(c->device);
  hipStream_t s = stream_of(c, stream);
  Index ix;
  c->sort_items = 0;  // the default sort tile
  st = build_index(c, points, uint32_t(n), false, false, s, &ix, eps, nullptr, nullptr);
  if (st != DBSCAN_OK) return st;
  unsigned long long* dcount = at<unsigned long long>(c, ix.L.count);
  launch_pairs_count(ix.nodes, ix.leaf, ix.keys, ix.bounds, ix.drop, uint32_t(n),
                     eps * eps, dcount, ix.status, 256, s);
  unsigned long long* h = reinterpret_cast<unsigned long long*>(c->host_status + 2);
  HIP_TRY(hipMemcpyAsync(h, dcount, 32, hipMemcpyDeviceToHost, s));
  st = finish(c, ix.status, false, s);
  if (st == DBSCAN_OK)
    for (int k = 0; k < 4; ++k) count[k] = int64_t(h[k]);
  return st;
}

// k nearest neighbours / core distances: the tree with full 63-bit codes
// (no eps to drop code bits for), then one walk per point.
static int knn_common(dbscan_ctx* c, const float* points, int64_t n, int32_t k,
                      int32_t* idx, float* d2, float* core, void* stream) {
  if (!c) return fail(DBSCAN_EINVAL, "null context");
  int st = check_args(points, n, 0.0f, 1, core ? static_cast<void*>(core) : idx);
  if (st != DBSCAN_OK) return st;
  if (k < 1 || k > KNN_MAX_K) return fail(DBSCAN_EINVAL, "k must be in [1, 32]");
  if (n > 0 && !core && !d2) return fail(DBSCAN_EINVAL, "null pointer");
  if (n == 0) return DBSCAN_OK;
  DeviceGuard g(c->device);
  hipStream_t s = stream_of(c, stream);
  Index ix;
  c->sort_items = 0;  // the default sort tile
  st = build_index(c, points, uint32_t(n), false, false, s, &ix, 0.0f, nullptr, nullptr);
  if (st != DBSCAN_OK) return st;
  launch_knn(ix.nodes, ix.leaf, ix.perm, uint32_t(n), ix.root, k, idx, d2, core, ix.status, s);
  HIP_TRY(hipGetLastError());
  return finish(c, ix.status, false, s);
}

int dbscan_knn(dbscan_ctx* c, const float* points, int64_t n, int32_t k, int32_t* indices,
               float* sq_dists, void* stream) {
  return knn_common(c, points, n, k, indices, sq_dists, nullptr, stream);
}

int dbscan_core_distances(dbscan_ctx* c, const float* points, int64_t n, int32_t min_pts,
                          float* sq_dists, void* stream) {
  return knn_common(c, points, n, min_pts, nullptr, nullptr, sq_dists, stream);
}

// Minimum spanning tree (mst.hip): the tree with full 63-bit codes, core
// distances by the kNN walk (min_pts > 1), then Borůvka rounds until n - 1
// edges are written (each round's edge count is read back: the host decides
// whether to run another), then the edges sorted by (w, lo, hi).
namespace {
struct MstLayout {
  size_t comp, flag, run, ends, rec, best_w, best_j, seed, lb, comp_best, comp_hi, comp_edge, core,
      lo, hi, w, ka, kb, va, vb, small, hist, tile_ctr, scan_status, sort_status, total;
};
MstLayout mst_layout(uint32_t n) {
  MstLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(std::max<size_t>(bytes, 4));
    return at;
  };
  L.comp = take(size_t(n) * 4);
  L.flag = take(size_t(n) * 4);
  L.run = take(size_t(n) * 4);
  L.ends = take(size_t(n) * 4);
  L.rec = take(size_t(n) * sizeof(MstRec));
  L.best_w = take(size_t(n) * 4);
  L.best_j = take(size_t(n) * 4);
  L.seed = take(size_t(n) * 4);
  L.lb = take(size_t(n) * 4);
  L.comp_best = take(size_t(n) * 8);
  L.comp_hi = take(size_t(n) * 4);
  L.comp_edge = take(size_t(n) * 8);
  L.core = take(size_t(n) * 4);
  L.lo = take(size_t(n) * 4);
  L.hi = take(size_t(n) * 4);
  L.w = take(size_t(n) * 4);
  L.ka = take(size_t(n) * 8);
  L.kb = take(size_t(n) * 8);
  L.va = take(size_t(n) * 4);
  L.vb = take(size_t(n) * 4);
  L.small = take(4 * 4);  // scan total, scan tile counter, edge count
  L.hist = take(SORT_PASSES * RADIX * 4);
  L.tile_ctr = take(SORT_PASSES * 4);
  L.scan_status = take(scan_status_words(n) * 4);
  L.sort_status = take(sort_status_words(n) * 4);
  L.total = o;
  return L;
}
}  // namespace

int dbscan_mst(dbscan_ctx* c, const float* points, int64_t n, int32_t min_pts, int32_t* edges,
               float* sq_weights, void* stream) {
  if (!c) return fail(DBSCAN_EINVAL, "null context");
  int st = check_args(points, n, 0.0f, 1, n > 1 ? static_cast<void*>(edges) : points);
  if (st != DBSCAN_OK) return st;
  if (min_pts < 1 || min_pts > KNN_MAX_K) return fail(DBSCAN_EINVAL, "min_pts must be in [1, 32]");
  if (n > 1 && !sq_weights) return fail(DBSCAN_EINVAL, "null pointer");
  if (n < 2) return DBSCAN_OK;
  DeviceGuard g(c->device);
  hipStream_t s = stream_of(c, stream);
  const uint32_t un = uint32_t(n), m = un - 1;
  const MstLayout L = mst_layout(un);
  if (c->mst_cap < L.total) {
    if (c->mst) {
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipFree(c->mst));
    }
    c->mst = nullptr;
    c->mst_cap = 0;
    if (hipMalloc(&c->mst, L.total) != hipSuccess) {
      (void)hipGetLastError();
      return fail(DBSCAN_ENOMEM, "hipMalloc of the spanning tree's buffers failed");
    }
    c->mst_cap = L.total;
  }
  char* B = c->mst;
  auto P = [&](size_t off) { return static_cast<void*>(B + off); };
  int32_t* comp = static_cast<int32_t*>(P(L.comp));
  uint32_t* flag = static_cast<uint32_t*>(P(L.flag));
  uint32_t* run = static_cast<uint32_t*>(P(L.run));
  uint32_t* ends = static_cast<uint32_t*>(P(L.ends));
  MstRec* rec = static_cast<MstRec*>(P(L.rec));
  float* best_w = static_cast<float*>(P(L.best_w));
  int32_t* best_j = static_cast<int32_t*>(P(L.best_j));
  int32_t* seed = static_cast<int32_t*>(P(L.seed));
  float* lb = static_cast<float*>(P(L.lb));
  auto* comp_best = static_cast<unsigned long long*>(P(L.comp_best));
  uint32_t* comp_hi = static_cast<uint32_t*>(P(L.comp_hi));
  int2* comp_edge = static_cast<int2*>(P(L.comp_edge));
  float* core = static_cast<float*>(P(L.core));
  uint32_t* lo = static_cast<uint32_t*>(P(L.lo));
  uint32_t* hi = static_cast<uint32_t*>(P(L.hi));
  float* w = static_cast<float*>(P(L.w));
  uint64_t* ka = static_cast<uint64_t*>(P(L.ka));
  uint64_t* kb = static_cast<uint64_t*>(P(L.kb));
  uint32_t* va = static_cast<uint32_t*>(P(L.va));
  uint32_t* vb = static_cast<uint32_t*>(P(L.vb));
  uint32_t* small = static_cast<uint32_t*>(P(L.small));  // total, scan counter, edge count
  uint32_t* count = small + 2;

  Index ix;
  c->sort_items = 0;  // the default sort tile
  st = build_index(c, points, un, false, false, s, &ix, 0.0f, nullptr, nullptr);
  if (st != DBSCAN_OK) return st;
  if (min_pts > 1)
    launch_knn(ix.nodes, ix.leaf, ix.perm, un, ix.root, min_pts, nullptr, nullptr, core,
               ix.status, s);
  int32_t* parent = at<int32_t>(c, ix.L.parent);  // every position its own root (the build)
  launch_mst_init(un, comp, comp_best, comp_hi, seed, lb, comp_edge, s);
  HIP_TRY(hipMemsetAsync(small, 0, 16, s));
  uint32_t done = 0;
  for (int round = 0; done < m; ++round) {
    if (round >= 64) return fail(DBSCAN_EDEVICE, "spanning tree: no convergence");
    HIP_TRY(hipMemsetAsync(small, 0, 8, s));  // the scan's total and tile counter
    HIP_TRY(hipMemsetAsync(P(L.scan_status), 0, scan_status_words(un) * 4, s));
    launch_mst_runs(un, comp, flag, run, ends, small, static_cast<uint32_t*>(P(L.scan_status)),
                    small + 1, ix.status, s);
    launch_mst_records(un, comp, run, ends, min_pts > 1 ? core : nullptr, ix.perm, rec, s);
    launch_mst_round(ix.nodes, ix.leaf, rec, run, ends, un, ix.root, ix.perm, parent, comp_best,
                     comp_hi,
                     comp_edge, best_w, best_j, seed, lb, count, lo, hi, w, ix.status, s);
    launch_mst_settle(un, parent, comp, comp_best, comp_hi, comp_edge, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(c->host_status, ix.status, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(c->host_status + 1, count, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c->host_status[0] != 0) return finish(c, ix.status, false, s);
    const uint32_t now = c->host_status[1];
    if (now <= done || now > m) return fail(DBSCAN_EDEVICE, "spanning tree: a round added no edge");
    done = now;
  }
  // (w, lo, hi) order: a stable sort by hi, then by (w, lo)
  SortScratch sc{static_cast<uint32_t*>(P(L.hist)), static_cast<uint32_t*>(P(L.tile_ctr)),
                 static_cast<uint32_t*>(P(L.sort_status)), ix.status};
  auto sort_prep = [&](const uint64_t* keys) -> int {
    HIP_TRY(hipMemsetAsync(sc.hist, 0, SORT_PASSES * RADIX * 4, s));
    HIP_TRY(hipMemsetAsync(sc.tile_ctr, 0, SORT_PASSES * 4, s));
    HIP_TRY(hipMemsetAsync(sc.status, 0, sort_first_status_words(m) * 4, s));
    launch_digit_histogram(keys, m, sc.hist, s);
    return DBSCAN_OK;
  };
  launch_mst_sort_keys_hi(m, hi, ka, s);
  st = sort_prep(ka);
  if (st != DBSCAN_OK) return st;
  const bool in_a1 = launch_radix_sort(ka, kb, va, vb, m, 4, true, sc, s);
  const uint32_t* order1 = in_a1 ? va : vb;
  uint32_t* vfree = in_a1 ? vb : va;
  // keys of the second sort in the free key buffer, its values beside them
  uint64_t* k2 = in_a1 ? kb : ka;
  uint64_t* k2b = in_a1 ? ka : kb;
  launch_mst_sort_keys_wlo(m, order1, lo, w, k2, vfree, s);
  st = sort_prep(k2);
  if (st != DBSCAN_OK) return st;
  uint32_t* v2b = const_cast<uint32_t*>(order1);  // order1 is consumed by now
  const bool in_a2 = launch_radix_sort(k2, k2b, vfree, v2b, m, 0, false, sc, s);
  launch_mst_out(m, in_a2 ? vfree : v2b, lo, hi, w, edges, sq_weights, s);
  HIP_TRY(hipGetLastError());
  return finish(c, ix.status, false, s);
}

namespace {
// the autotuner's last stage for a DenseBox pick with core points to find:
// the same options with counting by pair traversal instead of walks
std::vector<dbscan_options> pair_count_of(const dbscan_options& best, bool any_core) {
  std::vector<dbscan_options> v{best};
  if (best.algorithm == DBSCAN_ALGO_DENSEBOX && any_core) {
    dbscan_options o = best;
    o.flags ^= DBSCAN_FLAG_PAIR_COUNT;
    v.push_back(o);
  }
  return v;
}
}  // namespace

int dbscan_autotune(dbscan_ctx* c, const float* points, int64_t n, float eps, int32_t min_pts,
                    int32_t algorithm, int32_t* labels, dbscan_options* best, float* best_ms,
                    void* stream) {
  if (!c || !best) return fail(DBSCAN_EINVAL, "null pointer");
  int st = check_args(points, n, eps, min_pts, labels);
  if (st != DBSCAN_OK) return st;
  if (algorithm < DBSCAN_ALGO_AUTO || algorithm > DBSCAN_ALGO_DENSEBOX)
    return fail(DBSCAN_EINVAL, "unknown algorithm");
  const int32_t algo = algorithm == DBSCAN_ALGO_AUTO ? DBSCAN_ALGO_FDBSCAN : algorithm;
  if (n == 0) {
    *best = candidates(algo, min_pts)[0];
    if (best_ms) *best_ms = 0;
    return DBSCAN_OK;
  }
  hipStream_t s = stream_of(c, stream);
  auto run = [&](const dbscan_options& o) {
    return dbscan_cluster_ex(c, points, n, eps, min_pts, labels, stream, &o);
  };
  st = tune(c, s, candidates(algo, min_pts), best, best_ms, run);
  if (st != DBSCAN_OK) return st;
  st = tune(c, s, pair_count_of(*best, min_pts > 2), best, best_ms, run);
  if (st != DBSCAN_OK) return st;
  return tune(c, s, sort_tiles_of(*best), best, best_ms, run);
}

int dbscan_autotune_batched(dbscan_ctx* c, const float* points, const int64_t* offsets,
                            int32_t num_sets, const float* eps, const int32_t* min_pts,
                            int32_t* labels, dbscan_options* best, float* best_ms,
                            void* stream) {
  if (!c || !best) return fail(DBSCAN_EINVAL, "null pointer");
  if (num_sets < 0 || (num_sets > 0 && (!offsets || !min_pts)))
    return fail(DBSCAN_EINVAL, "null pointer");
  // DenseBox thresholds are absolute: multiples of the largest minPts
  int32_t mp_max = 1;
  for (int32_t k = 0; k < num_sets; ++k) mp_max = std::max(mp_max, min_pts[k]);
  std::vector<dbscan_options> cands = candidates(DBSCAN_ALGO_FDBSCAN, 1);
  for (const dbscan_options& d : candidates(DBSCAN_ALGO_DENSEBOX, mp_max)) {
    dbscan_options o = d;
    if (o.dense_threshold == mp_max) o.dense_threshold = 0;  // each set's own minPts
    cands.push_back(o);
  }
  hipStream_t s = stream_of(c, stream);
  auto run = [&](const dbscan_options& o) {
    return dbscan_cluster_batched(c, points, offsets, num_sets, eps, min_pts, labels, stream,
                                  &o);
  };
  int st = tune(c, s, cands, best, best_ms, run);
  if (st != DBSCAN_OK) return st;
  st = tune(c, s, pair_count_of(*best, mp_max > 2), best, best_ms, run);
  if (st != DBSCAN_OK) return st;
  return tune(c, s, sort_tiles_of(*best), best, best_ms, run);
}

const char* dbscan_strerror(int status) {
  switch (status) {
    case DBSCAN_OK: return "ok";
    case DBSCAN_EINVAL: return "invalid argument";
    case DBSCAN_ENONFINITE: return "non-finite coordinate";
    case DBSCAN_ENOMEM: return "out of device memory";
    case DBSCAN_EDEVICE: return "device error";
    case DBSCAN_ETOOBIG: return "job exceeds the memory budget";
    default: return "unknown status";
  }
}

const char* dbscan_last_error(void) { return g_last_error.c_str(); }

const char* dbscan_version(void) { return "dbscan-mi355x 0.1 (gfx950)"; }

}  // extern "C"
