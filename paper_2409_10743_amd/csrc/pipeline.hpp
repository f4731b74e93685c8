// Host-side launchers of the device kernels; internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace dbx {

// status word bits reported back to the host after a run
constexpr uint32_t STATUS_NONFINITE = 1u;
constexpr uint32_t STATUS_SORT_STALL = 2u;
constexpr uint32_t STATUS_TREE = 4u;   // malformed tree or traversal bound hit

// ---- radix sort (radix_sort.hip) ------------------------------------------
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 16;                        // default keys per thread
constexpr int SORT_ITEMS_MIN = 8;                     // smallest tile variant
constexpr int SORT_TILE_MIN = SORT_THREADS * SORT_ITEMS_MIN;
constexpr int RADIX = 256;
constexpr int SORT_PASSES = 8;                          // 8-bit digits of 64
constexpr uint32_t SORT_MAX_N = (1u << 30) - 1;         // 30-bit look-back counts

inline uint32_t sort_tiles(uint32_t n, int items) {
  const uint32_t tile = uint32_t(SORT_THREADS * items);
  return (n + tile - 1) / tile;
}
// words of look-back state for all passes of one sort of n keys (sized for
// the smallest tile, so any variant fits)
inline size_t sort_status_words(uint32_t n) {
  return size_t(SORT_PASSES) * sort_tiles(n, SORT_ITEMS_MIN) * RADIX;
}
// the words of pass 0 (any variant) at the start of that state: what must be
// zero when a sort starts
inline size_t sort_first_status_words(uint32_t n) {
  return size_t(sort_tiles(n, SORT_ITEMS_MIN)) * RADIX;
}

struct SortScratch {
  uint32_t* hist;      // [SORT_PASSES][RADIX] digit counts, zeroed
  uint32_t* tile_ctr;  // [SORT_PASSES] dynamic tile ids, zeroed
  uint32_t* status;    // [SORT_PASSES][tiles][RADIX] look-back words: the first
                       // pass's zeroed (sort_first_status_words), each pass
                       // clears the next pass's
  uint32_t* err;       // status word, STATUS_SORT_STALL set on a stalled wait
};

// The same sort with the first *drop / 8 passes skipped (the number is
// read on the device): the result always ends in the A buffers, and the
// first pass that runs takes the values to be 0..n-1.
void launch_radix_sort_dropped(uint64_t* ka, uint64_t* kb, uint32_t* va, uint32_t* vb,
                               uint32_t n, const uint32_t* drop, const SortScratch& sc,
                               hipStream_t s, void (*after_pass)(void*, int) = nullptr,
                               void* arg = nullptr, int items = 0);

// Digit histograms of keys already in memory (the morton kernel computes
// them itself while writing the keys).
void launch_digit_histogram(const uint64_t* keys, uint32_t n, uint32_t* hist,
                            hipStream_t s);
// LSD sort of (keys, vals) by the digits [first_pass, SORT_PASSES); passes
// alternate between the A and B buffers, starting from A.  If `iota_vals`,
// the input values are taken to be 0..n-1 and `va` is not read.  Returns
// true when the result ends in the A buffers.
// `after_pass(arg, p)`, if given, is called after pass p is enqueued.
// items: keys per thread of a tile (8, 12 or 16; 0 = SORT_ITEMS).
bool launch_radix_sort(uint64_t* ka, uint64_t* kb, uint32_t* va, uint32_t* vb,
                       uint32_t n, int first_pass, bool iota_vals,
                       const SortScratch& sc, hipStream_t s,
                       void (*after_pass)(void*, int) = nullptr, void* arg = nullptr,
                       int items = 0);

// ---- bounds, Morton codes, leaf scatter (morton.hip) -----------------------
// bounds[0..2] lo (ordered-int encoding), bounds[3..5] hi
// Zero the region, reset the bounds words, empty the build hand-over
// entries.
void launch_prep(uint32_t* zero_region, size_t zero_words, uint32_t* bounds, int4* pending,
                 uint32_t pending_entries, hipStream_t s);
void launch_bounds(const float* pts, uint32_t n, uint32_t* bounds,
                   uint32_t* status, hipStream_t s);
// Codes with their lowest droppable_code_bits(bounds, eps, n) bits cleared
// (eps <= 0: full 63-bit codes), written to keys_a if that drops an even
// number of whole sort passes, else to keys_b; the bit count goes to
// *drop_out (if not null) for launch_radix_sort_dropped and the walks.
void launch_morton(const float* pts, uint32_t n, const uint32_t* bounds, float eps,
                   uint64_t* keys_a, uint64_t* keys_b, uint32_t* drop_out, uint32_t* hist,
                   hipStream_t s);
// Sorted leaves, leaf[i] = point perm[i] (rope unset), plus the padding
// record leaf[n] (leaf holds n + 1 records); also initialises the
// per-point state and fills the build's hand-over entries with -1.
// leaf[i] = point perm[i], union-find state (parent[i] = i, flag 0;
// minlab INT_MAX and bestcore ~0 where given) and labels[i] = -1 (if given).
void launch_gather(const float* pts, const uint32_t* perm, uint32_t n,
                   float4* leaf, int32_t* parent, int32_t* minlab,
                   uint8_t* flag, unsigned long long* bestcore, int32_t* labels,
                   hipStream_t s);

// ---- LBVH (lbvh.hip) --------------------------------------------------------
constexpr int BUILD_LEAVES = 256;        // leaves per level-1 frame
constexpr int BUILD_FANOUT_LOG2 = 7;     // frames per next-level frame: 128
constexpr int BUILD_BLOCK = 256;         // = BUILD_LEAVES = 2 << BUILD_FANOUT_LOG2
static_assert(BUILD_BLOCK == BUILD_LEAVES && BUILD_BLOCK == (2 << BUILD_FANOUT_LOG2), "");
int build_levels(uint32_t n);
// int4 entries of hand-over state the build needs (all levels), -1 filled
size_t build_pending_entries(uint32_t n);
// Internal nodes in Karras' order (root = number 0), every leaf's and
// node's rope set.  other[k] (n - 1 words): exchange slots, set up by the
// build itself.  Keys may carry a set id in bits [set_shift, 64) (batched
// sets; 64 = a single set): ropes are then cut at set ends and set_root[s]
// receives the root of set s's subtree (for a single set, set_root[0] = the
// root).  `after_level(arg, lv)`, if given, is called after level lv is
// enqueued.  The level-1 frames gather their leaves: leaf j = input point
// perm[j] (with its rope; leaf[n] is a padding record), and they set up the
// union-find state of their points (parent[j] = j, flag[j] = 0; minlab[j] =
// INT_MAX, bestcore[j] = ~0 and deg[j] = 0 where given) and labels[j] = -1
// (if given).
// pending must have been emptied (launch_prep).
void launch_build(const uint64_t* keys, int set_shift, const float* pts, const uint32_t* perm,
                  float4* leaf, int32_t* parent, int32_t* minlab, uint8_t* flag,
                  unsigned long long* bestcore, int32_t* labels, uint32_t* deg, uint32_t n,
                  Node* nodes, int32_t* other,
                  int32_t* set_root, int4* pending, uint32_t* err, hipStream_t s,
                  void (*after_level)(void*, int) = nullptr, void* arg = nullptr);
// The clustering call's build: as launch_build without set bits, with each
// leaf's Morton code recomputed from its point (grid from `bounds`, the low
// *drop bits cleared, as the Morton kernel made them) and written to `keys`
// by the first level; the sort before it moved 32-bit halves of the codes.
void launch_build_coded(uint64_t* keys, const uint32_t* bounds, const uint32_t* drop,
                        const float* pts, const uint32_t* perm, float4* leaf, int32_t* parent,
                        int32_t* minlab, uint8_t* flag, unsigned long long* bestcore,
                        int32_t* labels, uint32_t* deg, uint32_t n, Node* nodes, int32_t* other,
                        int32_t* root, int4* pending, uint32_t* err, hipStream_t s,
                        void (*after_level)(void*, int) = nullptr, void* arg = nullptr);
// The same over box leaves (DenseBox primitives: Node records, payload in
// `left`, rope in `rope`); sets as in launch_build.  The primitive count is
// read from *n_dev (at most n_bound, which sizes the launches), so no host
// round trip is needed between the primitives and the build.
void launch_build_boxes(const uint64_t* keys, int set_shift, Node* prims, uint32_t n_bound,
                        const uint32_t* n_dev, Node* nodes, int32_t* other, int32_t* set_root,
                        int4* pending, uint32_t* err, hipStream_t s);

// ---- traversals (traverse.hip) ---------------------------------------------
// keys: the sorted Morton codes; bounds: the scene bounds words they were
// made with; drop: the number of low code bits the keys cleared (null: 0)
// (all three for the walks' early end).
void launch_count(const Node* nodes, const float4* leaf, const uint64_t* keys,
                  const uint32_t* bounds, const uint32_t* drop,
                  uint32_t n, const int32_t* root, float e2, int32_t min_pts, uint8_t* is_core,
                  uint32_t* err, int block, hipStream_t s);
// Core flags by pair traversal: each pair adds one to both points' counts
// in deg (zero beforehand; bit 31 set where the point's own walk found a
// pair), then is_core[i] = count + 1 >= min_pts.  No early exit: for
// fields where points have few neighbours.
// ncore (may be null; zeroed before): gets the number of core points.
void launch_count_pairs(const Node* nodes, const float4* leaf, const uint64_t* keys,
                        const uint32_t* bounds, const uint32_t* drop,
                        uint32_t n, float e2, int32_t min_pts, uint32_t* deg, uint8_t* is_core,
                        uint32_t* ncore, uint32_t* err, int block, hipStream_t s);
// minPts <= 2: every point with a neighbour is core; union every pair.
void launch_pairs_fof(const Node* nodes, const float4* leaf, const uint64_t* keys,
                      const uint32_t* bounds, const uint32_t* drop,
                      uint32_t n, float e2, const uint32_t* perm, int32_t* parent,
                      uint8_t* member, uint32_t* err, int block, hipStream_t s);
// minPts > 2: union core pairs, record each non-core point's smallest-index
// core neighbour.
// deg, ncore (may be null): neighbour counts and the number of core points
// from a counting pass by pair traversal; a point whose counting walk found
// no pair starts no walk (this one would find none either), and with no
// core point no walk starts.
void launch_pairs_core(const Node* nodes, const float4* leaf, const uint64_t* keys,
                       const uint32_t* bounds, const uint32_t* drop,
                       uint32_t n, float e2, const uint8_t* is_core, const uint32_t* perm,
                       int32_t* parent, unsigned long long* bestcore, const uint32_t* deg,
                       const uint32_t* ncore, uint32_t* err, int block, hipStream_t s);
// Pair traversal with F(i, j) = count: every pair exactly once.
void launch_pairs_count(const Node* nodes, const float4* leaf, const uint64_t* keys,
                        const uint32_t* bounds, const uint32_t* drop,
                        uint32_t n, float e2, unsigned long long* count, uint32_t* err,
                        int block, hipStream_t s);

// ---- k nearest neighbours (knn.hip) ----------------------------------------------
constexpr int32_t KNN_MAX_K = 32;
// k nearest neighbours (1 <= k <= KNN_MAX_K) of every point over the built
// tree, the point itself included, by (squared distance, input index): into
// out_idx / out_d2 (int32 / float [n][k], input order; -1 / +inf past n),
// or, with core_d2 (float[n], input order), only the k-th squared distance.
void launch_knn(const Node* nodes, const float4* leaf, const uint32_t* perm, uint32_t n,
                const int32_t* root, int32_t k, int32_t* out_idx, float* out_d2, float* core_d2,
                uint32_t* err, hipStream_t s);

// ---- minimum spanning trees (mst.hip) -------------------------------------------
// Per position (Morton-sorted leaf) record of a Borůvka round: the last
// position of the run of equal components starting here, the component (a
// union-find root position), the squared core distance and the input index.
struct alignas(16) MstRec {
  uint32_t run_end;
  int32_t comp;
  float core;
  uint32_t orig;
};
// every point its own component; no minima, no seeds
void launch_mst_init(uint32_t n, int32_t* comp, unsigned long long* comp_best, uint32_t* comp_hi,
                     int32_t* seed, float* lb, int2* comp_edge, hipStream_t s);
// runs of equal components: run[i] = number of runs ending before i, ends[r]
// = last position of run r (scan state zeroed; *total = the number of runs)
void launch_mst_runs(uint32_t n, const int32_t* comp, uint32_t* flag, uint32_t* run,
                     uint32_t* ends, uint32_t* total, uint32_t* scan_status, uint32_t* scan_ctr,
                     uint32_t* err, hipStream_t s);
// the round's records (core_in: squared core distances in input order, or
// null for zero)
void launch_mst_records(uint32_t n, const int32_t* comp, const uint32_t* run, const uint32_t* ends,
                        const float* core_in, const uint32_t* perm, MstRec* rec, hipStream_t s);
// one round: each component's least edge, written once (at out_*[*count++])
// and unioned into parent
void launch_mst_round(const Node* nodes, const float4* leaf, const MstRec* rec,
                      const uint32_t* run, const uint32_t* ends, uint32_t n,
                      const int32_t* root, const uint32_t* perm, int32_t* parent,
                      unsigned long long* comp_best, uint32_t* comp_hi, int2* comp_edge,
                      float* best_w, int32_t* best_j, int32_t* seed, float* lb, uint32_t* count,
                      uint32_t* out_lo, uint32_t* out_hi, float* out_w, uint32_t* err,
                      hipStream_t s);
// components = union-find roots; the round's minima cleared
void launch_mst_settle(uint32_t n, int32_t* parent, int32_t* comp, unsigned long long* comp_best,
                       uint32_t* comp_hi, int2* comp_edge, hipStream_t s);
// edge order (w, lo, hi): keys for a sort by hi (top word), then by (w, lo)
void launch_mst_sort_keys_hi(uint32_t m, const uint32_t* hi, uint64_t* key, hipStream_t s);
void launch_mst_sort_keys_wlo(uint32_t m, const uint32_t* order, const uint32_t* lo,
                              const float* w, uint64_t* key, uint32_t* val, hipStream_t s);
// edges[k] = (lo, hi), weights[k] = w of edge order[k]
void launch_mst_out(uint32_t m, const uint32_t* order, const uint32_t* lo, const uint32_t* hi,
                    const float* w, int32_t* edges, float* weights, hipStream_t s);

// ---- density probe (probe.hip) ---------------------------------------------------
// *out += sum over sets of n_k times an unbiased estimate of set k's mean
// eps-neighbour count (point itself left out), from min(n_k, s_max) evenly
// spread samples of the set (offsets, set_e2: device arrays); *out must be
// zeroed first.
void launch_density_probe(const float* pts, const int64_t* offsets, const float* set_e2,
                          uint32_t num_sets, uint32_t s_max, double* out, hipStream_t s);

// ---- labels (finalize.hip) --------------------------------------------------
// Labels of the sorted points into input order; labels must hold -1 for
// every point (the build or the gather writes it).  minlab (minPts > 2
// only) must hold INT_MAX per point.
void launch_final(uint32_t n, int32_t min_pts, const uint8_t* flag,
                  const unsigned long long* bestcore, const uint32_t* perm, int32_t* parent,
                  int32_t* minlab, int32_t* labels, hipStream_t s);
// dst[perm[i]] = src[i]: from sorted order back to input order
void launch_scatter_u8(const uint8_t* src, const uint32_t* perm, uint32_t n,
                       uint8_t* dst, hipStream_t s);

// ---- DenseBox (densebox.hip) -----------------------------------------------
// Per-set parameters of a DenseBox call, device arrays indexed by set id (a
// plain call is one set: shift 64, arrays of one).
struct DbSets {
  const float* e2;         // eps^2
  const int32_t* minpts;
  const int32_t* thresh;   // dense threshold T (>= minPts)
  const MortonGrid* grid;  // the cell grid (the walks' early end)
  const int32_t* root;     // subtree root of the set (written by the build)
  int shift;               // set id = key >> shift; 64: a single set
};
// The per-point and per-cell arrays the DenseBox walks read and write.
struct DbTables {
  const float4* pts;  // points in cell order
  const uint32_t* cell_start;
  const uint32_t* perm;
  const unsigned long long* cell_minorig;  // (input index << 32) | position, smallest
  const float4* cell_lo;
  const float4* cell_hi;
  int32_t* parent;
  uint8_t* flag;
  unsigned long long* bestcore;  // minPts > 2 only
};
// Cell keys (Morton code of the grid cell, side max(1/inv_h, extent/2^21))
// plus the digit histograms of the sort; *grid = the cell grid.
void launch_cell_keys(const float* pts, uint32_t n, const uint32_t* bounds, float inv_h,
                      uint64_t* keys, uint32_t* hist, MortonGrid* grid, hipStream_t s);
// words of look-back state of one exclusive scan of n values (zeroed)
size_t scan_status_words(uint32_t n);
void launch_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total,
                 uint32_t* status, uint32_t* tile_ctr, uint32_t* err, hipStream_t s);
// The cells of the sorted cell keys, in one scan: cid (cell of each sorted
// point), *ncells, cell_start[0..ncells] (cell_start[ncells] = n).
void launch_cells(const uint64_t* sorted_keys, uint32_t n, uint32_t* cid, uint32_t* ncells,
                  uint32_t* cell_start, uint32_t* scan_status, uint32_t* scan_ctr, uint32_t* err,
                  hipStream_t s);
// keys: the sorted cell keys (their set ids pick each cell's eps and T).
// Box and smallest index are computed, and needed, for cells with at least
// T points only.
void launch_cell_stats(const float4* pts, const uint32_t* perm, const uint64_t* keys, uint32_t n,
                       const uint32_t* ncells, const uint32_t* cell_start, const DbSets& sets,
                       float4* cell_lo, float4* cell_hi, unsigned long long* cell_minorig,
                       uint8_t* cell_dense, uint32_t* prim_count, hipStream_t s);
// a dense cell's points are joined directly to its representative, the
// point with the smallest input index (cell_minorig's low word)
void launch_make_prims(const float4* pts, const uint64_t* keys, uint32_t n, const uint32_t* cid,
                       const uint32_t* cell_start, const uint32_t* prim_start,
                       const uint8_t* cell_dense, const float4* cell_lo, const float4* cell_hi,
                       const unsigned long long* cell_minorig, Node* prims, uint64_t* pkey,
                       int32_t* parent, uint8_t* flag, uint32_t* deg, hipStream_t s);
// the one-set parameter table of a plain call
void launch_one_set(float e2, int32_t min_pts, int32_t thresh, float* e2o, int32_t* mpo,
                    int32_t* tho, hipStream_t s);
// block: a multiple of 64, at most 1024; the primitive count is *np_dev, at
// most np_bound (which sizes the launch)
// queue: 8 zeroed counters of the persistent walk (walk.hpp)
void launch_count_db(const Node* nodes, const Node* prims, const uint64_t* pkey,
                     uint32_t np_bound, const uint32_t* np_dev, const DbSets& sets,
                     const DbTables& t, uint32_t* queue, uint32_t* err, int block,
                     hipStream_t s);
// Core flags by pair traversal instead (the option): every pair of
// primitives within eps adds to the points' counts in deg[] (n words, zeroed
// by launch_make_prims), then the flags of the points outside dense cells
// are set from them.  queue: 8 zeroed counters (batched walks run
// persistently).
void launch_count_pairs_db(const Node* nodes, const Node* prims, const uint64_t* pkey,
                           uint32_t np_bound, const uint32_t* np_dev, const DbSets& sets,
                           const DbTables& t, uint32_t* deg, uint32_t* queue, uint32_t* err,
                           int block, hipStream_t s);
void launch_pairs_db(const Node* nodes, const Node* prims, const uint64_t* pkey,
                     uint32_t np_bound, const uint32_t* np_dev, const DbSets& sets,
                     const DbTables& t, uint32_t* queue, uint32_t* err, int block,
                     hipStream_t s);

// ---- batched sets (batched.hip) -----------------------------------------------
// Keys of every set: (set id << set_shift) | Morton code with `bits` bits per
// axis inside the set's own bounding box; set_root[s] = -1 for every set;
// grids[s] = set s's quantisation grid (for the walks' early end).
// With set_inv_h (DenseBox), the codes are those of grid cells of side
// max(1 / set_inv_h[s], extent / 2^bits) per axis instead.
void launch_set_morton(const float* pts, const int64_t* offsets, uint32_t num_sets, int bits,
                       int set_shift, const float* set_inv_h, uint64_t* keys, uint32_t* hist,
                       int32_t* set_root, MortonGrid* grids, uint32_t* status, hipStream_t s);
// queue: 8 zeroed counters of the persistent walk (walk.hpp)
void launch_count_sets(const Node* nodes, const float4* leaf, uint32_t n, const uint64_t* keys,
                       int set_shift, const int32_t* set_root, const float* set_e2,
                       const int32_t* set_minpts, const MortonGrid* grids, uint8_t* flag,
                       uint32_t* queue, uint32_t* err, int block, hipStream_t s);
void launch_pairs_sets(const Node* nodes, const float4* leaf, uint32_t n, const uint64_t* keys,
                       int set_shift, const float* set_e2, const int32_t* set_minpts,
                       const MortonGrid* grids, const uint32_t* perm, int32_t* parent,
                       uint8_t* flag, unsigned long long* bestcore, uint32_t* queue,
                       uint32_t* err, int block, hipStream_t s);
// labels are set-local: smallest input index in the cluster minus the
// set's offset (labels -1 and, with bestcore, minlab INT_MAX beforehand;
// bestcore null: no set has minPts > 2)
void launch_final_sets(uint32_t n, const uint64_t* keys, int set_shift, const int32_t* set_minpts,
                       const int64_t* offsets, const uint8_t* flag,
                       const unsigned long long* bestcore, const uint32_t* perm, int32_t* parent,
                       int32_t* minlab, int32_t* labels, hipStream_t s);

}  // namespace dbx
