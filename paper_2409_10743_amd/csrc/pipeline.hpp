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
constexpr int SORT_ITEMS = 12;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;  // keys per tile
constexpr int RADIX = 256;
constexpr int SORT_PASSES = 8;                          // 8-bit digits of 64
constexpr uint32_t SORT_MAX_N = (1u << 30) - 1;         // 30-bit look-back counts

inline uint32_t sort_tiles(uint32_t n) { return (n + SORT_TILE - 1) / SORT_TILE; }
// words of look-back state needed for all passes of one sort of n keys
inline size_t sort_status_words(uint32_t n) {
  return size_t(SORT_PASSES) * sort_tiles(n) * RADIX;
}

struct SortScratch {
  uint32_t* hist;      // [SORT_PASSES][RADIX] digit counts, zeroed
  uint32_t* tile_ctr;  // [SORT_PASSES] dynamic tile ids, zeroed
  uint32_t* status;    // [SORT_PASSES][tiles][RADIX] look-back words, zeroed
  uint32_t* err;       // status word, STATUS_SORT_STALL set on a stalled wait
};

// Digit histograms of keys already in memory (the morton kernel computes
// them itself while writing the keys).
void launch_digit_histogram(const uint64_t* keys, uint32_t n, uint32_t* hist,
                            hipStream_t s);
// LSD sort of (keys, vals) by the digits [first_pass, SORT_PASSES); passes
// alternate between the A and B buffers, starting from A.  If `iota_vals`,
// the input values are taken to be 0..n-1 and `va` is not read.  Returns
// true when the result ends in the A buffers.
// `after_pass(arg, p)`, if given, is called after pass p is enqueued.
bool launch_radix_sort(uint64_t* ka, uint64_t* kb, uint32_t* va, uint32_t* vb,
                       uint32_t n, int first_pass, bool iota_vals,
                       const SortScratch& sc, hipStream_t s,
                       void (*after_pass)(void*, int) = nullptr, void* arg = nullptr);

// ---- bounds, Morton codes, gather (morton.hip) ----------------------------
// bounds[0..2] lo (ordered-int encoding), bounds[3..5] hi
void launch_prep(uint32_t* zero_region, size_t zero_words, uint32_t* bounds,
                 hipStream_t s);
void launch_bounds(const float* pts, uint32_t n, uint32_t* bounds,
                   uint32_t* status, hipStream_t s);
void launch_morton(const float* pts, uint32_t n, const uint32_t* bounds,
                   uint64_t* keys, uint32_t* hist, hipStream_t s);
// Sorted float4 leaves + per-point state initialisation; also fills the
// build's hand-over entries with -1.
void launch_gather(const float* pts, const uint32_t* perm, uint32_t n,
                   float4* leaf, int32_t* parent, int32_t* minlab,
                   uint8_t* flag, unsigned long long* bestcore,
                   int4* pending, uint32_t pending_entries, hipStream_t s);

// ---- LBVH (lbvh.hip) --------------------------------------------------------
constexpr int BUILD_LEAVES = 256;        // leaves per level-1 frame
constexpr int BUILD_FANOUT_LOG2 = 7;     // frames per next-level frame: 128
constexpr int BUILD_BLOCK = 256;         // = BUILD_LEAVES = 2 << BUILD_FANOUT_LOG2
static_assert(BUILD_BLOCK == BUILD_LEAVES && BUILD_BLOCK == (2 << BUILD_FANOUT_LOG2), "");
int build_levels(uint32_t n);
// int4 entries of hand-over state the build needs (all levels), -1 filled
size_t build_pending_entries(uint32_t n);
// right[k]: right child of internal node k; other[k]: exchange slot (set
// up by the build itself); rend[k]: last leaf under internal node k.
void launch_build(const uint64_t* keys, const float4* leaf, uint32_t n,
                  Node* nodes, int32_t* right, int32_t* other, int32_t* rend,
                  int32_t* root, int4* pending, uint32_t* err, hipStream_t s);
void launch_ropes(Node* nodes, float4* leaf, const int32_t* right,
                  const int32_t* rend, uint32_t n, uint32_t* err, hipStream_t s);

// ---- traversals (traverse.hip) ---------------------------------------------
void launch_count(const Node* nodes, const float4* leaf, uint32_t n,
                  const int32_t* root, float e2, int32_t min_pts,
                  uint8_t* is_core, uint32_t* err, int block, hipStream_t s);
// minPts <= 2: every point with a neighbour is core; union every pair.
void launch_pairs_fof(const Node* nodes, const float4* leaf, uint32_t n,
                      float e2, int32_t* parent, uint8_t* member, uint32_t* err,
                      int block, hipStream_t s);
// minPts > 2: union core pairs, record each non-core point's smallest-index
// core neighbour.
void launch_pairs_core(const Node* nodes, const float4* leaf, uint32_t n,
                       float e2, const uint8_t* is_core, const uint32_t* perm,
                       int32_t* parent, unsigned long long* bestcore,
                       uint32_t* err, int block, hipStream_t s);
// Pair traversal with F(i, j) = count: every pair exactly once.
void launch_pairs_count(const Node* nodes, const float4* leaf, uint32_t n,
                        float e2, unsigned long long* count, uint32_t* err,
                        int block, hipStream_t s);

// ---- labels (finalize.hip) --------------------------------------------------
// 1) cluster root per point (written over parent; -1 = noise) and the
//    smallest input index per root;  2) labels in input order.
void launch_final_roots(uint32_t n, int32_t min_pts, const uint8_t* flag,
                        const unsigned long long* bestcore, const uint32_t* perm,
                        int32_t* parent, int32_t* minlab, hipStream_t s);
void launch_final_labels(uint32_t n, const uint32_t* perm, const int32_t* root,
                         const int32_t* minlab, int32_t* labels, hipStream_t s);
// dst[perm[i]] = src[i]: from sorted order back to input order
void launch_scatter_u8(const uint8_t* src, const uint32_t* perm, uint32_t n,
                       uint8_t* dst, hipStream_t s);

}  // namespace dbx
