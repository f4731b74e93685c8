// The stackless rope walk shared by every point traversal (sections 4.1,
// 4.2): at an internal node whose box is within eps of the query go to its
// left child, otherwise follow its rope; at a leaf test the point, then
// follow the leaf's rope; stop at the sentinel.
//
// One wave runs the walks of a chunk of consecutive (Morton-ordered)
// queries.  A lane whose walk ends takes the chunk's next query at once, so
// the wave does not idle until its longest walk of 64 is over.  Internal
// nodes and leaves go through the same step: a leaf is read as the box
// [p, p] (same load, same test; the box bound of a point box is exactly the
// point's squared distance), so the lanes of a wave never split into a leaf
// path and a node path, each paying its own memory latency.
//
// Early end.  Internal nodes are in Karras' order, so the node a rope leads
// to has its first leaf's number, and the walk, going right, meets leaves
// in increasing order.  Every neighbour's Morton code is at most
// khi = MortonGrid::upper_code(q): once a rope leads to a subtree whose
// first key exceeds khi, no leaf left in the walk can be a neighbour, and
// it ends.  (The first key is read with the node, in the same step.)
//
// The visitor V says whether its walks start at a rope target (pair walks:
// the query leaf's rope; a walk from a set's root does not, that node may
// be numbered by its last leaf), kStartIsRope, and holds the per-lane state
// of the lane's current query:
//   int32_t begin(uint32_t i, const float4& q)  first node of query i
//   uint64_t khi() const                        the early-end bound (all
//                                               ones: never end early)
//   float   e2() const                          squared radius (this query)
//   void    visit(bool leaf, bool near)         every step (statistics)
//   bool    hit(uint32_t i, int32_t j, const float4& q)
//                                               leaf j within eps; true ends
//                                               the walk early
//   void    end(uint32_t i)                     the walk of query i is over
#pragma once

#include "pipeline.hpp"

namespace dbx {

// Queries of one wave's chunk: 64 x walk_queries_per_lane(n).  More per
// lane keeps lanes busier (a lane takes a new query when its walk ends) but
// spreads the queries in flight over a longer stretch of the tree, which
// costs L2 hits, and for small n it leaves CUs idle: 4 per lane from 2^23
// queries, 2 from 2^22, else 1.
uint32_t walk_queries_per_lane(uint32_t n);
inline uint32_t walk_chunk_size(uint32_t n) { return 64u * walk_queries_per_lane(n); }

inline uint32_t walk_grid(uint32_t n, int block) {
  const uint32_t chunk = walk_chunk_size(n);
  const uint64_t waves = (uint64_t(n) + chunk - 1) / chunk;
  const uint32_t per_block = uint32_t(block) / 64;
  return uint32_t((waves + per_block - 1) / per_block);
}

// Box bound of `q` against the box [a.xyz, b.xyz]: the same arithmetic as
// box_sq_dist (no FMA, ((x + y) + z)).
__device__ __forceinline__ float box_sq_dist4(const float4& q, const float4& a, const float4& b) {
#pragma clang fp contract(off)
  const float gx = fmaxf(fmaxf(a.x - q.x, q.x - b.x), 0.0f);
  const float gy = fmaxf(fmaxf(a.y - q.y, q.y - b.y), 0.0f);
  const float gz = fmaxf(fmaxf(a.z - q.z, q.z - b.z), 0.0f);
  const float xx = gx * gx;
  const float yy = gy * gy;
  const float zz = gz * gz;
  const float s = xx + yy;
  return s + zz;
}

// Chunk of this wave: [c0, c1).  The grid is walk_grid(n, blockDim.x)
// blocks; blocks are dealt to XCDs so each XCD walks one contiguous
// stretch of queries (nearby queries share tree nodes in its L2).
__device__ __forceinline__ void walk_chunk(uint32_t n, uint32_t chunk, uint32_t& c0,
                                           uint32_t& c1) {
  const uint32_t wave = xcd_tile(blockIdx.x, gridDim.x) * (blockDim.x / 64) + threadIdx.x / 64;
  const uint64_t b = uint64_t(wave) * chunk;
  c0 = uint32_t(b < n ? b : n);
  c1 = uint32_t(b + chunk < n ? b + chunk : n);
}

// Lanes are refilled only once fewer than WALK_REFILL_AT of the 64 are
// still walking; in between, the wave runs a tight per-lane loop.
constexpr uint32_t WALK_REFILL_AT = 48;

struct WalkCfg {
  uint32_t chunk;      // queries per wave
  uint32_t refill_at;  // refill once fewer lanes than this are walking
  uint32_t* queue;     // persistent walks: 8 zeroed chunk counters; null: static chunks
};
inline WalkCfg walk_cfg(uint32_t n, uint32_t* queue = nullptr) {
  return WalkCfg{walk_chunk_size(n), WALK_REFILL_AT, queue};
}

// Persistent walks (PERSIST, with WalkCfg::queue): the grid holds only as
// many waves as the GPU runs at once, and every wave takes spans of
// WALK_GRAB chunks, one after another, from eight counters, one per XCD,
// each handing out a contiguous eighth of the spans.  A wave starts with its own XCD's counter (blockIdx % 8: blocks
// are dealt to the XCDs in turn), so nearby queries still share an L2, and
// takes the other counters' leftovers once its own is drained.  Query costs
// that differ a lot (sets of very different sizes and densities) are then
// balanced up to the end of the launch instead of per block.  Every wave
// leaves once all eight are drained.  All lanes of the wave call it.
// chunks a wave takes per counter increment: one (spans of 8 chunks made the
// batched walks up to 3.5x slower: a span over a dense sub-clump kept one
// wave busy long after the rest had finished)
constexpr uint32_t WALK_GRAB = 1;
__device__ __forceinline__ bool next_chunk(const WalkCfg& wc, uint32_t n, uint32_t& home,
                                           uint32_t& c0, uint32_t& c1) {
  const uint32_t span = wc.chunk * WALK_GRAB;  // a wave walks this many queries per take
  const uint32_t total = (n + span - 1) / span;
  for (uint32_t t = 0; t < 8; ++t) {
    const uint32_t x = (home + t) & 7u;
    const uint32_t lo = uint32_t(uint64_t(total) * x / 8);
    const uint32_t hi = uint32_t(uint64_t(total) * (x + 1) / 8);
    if (lo >= hi) continue;
    uint32_t id = 0;
    if ((threadIdx.x & 63) == 0) id = atomicAdd(wc.queue + x, 1u);
    id = __builtin_amdgcn_readfirstlane(id);
    if (id < hi - lo) {
      home = x;
      const uint64_t b = uint64_t(lo + id) * span;
      c0 = uint32_t(b);
      c1 = uint32_t(b + span < n ? b + span : n);
      return true;
    }
  }
  return false;
}

// Blocks of a persistent walk launch: as many as the GPU holds at once
// (a multiple of 8), at most `needed`.
uint32_t persistent_blocks(const void* kernel, int block, size_t lds, uint32_t needed);

// `leaf` must have one readable float4 past leaf n-1 (a leaf step reads 32
// bytes, like a node step, and ignores the second half).
// keys: the sorted Morton codes (read only when V::kBounded).
template <class V, bool PERSIST = false>
__device__ __forceinline__ void wave_walks(const Node* __restrict__ nodes,
                                           const float4* __restrict__ leaf,
                                           const uint64_t* __restrict__ keys, uint32_t n,
                                           WalkCfg wc, V& v, uint32_t* err) {
  uint32_t c0, c1;
  uint32_t home = blockIdx.x & 7u;
  bool drained = !PERSIST;  // no span left to take (static: the wave's one chunk)
  if (PERSIST) {
    if (!next_chunk(wc, n, home, c0, c1)) { c0 = c1 = n; drained = true; }
  } else {
    walk_chunk(n, wc.chunk, c0, c1);
  }
  const uint32_t refill_at = wc.refill_at;
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t head = c0;  // next unstarted query of the chunk (wave-uniform)
  uint32_t i = 0;
  bool have = false;   // lane holds query i whose end() is still due
  int32_t node = SENTINEL;
  uint32_t steps = 0;
  bool by_rope = false;  // node was reached through a rope: its number is its first leaf
  float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
  for (;;) {
    if (PERSIST && head >= c1 && !drained) {  // the next span
      if (next_chunk(wc, n, home, c0, c1)) head = c0;
      else drained = true;
    }
    // hand the chunk's next queries to the idle lanes
    const bool need = node == SENTINEL;
    const uint64_t m = __ballot(need);
    if (need) {
      if (have) { v.end(i); have = false; }
      const uint32_t idx = head + uint32_t(__popcll(m & lt));
      if (idx < c1) {
        i = idx;
        have = true;
        q = leaf[i];
        node = v.begin(i, q);
        steps = 0;
        by_rope = V::kStartIsRope;
      }
    }
    const uint32_t h = head + uint32_t(__popcll(m));
    head = h < c1 ? h : c1;
    if (__ballot(node != SENTINEL) == 0) {
      if (head >= c1 && (!PERSIST || drained)) break;
      continue;  // every new walk was empty: hand out more
    }
    // walk; stop early to refill once enough lanes are idle (and there is
    // something left to hand out).  The loop is wave-uniform: idle lanes
    // read leaf 0 (always readable) so that the loads need no branch.
    for (;;) {
      bool act = node != SENTINEL;
      const bool lf = is_leaf(node);
      const uint32_t idx = lf ? uint32_t(leaf_index(node)) : uint32_t(node);
      // a walk visits every node at most once: more than 2n steps, or a
      // reference outside the arrays, means a malformed tree (checked
      // without a branch; the rare failure takes one wave-uniform branch)
      steps += act ? 1u : 0u;
      const bool bad = act && (steps > 2 * n || idx >= (lf ? n : n - 1));
      if (__builtin_expect(__ballot(bad) != 0ull, 0)) {
        if (bad) atomicOr(err, STATUS_TREE);
        node = bad ? SENTINEL : node;
      }
      act = act && !bad;
      const float4* p = !act ? leaf
                        : lf ? leaf + idx
                             : reinterpret_cast<const float4*>(nodes + idx);
      const float4 a = p[0], p1 = p[1];
      const float4 b = lf ? a : p1;
      if (V::kBounded) {  // a rope target's number is its first leaf
        const uint32_t first = idx;
        const uint64_t kf = keys[act && by_rope ? first : 0u];
        if (act && by_rope && kf > v.khi()) {
          node = SENTINEL;
          act = false;
        }
      }
      if (act) {
        const bool near = box_sq_dist4(q, a, b) <= v.e2();
        v.visit(lf, near);
        // internal: left child (a.w) or rope (b.w); leaf: its rope (a.w = b.w)
        const bool down = near && !lf;
        int32_t next = down ? __float_as_int(a.w) : __float_as_int(b.w);
        if (near && lf && v.hit(i, leaf_index(node), q)) next = SENTINEL;
        node = next;
        by_rope = !down;
      }
      const uint32_t busy = uint32_t(__popcll(__ballot(node != SENTINEL)));
      if (busy == 0 || ((head < c1 || (PERSIST && !drained)) && busy < refill_at)) break;
    }
  }
  if (have) v.end(i);
}

}  // namespace dbx
