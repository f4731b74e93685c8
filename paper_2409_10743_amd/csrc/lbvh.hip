// Linear BVH over Morton-sorted leaves: Apetrei's bottom-up construction
// (section 4.2.1: faster than Karras' build), with the internal nodes laid
// out in Karras' order and the ropes of the stackless traversal written by
// the same pass.
//
// Construction.  delta(i) measures how different leaves i and i+1 are: the
// XOR of their codes, and for equal codes the XOR of the positions i^(i+1)
// (ranked below every differing pair), which splits runs of equal codes
// evenly.  A node covering leaves [l, r] is the left child of the node split
// at r when l = 0 or (r < n-1 and delta(r) < delta(l-1)), otherwise the
// right child of the node split at l-1.  Ties go to the smaller boundary
// index, a strict order, so every split gets exactly one left and one right
// child.  Each child swaps its outer range bound into a per-split slot
// (initially -1) with one acquire-release exchange: the first to arrive
// leaves, the second learns the parent's full range from the value it gets
// back, reads its sibling's box, finishes the parent and climbs on.
//
// Node order.  Internal nodes are numbered as in Karras' layout, which
// ArborX recovers after Apetrei's build (section 4.2.1): the node covering
// [l, r] is number r if it is the left child of its parent and number l if
// it is the right child, and the root is number 0.  So the children of the
// node split between leaves g and g+1 are number g (or leaf g) and number
// g+1 (or leaf g+1), and the numbers 0..n-2 are each used once.  A node's
// number is known as soon as it is finished: the thread that finishes it
// decides right away on which side of its parent it lies, and writes its
// record then.
//
// Ropes.  The rope of a node or leaf is where a stackless, left-first
// pre-order walk goes after its subtree: the right child of the lowest
// ancestor holding it in its left subtree, i.e. the right child of the split
// at its last leaf r.  That child covers [r+1, ...]; it is leaf r+1 exactly
// when leaf r+1 is a right child (r+1 is the last leaf, or delta(r+1) is not
// below delta(r)), else internal node r+1.  A rope is therefore a function
// of r and two deltas, written with the record: the sentinel when r is the
// last leaf (of its set), else r+1 as a leaf or a node.  A rope target's
// number is always its first leaf, which the traversal uses to stop early.
//
// Frames.  gfx950 has one L2 per XCD, so an exchange between threads of
// different workgroups needs agent scope, i.e. an L2 write-back before and
// an L2 invalidate after every exchange: far too slow for n of them.  So
// the climb runs in levels.  Level 1 gives each workgroup a frame of 256
// consecutive leaves; level k+1 frames hold 128 level-k frames.  A thread
// climbs while its parent's split lies strictly inside its frame (both
// leaves of the split in the frame); then every other thread that can touch
// that parent during this launch belongs to the same frame, i.e. the same
// workgroup, and workgroup scope is enough.  A node whose parent split is a
// frame edge is handed to the next level (at most two per frame: one per
// edge), which runs after a kernel boundary, so everything earlier levels
// wrote is visible there.  The last level is one frame holding all leaves.
//
// Batched sets: the keys carry the set id in their top bits (`set_shift`),
// so a boundary between sets has a larger delta than any boundary inside a
// set and every set is one complete subtree.  Ropes are cut at set ends
// (sets overlap in space, so boxes would not keep a walk inside its set),
// and the node spanning exactly a set is recorded as that set's root.  With
// no set bits (set_shift = 64) the only such node is the root.
#include <algorithm>
#include <type_traits>

#include "pipeline.hpp"

namespace dbx {

namespace {

// Leaves are points (FDBSCAN: float4 x, y, z, rope) or boxes (DenseBox
// primitives: Node records whose `left` holds the payload).  The levels
// above the first only load leaves.
struct PointLeaves {
  static constexpr bool kPoint = true;  // a record is one float4, its box [p, p]
  float4* leaf;
  __device__ void load(int32_t j, float4& lo, float4& hi) const { lo = hi = leaf[j]; }
  // 32 bytes from leaf j (the array has one record past the last leaf)
  __device__ const float4* rec(int32_t j) const { return leaf + j; }
};
// FDBSCAN's level-1 frames: leaf j is gathered from input point perm[j]
// here (a random 12-byte read) and written once, with its rope, together
// with the point's union-find state and label -1; later levels read the
// written leaves.
struct GatherLeaves {
  static constexpr bool kPoint = true;
  const float* pts;
  const uint32_t* perm;
  uint32_t n;
  float4* leaf;
  int32_t* parent;
  int32_t* minlab;               // null unless minPts > 2
  uint8_t* flag;
  unsigned long long* bestcore;  // null unless minPts > 2
  int32_t* labels;               // output, input order; null: none
  uint32_t* deg;                 // pair counts (core flags by pair traversal); null: none
  __device__ void load(int32_t j, float4& lo, float4& hi) const {
    const uint32_t o = min(perm[j], n - 1);  // a permutation unless the sort failed
    const float* p = pts + size_t(3) * o;
    lo = hi = make_float4(p[0], p[1], p[2], 0.0f);
  }
  __device__ void write_out(int32_t j, const float4& lo, const float4&, int32_t rope) const {
    leaf[j] = make_float4(lo.x, lo.y, lo.z, __int_as_float(rope));
    parent[j] = j;
    if (minlab) minlab[j] = 0x7fffffff;
    flag[j] = 0;
    if (bestcore) bestcore[j] = ~0ull;
    if (labels) labels[j] = -1;  // by input index: every index once
    if (deg) deg[j] = 0;
    if (uint32_t(j) == n - 1)  // the walks read one record past the last leaf
      leaf[n] = make_float4(0.f, 0.f, 0.f, __int_as_float(SENTINEL));
  }
};
// The clustering call's level-1 frames: as GatherLeaves, and each leaf's
// Morton code is computed here from its point with the grid and dropped
// bits the Morton kernel used (the same function of the same floats, so
// the same code): that call's sort moves 32-bit halves of the codes and
// does not write them.  The frame takes its deltas from these codes and
// writes them to `keys_out` for the upper levels and the walks' early end.
struct GatherCoded : GatherLeaves {
  const uint32_t* bounds;  // scene bounds words
  const uint32_t* drop;    // low code bits cleared
  uint64_t* keys_out;
};
template <class L>
struct codes_here : std::false_type {};
template <>
struct codes_here<GatherCoded> : std::true_type {};

struct BoxLeaves {
  static constexpr bool kPoint = false;
  Node* prim;
  __device__ const float4* rec(int32_t j) const {
    return reinterpret_cast<const float4*>(prim + j);
  }
  __device__ void load(int32_t j, float4& lo, float4& hi) const {
    const float4* q = reinterpret_cast<const float4*>(prim + j);
    lo = q[0];
    hi = q[1];
  }
  __device__ void write_out(int32_t j, const float4&, const float4&, int32_t rope) const {
    prim[j].rope = rope;
  }
};

__device__ __forceinline__ uint64_t set_mask_of(int set_shift) {
  return set_shift < 64 ? (~0ull << set_shift) : 0ull;
}
// does a set end at leaf q (q < n - 1)?
__device__ __forceinline__ bool set_cut(const uint64_t* __restrict__ keys, int32_t q,
                                        uint64_t mask) {
  return ((keys[q] ^ keys[q + 1]) & mask) != 0;
}
__device__ __forceinline__ uint32_t set_of(const uint64_t* __restrict__ keys, int32_t l,
                                           int set_shift) {
  return set_shift < 64 ? uint32_t(keys[l] >> set_shift) : 0u;
}

__device__ __forceinline__ uint64_t delta_of(uint64_t a, uint64_t b, int32_t i) {
  return a == b ? uint64_t(uint32_t(i) ^ uint32_t(i + 1)) : ((a ^ b) + (1ull << 32));
}
__device__ __forceinline__ uint64_t delta(const uint64_t* __restrict__ keys, int32_t i) {
  return delta_of(keys[i], keys[i + 1], i);
}

// Is [l, r] the left child of its parent (split at r) rather than the right
// child (split at l - 1)?  d_r = delta(r), d_lm1 = delta(l - 1); each is
// only used where it exists.
__device__ __forceinline__ bool left_side(int32_t l, int32_t r, int32_t last, uint64_t d_r,
                                          uint64_t d_lm1) {
  return l == 0 || (r != last && d_r < d_lm1);
}

// left child of the node [l, r] split at g: [l, g], number g or leaf g
__device__ __forceinline__ int32_t left_ref(int32_t l, int32_t g) {
  return l == g ? leaf_ref(g) : g;
}

// rope of a node or leaf whose last leaf is r; cut: a set ends at r,
// d_r = delta(r), d_r1 = delta(r + 1) (only used where they exist)
__device__ __forceinline__ int32_t rope_of(int32_t r, int32_t last, bool cut, uint64_t d_r,
                                           uint64_t d_r1) {
  if (r == last || cut) return SENTINEL;
  const bool leaf_next = r + 1 == last || !(d_r1 < d_r);
  return leaf_next ? leaf_ref(r + 1) : r + 1;
}

__device__ __forceinline__ void write_node(Node* nodes, int32_t k, const float4& lo,
                                           const float4& hi, int32_t left, int32_t rope) {
  float4* q = reinterpret_cast<float4*>(nodes + k);
  q[0] = make_float4(lo.x, lo.y, lo.z, __int_as_float(left));
  q[1] = make_float4(hi.x, hi.y, hi.z, __int_as_float(rope));
}

__device__ __forceinline__ void grow(float4& lo, float4& hi, const float4& slo,
                                     const float4& shi) {
  lo.x = fminf(lo.x, slo.x); lo.y = fminf(lo.y, slo.y); lo.z = fminf(lo.z, slo.z);
  hi.x = fmaxf(hi.x, shi.x); hi.y = fmaxf(hi.y, shi.y); hi.z = fmaxf(hi.z, shi.z);
}

// Level 1 of the build, all in LDS: one workgroup per 256-leaf frame.  The
// frame's deltas, leaves, exchange slots and finished nodes (by number:
// every node finished here has both range ends, so its number, in the
// frame) live in LDS; the exchange is an LDS swap.  At the end the frame's
// leaves and nodes go out whole, ropes included, in one coalesced pass,
// with the exchange slots later levels still need.  A point leaf's box is
// [p, p]: only its lower corner is kept, and the frame's codes share the
// node boxes' LDS (they are done with before the climb), so that eight
// workgroups fit a CU's LDS.
template <class Leaves>
__global__ __launch_bounds__(BUILD_BLOCK) void k_build_frame(
    const uint64_t* __restrict__ keys, Leaves lv, uint32_t n_bound,
    const uint32_t* __restrict__ n_dev, int set_shift, Node* __restrict__ nodes,
    int32_t* __restrict__ other, int32_t* __restrict__ set_root, int4* __restrict__ pend_out,
    uint32_t* __restrict__ err) {
  __shared__ uint64_t s_delta[BUILD_LEAVES + 2];  // delta of boundary f0-1+j at j
  __shared__ uint8_t s_cut[BUILD_LEAVES + 2];     // a set ends at boundary f0-1+j
  constexpr bool kPt = Leaves::kPoint;
  __shared__ float4 s_leaf[BUILD_LEAVES], s_leafhi[kPt ? 1 : BUILD_LEAVES];
  __shared__ float4 s_lo[BUILD_LEAVES], s_hi[BUILD_LEAVES];  // node number f0+k
  __shared__ int32_t s_left[BUILD_LEAVES], s_end[BUILD_LEAVES];  // its left child, last leaf
  __shared__ int32_t s_other[BUILD_LEAVES];  // exchange slot of split f0+k; -2 once finished
  const int32_t t = threadIdx.x;
  const uint32_t n = n_dev ? min(*n_dev, n_bound) : n_bound;
  const int32_t last = int32_t(n) - 1;
  const int32_t f0 = int32_t(blockIdx.x) * BUILD_LEAVES;
  if (f0 >= int32_t(n)) return;  // launched for the bound: the whole block
  const int32_t f1 = min(f0 + BUILD_LEAVES, int32_t(n));
  const int32_t m = f1 - f0;
  const uint64_t mask = set_mask_of(set_shift);
  // upper corner of leaf f0+k
  auto leaf_hi = [&](int32_t k) -> const float4& { return kPt ? s_leaf[k] : s_leafhi[k]; };
  auto load_leaf = [&](int32_t k) {
    float4 h;
    lv.load(f0 + k, s_leaf[k], kPt ? h : s_leafhi[k]);
  };
  if constexpr (codes_here<Leaves>::value) {
    // codes of leaves f0-1 .. f1+1 (at j = 0 .. m+2) from their points;
    // no set bits here.  In s_lo: read before the barrier ahead of the climb,
    // which writes s_lo.
    static_assert(sizeof(s_lo) >= (BUILD_LEAVES + 3) * sizeof(uint64_t), "codes fit s_lo");
    uint64_t* s_code = reinterpret_cast<uint64_t*>(s_lo);
    MortonGrid grid;
    grid.load(lv.bounds);
    const uint64_t cmask = ~0ull << *lv.drop;
    if (t < m) {
      load_leaf(t);
      const uint64_t c = grid.code(s_leaf[t].x, s_leaf[t].y, s_leaf[t].z) & cmask;
      s_code[t + 1] = c;
      lv.keys_out[f0 + t] = c;
    }
    if (t < 3) {  // leaves f0-1, f1 and f1+1, where they exist
      const int32_t b = t == 0 ? f0 - 1 : f1 - 1 + t;
      uint64_t c = 0;
      if (b >= 0 && b <= last) {
        float4 a, h;
        lv.load(b, a, h);
        c = grid.code(a.x, a.y, a.z) & cmask;
      }
      s_code[t == 0 ? 0 : m + t] = c;
    }
    __syncthreads();
    for (int32_t j = t; j <= m + 1; j += BUILD_BLOCK) {
      const int32_t b = f0 - 1 + j;
      const bool ok = b >= 0 && b < last;
      s_delta[j] = ok ? delta_of(s_code[j], s_code[j + 1], b) : 0ull;
      s_cut[j] = ok ? 0 : 1;
    }
  } else {
    for (int32_t j = t; j <= m + 1; j += BUILD_BLOCK) {
      const int32_t b = f0 - 1 + j;
      const bool ok = b >= 0 && b < last;
      s_delta[j] = ok ? delta(keys, b) : 0ull;
      s_cut[j] = ok ? set_cut(keys, b, mask) : 1;
    }
    if (t < m) load_leaf(t);
  }
  s_other[t] = -1;
  s_end[t] = -1;
  __syncthreads();
  auto D = [&](int32_t b) { return s_delta[b - f0 + 1]; };  // b in [f0-1, f1]
  // does [l, r] span a whole set? (l - 1 and r are set ends)
  auto spans = [&](int32_t l, int32_t r) { return s_cut[l - f0] && s_cut[r - f0 + 1]; };
  if (t < m) {
    const int32_t j0 = f0 + t;
    if (spans(j0, j0)) set_root[set_of(keys, j0, set_shift)] = leaf_ref(j0);
    if (n > 1) {
      int32_t l = j0, r = j0, g = -1;  // g: split of the node, -1 for the leaf
      float4 lo = s_leaf[t], hi = leaf_hi(t);
      for (;;) {
        const bool is_left = left_side(l, r, last, D(r), D(l - 1));
        if (g >= 0) {  // finished here: its number is known now
          const int32_t k = (is_left ? r : l) - f0;
          s_lo[k] = lo;
          s_hi[k] = hi;
          s_left[k] = left_ref(l, g);
          s_end[k] = r;
          if (spans(l, r)) set_root[set_of(keys, l, set_shift)] = k + f0;
        }
        const int32_t par = is_left ? r : l - 1;
        if (par < f0 || par > f1 - 2) {  // frame edge: hand over to level 2
          const int32_t ref = g < 0 ? leaf_ref(l) : (is_left ? r : l);
          pend_out[size_t(blockIdx.x) * 2 + (is_left ? 1 : 0)] = make_int4(ref, l, r, 0);
          break;
        }
        const int32_t k = par - f0;
        const int32_t bound = __hip_atomic_exchange(s_other + k, is_left ? l : r,
                                                    __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (bound < 0) break;  // first arrival: the sibling finishes the parent
        s_other[k] = -2;
        if (is_left) r = bound;
        else l = bound;
        // the sibling: the other child of split par, [par+1, r] or [l, par]
        const int32_t sl = is_left ? par + 1 : l, sr = is_left ? r : par;
        if (sl < f0 || sr > f1 - 1 || sl > sr) { atomicOr(err, STATUS_TREE); break; }
        if (sl == sr) {
          grow(lo, hi, s_leaf[sl - f0], leaf_hi(sl - f0));
        } else {
          const int32_t sk = (is_left ? sl : sr) - f0;  // right child: first leaf; left: last
          grow(lo, hi, s_lo[sk], s_hi[sk]);
        }
        g = par;
        if (l == 0 && r == last) {  // the root, number 0: this frame holds every leaf
          s_lo[0] = lo;
          s_hi[0] = hi;
          s_left[0] = left_ref(l, g);
          s_end[0] = r;
          if (spans(l, r)) set_root[set_of(keys, l, set_shift)] = 0;
          break;
        }
      }
    }
  }
  __syncthreads();
  // leaf f0+t and node number f0+t, whole, with their ropes; the exchange
  // slot of split f0+t unless it is finished (the frame's right edge split
  // is never touched here: -1)
  const int32_t p = f0 + t;
  if (t < m) {  // n = 1 too: the one leaf still goes out
    lv.write_out(p, s_leaf[t], leaf_hi(t), rope_of(p, last, s_cut[t + 1], D(p), D(p + 1)));
    const int32_t r = s_end[t];
    if (r >= 0)
      write_node(nodes, p, s_lo[t], s_hi[t], s_left[t],
                 rope_of(r, last, s_cut[r - f0 + 1], D(r), D(r + 1)));
    if (p < last && s_other[t] != -2) other[p] = s_other[t];
  }
}

// What a climbing thread keeps about the two ends of its node [l, r]: the
// deltas and set cuts there (so a step needs no key loads before its
// exchange).  cl: l = 0 or a set ends at l - 1; cr: r = last or a set ends
// at r.
struct Ends {
  uint64_t dl, dr, dr1;  // delta(l - 1), delta(r), delta(r + 1) where they exist
  bool cl, cr;
};

// the left end becomes l (keys l - 1, l)
__device__ __forceinline__ void set_left(Ends& E, const uint64_t* __restrict__ keys, int32_t l,
                                         uint64_t mask) {
  if (l == 0) {
    E.dl = 0;
    E.cl = true;
    return;
  }
  const uint64_t a = keys[l - 1], b = keys[l];
  E.dl = delta_of(a, b, l - 1);
  E.cl = ((a ^ b) & mask) != 0;
}
// the right end becomes r (keys r .. r + 2)
__device__ __forceinline__ void set_right(Ends& E, const uint64_t* __restrict__ keys, int32_t r,
                                          int32_t last, uint64_t mask) {
  if (r == last) {
    E.dr = E.dr1 = 0;
    E.cr = true;
    return;
  }
  const uint64_t a = keys[r], b = keys[r + 1];
  const uint64_t c = r + 1 < last ? keys[r + 2] : 0ull;
  E.dr = delta_of(a, b, r);
  E.dr1 = r + 1 < last ? delta_of(b, c, r + 1) : 0ull;
  E.cr = ((a ^ b) & mask) != 0;
}

// Levels k > 1 of the build: thread = one of the nodes handed up by the
// level-(k-1) frames inside this block's frame of `frame` leaves (two per
// frame; 2 * 128 per 256-thread block, or, for the top launch, one block
// over every leaf).
//
// Exchanges.  A split inside the frame is either half done already (one
// child finished in an earlier launch: other[split] holds its bound, and
// the thread finishing the other child here just reads it) or touched only
// in this launch, where its slot lives in an LDS hash table (split -> bound)
// instead of global memory: the exchange is an LDS atomic.  A first arrival
// that no thread of this launch completes is carried to other[] when the
// block ends, for a later level.
//
// Sibling hand-over in LDS.  Before its exchange a thread leaves, in its
// own LDS record, what the sibling will need from it: its box and what it
// knows about its outer end (the deltas and set cut there and other[] at
// that split).  The exchanged table value carries the thread's number with
// its bound.  The first arrival stops (a thread arrives first at most
// once), so its record stays put; the second arrival learns from the value
// it gets back whose record it is and takes box and end from LDS: a step between two
// nodes of the same launch costs no memory round trip.  Only a split whose
// first child finished in an earlier launch (other[] holds its bound) still
// loads the sibling's box, the keys around the node's new end and other[]
// at its candidate parent splits from memory, in one batch.  nodes is
// written and read by different threads of the same launch, ordered by the
// exchange: no __restrict__ on it.
//
// Table load: every key in the table has its first arrival in this launch,
// and a thread arrives first at most once, so a launch of T threads keys at
// most T splits: 2 slots per thread keep the load at most 1/2.
constexpr uint32_t LEVEL_TAB_FACTOR = 2;

// What a first arrival leaves for its sibling (one per thread).
struct SibRec {
  float lox, loy, loz, hix, hiy, hiz;
  uint64_t d0, d1;  // left child: delta(l - 1); right child: delta(r), delta(r + 1)
  int32_t o;        // other[] at that end's split (-1: none)
  int32_t cut;      // a set ends there
};
// LDS of a level launch of `threads` threads with a table of 2^tab_log2 slots
inline size_t level_lds(uint32_t threads, uint32_t tab_log2) {
  return (size_t(12) << tab_log2) + size_t(threads) * sizeof(SibRec);
}

__device__ __forceinline__ int32_t tab_slot(int32_t* s_key, uint32_t tab_log2, int32_t split) {
  const uint32_t m = (1u << tab_log2) - 1u;
  uint32_t h = (uint32_t(split) * 2654435761u) >> (32 - tab_log2);
  for (uint32_t t = 0; t <= m; ++t) {
    const int32_t k = atomicCAS(s_key + h, -1, split);
    if (k == -1 || k == split) return int32_t(h);
    h = (h + 1) & m;
  }
  return -1;  // full: cannot happen at load 1/2
}

template <class Leaves>
__global__ __launch_bounds__(1024) void k_build_level(
    const uint64_t* __restrict__ keys, Leaves lv, uint32_t n_bound,
    const uint32_t* __restrict__ n_dev, uint64_t frame, uint32_t entries, uint32_t tab_log2,
    int set_shift, Node* nodes, int32_t* __restrict__ other, int32_t* set_root,
    const int4* __restrict__ pend_in, int4* __restrict__ pend_out, uint32_t* err) {
  // split keys; their values: -1 empty, -2 both children met, else the first
  // arrival's (thread << 32 | bound); then one SibRec per thread
  extern __shared__ int32_t s_tab[];
  const uint32_t tab = 1u << tab_log2;
  int32_t* s_key = s_tab;
  int64_t* s_val = reinterpret_cast<int64_t*>(s_tab + tab);
  SibRec* s_rec = reinterpret_cast<SibRec*>(s_tab + 3 * tab);
  for (uint32_t h = threadIdx.x; h < tab; h += blockDim.x) {
    s_key[h] = -1;
    s_val[h] = -1;
  }
  __syncthreads();
  const uint32_t n = n_dev ? min(*n_dev, n_bound) : n_bound;
  const int32_t last = int32_t(n) - 1;
  const int64_t f0 = int64_t(blockIdx.x) * int64_t(frame);
  const int64_t f1 = min(f0 + int64_t(frame), int64_t(n));
  const uint64_t mask = set_mask_of(set_shift);
  const size_t slot = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int4 e = make_int4(SENTINEL, 0, 0, 0);
  if (slot < entries) e = pend_in[slot];
  int32_t ref = e.x, l = e.y, r = e.z, g = -1;
  bool live = ref != SENTINEL;  // no early return: every thread reaches the carry below
  float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
  Ends E{};
  int32_t o_r = -1, o_l = -1;  // other[r], other[l - 1]: a half-done split there
  if (live) {
    if (is_leaf(ref)) {
      lv.load(leaf_index(ref), lo, hi);
    } else {
      const float4* q = reinterpret_cast<const float4*>(nodes + ref);
      lo = q[0];
      hi = q[1];
    }
    set_left(E, keys, l, mask);
    set_right(E, keys, r, last, mask);
    o_r = r < last ? other[r] : -1;
    o_l = l > 0 ? other[l - 1] : -1;
  }
  while (live) {
    const bool is_left = left_side(l, r, last, E.dr, E.dl);
    if (g >= 0) {  // finished in this launch: write it under its number
      ref = is_left ? r : l;
      write_node(nodes, ref, lo, hi, left_ref(l, g), rope_of(r, last, E.cr, E.dr, E.dr1));
      if (E.cl && E.cr) set_root[set_of(keys, l, set_shift)] = ref;  // spans a whole set
      g = -1;
    }
    const int32_t par = is_left ? r : l - 1;
    if (par < f0 || par > f1 - 2) {  // the split is a frame edge: to the next level
      pend_out[size_t(blockIdx.x) * 2 + (is_left ? 1 : 0)] = make_int4(ref, l, r, 0);
      break;
    }
    int32_t bound = is_left ? o_r : o_l;  // the other child finished in an earlier launch
    int32_t who = -1;  // the sibling's thread, when it finished in this launch
    if (bound < 0) {
      const int32_t h = tab_slot(s_key, tab_log2, par);
      if (h < 0) {
        atomicOr(err, STATUS_TREE);
        break;
      }
      // for the sibling, should this be the first arrival: box and outer end
      SibRec& mine = s_rec[threadIdx.x];
      mine.lox = lo.x; mine.loy = lo.y; mine.loz = lo.z;
      mine.hix = hi.x; mine.hiy = hi.y; mine.hiz = hi.z;
      mine.d0 = is_left ? E.dl : E.dr;
      mine.d1 = E.dr1;
      mine.o = is_left ? o_l : o_r;
      mine.cut = is_left ? E.cl : E.cr;
      const int64_t v = (int64_t(threadIdx.x) << 32) | int64_t(uint32_t(is_left ? l : r));
      const int64_t got = __hip_atomic_exchange(s_val + h, v, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_WORKGROUP);
      if (got < 0) break;  // first arrival: the sibling finishes the parent (or later)
      bound = int32_t(uint32_t(got));
      who = int32_t(got >> 32);
      s_val[h] = -2;       // both children met here: nothing to carry on
    }
    if (is_left) r = bound;
    else l = bound;
    const int32_t sl = is_left ? par + 1 : l, sr = is_left ? r : par;
    if (sl < 0 || sr > last || sl > sr || l > par || par >= r ||
        who >= int32_t(blockDim.x)) {
      atomicOr(err, STATUS_TREE);
      break;
    }
    if (who >= 0) {  // the sibling's box and outer end, from its record
      const SibRec& sib = s_rec[who];
      grow(lo, hi, make_float4(sib.lox, sib.loy, sib.loz, 0.f),
           make_float4(sib.hix, sib.hiy, sib.hiz, 0.f));
      if (is_left) {  // the right end is now the sibling's right end
        E.dr = sib.d0;
        E.dr1 = sib.d1;
        E.cr = sib.cut != 0;
        o_r = sib.o;
      } else {        // the left end is now the sibling's left end
        E.dl = sib.d0;
        E.cl = sib.cut != 0;
        o_l = sib.o;
      }
      g = par;
      if (l == 0 && r == last) {  // the root, number 0
        write_node(nodes, 0, lo, hi, left_ref(l, g), SENTINEL);
        if (E.cl && E.cr) set_root[set_of(keys, l, set_shift)] = 0;
        break;
      }
      continue;
    }
    // the sibling's box, the keys around the new end and other[] at the new
    // node's candidate parent splits, loaded together (no branch between
    // the loads: a leaf is read as 32 bytes too)
    const bool sleaf = sl == sr;
    const float4* sp =
        sleaf ? lv.rec(sl) : reinterpret_cast<const float4*>(nodes + (is_left ? sl : sr));
    const float4 sa = sp[0], sb = sp[1];
    const int32_t x = bound;
    const uint64_t k0 = keys[x > 0 ? x - 1 : 0], k1 = keys[x];
    const uint64_t k2 = keys[x < last ? x + 1 : last], k3 = keys[x + 1 < last ? x + 2 : last];
    const int32_t ox = other[x < last ? x : 0], oxm = other[x > 0 ? x - 1 : 0];
    // both readings computed, one kept: selects, so that every load above
    // is issued before the first wait
    const uint64_t dr = x < last ? delta_of(k1, k2, x) : 0ull;
    const uint64_t dr1 = x + 1 < last ? delta_of(k2, k3, x + 1) : 0ull;
    const bool cr = x == last || ((k1 ^ k2) & mask) != 0;
    const uint64_t dl = x > 0 ? delta_of(k0, k1, x - 1) : 0ull;
    const bool cl = x == 0 || ((k0 ^ k1) & mask) != 0;
    E.dr = is_left ? dr : E.dr;  // the right end is now x
    E.dr1 = is_left ? dr1 : E.dr1;
    E.cr = is_left ? cr : E.cr;
    o_r = is_left ? (x < last ? ox : -1) : o_r;
    E.dl = is_left ? E.dl : dl;  // the left end is now x
    E.cl = is_left ? E.cl : cl;
    o_l = is_left ? o_l : (x > 0 ? oxm : -1);
    grow(lo, hi, sa, sleaf && Leaves::kPoint ? sa : sb);
    g = par;
    if (l == 0 && r == last) {  // the root, number 0
      write_node(nodes, 0, lo, hi, left_ref(l, g), SENTINEL);
      if (E.cl && E.cr) set_root[set_of(keys, l, set_shift)] = 0;
      break;
    }
  }
  // first arrivals nobody here completed: to other[], for a later level
  __syncthreads();
  for (uint32_t h = threadIdx.x; h < tab; h += blockDim.x) {
    const int32_t k = s_key[h];
    const int64_t v = s_val[h];
    if (k >= 0 && v >= 0) other[k] = int32_t(uint32_t(v));
  }
}

}  // namespace

int build_levels(uint32_t n) {
  int levels = 1;
  uint64_t frame = BUILD_LEAVES;
  while (frame < n) { frame <<= BUILD_FANOUT_LOG2; ++levels; }
  return levels;
}

// Level lv writes two entries per frame into a region the next level reads
// in whole blocks of BUILD_BLOCK entries (one block per next-level frame).
static size_t level_region(uint32_t frames) {
  return size_t((frames + (1u << BUILD_FANOUT_LOG2) - 1) >> BUILD_FANOUT_LOG2) * BUILD_BLOCK;
}

size_t build_pending_entries(uint32_t n) {
  size_t total = 0;
  uint64_t frame = BUILD_LEAVES;
  for (int lv = 1, levels = build_levels(n); lv <= levels; ++lv) {
    total += level_region(uint32_t((n + frame - 1) / frame));
    frame <<= BUILD_FANOUT_LOG2;
  }
  return total;
}

namespace {
// Hand-over entries one workgroup takes to the root.  Not more: the top
// climb is a chain of dependent memory round trips, and 1,024 entries on
// one CU took 120 us on the 2^24-point field where a level launch of four
// workgroups and a top block of 256 threads take 80 us.
constexpr uint32_t BUILD_TOP_ENTRIES = 256;

// log2 of the exchange table slots of a level block of `threads` threads
uint32_t level_tab_log2(uint32_t threads) {
  uint32_t t = 6;
  while ((1u << t) < threads * LEVEL_TAB_FACTOR) ++t;
  return t;
}

// FrameLeaves: the leaves as level 1 reads and writes them; Leaves: as the
// later levels read them
// n: the leaf count, or with n_dev an upper bound of the count held in
// device memory at *n_dev (the launches are sized for the bound; frames past
// the count exit at once)
template <class FrameLeaves, class Leaves>
void build_impl(const uint64_t* keys, int set_shift, FrameLeaves flv, Leaves lv, uint32_t n,
                const uint32_t* n_dev, Node* nodes, int32_t* other, int32_t* root,
                int4* pending, uint32_t* err, hipStream_t s, void (*after_level)(void*, int),
                void* arg) {
  if (n == 0) return;
  const int levels = build_levels(n);
  uint64_t frame = BUILD_LEAVES;
  const int4* pin = nullptr;
  int4* pout = pending;
  uint32_t entries = 0;  // hand-over entries the previous level wrote (its region)
  for (int lv_i = 1; lv_i <= levels; ++lv_i) {
    const uint32_t frames = uint32_t((n + frame - 1) / frame);
    if (lv_i == 1) {
      hipLaunchKernelGGL(k_build_frame<FrameLeaves>, dim3(frames), dim3(BUILD_BLOCK), 0, s, keys,
                         flv, n, n_dev, set_shift, nodes, other, root, pout, err);
    } else if (entries <= BUILD_TOP_ENTRIES) {
      // few enough nodes left for one workgroup: it climbs them all to the
      // root (one frame over every leaf), in place of the remaining levels
      const uint32_t threads = (entries + 63) / 64 * 64;
      const uint32_t tl = level_tab_log2(threads);
      hipLaunchKernelGGL(k_build_level<Leaves>, dim3(1), dim3(threads), level_lds(threads, tl), s,
                         keys,
                         lv, n, n_dev, uint64_t(n), entries, tl, set_shift, nodes, other, root,
                         pin, pout, err);
      if (after_level) after_level(arg, lv_i);
      return;
    } else {
      const uint32_t tl = level_tab_log2(BUILD_BLOCK);
      hipLaunchKernelGGL(k_build_level<Leaves>, dim3(frames), dim3(BUILD_BLOCK),
                         level_lds(BUILD_BLOCK, tl), s,
                         keys, lv, n, n_dev, frame, uint32_t(frames) * BUILD_BLOCK, tl, set_shift,
                         nodes, other, root, pin, pout, err);
    }
    if (after_level) after_level(arg, lv_i);
    pin = pout;
    entries = uint32_t(level_region(frames));
    pout += entries;
    frame <<= BUILD_FANOUT_LOG2;
  }
}

}  // namespace

void launch_build(const uint64_t* keys, int set_shift, const float* pts, const uint32_t* perm,
                  float4* leaf, int32_t* parent, int32_t* minlab, uint8_t* flag,
                  unsigned long long* bestcore, int32_t* labels, uint32_t* deg, uint32_t n,
                  Node* nodes, int32_t* other, int32_t* set_root, int4* pending, uint32_t* err,
                  hipStream_t s, void (*after_level)(void*, int), void* arg) {
  build_impl(keys, set_shift,
             GatherLeaves{pts, perm, n, leaf, parent, minlab, flag, bestcore, labels, deg},
             PointLeaves{leaf}, n, nullptr, nodes, other, set_root, pending, err, s, after_level,
             arg);
}

void launch_build_coded(uint64_t* keys, const uint32_t* bounds, const uint32_t* drop,
                        const float* pts, const uint32_t* perm, float4* leaf, int32_t* parent,
                        int32_t* minlab, uint8_t* flag, unsigned long long* bestcore,
                        int32_t* labels, uint32_t* deg, uint32_t n, Node* nodes, int32_t* other,
                        int32_t* root, int4* pending, uint32_t* err, hipStream_t s,
                        void (*after_level)(void*, int), void* arg) {
  GatherCoded g;
  static_cast<GatherLeaves&>(g) =
      GatherLeaves{pts, perm, n, leaf, parent, minlab, flag, bestcore, labels, deg};
  g.bounds = bounds;
  g.drop = drop;
  g.keys_out = keys;
  build_impl(keys, 64, g, PointLeaves{leaf}, n, nullptr, nodes, other, root, pending, err, s,
             after_level, arg);
}

void launch_build_boxes(const uint64_t* keys, int set_shift, Node* prims, uint32_t n_bound,
                        const uint32_t* n_dev, Node* nodes, int32_t* other, int32_t* set_root,
                        int4* pending, uint32_t* err, hipStream_t s) {
  build_impl(keys, set_shift, BoxLeaves{prims}, BoxLeaves{prims}, n_bound, n_dev, nodes, other,
             set_root, pending, err, s, nullptr, nullptr);
}

}  // namespace dbx
