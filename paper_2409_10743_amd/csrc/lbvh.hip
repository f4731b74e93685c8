// Linear BVH over Morton-sorted leaves: Apetrei's bottom-up construction
// (section 4.2.1: faster than Karras' build) followed by a separate pass that
// sets the ropes used by the stackless traversal.
//
// Construction.  delta(i) measures how different leaves i and i+1 are: the
// XOR of their codes, and for equal codes the XOR of the positions i^(i+1)
// (ranked below every differing pair), which splits runs of equal codes
// evenly.  A node covering leaves [l, r] is the left child of internal node
// r when l = 0 or (r < n-1 and delta(r) < delta(l-1)), otherwise the right
// child of internal node l-1.  Ties go to the smaller boundary index, a
// strict order, so every internal node gets exactly one left and one right
// child.  Each child swaps its outer range bound into a per-parent slot
// (initially -1) with one acquire-release exchange: the first to arrive
// leaves, the second learns the parent's full range from the value it gets
// back, sees its sibling's box, writes the parent's box and climbs on.
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
// Ropes.  The rope of a node is where a stackless, left-first pre-order
// walk goes after the node's subtree: the right child of the lowest ancestor
// holding the node in its left subtree.  That ancestor is internal node r,
// r being the last leaf the node covers, so rope = right(r), or the sentinel
// when r = n-1 (the right-most path).  No reordering of nodes is needed.
// Batched sets: the keys carry the set id in their top bits (`set_shift`),
// so a boundary between sets has a larger delta than any boundary inside a
// set and every set is one complete subtree.  Ropes are cut at set ends
// (sets overlap in space, so boxes would not keep a walk inside its set),
// and the node spanning exactly a set is recorded as that set's root.  With
// no set bits (set_shift = 64) the only such node is the root.
// Level 1 knows right(r) whenever that child was finished inside the frame,
// which holds for nearly every node: it writes those leaves and nodes whole,
// once.  The rest (nodes whose r is the frame's last leaf or whose right(r)
// crosses the frame edge, and nodes finished at higher levels) are listed
// and patched by k_ropes after the last level.
#include <algorithm>

#include "pipeline.hpp"

namespace dbx {

namespace {

// Leaves are points (FDBSCAN: float4 x, y, z, rope) or boxes (DenseBox
// primitives: Node records whose `left` holds the payload).
struct PointLeaves {
  float4* leaf;
  __device__ void load(int32_t j, float4& lo, float4& hi) const { lo = hi = leaf[j]; }
  // whole record, coalesced, when the frame writes its leaves out
  __device__ void write_out(int32_t j, const float4& lo, const float4&, int32_t rope) const {
    leaf[j] = make_float4(lo.x, lo.y, lo.z, __int_as_float(rope));
  }
  __device__ void set_rope(int32_t j, int32_t rope) const { leaf[j].w = __int_as_float(rope); }
};
struct BoxLeaves {
  Node* prim;
  __device__ void load(int32_t j, float4& lo, float4& hi) const {
    const float4* q = reinterpret_cast<const float4*>(prim + j);
    lo = q[0];
    hi = q[1];
  }
  __device__ void write_out(int32_t j, const float4&, const float4&, int32_t rope) const {
    prim[j].rope = rope;
  }
  __device__ void set_rope(int32_t j, int32_t rope) const { prim[j].rope = rope; }
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

__device__ __forceinline__ uint64_t delta(const uint64_t* __restrict__ keys, int32_t i) {
  uint64_t a = keys[i], b = keys[i + 1];
  return a == b ? uint64_t(uint32_t(i) ^ uint32_t(i + 1)) : ((a ^ b) + (1ull << 32));
}

// One climb step at interior parent `par` of the node `node` = [l, r]:
// link it, exchange, and, for the second arrival, finish the parent.
// Returns false when the climb stops here (first arrival, or a bad tree).
// Fix-up list: each level-1 frame owns FIX_PER_FRAME entries and a count.
// An internal node p goes into the region of the frame holding leaf p; a
// frame holds at most 256 leaves and 256 splits, so its region never
// overflows for a well-formed tree.  Nodes finished above level 1 take a
// slot with an atomic on their frame's count: these atomics are spread over
// all frames, never one shared counter.
struct FixList {
  int2* entries;
  uint32_t* cnt;
  uint32_t* err;
  __device__ void push(int32_t p, int2 e) const {
    const uint32_t f = uint32_t(p) / BUILD_LEAVES;
    const uint32_t k = atomicAdd(cnt + f, 1u);
    if (k < FIX_PER_FRAME) entries[size_t(f) * FIX_PER_FRAME + k] = e;
    else atomicOr(err, STATUS_TREE);
  }
};

template <class Leaves>
__device__ __forceinline__ bool climb_step(const Leaves& lv, Node* nodes,
                                           int32_t* right, int32_t* other, const FixList& fx,
                                           uint32_t* err, const uint64_t* keys,
                                           int set_shift, int32_t* set_root,
                                           int32_t last, bool is_left, int32_t par,
                                           int32_t& node, int32_t& l, int32_t& r, float& lox,
                                           float& loy, float& loz, float& hix, float& hiy,
                                           float& hiz) {
  if (is_left) nodes[par].left = node;
  else right[par] = node;
  const int32_t bound = __hip_atomic_exchange(other + par, is_left ? l : r, __ATOMIC_ACQ_REL,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
  if (bound < 0) return false;  // first arrival: the sibling finishes the parent
  int32_t sib;
  if (is_left) { r = bound; sib = right[par]; }
  else { l = bound; sib = nodes[par].left; }
  const bool sib_ok = is_leaf(sib) ? leaf_index(sib) <= last : (sib >= 0 && sib < last);
  if (!sib_ok || l < 0 || r > last || l > r) { atomicOr(err, STATUS_TREE); return false; }
  float slx, sly, slz, shx, shy, shz;
  if (is_leaf(sib)) {
    float4 ql, qh;
    lv.load(leaf_index(sib), ql, qh);
    slx = ql.x; sly = ql.y; slz = ql.z; shx = qh.x; shy = qh.y; shz = qh.z;
  } else {
    const Node& sn = nodes[sib];
    slx = sn.lox; sly = sn.loy; slz = sn.loz; shx = sn.hix; shy = sn.hiy; shz = sn.hiz;
  }
  lox = fminf(lox, slx); loy = fminf(loy, sly); loz = fminf(loz, slz);
  hix = fmaxf(hix, shx); hiy = fmaxf(hiy, shy); hiz = fmaxf(hiz, shz);
  Node& pn = nodes[par];
  pn.lox = lox; pn.loy = loy; pn.loz = loz;
  pn.hix = hix; pn.hiy = hiy; pn.hiz = hiz;
  fx.push(par, make_int2(par, r));  // rope set by k_ropes
  node = par;
  const uint64_t mask = set_mask_of(set_shift);
  if ((l == 0 || set_cut(keys, l - 1, mask)) && (r == last || set_cut(keys, r, mask)))
    set_root[set_of(keys, l, set_shift)] = par;
  return true;
}

// Level 1 of the build, all in LDS: one workgroup per 256-leaf frame.  The
// frame's delta values, leaves, exchange slots, child references and boxes
// live in LDS (the exchange is an LDS swap); at the end the frame's
// internal nodes go out to memory in one coalesced pass, together with the
// state later levels need: the exchange slot of every split in the frame
// (-1 for the frame's right edge), child references set so far, and the
// range end of every finished node.
// Appends one entry per lane with `want` set to the frame's own list
// (count in LDS); all lanes of the wave call it.
__device__ __forceinline__ void wave_append(int2* list, uint32_t* lds_count, bool want, int2 e) {
  const uint64_t m = __ballot(want);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll(static_cast<long long>(m)) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(lds_count, uint32_t(__popcll(m)));
  base = __shfl(base, leader, 64);
  const uint64_t below = lane ? (m & (~0ull >> (64 - lane))) : 0ull;
  if (want) list[base + __popcll(below)] = e;
}

template <class Leaves>
__global__ __launch_bounds__(BUILD_BLOCK) void k_build_frame(
    const uint64_t* __restrict__ keys, Leaves lv, uint32_t n, int set_shift,
    Node* __restrict__ nodes, int32_t* __restrict__ right, int32_t* __restrict__ other,
    int32_t* __restrict__ set_root, int4* __restrict__ pend_out, int2* __restrict__ fix_frame,
    uint32_t* __restrict__ fix_cnt, uint32_t* __restrict__ err) {
  __shared__ uint64_t s_delta[BUILD_LEAVES + 1];  // boundary f0-1+j at j
  __shared__ uint32_t s_fix_cnt;
  __shared__ float4 s_leaf[BUILD_LEAVES], s_leafhi[BUILD_LEAVES];
  __shared__ float4 s_lo[BUILD_LEAVES], s_hi[BUILD_LEAVES];
  __shared__ int32_t s_other[BUILD_LEAVES], s_left[BUILD_LEAVES], s_right[BUILD_LEAVES],
      s_end[BUILD_LEAVES];
  __shared__ uint8_t s_cut[BUILD_LEAVES + 1];  // a set ends at boundary f0-1+j
  const int32_t t = threadIdx.x;
  const int32_t last = int32_t(n) - 1;
  const int32_t f0 = int32_t(blockIdx.x) * BUILD_LEAVES;
  const int32_t f1 = min(f0 + BUILD_LEAVES, int32_t(n));
  const int32_t m = f1 - f0;
  const uint64_t mask = set_mask_of(set_shift);
  for (int32_t j = t; j <= m; j += BUILD_BLOCK) {
    const int32_t b = f0 - 1 + j;
    const bool ok = b >= 0 && b < last;
    s_delta[j] = ok ? delta(keys, b) : 0ull;
    s_cut[j] = ok ? set_cut(keys, b, mask) : 1;
  }
  if (t < m) lv.load(f0 + t, s_leaf[t], s_leafhi[t]);
  s_other[t] = -1;
  s_left[t] = SENTINEL;
  s_right[t] = SENTINEL;
  s_end[t] = -1;
  if (t == 0) s_fix_cnt = 0;
  __syncthreads();
  // does [l, r] span a whole set? (l - 1 and r are set ends; both in frame)
  auto spans = [&](int32_t l, int32_t r) { return s_cut[l - f0] && s_cut[r - f0 + 1]; };
  if (t < m) {
    if (spans(f0 + t, f0 + t)) set_root[set_of(keys, f0 + t, set_shift)] = leaf_ref(f0 + t);
    if (n > 1) {
      int32_t node = leaf_ref(f0 + t), l = f0 + t, r = f0 + t;
      float4 lo = s_leaf[t], hi = s_leafhi[t];
      for (;;) {
        const bool is_left =
            (l == 0) || (r != last && s_delta[r - f0 + 1] < s_delta[l - 1 - f0 + 1]);
        const int32_t par = is_left ? r : l - 1;
        if (par < f0 || par > f1 - 2) {  // frame edge: hand over to level 2
          pend_out[size_t(blockIdx.x) * 2 + (is_left ? 1 : 0)] = make_int4(node, l, r, 0);
          break;
        }
        const int32_t k = par - f0;
        if (is_left) s_left[k] = node;
        else s_right[k] = node;
        const int32_t bound = __hip_atomic_exchange(s_other + k, is_left ? l : r,
                                                    __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (bound < 0) break;
        int32_t sib;
        if (is_left) { r = bound; sib = s_right[k]; }
        else { l = bound; sib = s_left[k]; }
        const int32_t si = is_leaf(sib) ? leaf_index(sib) - f0 : sib - f0;
        if (si < 0 || si >= m || l > r) { atomicOr(err, STATUS_TREE); break; }
        const float4 slo = is_leaf(sib) ? s_leaf[si] : s_lo[si];
        const float4 shi = is_leaf(sib) ? s_leafhi[si] : s_hi[si];
        lo.x = fminf(lo.x, slo.x); lo.y = fminf(lo.y, slo.y); lo.z = fminf(lo.z, slo.z);
        hi.x = fmaxf(hi.x, shi.x); hi.y = fmaxf(hi.y, shi.y); hi.z = fmaxf(hi.z, shi.z);
        s_lo[k] = lo;
        s_hi[k] = hi;
        s_end[k] = r;
        node = par;
        if (spans(l, r)) set_root[set_of(keys, l, set_shift)] = par;
        if (l == 0 && r == last) break;
      }
    }
  }
  __syncthreads();
  // Write out split f0 + t (internal node) and leaf f0 + t with their ropes
  // where right(r) is known here; the frame's right edge split only resets
  // its exchange slot for the next level.
  const int32_t p = f0 + t;
  // right child of split q if it was finished in this frame, else -2
  auto known_right = [&](int32_t q) -> int32_t {
    if (q == last || s_cut[q - f0 + 1]) return SENTINEL;  // right-most path of the set
    if (q < f0 || q > f1 - 2) return -2;
    return s_right[q - f0] != SENTINEL ? s_right[q - f0] : -2;
  };
  bool fix_leaf = false, fix_node = false;
  int32_t node_end = -1;
  if (t < m && n > 1) {
    const int32_t lr = known_right(p);
    lv.write_out(p, s_leaf[t], s_leafhi[t], lr == -2 ? SENTINEL : lr);
    fix_leaf = lr == -2;
    if (p < last) {
      if (t == m - 1) {
        other[p] = -1;
      } else {
        other[p] = s_other[t];
        if (s_right[t] != SENTINEL) right[p] = s_right[t];
        if (s_end[t] >= 0) {
          node_end = s_end[t];
          const int32_t nr = known_right(node_end);
          fix_node = nr == -2;
          const float4 lo = s_lo[t], hi = s_hi[t];
          reinterpret_cast<float4*>(nodes + p)[0] =
              make_float4(lo.x, lo.y, lo.z, __int_as_float(s_left[t]));
          reinterpret_cast<float4*>(nodes + p)[1] =
              make_float4(hi.x, hi.y, hi.z, __int_as_float(nr == -2 ? SENTINEL : nr));
        } else if (s_left[t] != SENTINEL) {
          nodes[p].left = s_left[t];
        }
      }
    }
  }
  int2* mine = fix_frame + size_t(blockIdx.x) * FIX_PER_FRAME;
  wave_append(mine, &s_fix_cnt, fix_leaf, make_int2(leaf_ref(p), p));
  wave_append(mine, &s_fix_cnt, fix_node, make_int2(p, node_end));
  __syncthreads();
  if (t == 0) fix_cnt[blockIdx.x] = s_fix_cnt;  // later levels add to it
}

// Levels k > 1 of the build: thread = one of the 2 * 128 nodes handed up by
// the 128 level-(k-1) frames inside this block's frame.  nodes/right/other
// are written and read by different threads of the same launch, ordered by
// the exchange: no __restrict__ on them.
template <class Leaves>
__global__ __launch_bounds__(BUILD_BLOCK) void k_build_level(
    const uint64_t* __restrict__ keys, Leaves lv, uint32_t n, int level, int set_shift,
    Node* nodes, int32_t* right, int32_t* other, int32_t* set_root,
    const int4* __restrict__ pend_in, int4* __restrict__ pend_out, int2* fix_frame,
    uint32_t* fix_cnt, uint32_t* err) {
  const FixList fx{fix_frame, fix_cnt, err};
  const int32_t last = int32_t(n) - 1;
  const uint64_t frame = uint64_t(BUILD_LEAVES) << (BUILD_FANOUT_LOG2 * (level - 1));
  const int64_t f0 = int64_t(blockIdx.x) * int64_t(frame);
  const int64_t f1 = min(f0 + int64_t(frame), int64_t(n));
  int32_t node, l, r;
  float lox, loy, loz, hix, hiy, hiz;
  {
    const int4 e = pend_in[size_t(blockIdx.x) * BUILD_BLOCK + threadIdx.x];
    node = e.x;
    if (node == SENTINEL) return;
    l = e.y;
    r = e.z;
    if (is_leaf(node)) {
      float4 ql, qh;
      lv.load(leaf_index(node), ql, qh);
      lox = ql.x; loy = ql.y; loz = ql.z; hix = qh.x; hiy = qh.y; hiz = qh.z;
    } else {
      const Node& nd = nodes[node];
      lox = nd.lox; loy = nd.loy; loz = nd.loz; hix = nd.hix; hiy = nd.hiy; hiz = nd.hiz;
    }
  }
  for (;;) {
    const bool is_left = (l == 0) || (r != last && delta(keys, r) < delta(keys, l - 1));
    const int32_t par = is_left ? r : l - 1;
    if (par < f0 || par > f1 - 2) {
      // the split is a frame edge: hand the node to the next level
      pend_out[size_t(blockIdx.x) * 2 + (is_left ? 1 : 0)] = make_int4(node, l, r, 0);
      return;
    }
    if (!climb_step(lv, nodes, right, other, fx, err, keys, set_shift, set_root, last,
                    is_left, par, node, l, r, lox, loy, loz, hix, hiy, hiz))
      return;
    if (l == 0 && r == last) return;
  }
}

// One wave per level-1 frame: set the ropes of the frame's fix-up entries.
template <class Leaves>
__global__ __launch_bounds__(256) void k_ropes(Node* __restrict__ nodes, Leaves lv,
                                              const uint64_t* __restrict__ keys, int set_shift,
                                              const int32_t* __restrict__ right,
                                              const int2* __restrict__ fix_frame,
                                              const uint32_t* __restrict__ fix_cnt, uint32_t n,
                                              uint32_t* __restrict__ err) {
  const uint32_t frames = (n + BUILD_LEAVES - 1) / BUILD_LEAVES;
  const uint32_t f = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (f >= frames) return;
  const uint32_t count = min(fix_cnt[f], uint32_t(FIX_PER_FRAME));
  const int2* list = fix_frame + size_t(f) * FIX_PER_FRAME;
  const int32_t last = int32_t(n) - 1;
  const uint64_t mask = set_mask_of(set_shift);
  for (uint32_t k = threadIdx.x & 63; k < count; k += 64) {
    const int2 e = list[k];
    int32_t r = e.y;
    if (r < 0 || r > last) {  // only if the build failed
      atomicOr(err, STATUS_TREE);
      r = last;
    }
    const int32_t rope = (r == last || set_cut(keys, r, mask)) ? SENTINEL : right[r];
    if (is_leaf(e.x)) lv.set_rope(leaf_index(e.x), rope);
    else nodes[e.x].rope = rope;
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
template <class Leaves>
void build_impl(const uint64_t* keys, int set_shift, Leaves lv, uint32_t n, Node* nodes,
                int32_t* right, int32_t* other, int32_t* root, int4* pending, int2* fixups,
                uint32_t* fix_cnt, uint32_t* err, hipStream_t s, void (*after_level)(void*, int),
                void* arg) {
  if (n == 0) return;
  const int levels = build_levels(n);
  uint64_t frame = BUILD_LEAVES;
  const int4* pin = nullptr;
  int4* pout = pending;
  for (int lv_i = 1; lv_i <= levels; ++lv_i) {
    const uint32_t frames = uint32_t((n + frame - 1) / frame);
    if (lv_i == 1)
      hipLaunchKernelGGL(k_build_frame<Leaves>, dim3(frames), dim3(BUILD_BLOCK), 0, s, keys, lv,
                         n, set_shift, nodes, right, other, root, pout, fixups, fix_cnt, err);
    else
      hipLaunchKernelGGL(k_build_level<Leaves>, dim3(frames), dim3(BUILD_BLOCK), 0, s, keys, lv,
                         n, lv_i, set_shift, nodes, right, other, root, pin, pout, fixups,
                         fix_cnt, err);
    if (after_level) after_level(arg, lv_i);
    pin = pout;
    pout += level_region(frames);
    frame <<= BUILD_FANOUT_LOG2;
  }
}

template <class Leaves>
void ropes_impl(Node* nodes, Leaves lv, const uint64_t* keys, int set_shift,
                const int32_t* right, const int2* fixups, const uint32_t* fix_cnt, uint32_t n,
                uint32_t* err, hipStream_t s) {
  if (n < 2) return;
  const uint32_t frames = (n + BUILD_LEAVES - 1) / BUILD_LEAVES;
  hipLaunchKernelGGL(k_ropes<Leaves>, dim3((frames + 3) / 4), dim3(256), 0, s, nodes, lv, keys,
                     set_shift, right, fixups, fix_cnt, n, err);
}
}  // namespace

void launch_build(const uint64_t* keys, int set_shift, float4* leaf, uint32_t n, Node* nodes,
                  int32_t* right, int32_t* other, int32_t* set_root, int4* pending,
                  int2* fixups, uint32_t* fix_cnt, uint32_t* err, hipStream_t s,
                  void (*after_level)(void*, int), void* arg) {
  build_impl(keys, set_shift, PointLeaves{leaf}, n, nodes, right, other, set_root, pending,
             fixups, fix_cnt, err, s, after_level, arg);
}

void launch_build_boxes(const uint64_t* keys, Node* prims, uint32_t n, Node* nodes,
                        int32_t* right, int32_t* other, int32_t* root, int4* pending,
                        int2* fixups, uint32_t* fix_cnt, uint32_t* err, hipStream_t s) {
  build_impl(keys, 64, BoxLeaves{prims}, n, nodes, right, other, root, pending, fixups, fix_cnt,
             err, s, nullptr, nullptr);
}

void launch_ropes(const uint64_t* keys, int set_shift, Node* nodes, float4* leaf,
                  const int32_t* right, const int2* fixups, const uint32_t* fix_cnt, uint32_t n,
                  uint32_t* err, hipStream_t s) {
  ropes_impl(nodes, PointLeaves{leaf}, keys, set_shift, right, fixups, fix_cnt, n, err, s);
}

void launch_ropes_boxes(const uint64_t* keys, Node* nodes, Node* prims, const int32_t* right,
                        const int2* fixups, const uint32_t* fix_cnt, uint32_t n, uint32_t* err,
                        hipStream_t s) {
  ropes_impl(nodes, BoxLeaves{prims}, keys, 64, right, fixups, fix_cnt, n, err, s);
}

}  // namespace dbx
