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
#include "pipeline.hpp"

namespace dbx {

namespace {

__device__ __forceinline__ uint64_t delta(const uint64_t* __restrict__ keys, int32_t i) {
  uint64_t a = keys[i], b = keys[i + 1];
  return a == b ? uint64_t(uint32_t(i) ^ uint32_t(i + 1)) : ((a ^ b) + (1ull << 32));
}

// One climb step at interior parent `par` of the node `node` = [l, r]:
// link it, exchange, and, for the second arrival, finish the parent.
// Returns false when the climb stops here (first arrival, or a bad tree).
__device__ __forceinline__ bool climb_step(const float4* __restrict__ leaf, Node* nodes,
                                           int32_t* right, int32_t* other, int32_t* rend,
                                           uint32_t* err,
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
    float4 q = leaf[leaf_index(sib)];
    slx = shx = q.x; sly = shy = q.y; slz = shz = q.z;
  } else {
    const Node& sn = nodes[sib];
    slx = sn.lox; sly = sn.loy; slz = sn.loz; shx = sn.hix; shy = sn.hiy; shz = sn.hiz;
  }
  lox = fminf(lox, slx); loy = fminf(loy, sly); loz = fminf(loz, slz);
  hix = fmaxf(hix, shx); hiy = fmaxf(hiy, shy); hiz = fmaxf(hiz, shz);
  Node& pn = nodes[par];
  pn.lox = lox; pn.loy = loy; pn.loz = loz;
  pn.hix = hix; pn.hiy = hiy; pn.hiz = hiz;
  rend[par] = r;  // range end, turned into the rope by k_ropes
  node = par;
  return true;
}

// Level 1 of the build, all in LDS: one workgroup per 256-leaf frame.  The
// frame's delta values, leaves, exchange slots, child references and boxes
// live in LDS (the exchange is an LDS swap); at the end the frame's
// internal nodes go out to memory in one coalesced pass, together with the
// state later levels need: the exchange slot of every split in the frame
// (-1 for the frame's right edge), child references set so far, and the
// range end of every finished node.
__global__ __launch_bounds__(BUILD_BLOCK) void k_build_frame(
    const uint64_t* __restrict__ keys, const float4* __restrict__ leaf, uint32_t n,
    Node* __restrict__ nodes, int32_t* __restrict__ right, int32_t* __restrict__ other,
    int32_t* __restrict__ rend, int32_t* __restrict__ root, int4* __restrict__ pend_out,
    uint32_t* __restrict__ err) {
  __shared__ uint64_t s_delta[BUILD_LEAVES + 1];  // boundary f0-1+j at j
  __shared__ float4 s_leaf[BUILD_LEAVES];
  __shared__ float4 s_lo[BUILD_LEAVES], s_hi[BUILD_LEAVES];
  __shared__ int32_t s_other[BUILD_LEAVES], s_left[BUILD_LEAVES], s_right[BUILD_LEAVES],
      s_end[BUILD_LEAVES];
  const int32_t t = threadIdx.x;
  const int32_t last = int32_t(n) - 1;
  const int32_t f0 = int32_t(blockIdx.x) * BUILD_LEAVES;
  const int32_t f1 = min(f0 + BUILD_LEAVES, int32_t(n));
  const int32_t m = f1 - f0;
  for (int32_t j = t; j <= m; j += BUILD_BLOCK) {
    const int32_t b = f0 - 1 + j;
    s_delta[j] = (b >= 0 && b < last) ? delta(keys, b) : 0ull;
  }
  if (t < m) s_leaf[t] = leaf[f0 + t];
  s_other[t] = -1;
  s_left[t] = SENTINEL;
  s_right[t] = SENTINEL;
  s_end[t] = -1;
  __syncthreads();
  if (t < m) {
    if (n == 1) {
      *root = leaf_ref(0);
    } else {
      int32_t node = leaf_ref(f0 + t), l = f0 + t, r = f0 + t;
      float4 lo = s_leaf[t], hi = lo;
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
        const float4 shi = is_leaf(sib) ? s_leaf[si] : s_hi[si];
        lo.x = fminf(lo.x, slo.x); lo.y = fminf(lo.y, slo.y); lo.z = fminf(lo.z, slo.z);
        hi.x = fmaxf(hi.x, shi.x); hi.y = fmaxf(hi.y, shi.y); hi.z = fmaxf(hi.z, shi.z);
        s_lo[k] = lo;
        s_hi[k] = hi;
        s_end[k] = r;
        node = par;
        if (l == 0 && r == last) { *root = par; break; }
      }
    }
  }
  __syncthreads();
  // write out split f0 + t (the frame's right edge split only resets its slot)
  const int32_t p = f0 + t;
  if (t < m && p < last) {
    if (t == m - 1) {
      other[p] = -1;
    } else {
      other[p] = s_other[t];
      if (s_right[t] != SENTINEL) right[p] = s_right[t];
      if (s_end[t] >= 0) {
        const float4 lo = s_lo[t], hi = s_hi[t];
        reinterpret_cast<float4*>(nodes + p)[0] =
            make_float4(lo.x, lo.y, lo.z, __int_as_float(s_left[t]));
        reinterpret_cast<float4*>(nodes + p)[1] = make_float4(hi.x, hi.y, hi.z, 0.0f);
        rend[p] = s_end[t];
      } else if (s_left[t] != SENTINEL) {
        nodes[p].left = s_left[t];
      }
    }
  }
}

// Levels k > 1 of the build: thread = one of the 2 * 128 nodes handed up by
// the 128 level-(k-1) frames inside this block's frame.  nodes/right/other
// are written and read by different threads of the same launch, ordered by
// the exchange: no __restrict__ on them.
__global__ __launch_bounds__(BUILD_BLOCK) void k_build_level(
    const uint64_t* __restrict__ keys, const float4* __restrict__ leaf, uint32_t n, int level,
    Node* nodes, int32_t* right, int32_t* other, int32_t* rend, int32_t* root,
    const int4* __restrict__ pend_in, int4* __restrict__ pend_out, uint32_t* err) {
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
      const float4 p = leaf[leaf_index(node)];
      lox = hix = p.x; loy = hiy = p.y; loz = hiz = p.z;
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
    if (!climb_step(leaf, nodes, right, other, rend, err, last, is_left, par, node, l, r, lox,
                    loy, loz, hix, hiy, hiz))
      return;
    if (l == 0 && r == last) { *root = node; return; }
  }
}

__global__ __launch_bounds__(256) void k_ropes(Node* __restrict__ nodes, float4* __restrict__ leaf,
                                              const int32_t* __restrict__ right,
                                              const int32_t* __restrict__ rend, uint32_t n,
                                              uint32_t* __restrict__ err) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < 2 || t >= 2 * n - 1) return;
  const int32_t last = int32_t(n) - 1;
  if (t < n - 1) {
    int32_t r = rend[t];
    if (r < 0 || r > last) {  // only if the build failed
      atomicOr(err, STATUS_TREE);
      r = last;
    }
    nodes[t].rope = (r == last) ? SENTINEL : right[r];
  } else {
    int32_t j = int32_t(t - (n - 1));
    leaf[j].w = __int_as_float(j == last ? SENTINEL : right[j]);
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

void launch_build(const uint64_t* keys, const float4* leaf, uint32_t n, Node* nodes,
                  int32_t* right, int32_t* other, int32_t* rend, int32_t* root, int4* pending,
                  uint32_t* err, hipStream_t s) {
  if (n == 0) return;
  const int levels = build_levels(n);
  uint64_t frame = BUILD_LEAVES;
  const int4* pin = nullptr;
  int4* pout = pending;
  for (int lv = 1; lv <= levels; ++lv) {
    const uint32_t frames = uint32_t((n + frame - 1) / frame);
    if (lv == 1)
      hipLaunchKernelGGL(k_build_frame, dim3(frames), dim3(BUILD_BLOCK), 0, s, keys, leaf, n,
                         nodes, right, other, rend, root, pout, err);
    else
      hipLaunchKernelGGL(k_build_level, dim3(frames), dim3(BUILD_BLOCK), 0, s, keys, leaf, n, lv,
                         nodes, right, other, rend, root, pin, pout, err);
    pin = pout;
    pout += level_region(frames);
    frame <<= BUILD_FANOUT_LOG2;
  }
}

void launch_ropes(Node* nodes, float4* leaf, const int32_t* right, const int32_t* rend,
                  uint32_t n, uint32_t* err, hipStream_t s) {
  if (n < 2) return;
  uint32_t t = 2 * n - 1;
  hipLaunchKernelGGL(k_ropes, dim3((t + 255) / 256), dim3(256), 0, s, nodes, leaf, right, rend, n,
                     err);
}

}  // namespace dbx
