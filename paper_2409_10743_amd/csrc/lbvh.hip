// Linear BVH over Morton-sorted leaves: Apetrei's bottom-up construction
// (section 4.2.1: faster than Karras' build) followed by a separate pass that
// sets the ropes used by the stackless traversal.
//
// Construction.  delta(i) measures how different leaves i and i+1 are: the
// XOR of their codes, and for equal codes the XOR of the positions i^(i+1)
// (ranked below every differing pair), which splits runs of equal codes
// evenly.  One thread per leaf climbs: a node covering leaves [l, r] is the
// left child of internal node r when l = 0 or (r < n-1 and delta(r) <
// delta(l-1)), otherwise the right child of internal node l-1.  Ties go to
// the smaller boundary index, a strict order, so every internal node gets
// exactly one left and one right child.  Each child swaps its outer range
// bound into a per-parent slot (initially -1) with one acquire-release
// exchange: the first to arrive leaves, the second learns the parent's full
// range from the value it gets back, sees its sibling's box (release/acquire
// order), writes the parent's box and climbs on.
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

__global__ __launch_bounds__(256) void k_build(const uint64_t* __restrict__ keys,
                                              const float4* __restrict__ leaf, uint32_t n,
                                              Node* nodes, int32_t* right, int32_t* other,
                                              int32_t* root, uint32_t* err) {
  // nodes/right/other are written and read by different threads within this
  // kernel, ordered by the exchange below: no __restrict__ on them
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (n == 1) { *root = leaf_ref(0); return; }
  const int32_t last = int32_t(n) - 1;
  float4 p = leaf[i];
  float lox = p.x, loy = p.y, loz = p.z, hix = p.x, hiy = p.y, hiz = p.z;
  int32_t l = int32_t(i), r = int32_t(i);
  int32_t node = leaf_ref(int32_t(i));
  for (;;) {
    const bool is_left = (l == 0) || (r != last && delta(keys, r) < delta(keys, l - 1));
    const int32_t par = is_left ? r : l - 1;
    if (is_left) nodes[par].left = node;
    else right[par] = node;
    const int32_t bound = __hip_atomic_exchange(other + par, is_left ? l : r, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (bound < 0) return;  // first arrival: the sibling finishes the parent
    int32_t sib;
    if (is_left) { r = bound; sib = right[par]; }
    else { l = bound; sib = nodes[par].left; }
    const bool sib_ok = is_leaf(sib) ? leaf_index(sib) <= last : (sib >= 0 && sib < last);
    if (!sib_ok || l < 0 || r > last || l > r) { atomicOr(err, STATUS_TREE); return; }
    float slx, sly, slz, shx, shy, shz;
    if (is_leaf(sib)) {
      float4 q = leaf[leaf_index(sib)];
      slx = shx = q.x; sly = shy = q.y; slz = shz = q.z;
    } else {
      const Node& s = nodes[sib];
      slx = s.lox; sly = s.loy; slz = s.loz; shx = s.hix; shy = s.hiy; shz = s.hiz;
    }
    lox = fminf(lox, slx); loy = fminf(loy, sly); loz = fminf(loz, slz);
    hix = fmaxf(hix, shx); hiy = fmaxf(hiy, shy); hiz = fmaxf(hiz, shz);
    Node& pn = nodes[par];
    pn.lox = lox; pn.loy = loy; pn.loz = loz;
    pn.hix = hix; pn.hiy = hiy; pn.hiz = hiz;
    pn.rope = r;  // range end, turned into the rope by k_ropes
    node = par;
    if (l == 0 && r == last) { *root = par; return; }
  }
}

__global__ __launch_bounds__(256) void k_ropes(Node* __restrict__ nodes, float4* __restrict__ leaf,
                                              const int32_t* __restrict__ right, uint32_t n,
                                              uint32_t* __restrict__ err) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < 2 || t >= 2 * n - 1) return;
  const int32_t last = int32_t(n) - 1;
  if (t < n - 1) {
    int32_t r = nodes[t].rope;
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

void launch_build(const uint64_t* keys, const float4* leaf, uint32_t n, Node* nodes,
                  int32_t* right, int32_t* other, int32_t* root, uint32_t* err, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_build, dim3((n + 255) / 256), dim3(256), 0, s, keys, leaf, n, nodes,
                     right, other, root, err);
}

void launch_ropes(Node* nodes, float4* leaf, const int32_t* right, uint32_t n, uint32_t* err,
                  hipStream_t s) {
  if (n < 2) return;
  uint32_t t = 2 * n - 1;
  hipLaunchKernelGGL(k_ropes, dim3((t + 255) / 256), dim3(256), 0, s, nodes, leaf, right, n, err);
}

}  // namespace dbx
