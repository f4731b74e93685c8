// Stackless BVH traversals with fused callbacks (sections 4.1, 4.2, 4.3.3).
//
// One lane per query, queries in Morton order so the 64 lanes of a wave
// walk nearby parts of the tree (section 3.2).  The walk is a left-first
// pre-order over ropes (section 4.2.1): at an internal node whose box is
// within eps of the query go to its left child, otherwise follow its rope;
// at a leaf test the point, then follow the leaf's rope; stop at the
// sentinel.  Nothing is stored per neighbour: the work on a found pair is
// done on the spot (the "callback"), so memory stays O(n).
//
//  * counting (Algorithm 2, preprocessing; only needed when minPts > 2):
//    walk from the root and stop as soon as minPts neighbours are found
//    (early termination, section 4.1.2);
//  * main phase (Algorithm 2, pair loop) with pair traversal (section
//    4.2.3): lane i starts at the rope of its own leaf, which visits exactly
//    the leaves j > i in pre-order, so every pair is handled once.
#include "pipeline.hpp"

namespace dbx {

namespace {

__device__ __forceinline__ Node load_node(const Node* __restrict__ nodes, int32_t k) {
  const float4* p = reinterpret_cast<const float4*>(nodes + k);
  float4 a = p[0], b = p[1];
  Node nd;
  nd.lox = a.x; nd.loy = a.y; nd.loz = a.z; nd.left = __float_as_int(a.w);
  nd.hix = b.x; nd.hiy = b.y; nd.hiz = b.z; nd.rope = __float_as_int(b.w);
  return nd;
}

__device__ __forceinline__ uint32_t query_index() {
  return xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

// A walk visits every node at most once, so more than 2n steps, or a
// reference outside the arrays, means a malformed tree: report, don't loop.
__device__ __forceinline__ bool bad_ref(int32_t node, uint32_t n, uint32_t& steps) {
  if (++steps > 2 * n) return true;
  return is_leaf(node) ? uint32_t(leaf_index(node)) >= n : uint32_t(node) >= n - 1;
}

__global__ void k_count(const Node* __restrict__ nodes, const float4* __restrict__ leaf,
                        uint32_t n, const int32_t* __restrict__ root, float e2,
                        int32_t min_pts, uint8_t* __restrict__ is_core, uint32_t* err) {
  const uint32_t i = query_index();
  if (i >= n) return;
  const float4 q = leaf[i];
  int32_t cnt = 0;
  int32_t node = *root;
  uint32_t steps = 0;
  while (node != SENTINEL) {
    if (bad_ref(node, n, steps)) { atomicOr(err, STATUS_TREE); break; }
    if (!is_leaf(node)) {
      Node nd = load_node(nodes, node);
      node = box_sq_dist(q.x, q.y, q.z, nd) <= e2 ? nd.left : nd.rope;
    } else {
      float4 p = leaf[leaf_index(node)];
      if (sq_dist(q.x, q.y, q.z, p.x, p.y, p.z) <= e2) {
        if (++cnt >= min_pts) break;  // early termination
      }
      node = __float_as_int(p.w);
    }
  }
  is_core[i] = cnt >= min_pts;
}

enum PairMode { FOF = 0, CORE = 1, COUNT = 2 };

template <int MODE>
__global__ void k_pairs(const Node* __restrict__ nodes, const float4* __restrict__ leaf,
                        uint32_t n, float e2, const uint8_t* __restrict__ is_core,
                        const uint32_t* __restrict__ perm, int32_t* parent, uint8_t* member,
                        unsigned long long* bestcore, unsigned long long* count,
                        uint32_t* err) {
  const uint32_t i = query_index();
  unsigned long long found = 0;
  if (i < n) {
    const float4 q = leaf[i];
    const bool ci = MODE == CORE ? is_core[i] != 0 : true;
    int32_t node = __float_as_int(q.w);  // rope of leaf i: leaves j > i only
    uint32_t steps = 0;
    while (node != SENTINEL) {
      if (bad_ref(node, n, steps)) { atomicOr(err, STATUS_TREE); break; }
      if (!is_leaf(node)) {
        Node nd = load_node(nodes, node);
        node = box_sq_dist(q.x, q.y, q.z, nd) <= e2 ? nd.left : nd.rope;
      } else {
        const int32_t j = leaf_index(node);
        const float4 p = leaf[j];
        if (sq_dist(q.x, q.y, q.z, p.x, p.y, p.z) <= e2) {
          ++found;
          if (MODE == FOF) {
            uf_union(parent, int32_t(i), j);
            member[j] = 1;
          } else if (MODE == CORE) {
            const bool cj = is_core[j] != 0;
            if (ci && cj) {
              uf_union(parent, int32_t(i), j);
            } else if (ci) {
              atomicMin(bestcore + j, (static_cast<unsigned long long>(perm[i]) << 32) | i);
            } else if (cj) {
              atomicMin(bestcore + i, (static_cast<unsigned long long>(perm[j]) << 32) | uint32_t(j));
            }
          }
        }
        node = __float_as_int(p.w);
      }
    }
    if (MODE == FOF && found) member[i] = 1;
  }
  if (MODE == COUNT) {
    for (int o = 32; o > 0; o >>= 1) found += __shfl_xor(found, o, 64);
    if ((threadIdx.x & 63) == 0 && found) atomicAdd(count, found);
  }
}

uint32_t grid_for(uint32_t n, int block) { return (n + block - 1) / block; }

}  // namespace

void launch_count(const Node* nodes, const float4* leaf, uint32_t n, const int32_t* root,
                  float e2, int32_t min_pts, uint8_t* is_core, uint32_t* err, int block,
                  hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_count, dim3(grid_for(n, block)), dim3(block), 0, s, nodes, leaf, n, root,
                     e2, min_pts, is_core, err);
}

void launch_pairs_fof(const Node* nodes, const float4* leaf, uint32_t n, float e2,
                      int32_t* parent, uint8_t* member, uint32_t* err, int block, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_pairs<FOF>, dim3(grid_for(n, block)), dim3(block), 0, s, nodes, leaf, n,
                     e2, nullptr, nullptr, parent, member, nullptr, nullptr, err);
}

void launch_pairs_core(const Node* nodes, const float4* leaf, uint32_t n, float e2,
                       const uint8_t* is_core, const uint32_t* perm, int32_t* parent,
                       unsigned long long* bestcore, uint32_t* err, int block, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_pairs<CORE>, dim3(grid_for(n, block)), dim3(block), 0, s, nodes, leaf, n,
                     e2, is_core, perm, parent, nullptr, bestcore, nullptr, err);
}

void launch_pairs_count(const Node* nodes, const float4* leaf, uint32_t n, float e2,
                        unsigned long long* count, uint32_t* err, int block, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_pairs<COUNT>, dim3(grid_for(n, block)), dim3(block), 0, s, nodes, leaf,
                     n, e2, nullptr, nullptr, nullptr, nullptr, nullptr, count, err);
}

}  // namespace dbx
