// k nearest neighbours over the linear BVH (section 3.2: the nearest
// search, which finds a given number of the closest points whatever their
// distance), and from them HDBSCAN*'s core distance (section 5: the
// distance to the minPts-th nearest neighbour, the point itself counted).
//
// The answer is unique: the k points j (the query included) with the
// smallest pairs (D(q, j), input index of j), D the binary32 squared
// distance of the DBSCAN predicate; past n points the entries are -1 and
// +inf.
//
// Each lane owns one query (sorted order, so a wave's 64 queries are
// Morton neighbours) and keeps its k best pairs in registers, sorted; the
// list is K long (K >= k, a compiled size) and the k-th entry is the
// pruning radius.  It is seeded with the k points around the query in
// Morton order, which already bound the k-th distance tightly, then the
// rope walk from the root visits every node whose box bound does not
// exceed that radius (a point whose D equals the radius may still enter
// with a smaller index, so only a larger bound prunes).  The radius only
// shrinks, and any true neighbour's D is at most the radius at every
// moment, so no true neighbour's leaf is ever pruned.  Leaves of the seed
// range are skipped by the walk (they are in the list already).
#include "pipeline.hpp"

namespace dbx {

namespace {

constexpr int32_t NO_POINT = 0x7fffffff;  // an empty slot: (+inf, NO_POINT)

// (d, o) comes before (e, p): smaller distance, then smaller input index
__device__ __forceinline__ bool before(float d, int32_t o, float e, int32_t p) {
  return d < e || (d == e && o < p);
}

template <int K>
struct BestK {
  float d[K];
  int32_t o[K];
  float kd;   // the k-th entry: the pruning radius
  int32_t ko;
  __device__ void clear() {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      d[t] = INFINITY;
      o[t] = NO_POINT;
    }
    kd = INFINITY;
    ko = NO_POINT;
  }
  // insert (x, y) in order if it comes before the k-th entry; every index
  // below is a compile-time constant, so the list stays in registers
  __device__ void insert(float x, int32_t y, int32_t k) {
    if (!before(x, y, kd, ko)) return;
#pragma unroll
    for (int t = K - 1; t > 0; --t) {
      if (before(x, y, d[t - 1], o[t - 1])) {
        d[t] = d[t - 1];
        o[t] = o[t - 1];
      } else if (before(x, y, d[t], o[t])) {
        d[t] = x;
        o[t] = y;
      }
    }
    if (before(x, y, d[0], o[0])) {
      d[0] = x;
      o[0] = y;
    }
#pragma unroll
    for (int t = 0; t < K; ++t)
      if (t == k - 1) {
        kd = d[t];
        ko = o[t];
      }
  }
};

__device__ __forceinline__ float point_sq_dist(const float4& a, const float4& b) {
  return sq_dist(a.x, a.y, a.z, b.x, b.y, b.z);
}

// One query per thread.  out_idx/out_d2 (input order, rows of k), or with
// core_d2 only the k-th squared distance of every point.
template <int K>
__global__ __launch_bounds__(256) void k_knn(const Node* __restrict__ nodes,
                                             const float4* __restrict__ leaf,
                                             const uint32_t* __restrict__ perm, uint32_t n,
                                             const int32_t* __restrict__ root, int32_t k,
                                             int32_t* __restrict__ out_idx,
                                             float* __restrict__ out_d2,
                                             float* __restrict__ core_d2,
                                             uint32_t* __restrict__ err) {
  const uint32_t i = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 q = leaf[i];
  BestK<K> best;
  best.clear();
  // seed: m = min(k, n) consecutive leaves around the query
  const uint32_t m = min(uint32_t(k), n);
  const uint32_t half = m / 2;
  const uint32_t a = min(i > half ? i - half : 0u, n - m);
  const uint32_t b = a + m - 1;
  for (uint32_t j = a; j <= b; ++j) best.insert(point_sq_dist(q, leaf[j]), int32_t(perm[j]), k);
  // the rope walk from the root with the shrinking radius
  int32_t node = *root;
  uint32_t steps = 0;
  while (node != SENTINEL) {
    if (++steps > 2 * n) {  // a walk visits every node at most once
      atomicOr(err, STATUS_TREE);
      break;
    }
    if (is_leaf(node)) {
      const uint32_t j = uint32_t(leaf_index(node));
      if (j >= n) {
        atomicOr(err, STATUS_TREE);
        break;
      }
      const float4 p = leaf[j];
      if (j < a || j > b) best.insert(point_sq_dist(q, p), int32_t(perm[j]), k);
      node = __float_as_int(p.w);
    } else {
      if (uint32_t(node) + 1 >= n) {
        atomicOr(err, STATUS_TREE);
        break;
      }
      const Node nd = nodes[node];
      node = box_sq_dist(q.x, q.y, q.z, nd) <= best.kd ? nd.left : nd.rope;
    }
  }
  const uint32_t row = perm[i];
  if (core_d2) {
    core_d2[row] = best.kd;
    return;
  }
#pragma unroll
  for (int t = 0; t < K; ++t)
    if (t < k) {
      out_idx[size_t(row) * k + t] = best.o[t] == NO_POINT ? -1 : best.o[t];
      out_d2[size_t(row) * k + t] = best.d[t];
    }
}

template <int K>
void launch_knn_k(const Node* nodes, const float4* leaf, const uint32_t* perm, uint32_t n,
                  const int32_t* root, int32_t k, int32_t* out_idx, float* out_d2,
                  float* core_d2, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_knn<K>, dim3((n + 255) / 256), dim3(256), 0, s, nodes, leaf, perm, n,
                     root, k, out_idx, out_d2, core_d2, err);
}

}  // namespace

void launch_knn(const Node* nodes, const float4* leaf, const uint32_t* perm, uint32_t n,
                const int32_t* root, int32_t k, int32_t* out_idx, float* out_d2, float* core_d2,
                uint32_t* err, hipStream_t s) {
  if (n == 0) return;
  if (k <= 4) launch_knn_k<4>(nodes, leaf, perm, n, root, k, out_idx, out_d2, core_d2, err, s);
  else if (k <= 8) launch_knn_k<8>(nodes, leaf, perm, n, root, k, out_idx, out_d2, core_d2, err, s);
  else if (k <= 16)
    launch_knn_k<16>(nodes, leaf, perm, n, root, k, out_idx, out_d2, core_d2, err, s);
  else launch_knn_k<32>(nodes, leaf, perm, n, root, k, out_idx, out_d2, core_d2, err, s);
}

}  // namespace dbx
