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
// Each lane holds one query at a time (sorted order, so a wave's queries
// are Morton neighbours) and keeps its k best pairs in registers, sorted;
// the list is K long (K >= k, a compiled size) and the k-th entry is the
// pruning radius.  It is seeded with the k points around the query in
// Morton order, which already bound the k-th distance tightly, then the
// rope walk from the root visits every node whose box bound does not
// exceed that radius (a point whose D equals the radius may still enter
// with a smaller index, so only a larger bound prunes).  The radius only
// shrinks, and any true neighbour's D is at most the radius at every
// moment, so no true neighbour's leaf is ever pruned.  Leaves of the seed
// range are skipped by the walk (they are in the list already).
#include "walk.hpp"

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

// The search runs in the wave walk of the clustering traversals
// (walk.hpp): a lane whose walk ends takes the chunk's next query, so a wave
// does not wait for its longest search (against one query per thread: 40.9
// → 31.7 ms at k = 8 and 106 → 54 ms at k = 16 on the 2^24-point field).
// The pruning radius is the visitor's current k-th distance; leaves come
// to hit() when their squared distance is within it.
template <int K>
struct KnnVisit {
  static constexpr bool kBounded = false;
  static constexpr bool kStartIsRope = false;  // the root
  const float4* leaf;
  const uint32_t* perm;
  uint32_t n;
  int32_t root, k;
  int32_t* out_idx;
  float* out_d2;
  float* core_d2;
  BestK<K> best;
  uint32_t a, b;  // the seed range: already in the list
  __device__ uint64_t khi() const { return ~0ull; }
  __device__ int32_t begin(uint32_t i, const float4& q) {
    best.clear();
    const uint32_t m = min(uint32_t(k), n);
    const uint32_t half = m / 2;
    a = min(i > half ? i - half : 0u, n - m);
    b = a + m - 1;
    for (uint32_t j = a; j <= b; ++j) best.insert(point_sq_dist(q, leaf[j]), int32_t(perm[j]), k);
    return root;
  }
  __device__ float e2() const { return best.kd; }
  __device__ void visit(bool, bool) {}
  __device__ bool hit(uint32_t, int32_t j, const float4& q) {
    if (uint32_t(j) < a || uint32_t(j) > b)
      best.insert(point_sq_dist(q, leaf[j]), int32_t(perm[j]), k);
    return false;
  }
  __device__ void end(uint32_t i) {
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
};

template <int K>
__global__ void k_knn_waves(const Node* __restrict__ nodes, const float4* __restrict__ leaf,
                            const uint32_t* __restrict__ perm, uint32_t n, WalkCfg wc,
                            const int32_t* __restrict__ root, int32_t k,
                            int32_t* __restrict__ out_idx, float* __restrict__ out_d2,
                            float* __restrict__ core_d2, uint32_t* __restrict__ err) {
  KnnVisit<K> v{leaf, perm, n, *root, k, out_idx, out_d2, core_d2, {}, 0, 0};
  wave_walks(nodes, leaf, nullptr, n, wc, v, err);
}

template <int K>
void launch_knn_k(const Node* nodes, const float4* leaf, const uint32_t* perm, uint32_t n,
                  const int32_t* root, int32_t k, int32_t* out_idx, float* out_d2,
                  float* core_d2, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_knn_waves<K>, dim3(walk_grid(n, 256)), dim3(256), 0, s, nodes, leaf, perm,
                     n, walk_cfg(n), root, k, out_idx, out_d2, core_d2, err);
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
