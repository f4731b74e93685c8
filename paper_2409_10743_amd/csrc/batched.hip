// Batched clustering: many independent point sets (given as CSR offsets)
// clustered in one pass of the whole path, each with its own eps and minPts,
// each result identical to clustering that set alone (labels are set-local
// input indices).
//
// The sets share one key space: key = (set id << set_shift) | Morton code of
// the point within its own set's bounding box (set_shift/3 bits per axis).
// One radix sort orders all points, one build makes every set a complete
// subtree (a boundary between sets has a larger delta than any boundary
// inside a set), ropes are cut at set ends, and each traversal lane reads its
// set's parameters and subtree root from its key's top bits.
#include <algorithm>

#include "walk.hpp"

namespace dbx {

namespace {

__device__ __forceinline__ float block_min(float v, float* s_red) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = s_red[0];
  for (int w = 1; w < int(blockDim.x >> 6); ++w) r = fminf(r, s_red[w]);
  __syncthreads();
  return r;
}
__device__ __forceinline__ float block_max(float v, float* s_red) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = s_red[0];
  for (int w = 1; w < int(blockDim.x >> 6); ++w) r = fmaxf(r, s_red[w]);
  __syncthreads();
  return r;
}

// One workgroup per set: the set's bounding box, then its keys (set id in
// the top bits, `bits` per axis of Morton code below) and digit histograms.
// The set's grid goes to grids[set] for the walks' early end.  With
// set_inv_h (DenseBox) the grid is that of the set's cells, side
// max(1 / set_inv_h[set], extent / 2^bits).
__global__ __launch_bounds__(256) void k_set_morton(const float* __restrict__ pts,
                                                   const int64_t* __restrict__ offsets,
                                                   int bits, int set_shift,
                                                   const float* __restrict__ set_inv_h,
                                                   uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ hist,
                                                   int32_t* __restrict__ set_root,
                                                   MortonGrid* __restrict__ grids,
                                                   uint32_t* __restrict__ status) {
  __shared__ uint32_t sh[SORT_PASSES * RADIX];
  __shared__ float s_red[4];
  const uint32_t set = blockIdx.x;
  if (threadIdx.x == 0) set_root[set] = SENTINEL;  // the build sets it (non-empty sets)
  const uint32_t b = uint32_t(offsets[set]), e = uint32_t(offsets[set + 1]);
  if (b >= e) return;
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x) sh[t] = 0;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (uint32_t i = b + threadIdx.x; i < e; i += blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float v = pts[size_t(3) * i + a];
      bad |= !isfinite(v);
      lo[a] = fminf(lo[a], v);
      hi[a] = fmaxf(hi[a], v);
    }
  }
  if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(status, STATUS_NONFINITE);
  MortonGrid g;
  g.maxc = float((1u << bits) - 1u);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = block_min(lo[a], s_red);
    const float top = block_max(hi[a], s_red);
    const float ext = top - g.lo[a];
    g.s[a] = ext > 0.0f ? float(1u << bits) / ext : 0.0f;
    if (set_inv_h && ext > 0.0f) g.s[a] = fminf(set_inv_h[set], g.s[a]);  // DenseBox cells
  }
  if (threadIdx.x == 0) grids[set] = g;
  const uint64_t tag = uint64_t(set) << set_shift;
  for (uint32_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    const float* p = pts + size_t(3) * i;
    const uint64_t code = tag | g.code(p[0], p[1], p[2]);
    keys[i] = code;
    count_digits_wave(sh, code, SORT_PASSES);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x)
    if (sh[t]) atomicAdd(&hist[t], sh[t]);
}

// the early-end bound of a query of set `set` (its codes carry the set id)
__device__ __forceinline__ uint64_t set_upper_code(const MortonGrid* grids, uint32_t set,
                                                   int set_shift, const float4& q, float e2) {
  const MortonGrid g = grids[set];
  return (uint64_t(set) << set_shift) | g.upper_code(q, e2);
}

// Counting for the points of sets with minPts > 2, from their set's root.
struct CountSets {
  static constexpr bool kBounded = true;
  static constexpr bool kStartIsRope = false;  // the set's root
  __device__ uint64_t khi() const { return hi; }
  const uint64_t* keys;
  int set_shift;
  const int32_t* set_root;
  const float* set_e2;
  const int32_t* set_minpts;
  uint8_t* flag;
  const MortonGrid* grids;
  float r2;
  int32_t min_pts, cnt;
  uint64_t hi;
  __device__ int32_t begin(uint32_t i, const float4& q) {
    const uint32_t set = uint32_t(keys[i] >> set_shift);
    min_pts = set_minpts[set];
    r2 = set_e2[set];
    cnt = 0;
    if (min_pts <= 2) return SENTINEL;
    hi = set_upper_code(grids, set, set_shift, q, r2);
    return set_root[set];
  }
  __device__ float e2() const { return r2; }
  __device__ void visit(bool, bool) {}
  __device__ bool hit(uint32_t, int32_t, const float4&) { return ++cnt >= min_pts; }
  __device__ void end(uint32_t i) {
    if (min_pts > 2) flag[i] = cnt >= min_pts;  // minPts <= 2: the pair phase sets it
  }
};

template <bool PERSIST>
__global__ void k_count_sets(const Node* __restrict__ nodes, const float4* __restrict__ leaf,
                             uint32_t n, WalkCfg wc,
                             const uint64_t* __restrict__ keys,
                             int set_shift, const int32_t* __restrict__ set_root,
                             const float* __restrict__ set_e2,
                             const int32_t* __restrict__ set_minpts,
                             const MortonGrid* __restrict__ grids,
                             uint8_t* __restrict__ flag, uint32_t* __restrict__ err) {
  CountSets v{keys, set_shift, set_root, set_e2, set_minpts, flag, grids, 0.f, 0, 0, 0};
  wave_walks<decltype(v), PERSIST>(nodes, leaf, keys, n, wc, v, err);
}

// Pair traversal; each lane runs the minPts <= 2 or the minPts > 2 rule of
// its own set (both ends of a pair are always in the same set).
struct PairSets {
  static constexpr bool kBounded = true;
  static constexpr bool kStartIsRope = true;  // the query leaf's rope
  __device__ uint64_t khi() const { return hi; }
  const uint64_t* keys;
  int set_shift;
  const float* set_e2;
  const int32_t* set_minpts;
  const uint32_t* perm;
  int32_t* parent;
  uint8_t* flag;
  unsigned long long* bestcore;
  const MortonGrid* grids;
  float r2;
  bool core_mode, ci, found;
  uint64_t hi;
  int32_t ri;  // an ancestor of the query's point in the union-find forest
  __device__ int32_t begin(uint32_t i, const float4& q) {
    const uint32_t set = uint32_t(keys[i] >> set_shift);
    r2 = set_e2[set];
    hi = set_upper_code(grids, set, set_shift, q, r2);
    core_mode = set_minpts[set] > 2;
    ci = core_mode ? flag[i] != 0 : true;
    found = false;
    ri = int32_t(i);
    return __float_as_int(q.w);
  }
  __device__ float e2() const { return r2; }
  __device__ void visit(bool, bool) {}
  __device__ bool hit(uint32_t i, int32_t j, const float4&) {
    if (!core_mode) {
      found = true;
      ri = uf_union(parent, perm, ri, j);
      flag[j] = 1;
      return false;
    }
    const bool cj = flag[j] != 0;
    if (ci && cj) ri = uf_union(parent, perm, ri, j);
    else if (ci) atomicMin(bestcore + j, (static_cast<unsigned long long>(perm[i]) << 32) | i);
    else if (cj)
      atomicMin(bestcore + i, (static_cast<unsigned long long>(perm[j]) << 32) | uint32_t(j));
    return false;
  }
  __device__ void end(uint32_t i) {
    if (!core_mode && found) flag[i] = 1;
  }
};

template <bool PERSIST>
__global__ void k_pairs_sets(const Node* __restrict__ nodes, const float4* __restrict__ leaf,
                             uint32_t n, WalkCfg wc,
                             const uint64_t* __restrict__ keys,
                             int set_shift,
                             const float* __restrict__ set_e2,
                             const int32_t* __restrict__ set_minpts,
                             const MortonGrid* __restrict__ grids,
                             const uint32_t* __restrict__ perm, int32_t* parent, uint8_t* flag,
                             unsigned long long* bestcore, uint32_t* err) {
  PairSets v{keys, set_shift, set_e2, set_minpts, perm, parent, flag, bestcore, grids,
             0.f, false, true, false, 0, 0};
  wave_walks<decltype(v), PERSIST>(nodes, leaf, keys, n, wc, v, err);
}


// Labels as in finalize.hip, each point by its own set's minPts: a
// clustered point's label is the smallest input index of its cluster (the
// root's, or a border point's, collected in minlab) minus the set's offset;
// noise keeps the -1 the build wrote.
constexpr int FINAL_ITEMS = 4;  // points per thread, 256 apart: their chains climb together
constexpr uint32_t FINAL_TILE = 256u * FINAL_ITEMS;

// Where the chain of point i starts (-1: noise), by its set's minPts mp.
__device__ __forceinline__ int32_t set_chain_start(uint32_t i, int32_t mp,
                                                   const uint8_t* __restrict__ flag,
                                                   const unsigned long long* __restrict__ bestcore) {
  if (mp == 1 || flag[i]) return int32_t(i);
  if (mp <= 2) return -1;
  const unsigned long long b = bestcore[i];
  return b == ~0ull ? -1 : int32_t(uint32_t(b));
}

// no set with minPts > 2: one pass
__global__ __launch_bounds__(256) void k_final_labels_sets(
    uint32_t n, const uint64_t* __restrict__ keys, int set_shift,
    const int32_t* __restrict__ set_minpts, const int64_t* __restrict__ offsets,
    const uint8_t* __restrict__ flag, const uint32_t* __restrict__ perm,
    const int32_t* __restrict__ parent, int32_t* __restrict__ labels) {
  const uint32_t i0 = blockIdx.x * FINAL_TILE + threadIdx.x;
  int32_t x[FINAL_ITEMS];
  uint32_t set[FINAL_ITEMS];
#pragma unroll
  for (int k = 0; k < FINAL_ITEMS; ++k) {
    const uint32_t i = i0 + 256u * k;
    set[k] = i < n ? uint32_t(keys[i] >> set_shift) : 0u;
    x[k] = i < n ? set_chain_start(i, set_minpts[set[k]], flag, nullptr) : -1;
  }
  uf_roots_final(parent, x);
#pragma unroll
  for (int k = 0; k < FINAL_ITEMS; ++k) {
    const uint32_t i = i0 + 256u * k;
    if (x[k] < 0) continue;
    const uint32_t o = perm[i];
    if (o < n) labels[o] = int32_t(perm[x[k]]) - int32_t(offsets[set[k]]);
  }
}

// some set with minPts > 2: roots and border minima, then labels
__global__ __launch_bounds__(256) void k_final_roots_sets(
    uint32_t n, const uint64_t* __restrict__ keys, int set_shift,
    const int32_t* __restrict__ set_minpts, const uint8_t* __restrict__ flag,
    const unsigned long long* __restrict__ bestcore, const uint32_t* __restrict__ perm,
    int32_t* parent, int32_t* __restrict__ minlab) {
  const uint32_t i0 = blockIdx.x * FINAL_TILE + threadIdx.x;
  int32_t x[FINAL_ITEMS], mp[FINAL_ITEMS];
#pragma unroll
  for (int k = 0; k < FINAL_ITEMS; ++k) {
    const uint32_t i = i0 + 256u * k;
    mp[k] = i < n ? set_minpts[uint32_t(keys[i] >> set_shift)] : 0;
    x[k] = i < n ? set_chain_start(i, mp[k], flag, bestcore) : -1;
  }
  uf_roots_final(parent, x);
#pragma unroll
  for (int k = 0; k < FINAL_ITEMS; ++k) {
    const uint32_t i = i0 + 256u * k;
    if (i >= n) continue;
    if (x[k] >= 0 && mp[k] > 2 && !flag[i]) atomicMin(minlab + x[k], int32_t(perm[i]));
    parent[i] = x[k];
  }
}

__global__ __launch_bounds__(256) void k_final_border_labels_sets(
    uint32_t n, const uint64_t* __restrict__ keys, int set_shift,
    const int64_t* __restrict__ offsets, const uint32_t* __restrict__ perm,
    const int32_t* __restrict__ root, const int32_t* __restrict__ minlab,
    int32_t* __restrict__ labels) {
  const uint32_t i0 = blockIdx.x * FINAL_TILE + threadIdx.x;
#pragma unroll
  for (int k = 0; k < FINAL_ITEMS; ++k) {
    const uint32_t i = i0 + 256u * k;
    if (i >= n) break;
    const int32_t r = root[i];
    if (r < 0) continue;  // noise: already -1
    const uint32_t o = perm[i];
    const int32_t base = int32_t(offsets[uint32_t(keys[i] >> set_shift)]);
    if (o < n) labels[o] = min(int32_t(perm[r]), minlab[r]) - base;
  }
}

}  // namespace

// Which batched FDBSCAN walks run persistently by default (see walk.hpp):
// neither; on the 4,096 sub-halo sets the static chunks were faster (count
// 31 against 38 ms, pairs 147 against 155 ms).
constexpr bool SETS_PERSIST_COUNT = false;
constexpr bool SETS_PERSIST_PAIRS = false;

void launch_set_morton(const float* pts, const int64_t* offsets, uint32_t num_sets, int bits,
                       int set_shift, const float* set_inv_h, uint64_t* keys, uint32_t* hist,
                       int32_t* set_root, MortonGrid* grids, uint32_t* status, hipStream_t s) {
  if (num_sets == 0) return;
  hipLaunchKernelGGL(k_set_morton, dim3(num_sets), dim3(256), 0, s, pts, offsets, bits, set_shift,
                     set_inv_h, keys, hist, set_root, grids, status);
}

void launch_count_sets(const Node* nodes, const float4* leaf, uint32_t n, const uint64_t* keys,
                       int set_shift, const int32_t* set_root, const float* set_e2,
                       const int32_t* set_minpts, const MortonGrid* grids, uint8_t* flag,
                       uint32_t* queue, uint32_t* err, int block, hipStream_t s) {
  if (n == 0) return;
  if (SETS_PERSIST_COUNT) {
    const uint32_t grid = persistent_blocks(reinterpret_cast<const void*>(&k_count_sets<true>),
                                            block, 0, walk_grid(n, block));
    hipLaunchKernelGGL(k_count_sets<true>, dim3(grid), dim3(block), 0, s, nodes, leaf, n,
                       walk_cfg(n, queue), keys, set_shift, set_root, set_e2, set_minpts, grids,
                       flag, err);
  } else {
    hipLaunchKernelGGL(k_count_sets<false>, dim3(walk_grid(n, block)), dim3(block), 0, s, nodes,
                       leaf, n, walk_cfg(n), keys, set_shift, set_root, set_e2, set_minpts, grids,
                       flag, err);
  }
}

void launch_pairs_sets(const Node* nodes, const float4* leaf, uint32_t n, const uint64_t* keys,
                       int set_shift, const float* set_e2, const int32_t* set_minpts,
                       const MortonGrid* grids, const uint32_t* perm, int32_t* parent,
                       uint8_t* flag, unsigned long long* bestcore, uint32_t* queue,
                       uint32_t* err, int block, hipStream_t s) {
  if (n == 0) return;
  if (SETS_PERSIST_PAIRS) {
    const uint32_t grid = persistent_blocks(reinterpret_cast<const void*>(&k_pairs_sets<true>),
                                            block, 0, walk_grid(n, block));
    hipLaunchKernelGGL(k_pairs_sets<true>, dim3(grid), dim3(block), 0, s, nodes, leaf, n,
                       walk_cfg(n, queue), keys, set_shift, set_e2, set_minpts, grids, perm,
                       parent, flag, bestcore, err);
  } else {
    hipLaunchKernelGGL(k_pairs_sets<false>, dim3(walk_grid(n, block)), dim3(block), 0, s, nodes,
                       leaf, n, walk_cfg(n), keys, set_shift, set_e2, set_minpts, grids, perm,
                       parent, flag, bestcore, err);
  }
}

void launch_final_sets(uint32_t n, const uint64_t* keys, int set_shift, const int32_t* set_minpts,
                       const int64_t* offsets, const uint8_t* flag,
                       const unsigned long long* bestcore, const uint32_t* perm, int32_t* parent,
                       int32_t* minlab, int32_t* labels, hipStream_t s) {
  if (n == 0) return;
  const uint32_t g = (n + FINAL_TILE - 1) / FINAL_TILE;
  if (!bestcore) {  // no set with minPts > 2
    hipLaunchKernelGGL(k_final_labels_sets, dim3(g), dim3(256), 0, s, n, keys, set_shift,
                       set_minpts, offsets, flag, perm, parent, labels);
    return;
  }
  hipLaunchKernelGGL(k_final_roots_sets, dim3(g), dim3(256), 0, s, n, keys, set_shift,
                     set_minpts, flag, bestcore, perm, parent, minlab);
  hipLaunchKernelGGL(k_final_border_labels_sets, dim3(g), dim3(256), 0, s, n, keys, set_shift,
                     offsets, perm, parent, minlab, labels);
}

}  // namespace dbx
