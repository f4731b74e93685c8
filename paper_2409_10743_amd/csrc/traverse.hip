// Stackless BVH traversals with fused callbacks (sections 4.1, 4.2, 4.3.3).
//
// One lane per query at a time, queries in Morton order so the 64 lanes of a
// wave walk nearby parts of the tree (section 3.2); the walk itself (a
// left-first pre-order over ropes, section 4.2.1) is in walk.hpp.  Nothing
// is stored per neighbour: the work on a found pair is done on the spot (the
// "callback"), so memory stays O(n).
//
//  * counting (Algorithm 2, preprocessing; only needed when minPts > 2):
//    walk from the root and stop as soon as minPts neighbours are found
//    (early termination, section 4.1.2);
//  * main phase (Algorithm 2, pair loop) with pair traversal (section
//    4.2.3): lane i starts at the rope of its own leaf, which visits exactly
//    the leaves j > i in pre-order, so every pair is handled once;
//  * counting by pair traversal (an option): every pair adds one to both
//    points' neighbour counts.  No early exit, but no walk from the root
//    either: cheaper where points have few neighbours.
#include <map>
#include <mutex>
#include <utility>

#include "walk.hpp"

namespace dbx {

namespace {

// counting: walk from the root, stop at minPts neighbours
struct CountCore {
  static constexpr bool kBounded = true;
  static constexpr bool kStartIsRope = false;  // the root
  int32_t root, min_pts, cnt;
  float r2;
  uint8_t* is_core;
  MortonGrid grid;
  uint64_t hi, mask;
  __device__ int32_t begin(uint32_t, const float4& q) {
    cnt = 0;
    hi = grid.upper_code(q, r2) & mask;
    return root;
  }
  __device__ uint64_t khi() const { return hi; }
  __device__ float e2() const { return r2; }
  __device__ void visit(bool, bool) {}
  __device__ bool hit(uint32_t, int32_t, const float4&) { return ++cnt >= min_pts; }
  __device__ void end(uint32_t i) { is_core[i] = cnt >= min_pts; }
};

__global__ void k_count(const Node* __restrict__ nodes, const float4* __restrict__ leaf,
                        const uint64_t* __restrict__ keys, const uint32_t* __restrict__ bounds,
                        const uint32_t* drop, uint32_t n, WalkCfg wc,
                        const int32_t* __restrict__ root, float e2, int32_t min_pts,
                        uint8_t* __restrict__ is_core, uint32_t* err) {
  CountCore v{*root, min_pts, 0, e2, is_core, {}, 0, ~0ull << (drop ? *drop : 0u)};
  v.grid.load(bounds);
  wave_walks(nodes, leaf, keys, n, wc, v, err);
}

enum PairMode { FOF = 0, CORE = 1, COUNT = 2, DEGREE = 3 };

// Counting by pair traversal: the top bit of a point's count marks that
// its own walk (leaves after it) found a pair.
constexpr uint32_t DEG_FORWARD = 1u << 31;
static_assert(SORT_MAX_N < DEG_FORWARD / 2, "counts below 2^30 leave the bit free");

// pair traversal: query i starts at its own leaf's rope (leaves j > i only)
template <int MODE>
struct PairVisit {
  static constexpr bool kBounded = true;
  static constexpr bool kStartIsRope = true;  // the query leaf's rope
  float r2;
  const uint8_t* is_core;
  const uint32_t* perm;
  int32_t* parent;
  uint8_t* member;
  unsigned long long* bestcore;
  bool ci, found;
  int32_t ri;  // an ancestor of the query's point in the union-find forest
  uint32_t pairs, visits, descents, leaves;  // COUNT only: this query's counts
  unsigned long long tot[4];                 // COUNT only: this lane's totals
  MortonGrid grid;
  uint64_t hi, mask;
  // DEGREE: neighbour counts (self excluded) with DEG_FORWARD set where the
  // point's own walk found a pair; CORE: the same, read (or null)
  uint32_t* deg;
  __device__ uint64_t khi() const { return hi; }
  __device__ int32_t begin(uint32_t i, const float4& q) {
    found = false;
    ri = int32_t(i);
    // the counting walk from i found no pair: neither will this one
    if (MODE == CORE && deg && !(deg[i] & DEG_FORWARD)) return SENTINEL;
    hi = grid.upper_code(q, r2) & mask;
    if (MODE == COUNT || MODE == DEGREE) pairs = visits = descents = leaves = 0;
    if (MODE == CORE) ci = is_core[i] != 0;
    return __float_as_int(q.w);
  }
  __device__ float e2() const { return r2; }
  __device__ void visit(bool lf, bool near) {
    if (MODE == COUNT) {
      if (lf) {
        ++leaves;
      } else {
        ++visits;
        if (near) ++descents;
      }
    }
  }
  __device__ bool hit(uint32_t i, int32_t j, const float4&) {
    if (MODE == FOF) {
      found = true;
      ri = uf_union(parent, perm, ri, j);
      member[j] = 1;
    } else if (MODE == CORE) {
      const bool cj = is_core[j] != 0;
      if (ci && cj) ri = uf_union(parent, perm, ri, j);
      else if (ci) atomicMin(bestcore + j, (static_cast<unsigned long long>(perm[i]) << 32) | i);
      else if (cj)
        atomicMin(bestcore + i, (static_cast<unsigned long long>(perm[j]) << 32) | uint32_t(j));
    } else if (MODE == DEGREE) {
      ++pairs;
      atomicAdd(deg + j, 1u);
    } else {
      ++pairs;
    }
    return false;
  }
  __device__ void end(uint32_t i) {
    if (MODE == FOF && found) member[i] = 1;
    // others may add to it too; counts stay below 2^30 (n does)
    if (MODE == DEGREE && pairs) atomicAdd(deg + i, pairs | DEG_FORWARD);
    if (MODE == COUNT) {  // a query's counts are below 2n, so 32 bits hold them
      tot[0] += pairs; tot[1] += visits; tot[2] += descents; tot[3] += leaves;
    }
  }
};

// one atomic per wave with the wave's sum
__device__ __forceinline__ void wave_add(unsigned long long* dst, unsigned long long x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  if ((threadIdx.x & 63) == 0 && x) atomicAdd(dst, x);
}

template <int MODE>
__global__ void k_pairs(const Node* __restrict__ nodes, const float4* __restrict__ leaf,
                        const uint64_t* __restrict__ keys, const uint32_t* __restrict__ bounds,
                        const uint32_t* drop, uint32_t n, WalkCfg wc, float e2,
                        const uint8_t* __restrict__ is_core, const uint32_t* __restrict__ perm,
                        int32_t* parent, uint8_t* member, unsigned long long* bestcore,
                        unsigned long long* count, uint32_t* deg, const uint32_t* ncore,
                        uint32_t* err) {
  // ncore (CORE only, may be null): the number of core points; with none
  // there is nothing for the main phase to join or attach
  if (MODE == CORE && ncore && *ncore == 0u) return;
  PairVisit<MODE> v{e2, is_core, perm, parent, member, bestcore, true, false, 0, 0, 0, 0, 0,
                    {0, 0, 0, 0}, {}, 0, ~0ull << (drop ? *drop : 0u), deg};
  v.grid.load(bounds);
  wave_walks(nodes, leaf, keys, n, wc, v, err);
  if (MODE == COUNT) {  // pairs, internal visits, descents, leaf tests
    wave_add(count, v.tot[0]);
    wave_add(count + 1, v.tot[1]);
    wave_add(count + 2, v.tot[2]);
    wave_add(count + 3, v.tot[3]);
  }
}

// core flags from the pair counts: the point itself counts too
// (and the number of core points, one atomic per wave)
__global__ __launch_bounds__(256) void k_degree_flags(uint32_t n, const uint32_t* __restrict__ deg,
                                                     int32_t min_pts, uint8_t* __restrict__ flag,
                                                     uint32_t* __restrict__ ncore) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool core = i < n && int64_t(deg[i] & ~DEG_FORWARD) + 1 >= int64_t(min_pts);
  if (i < n) flag[i] = core;
  const uint64_t m = __ballot(core);
  if (ncore && m && (threadIdx.x & 63) == 0) atomicAdd(ncore, uint32_t(__popcll(m)));
}

}  // namespace

uint32_t walk_queries_per_lane(uint32_t n) {
  return n >= (1u << 23) ? 4u : n >= (1u << 22) ? 2u : 1u;
}

uint32_t persistent_blocks(const void* kernel, int block, size_t lds, uint32_t needed) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, uint32_t> cache;  // per kernel and block size
  uint32_t fit = 0;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find({kernel, block});
    if (it != cache.end()) fit = it->second;
  }
  if (fit == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess ||
        cus < 1 || per_cu < 1) {
      (void)hipGetLastError();
      return (needed + 7) / 8 * 8;  // every chunk group its own block: still correct
    }
    fit = (uint32_t(cus) * uint32_t(per_cu) + 7) / 8 * 8;
    std::lock_guard<std::mutex> g(mu);
    cache[{kernel, block}] = fit;
  }
  return std::max(8u, std::min(fit, (needed + 7) / 8 * 8));
}

void launch_count(const Node* nodes, const float4* leaf, const uint64_t* keys,
                  const uint32_t* bounds, const uint32_t* drop, uint32_t n, const int32_t* root,
                  float e2, int32_t min_pts, uint8_t* is_core, uint32_t* err, int block,
                  hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_count, dim3(walk_grid(n, block)), dim3(block), 0, s, nodes, leaf, keys,
                     bounds, drop, n, walk_cfg(n), root, e2, min_pts, is_core, err);
}

void launch_pairs_fof(const Node* nodes, const float4* leaf, const uint64_t* keys,
                      const uint32_t* bounds, const uint32_t* drop, uint32_t n, float e2,
                      const uint32_t* perm, int32_t* parent, uint8_t* member, uint32_t* err,
                      int block, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_pairs<FOF>, dim3(walk_grid(n, block)), dim3(block), 0, s, nodes, leaf,
                     keys, bounds, drop, n, walk_cfg(n), e2, nullptr, perm, parent,
                     member, nullptr, nullptr, nullptr, nullptr, err);
}

void launch_pairs_core(const Node* nodes, const float4* leaf, const uint64_t* keys,
                       const uint32_t* bounds, const uint32_t* drop, uint32_t n, float e2,
                       const uint8_t* is_core, const uint32_t* perm, int32_t* parent,
                       unsigned long long* bestcore, const uint32_t* deg,
                       const uint32_t* ncore, uint32_t* err, int block, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_pairs<CORE>, dim3(walk_grid(n, block)), dim3(block), 0, s, nodes, leaf,
                     keys, bounds, drop, n, walk_cfg(n), e2, is_core, perm, parent, nullptr,
                     bestcore, nullptr, const_cast<uint32_t*>(deg), ncore, err);
}

void launch_pairs_count(const Node* nodes, const float4* leaf, const uint64_t* keys,
                        const uint32_t* bounds, const uint32_t* drop, uint32_t n, float e2,
                        unsigned long long* count, uint32_t* err, int block, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_pairs<COUNT>, dim3(walk_grid(n, block)), dim3(block), 0, s, nodes, leaf,
                     keys, bounds, drop, n, walk_cfg(n), e2, nullptr, nullptr, nullptr,
                     nullptr, nullptr, count, nullptr, nullptr, err);
}

void launch_count_pairs(const Node* nodes, const float4* leaf, const uint64_t* keys,
                        const uint32_t* bounds, const uint32_t* drop, uint32_t n, float e2,
                        int32_t min_pts, uint32_t* deg, uint8_t* is_core, uint32_t* ncore,
                        uint32_t* err, int block, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_pairs<DEGREE>, dim3(walk_grid(n, block)), dim3(block), 0, s, nodes, leaf,
                     keys, bounds, drop, n, walk_cfg(n), e2, nullptr, nullptr, nullptr,
                     nullptr, nullptr, nullptr, deg, nullptr, err);
  hipLaunchKernelGGL(k_degree_flags, dim3((n + 255) / 256), dim3(256), 0, s, n, deg, min_pts,
                     is_core, ncore);
}

}  // namespace dbx
