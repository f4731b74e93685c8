// Label finalisation: turn the union-find forest into one label per point,
// in input order.  The paper leaves this step implicit; the labelling rule
// here (section 3.1 definitions, with the border rule made deterministic):
//   - a core point belongs to the cluster of its union-find root;
//   - a non-core point with a core neighbour (a border point) belongs to the
//     cluster of its smallest-input-index core neighbour;
//   - every other point is noise, label -1;
//   - a cluster's label is the smallest input index among its members.
// With minPts <= 2 every point with a neighbour is core (minPts = 1: every
// point), so there are no border points.
#include "pipeline.hpp"

namespace dbx {

namespace {

constexpr int FINAL_ITEMS = 4;  // points per thread, 256 apart: their chains climb together
constexpr uint32_t FINAL_TILE = 256u * FINAL_ITEMS;

// Where the chain of point i starts (-1: noise): the point itself (core, or
// every member with minPts <= 2) or its smallest-index core neighbour
// (border).
__device__ __forceinline__ int32_t chain_start(uint32_t i, int32_t min_pts,
                                               const uint8_t* __restrict__ flag,
                                               const unsigned long long* __restrict__ bestcore) {
  if (min_pts == 1 || flag[i]) return int32_t(i);
  if (min_pts <= 2) return -1;
  const unsigned long long b = bestcore[i];
  return b == ~0ull ? -1 : int32_t(uint32_t(b));
}

// minPts <= 2, one pass: every member is in the union-find, whose root is
// the member with the smallest input index, i.e. the label.  Noise keeps
// the -1 the build wrote (coalesced, by input index), so only clustered
// points are written, scattered to input order: in sparse fields most
// points are noise.
__global__ __launch_bounds__(256) void k_final_labels(
    uint32_t n, int32_t min_pts, const uint8_t* __restrict__ flag, const uint32_t* __restrict__ perm,
    const int32_t* __restrict__ parent, int32_t* __restrict__ labels) {
  const uint32_t i0 = blockIdx.x * FINAL_TILE + threadIdx.x;
  int32_t x[FINAL_ITEMS];
  uint32_t o[FINAL_ITEMS];
#pragma unroll
  for (int k = 0; k < FINAL_ITEMS; ++k) {
    const uint32_t i = i0 + 256u * k;
    x[k] = i < n ? chain_start(i, min_pts, flag, nullptr) : -1;
    o[k] = x[k] >= 0 ? perm[i] : n;
  }
  uf_roots_final(parent, x);
#pragma unroll
  for (int k = 0; k < FINAL_ITEMS; ++k)
    if (x[k] >= 0 && o[k] < n) labels[o[k]] = int32_t(perm[x[k]]);
}

// minPts > 2: border points are not in the union-find and may have the
// smallest index of their cluster.  First pass: every point's root (written
// over parent[i], or -1; a root is an ancestor, so other points' chains only
// get shorter) and, for border points, atomicMin of the input index into
// minlab[root].  Second pass: label = min(input index of the root, minlab).
__global__ __launch_bounds__(256) void k_final_roots(
    uint32_t n, int32_t min_pts, const uint8_t* __restrict__ flag,
    const unsigned long long* __restrict__ bestcore, const uint32_t* __restrict__ perm,
    int32_t* parent, int32_t* __restrict__ minlab) {
  const uint32_t i0 = blockIdx.x * FINAL_TILE + threadIdx.x;
  int32_t x[FINAL_ITEMS];
#pragma unroll
  for (int k = 0; k < FINAL_ITEMS; ++k) {
    const uint32_t i = i0 + 256u * k;
    x[k] = i < n ? chain_start(i, min_pts, flag, bestcore) : -1;
  }
  uf_roots_final(parent, x);
#pragma unroll
  for (int k = 0; k < FINAL_ITEMS; ++k) {
    const uint32_t i = i0 + 256u * k;
    if (i >= n) continue;
    if (x[k] >= 0 && !flag[i]) atomicMin(minlab + x[k], int32_t(perm[i]));
    parent[i] = x[k];
  }
}

__global__ __launch_bounds__(256) void k_final_border_labels(uint32_t n,
                                                            const uint32_t* __restrict__ perm,
                                                            const int32_t* __restrict__ root,
                                                            const int32_t* __restrict__ minlab,
                                                            int32_t* __restrict__ labels) {
  const uint32_t i0 = blockIdx.x * FINAL_TILE + threadIdx.x;
#pragma unroll
  for (int k = 0; k < FINAL_ITEMS; ++k) {
    const uint32_t i = i0 + 256u * k;
    if (i >= n) break;
    const int32_t r = root[i];
    if (r < 0) continue;  // noise: already -1
    const uint32_t o = perm[i];
    if (o < n) labels[o] = min(int32_t(perm[r]), minlab[r]);
  }
}

__global__ __launch_bounds__(256) void k_scatter_u8(const uint8_t* __restrict__ src,
                                                   const uint32_t* __restrict__ perm, uint32_t n,
                                                   uint8_t* __restrict__ dst) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && perm[i] < n) dst[perm[i]] = src[i];
}

}  // namespace

void launch_scatter_u8(const uint8_t* src, const uint32_t* perm, uint32_t n, uint8_t* dst,
                       hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_scatter_u8, dim3((n + 255) / 256), dim3(256), 0, s, src, perm, n, dst);
}

void launch_final(uint32_t n, int32_t min_pts, const uint8_t* flag,
                  const unsigned long long* bestcore, const uint32_t* perm, int32_t* parent,
                  int32_t* minlab, int32_t* labels, hipStream_t s) {
  if (n == 0) return;
  const uint32_t g = (n + FINAL_TILE - 1) / FINAL_TILE;
  if (min_pts <= 2) {
    hipLaunchKernelGGL(k_final_labels, dim3(g), dim3(256), 0, s, n, min_pts, flag, perm, parent,
                       labels);
    return;
  }
  hipLaunchKernelGGL(k_final_roots, dim3(g), dim3(256), 0, s, n, min_pts, flag, bestcore, perm,
                     parent, minlab);
  hipLaunchKernelGGL(k_final_border_labels, dim3(g), dim3(256), 0, s, n, perm, parent, minlab,
                     labels);
}

}  // namespace dbx
