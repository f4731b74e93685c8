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

// First pass: cluster root of every point (or -1; the chains are
// compressed onto it on the way), and the smallest input index per root.
// The root is written over parent[i]; that only shortens other points'
// chains (a root is an ancestor), and noise points are
// singletons nobody else's chain passes through.  It also sets every label
// to -1 (coalesced: input index i, whatever point sits at sorted position
// i), so the second pass only writes the labels of clustered points: for
// sparse fields most points are noise, and those scattered 4-byte writes
// are the expensive part.
__global__ __launch_bounds__(256) void k_final_roots(
    uint32_t n, int32_t min_pts, const uint8_t* __restrict__ flag,
    const unsigned long long* __restrict__ bestcore, const uint32_t* __restrict__ perm,
    int32_t* parent, int32_t* __restrict__ minlab, int32_t* __restrict__ labels) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i < n;  // no early return: the wave combines its minima
  int32_t r = -1;
  if (ok) {
    labels[i] = -1;
    if (min_pts <= 2) {
      r = (min_pts == 1 || flag[i]) ? uf_root_final(parent, int32_t(i)) : -1;
    } else if (flag[i]) {  // core
      r = uf_root_final(parent, int32_t(i));
    } else {
      unsigned long long b = bestcore[i];
      r = b == ~0ull ? -1 : uf_root_final(parent, int32_t(uint32_t(b)));
    }
  }
  wave_min_by_key(minlab, r, r >= 0 ? int32_t(perm[i]) : 0);
  if (ok) parent[i] = r;
}

__global__ __launch_bounds__(256) void k_final_labels(uint32_t n, const uint32_t* __restrict__ perm,
                                                     const int32_t* __restrict__ root,
                                                     const int32_t* __restrict__ minlab,
                                                     int32_t* __restrict__ labels) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t r = root[i];
  if (r < 0) return;  // noise: already -1
  const uint32_t o = perm[i];
  if (o < n) labels[o] = minlab[r];
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

void launch_final_roots(uint32_t n, int32_t min_pts, const uint8_t* flag,
                        const unsigned long long* bestcore, const uint32_t* perm,
                        int32_t* parent, int32_t* minlab, int32_t* labels, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_final_roots, dim3((n + 255) / 256), dim3(256), 0, s, n, min_pts, flag,
                     bestcore, perm, parent, minlab, labels);
}

void launch_final_labels(uint32_t n, const uint32_t* perm, const int32_t* root,
                         const int32_t* minlab, int32_t* labels, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_final_labels, dim3((n + 255) / 256), dim3(256), 0, s, n, perm, root,
                     minlab, labels);
}

}  // namespace dbx
