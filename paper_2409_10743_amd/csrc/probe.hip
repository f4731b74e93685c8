// Density probe behind DBSCAN_ALGO_AUTO: an estimate of the mean number of
// eps-neighbours per point (the point itself left out), from which the
// call picks FDBSCAN or DenseBox.  DenseBox (section 4.3.4) pays off where
// points have many neighbours, so that grid cells of side eps/sqrt(3) hold
// at least minPts points and whole cells replace distance tests; where
// neighbours are few its cell pass is pure overhead.
//
// Per set: S = min(n, s_max) sample points, evenly spread over the set's
// index range; c = number of ordered sample pairs (i != j) within eps;
// c / S * (n - 1) / (S - 1) estimates the mean neighbour count of the set
// without bias (each of the n - 1 other points is a neighbour with the
// same probability as each of the S - 1 other samples).  The sum over sets
// of n times that estimate is accumulated in *out (double).  The result
// does not affect labels, only which algorithm computes them.
#include "pipeline.hpp"

namespace dbx {

namespace {

constexpr int PROBE_THREADS = 256;

// one block per (set, 256 sample rows); sample columns through LDS tiles
__global__ __launch_bounds__(PROBE_THREADS) void k_density_probe(
    const float* __restrict__ pts, const int64_t* __restrict__ offsets,
    const float* __restrict__ set_e2, uint32_t s_max, uint32_t row_blocks,
    double* __restrict__ out) {
  __shared__ float4 tile[PROBE_THREADS];
  __shared__ uint32_t s_sum;
  const uint32_t set = blockIdx.x / row_blocks;
  const uint32_t r0 = (blockIdx.x % row_blocks) * PROBE_THREADS;
  const int64_t a = offsets[set], n = offsets[set + 1] - a;
  const uint32_t S = uint32_t(n < int64_t(s_max) ? n : int64_t(s_max));
  if (S < 2 || r0 >= S) return;  // whole block: uniform
  const float e2 = set_e2[set];
  auto sample = [&](uint32_t s) {
    const float* p = pts + 3 * (a + int64_t(s) * n / S);
    return make_float4(p[0], p[1], p[2], 0.f);
  };
  const uint32_t row = r0 + threadIdx.x;
  const float4 q = row < S ? sample(row) : make_float4(0.f, 0.f, 0.f, 0.f);
  if (threadIdx.x == 0) s_sum = 0;
  uint32_t cnt = 0;
  for (uint32_t c0 = 0; c0 < S; c0 += PROBE_THREADS) {
    __syncthreads();
    if (c0 + threadIdx.x < S) tile[threadIdx.x] = sample(c0 + threadIdx.x);
    __syncthreads();
    const uint32_t m = S - c0 < PROBE_THREADS ? S - c0 : PROBE_THREADS;
    if (row < S)
      for (uint32_t j = 0; j < m; ++j) {
        const float4 p = tile[j];
        cnt += (c0 + j != row && sq_dist(q.x, q.y, q.z, p.x, p.y, p.z) <= e2) ? 1u : 0u;
      }
  }
  atomicAdd(&s_sum, cnt);
  __syncthreads();
  if (threadIdx.x == 0 && s_sum)
    atomicAdd(out, double(s_sum) / double(S) * double(n - 1) / double(S - 1) * double(n));
}

}  // namespace

void launch_density_probe(const float* pts, const int64_t* offsets, const float* set_e2,
                          uint32_t num_sets, uint32_t s_max, double* out, hipStream_t s) {
  if (num_sets == 0) return;
  const uint32_t rb = (s_max + PROBE_THREADS - 1) / PROBE_THREADS;
  hipLaunchKernelGGL(k_density_probe, dim3(num_sets * rb), dim3(PROBE_THREADS), 0, s, pts,
                     offsets, set_e2, s_max, rb, out);
}

}  // namespace dbx
