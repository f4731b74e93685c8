// Scene bounds, 64-bit Morton codes and the sorted leaf array.
//
// The leaves are written by scattering the points (read in input order) to
// their sorted positions: on this GPU a random 16-byte write costs about a
// 32-byte sector, a random 12-byte read a whole 128-byte line.
//
// Section 3.2: the scene bounding volume encloses all objects; LBVH orders
// the objects along a Z-curve.  Section 4.2.2: 64-bit codes (21 bits per
// axis here) instead of 32-bit ones, which leave far fewer points sharing a
// code.  A point's grid coordinate on axis a is
//     q_a = min(floor((p_a - lo_a) * s_a), 2^21 - 1),  s_a = 2^21 / (hi_a - lo_a)
// in binary32 (s_a = 0 for a zero extent); bit b of q_x, q_y, q_z goes to
// bit 3b+2, 3b+1, 3b of the code.  The codes only shape the tree: any order
// of the points gives the same clustering.
#include <algorithm>

#include "pipeline.hpp"

namespace dbx {

namespace {

__global__ void k_prep(uint32_t* __restrict__ z, size_t words, uint32_t* __restrict__ bounds) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < words; i += stride) z[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < 6)
    bounds[threadIdx.x] = threadIdx.x < 3 ? 0xffffffffu : 0u;  // lo = +max, hi = -max
}

__device__ __forceinline__ float wave_min(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

__global__ __launch_bounds__(256) void k_bounds(const float* __restrict__ pts, uint32_t n,
                                               uint32_t* __restrict__ bounds,
                                               uint32_t* __restrict__ status) {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float v = pts[size_t(3) * i + a];
      bad |= !isfinite(v);
      lo[a] = fminf(lo[a], v);
      hi[a] = fmaxf(hi[a], v);
    }
  }
  __shared__ float s_lo[3][4], s_hi[3][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float l = wave_min(lo[a]), h = wave_max(hi[a]);
    if (lane == 0) { s_lo[a][wave] = l; s_hi[a][wave] = h; }
  }
  if (__ballot(bad) != 0ull && lane == 0) atomicOr(status, STATUS_NONFINITE);
  __syncthreads();
  if (threadIdx.x < 3) {
    int a = threadIdx.x;
    float l = fminf(fminf(s_lo[a][0], s_lo[a][1]), fminf(s_lo[a][2], s_lo[a][3]));
    float h = fmaxf(fmaxf(s_hi[a][0], s_hi[a][1]), fmaxf(s_hi[a][2], s_hi[a][3]));
    atomicMin(&bounds[a], f2ord(l));
    atomicMax(&bounds[3 + a], f2ord(h));
  }
}

// spread the low 21 bits of v to every third bit of a 64-bit word
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x001f00000000ffffull;
  x = (x | (x << 16)) & 0x001f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t quantise(float p, float lo, float s) {
#pragma clang fp contract(off)
  float t = (p - lo) * s;
  t = fminf(fmaxf(floorf(t), 0.0f), float((1u << MORTON_BITS) - 1));  // NaN -> 0
  return uint32_t(t);
}

__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ pts, uint32_t n,
                                               const uint32_t* __restrict__ bounds,
                                               uint64_t* __restrict__ keys,
                                               uint32_t* __restrict__ hist) {
  __shared__ uint32_t sh[SORT_PASSES * RADIX];
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x) sh[t] = 0;
  float lo[3], s[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = ord2f(bounds[a]);
    float ext = ord2f(bounds[3 + a]) - lo[a];
    s[a] = ext > 0.0f ? float(1u << MORTON_BITS) / ext : 0.0f;  // IEEE division
  }
  __syncthreads();
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float* p = pts + size_t(3) * i;
    uint64_t code = (spread3(quantise(p[0], lo[0], s[0])) << 2) |
                    (spread3(quantise(p[1], lo[1], s[1])) << 1) |
                    spread3(quantise(p[2], lo[2], s[2]));
    keys[i] = code;
#pragma unroll
    for (int q = 0; q < SORT_PASSES; ++q)
      atomicAdd(&sh[q * RADIX + ((code >> (8 * q)) & 0xff)], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x)
    if (sh[t]) atomicAdd(&hist[t], sh[t]);
}

__global__ __launch_bounds__(256) void k_scatter(
    const float* __restrict__ pts, const uint32_t* inv, uint32_t n, float4* __restrict__ leaf,
    int32_t* parent, int32_t* __restrict__ minlab, uint8_t* __restrict__ flag,
    unsigned long long* __restrict__ bestcore, int4* __restrict__ pending,
    uint32_t pending_entries) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t k = i; k < pending_entries; k += gridDim.x * blockDim.x)
    pending[k] = make_int4(SENTINEL, 0, 0, 0);
  if (i >= n) return;
  const uint32_t s = inv[i];  // read before parent[i] (which may alias inv) is set
  const float* p = pts + size_t(3) * i;
  if (s < n) leaf[s] = make_float4(p[0], p[1], p[2], __int_as_float(SENTINEL));
  parent[i] = int32_t(i);
  minlab[i] = 0x7fffffff;
  flag[i] = 0;
  if (bestcore) bestcore[i] = ~0ull;
}

uint32_t stream_blocks(uint32_t n) { return std::max(1u, std::min((n + 255) / 256, 4096u)); }

}  // namespace

void launch_prep(uint32_t* zero_region, size_t zero_words, uint32_t* bounds, hipStream_t s) {
  uint32_t blocks = uint32_t(std::min<size_t>((zero_words + 255) / 256 + 1, 4096));
  hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(256), 0, s, zero_region, zero_words, bounds);
}

void launch_bounds(const float* pts, uint32_t n, uint32_t* bounds, uint32_t* status,
                   hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_bounds, dim3(stream_blocks(n)), dim3(256), 0, s, pts, n, bounds, status);
}

void launch_morton(const float* pts, uint32_t n, const uint32_t* bounds, uint64_t* keys,
                   uint32_t* hist, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_morton, dim3(stream_blocks(n)), dim3(256), 0, s, pts, n, bounds, keys,
                     hist);
}

void launch_scatter(const float* pts, const uint32_t* inv, uint32_t n, float4* leaf,
                    int32_t* parent, int32_t* minlab, uint8_t* flag,
                    unsigned long long* bestcore, int4* pending, uint32_t pending_entries,
                    hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, s, pts, inv, n, leaf,
                     parent, minlab, flag, bestcore, pending, pending_entries);
}

}  // namespace dbx
