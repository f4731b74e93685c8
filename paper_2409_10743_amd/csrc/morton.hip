// Scene bounds, 64-bit Morton codes and the sorted leaf array.

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

__global__ void k_prep(uint32_t* __restrict__ z, size_t words, uint32_t* __restrict__ bounds,
                       int4* __restrict__ pending, uint32_t pending_entries) {
  const size_t i0 = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = i0; i < words; i += stride) z[i] = 0u;
  // build hand-over entries: empty until a frame hands a node up
  for (size_t i = i0; i < pending_entries; i += stride) pending[i] = make_int4(SENTINEL, 0, 0, 0);
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

__device__ __forceinline__ void take_axis(float* lo, float* hi, uint32_t axis, float v) {
  // axis in {0, 1, 2}; selects instead of a dynamic register index
  lo[0] = axis == 0 ? fminf(lo[0], v) : lo[0];
  hi[0] = axis == 0 ? fmaxf(hi[0], v) : hi[0];
  lo[1] = axis == 1 ? fminf(lo[1], v) : lo[1];
  hi[1] = axis == 1 ? fmaxf(hi[1], v) : hi[1];
  lo[2] = axis == 2 ? fminf(lo[2], v) : lo[2];
  hi[2] = axis == 2 ? fmaxf(hi[2], v) : hi[2];
}

// Per-axis min/max of the n points and a non-finite flag.  With a 16-byte
// aligned array the coordinates are read as float4s: the 4 values of float4
// number v are coordinates v, v+1, v+2, v (mod 3) of the flat x,y,z array,
// since 4v = v (mod 3).
template <bool VEC>
__global__ __launch_bounds__(256) void k_bounds(const float* __restrict__ pts, uint32_t n,
                                               uint32_t* __restrict__ bounds,
                                               uint32_t* __restrict__ status) {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  const uint64_t gid = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  if (VEC) {
    const uint64_t total = 3ull * n, nv = total / 4;
    const float4* p4 = reinterpret_cast<const float4*>(pts);
    auto take4 = [&](const float4& x, uint64_t v) {
      bad |= !(isfinite(x.x) && isfinite(x.y) && isfinite(x.z) && isfinite(x.w));
      const uint32_t r = uint32_t(v % 3);
      const float m = fminf(x.x, x.w), M = fmaxf(x.x, x.w);
      // axis r: x.x and x.w; axis r+1: x.y; axis r+2: x.z
      const float l0 = r == 0 ? m : (r == 1 ? x.z : x.y), h0 = r == 0 ? M : (r == 1 ? x.z : x.y);
      const float l1 = r == 1 ? m : (r == 2 ? x.z : x.y), h1 = r == 1 ? M : (r == 2 ? x.z : x.y);
      const float l2 = r == 2 ? m : (r == 0 ? x.z : x.y), h2 = r == 2 ? M : (r == 0 ? x.z : x.y);
      lo[0] = fminf(lo[0], l0); hi[0] = fmaxf(hi[0], h0);
      lo[1] = fminf(lo[1], l1); hi[1] = fmaxf(hi[1], h1);
      lo[2] = fminf(lo[2], l2); hi[2] = fmaxf(hi[2], h2);
    };
    // four loads in flight per thread
    uint64_t v = gid;
    for (; v + 3 * stride < nv; v += 4 * stride) {
      const float4 x0 = p4[v], x1 = p4[v + stride], x2 = p4[v + 2 * stride],
                   x3 = p4[v + 3 * stride];
      take4(x0, v);
      take4(x1, v + stride);
      take4(x2, v + 2 * stride);
      take4(x3, v + 3 * stride);
    }
    for (; v < nv; v += stride) take4(p4[v], v);
    if (gid == 0)
      for (uint64_t e = nv * 4; e < total; ++e) {
        const float v = pts[e];
        bad |= !isfinite(v);
        take_axis(lo, hi, uint32_t(e % 3), v);
      }
  } else {
    for (uint64_t i = gid; i < n; i += stride) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        float v = pts[3 * i + a];
        bad |= !isfinite(v);
        lo[a] = fminf(lo[a], v);
        hi[a] = fmaxf(hi[a], v);
      }
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


// Digit counts of the passes the sort runs (digits below `first` are all
// zero and their passes skipped: counting them would pile every lane of a
// wave onto one LDS bin).
__device__ __forceinline__ void count_digits(uint32_t* sh, uint64_t code, int first) {
#pragma unroll
  for (int q = 0; q < SORT_PASSES; ++q)
    if (q >= first) atomicAdd(&sh[q * RADIX + ((code >> (8 * q)) & 0xff)], 1u);
}

// Codes of all points plus the digit counts of every sort pass.  With a
// 16-byte aligned point array a thread codes 4 points from 3 float4 loads
// and writes their keys as two 16-byte stores.
// The lowest `drop` code bits are cleared, drop = droppable_code_bits()
// (all blocks compute the same value; block 0 also stores it for the sort
// and the walks).  The sort then skips drop / 8 passes and always ends in
// the first key buffer, so the codes go to the first buffer if it skips an
// even number of passes, else to the second.  With `drop_out` (the
// clustering call's sort, which moves 32-bit words) a code is written as
// its two halves, the low one to 32-bit word i of that buffer and the high
// one to word n + i, or, when the low half is all dropped, the high half
// alone to word i.
template <bool VEC>
__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ pts, uint32_t n,
                                               const uint32_t* __restrict__ bounds, float eps,
                                               uint64_t* __restrict__ keys_a,
                                               uint64_t* __restrict__ keys_b,
                                               uint32_t* __restrict__ drop_out,
                                               uint32_t* __restrict__ hist) {
  __shared__ uint32_t sh[SORT_PASSES * RADIX];
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x) sh[t] = 0;
  MortonGrid grid;
  grid.load(bounds);
  const int drop = droppable_code_bits(bounds, eps, n);
  const uint64_t mask = ~0ull << drop;
  const int first = drop / 8;  // first sort pass that runs
  uint64_t* keys = (first % 2 == 0) ? keys_a : keys_b;
  if (blockIdx.x == 0 && threadIdx.x == 0 && drop_out) *drop_out = uint32_t(drop);
  // 32-bit words for the clustering call's sort: lo[i] and hi[i] (hi = lo + n),
  // or the high half alone in lo[i] once the low half is dropped
  const bool split = drop_out != nullptr;
  const bool halves = split && first < 4;
  uint32_t* lo32 = reinterpret_cast<uint32_t*>(keys);
  uint32_t* hi32 = lo32 + n;
  auto put = [&](uint32_t i, uint64_t c) {
    if (!split) {
      keys[i] = c;
    } else if (halves) {
      lo32[i] = uint32_t(c);
      hi32[i] = uint32_t(c >> 32);
    } else {
      lo32[i] = uint32_t(c >> 32);
    }
  };
  __syncthreads();
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t first_scalar = 0;
  if (VEC) {
    const uint32_t groups = n / 4;
    const float4* p4 = reinterpret_cast<const float4*>(pts);
    ulonglong2* k2 = reinterpret_cast<ulonglong2*>(keys);
    auto code4 = [&](uint32_t g, const float4& a, const float4& b, const float4& c) {
      const uint64_t c0 = grid.code(a.x, a.y, a.z) & mask;
      const uint64_t c1 = grid.code(a.w, b.x, b.y) & mask;
      const uint64_t c2 = grid.code(b.z, b.w, c.x) & mask;
      const uint64_t c3 = grid.code(c.y, c.z, c.w) & mask;
      if (!split) {
        k2[2 * size_t(g)] = make_ulonglong2(c0, c1);
        k2[2 * size_t(g) + 1] = make_ulonglong2(c2, c3);
      } else if (halves) {  // 4-aligned word groups: n may be odd, so no 16-byte stores at n + i
        put(4 * g, c0); put(4 * g + 1, c1); put(4 * g + 2, c2); put(4 * g + 3, c3);
      } else {
        reinterpret_cast<uint4*>(lo32)[g] =
            make_uint4(uint32_t(c0 >> 32), uint32_t(c1 >> 32), uint32_t(c2 >> 32),
                       uint32_t(c3 >> 32));
      }
      count_digits(sh, c0, first);
      count_digits(sh, c1, first);
      count_digits(sh, c2, first);
      count_digits(sh, c3, first);
    };
    // two groups (six loads) in flight per thread
    uint32_t g = gid;
    for (; uint64_t(g) + stride < groups; g += 2 * stride) {
      const size_t f = 3 * size_t(g), h = 3 * size_t(g + stride);
      const float4 a0 = p4[f], b0 = p4[f + 1], c0 = p4[f + 2];
      const float4 a1 = p4[h], b1 = p4[h + 1], c1 = p4[h + 2];
      code4(g, a0, b0, c0);
      code4(g + stride, a1, b1, c1);
    }
    for (; g < groups; g += stride) {
      const size_t f = 3 * size_t(g);
      code4(g, p4[f], p4[f + 1], p4[f + 2]);
    }
    first_scalar = groups * 4;
  }
  for (uint32_t i = first_scalar + gid; i < n; i += stride) {
    const float* p = pts + size_t(3) * i;
    const uint64_t code = grid.code(p[0], p[1], p[2]) & mask;
    put(i, code);
    count_digits(sh, code, first);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x)
    if (sh[t]) atomicAdd(&hist[t], sh[t]);
}

__global__ __launch_bounds__(256) void k_gather(
    const float* __restrict__ pts, const uint32_t* __restrict__ perm, uint32_t n,
    float4* __restrict__ leaf, int32_t* __restrict__ parent, int32_t* __restrict__ minlab,
    uint8_t* __restrict__ flag, unsigned long long* __restrict__ bestcore,
    int32_t* __restrict__ labels) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) leaf[n] = make_float4(0.f, 0.f, 0.f, __int_as_float(SENTINEL));  // padding
  if (i >= n) return;
  const uint32_t o = min(perm[i], n - 1);  // a permutation unless the sort failed
  const float* p = pts + size_t(3) * o;
  leaf[i] = make_float4(p[0], p[1], p[2], __int_as_float(SENTINEL));
  parent[i] = int32_t(i);
  if (minlab) minlab[i] = 0x7fffffff;
  flag[i] = 0;
  if (bestcore) bestcore[i] = ~0ull;
  if (labels) labels[i] = -1;  // by input index: every index once
}

// Reductions into a few global words (bounds, digit counts): 1024 blocks of
// 256 threads keep every CU busy while bounding the closing global atomics.
uint32_t reduce_blocks(uint32_t n) { return std::max(1u, std::min((n + 1023) / 1024, 1024u)); }
// the bounds pass: two blocks per CU (1,024 or 2,048 blocks were slower:
// 0.056 and 0.071 against 0.046 ms over 2^24 points; the Morton pass, which
// also writes the codes, stays on reduce_blocks: 0.066 against 0.069 ms)
uint32_t bounds_blocks(uint32_t n) { return std::max(1u, std::min((n + 1023) / 1024, 512u)); }

}  // namespace

void launch_prep(uint32_t* zero_region, size_t zero_words, uint32_t* bounds, int4* pending,
                 uint32_t pending_entries, hipStream_t s) {
  const size_t work = std::max<size_t>(zero_words, pending_entries);
  uint32_t blocks = uint32_t(std::min<size_t>((work + 255) / 256 + 1, 4096));
  hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(256), 0, s, zero_region, zero_words, bounds,
                     pending, pending_entries);
}

void launch_bounds(const float* pts, uint32_t n, uint32_t* bounds, uint32_t* status,
                   hipStream_t s) {
  if (n == 0) return;
  if (reinterpret_cast<uintptr_t>(pts) % 16 == 0)
    hipLaunchKernelGGL(k_bounds<true>, dim3(bounds_blocks(n)), dim3(256), 0, s, pts, n, bounds,
                       status);
  else
    hipLaunchKernelGGL(k_bounds<false>, dim3(reduce_blocks(n)), dim3(256), 0, s, pts, n, bounds,
                       status);
}

void launch_morton(const float* pts, uint32_t n, const uint32_t* bounds, float eps,
                   uint64_t* keys_a, uint64_t* keys_b, uint32_t* drop_out, uint32_t* hist,
                   hipStream_t s) {
  if (n == 0) return;
  // the point array may not be 16-byte aligned (arena buffers are)
  const bool vec = reinterpret_cast<uintptr_t>(pts) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(keys_a) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(keys_b) % 16 == 0;
  if (vec)
    hipLaunchKernelGGL(k_morton<true>, dim3(reduce_blocks(n)), dim3(256), 0, s, pts, n, bounds,
                       eps, keys_a, keys_b, drop_out, hist);
  else
    hipLaunchKernelGGL(k_morton<false>, dim3(reduce_blocks(n)), dim3(256), 0, s, pts, n, bounds,
                       eps, keys_a, keys_b, drop_out, hist);
}

void launch_gather(const float* pts, const uint32_t* perm, uint32_t n, float4* leaf,
                   int32_t* parent, int32_t* minlab, uint8_t* flag,
                   unsigned long long* bestcore, int32_t* labels, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, s, pts, perm, n, leaf,
                     parent, minlab, flag, bestcore, labels);
}

}  // namespace dbx
