// Device-side building blocks shared by the DBSCAN kernels (gfx950 only).
//
// Layout of the linear BVH (paper, section 3.2 and 4.2.1):
//   internal node k (0 <= k < n-1), 32 bytes:  float lo[3]; int left;
//                                              float hi[3]; int rope;
//   leaf j (0 <= j < n), 16 bytes:             float x, y, z; int rope
//     (the leaf array is the points in Morton order; the rope sits in .w)
//   node references: k >= 0 internal, (j | LEAF_BIT) a leaf, SENTINEL = -1.
// Internal nodes are in Karras' order: the node covering leaves [l, r] is
// number r if it is its parent's left child, number l if the right child,
// and the root is number 0; so a rope target's number is its first leaf.
// Every reference fits in 32 bits for n < 2^31.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dbx {

constexpr int32_t LEAF_BIT = int32_t(0x80000000u);
constexpr int32_t SENTINEL = -1;
constexpr int MORTON_BITS = 21;           // per axis, 63-bit codes

struct alignas(16) Node {
  float lox, loy, loz;
  int32_t left;
  float hix, hiy, hiz;
  int32_t rope;
};
static_assert(sizeof(Node) == 32, "node must be 32 bytes");

__device__ __forceinline__ bool is_leaf(int32_t ref) { return ref < -1; }
__device__ __forceinline__ int32_t leaf_ref(int32_t j) { return j | LEAF_BIT; }
__device__ __forceinline__ int32_t leaf_index(int32_t ref) { return ref & 0x7fffffff; }

// ---- the one distance predicate (section 3.1, eps-neighbourhood) ---------
// Squared Euclidean distance in binary32, ((dx*dx + dy*dy) + dz*dz), every
// operation rounded on its own.  The library is compiled with
// -ffp-contract=off; the pragma keeps this true even if that flag is lost.
__device__ __forceinline__ float sq_dist(float ax, float ay, float az,
                                         float bx, float by, float bz) {
#pragma clang fp contract(off)
  float dx = ax - bx;
  float dy = ay - by;
  float dz = az - bz;
  float xx = dx * dx;
  float yy = dy * dy;
  float zz = dz * dz;
  float s = xx + yy;
  return s + zz;
}

// Lower bound of sq_dist(q, p) over all p in the box [lo, hi].  For p in the
// box, |fl(p_a - q_a)| >= fl(lo_a - q_a) (resp. fl(q_a - hi_a)) because
// rounding is monotone, and squares and sums are monotone too, so pruning a
// box whose bound exceeds e2 never drops a point that passes the predicate.
__device__ __forceinline__ float box_sq_dist(float qx, float qy, float qz,
                                             const Node& nd) {
#pragma clang fp contract(off)
  float gx = fmaxf(fmaxf(nd.lox - qx, qx - nd.hix), 0.0f);
  float gy = fmaxf(fmaxf(nd.loy - qy, qy - nd.hiy), 0.0f);
  float gz = fmaxf(fmaxf(nd.loz - qz, qz - nd.hiz), 0.0f);
  float xx = gx * gx;
  float yy = gy * gy;
  float zz = gz * gz;
  float s = xx + yy;
  return s + zz;
}

// ---- scoped atomics --------------------------------------------------------
// gfx950 has one L2 per XCD; agent scope makes accesses coherent across them.
template <class T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T ld_wg(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <class T>
__device__ __forceinline__ void st_wg(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <class T>
__device__ __forceinline__ T cas_agent(T* p, T expected, T desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the value found (== the old expected on success)
}

// ---- lock-free union-find (section 4.3, disjoint sets) --------------------
// parent[] over Morton-sorted positions, roots ordered by key[] (the sort's
// permutation: a position's input index).  Invariant: a non-root x always
// has key[parent[x]] < key[x], so the forest stays acyclic whatever order
// racing writes land in, every value ever stored is an ancestor, and the
// root of a set is its member with the smallest input index: the cluster's
// label.  Roots are hooked by CAS (the one with the larger key under the
// other); path halving uses plain relaxed stores, which only ever touch
// non-roots and so never undo a hook.
//
// The finds read and halve at workgroup scope: a load may hit a stale line
// in the CU's own cache.  That is safe.  Every value parent[x] ever held is
// a node of x's set with a smaller key, so a stale read still moves down a
// chain of x's set with strictly decreasing keys, and a stale "root" r is
// still in the set.  A union that ends because both finds met the same node
// joins two nodes that are already connected; one whose CAS expects a stale
// root fails (the CAS is at agent scope and sees the true value) and
// continues from the value it found, whose key is smaller: so every union
// ends.  Finds after the kernel (label finalisation) run in a later launch
// and see the final forest.
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
  for (;;) {
    int32_t p = ld_wg(parent + x);
    if (p == x) return x;
    int32_t gp = ld_wg(parent + p);
    if (gp == p) return p;
    st_wg(parent + x, gp);
    x = gp;
  }
}

// Union of the sets of a and b.  Returns a node that is, at return, an
// ancestor of both (the merged root or, if others hooked it meanwhile, one
// of its descendants): a walk that unions one point with many neighbours
// passes it back as `a` and so starts each find from high up its chain.
__device__ __forceinline__ int32_t uf_union(int32_t* parent, const uint32_t* __restrict__ key,
                                            int32_t a, int32_t b) {
  for (;;) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return a;
    if (key[a] > key[b]) { int32_t t = a; a = b; b = t; }
    int32_t seen = cas_agent(parent + b, b, a);
    if (seen == b) return a;
    b = seen;  // b was hooked under `seen` meanwhile: continue from there
  }
}

// Roots of K points at once, once the forest no longer changes: the K
// chains climb in lockstep, so a thread keeps K independent loads in flight
// (the chains are short; their latency, not bandwidth, bounds the final
// pass).  x[k] < 0: no point there, left as is.  Plain loads, no writes.
template <int K>
__device__ __forceinline__ void uf_roots_final(const int32_t* parent, int32_t (&x)[K]) {
  int32_t p[K];
#pragma unroll
  for (int k = 0; k < K; ++k) p[k] = x[k] >= 0 ? parent[x[k]] : x[k];
  bool more = true;
  while (more) {
    more = false;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (p[k] != x[k]) {
        x[k] = p[k];
        p[k] = parent[x[k]];
        more = true;
      }
  }
}

// ---- Morton codes (section 4.2.2) ------------------------------------------
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

// grid coordinate of p on one axis: min(floor((p - lo) * s), maxc) in
// binary32, s = (maxc + 1) / extent (0 for a zero extent), maxc = 2^b - 1
// for b bits per axis; monotone in p
__device__ __forceinline__ uint32_t quantise(float p, float lo, float s,
                                             float maxc = float((1u << MORTON_BITS) - 1)) {
#pragma clang fp contract(off)
  float t = (p - lo) * s;
  t = fminf(fmaxf(floorf(t), 0.0f), maxc);  // NaN -> 0
  return uint32_t(t);
}

__device__ __forceinline__ uint64_t morton_of(float x, float y, float z, const float* lo,
                                              const float* s,
                                              float maxc = float((1u << MORTON_BITS) - 1)) {
  return (spread3(quantise(x, lo[0], s[0], maxc)) << 2) |
         (spread3(quantise(y, lo[1], s[1], maxc)) << 1) | spread3(quantise(z, lo[2], s[2], maxc));
}

// Ordered-integer view of a float for atomic min/max of scene bounds.
__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float ord2f(uint32_t u) {
  uint32_t b = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  float f;
  __builtin_memcpy(&f, &b, 4);
  return f;
}

// Low code bits a clustering call may drop (a multiple of 8 up to 40: whole
// sort passes).  The codes only shape the tree; the walks prune with exact
// boxes.  A drop is taken if the grid cells it leaves are
//  * at most eps/2 wide on every axis: points that then share a code lie
//    within 0.87 eps of each other, mutual neighbours that the walks meet
//    together anyway; or
//  * at most 2.5 eps wide and so small against the point density that the
//    field holds at most 1/16 point per cell on average (n times a cell's
//    share of the bounding box): codes are then nearly all distinct, and
//    the tree over them is as good as over finer ones.
// Bit b of a code belongs to axis z, y, x for b % 3 = 0, 1, 2.  eps <= 0:
// none.
__device__ inline int droppable_code_bits(const uint32_t* bounds, float eps, uint32_t n) {
  if (!(eps > 0.0f)) return 0;
  int best = 0;
  for (int d = 8; d <= 40; d += 8) {
    bool fine = true, coarse = true;
    double per_cell = double(n);
    for (int a = 0; a < 3; ++a) {  // x, y, z
      const int off = 2 - a;       // the axis' bit position within a triple
      const int dropped = d > off ? (d - off + 2) / 3 : 0;
      const double share = ldexp(1.0, dropped - MORTON_BITS);  // cell / extent
      const double ext = double(ord2f(bounds[3 + a])) - double(ord2f(bounds[a]));
      fine = fine && ext * share <= 0.5 * double(eps);
      coarse = coarse && ext * share <= 2.5 * double(eps);
      if (ext > 0.0) per_cell *= share;
    }
    if (fine || (coarse && per_cell <= 1.0 / 16.0)) best = d;
  }
  return best;
}

// The grid the Morton codes quantise to, from the scene bounds words
// (bounds[0..2] lo, [3..5] hi, ordered ints).
// (Batched sets: one grid per set, b bits per axis, maxc = 2^b - 1.)
struct MortonGrid {
  float lo[3], s[3];
  float maxc;
  __device__ void load(const uint32_t* bounds) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = ord2f(bounds[a]);
      const float ext = ord2f(bounds[3 + a]) - lo[a];
      s[a] = ext > 0.0f ? float(1u << MORTON_BITS) / ext : 0.0f;  // IEEE division
    }
    maxc = float((1u << MORTON_BITS) - 1);
  }
  __device__ uint64_t code(float x, float y, float z) const {
    return morton_of(x, y, z, lo, s, maxc);
  }
  // A code no smaller than that of any point p with sq_dist(q, p) <= e2.
  // Such a p has |p_a - q_a| <= sqrt(e2) (1 + 3u) on every axis (u = 2^-24),
  // so p_a <= h_a = q_a + pad (pad covers that and the rounding of the sum,
  // and an absolute 1e-22 for e2 that underflow); quantise() and the
  // interleaving are monotone, so code(p) <= code(h).
  __device__ uint64_t upper_code(const float4& q, float e2) const {
    const float pad = sqrtf(e2) * 1.0001f + 1e-22f;
    const float hx = q.x + (pad + fabsf(q.x) * 1e-6f);
    const float hy = q.y + (pad + fabsf(q.y) * 1e-6f);
    const float hz = q.z + (pad + fabsf(q.z) * 1e-6f);
    return code(hx, hy, hz);
  }
};

// Digit counts of the sort passes for one key per active lane, into the LDS
// table sh[pass][digit].  Where every active lane has the same digit (code
// bits that are constant across the points, or a batched set's id) the wave
// adds its count with one atomic instead of piling 64 onto one bin.
__device__ __forceinline__ void count_digits_wave(uint32_t* sh, uint64_t code, int passes) {
  const uint64_t active = __ballot(true);
  const int first = __ffsll(static_cast<long long>(active)) - 1;
  const int lane = threadIdx.x & 63;
  for (int q = 0; q < passes; ++q) {
    const uint32_t d = uint32_t(code >> (8 * q)) & 0xffu;
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
    if (__ballot(d == d0) == active) {
      if (lane == first) atomicAdd(&sh[q * 256 + d0], uint32_t(__popcll(active)));
    } else {
      atomicAdd(&sh[q * 256 + d], 1u);
    }
  }
}

// XCD-aware block order: the hardware deals consecutive workgroups to the
// 8 XCDs round-robin; remap so each XCD works on one contiguous stretch of
// tiles (Morton-adjacent queries share tree nodes in that XCD's L2).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb) {
  constexpr uint32_t X = 8;
  uint32_t per = nb / X, extra = nb % X;
  uint32_t xcd = b % X, slot = b / X;
  // XCDs below `extra` own per+1 tiles
  uint32_t base = xcd * per + (xcd < extra ? xcd : extra);
  return base + slot;
}

}  // namespace dbx
