// Device-side building blocks shared by the DBSCAN kernels (gfx950 only).
//
// Layout of the linear BVH (paper, section 3.2 and 4.2.1):
//   internal node k (0 <= k < n-1), 32 bytes:  float lo[3]; int left;
//                                              float hi[3]; int rope;
//   leaf j (0 <= j < n), 16 bytes:             float x, y, z; int rope
//     (the leaf array is the points in Morton order; the rope sits in .w)
//   node references: k >= 0 internal, (j | LEAF_BIT) a leaf, SENTINEL = -1.
// Internal node k is the one whose split lies between leaves k and k+1
// (the Apetrei numbering), so every reference fits in 32 bits for n < 2^31.
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
__device__ __forceinline__ T cas_agent(T* p, T expected, T desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the value found (== the old expected on success)
}

// ---- lock-free union-find (section 4.3, disjoint sets) --------------------
// parent[] over Morton-sorted positions.  Invariant: a non-root x always has
// parent[x] < x, so the forest stays acyclic whatever order racing writes
// land in, and every value ever stored is an ancestor.  Roots are hooked by
// CAS (larger root under smaller); path halving uses plain relaxed stores,
// which only ever touch non-roots and so never undo a hook.
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
  for (;;) {
    int32_t p = ld_agent(parent + x);
    if (p == x) return x;
    int32_t gp = ld_agent(parent + p);
    if (gp == p) return p;
    st_agent(parent + x, gp);
    x = gp;
  }
}

__device__ __forceinline__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
  for (;;) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a > b) { int32_t t = a; a = b; b = t; }
    int32_t seen = cas_agent(parent + b, b, a);
    if (seen == b) return;
    b = seen;  // b was hooked under `seen` meanwhile: continue from there
  }
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
