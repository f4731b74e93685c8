// FDBSCAN-DenseBox (section 4.3.4): a regular grid of cell side eps/sqrt(3)
// is laid over the points, so a cell's diameter is at most eps; a cell with
// at least minPts points is "dense": all its points are core and no distance
// between two of them needs computing.  The BVH is built over a mix of
// primitives -- dense cells (as boxes) and the points outside dense cells --
// and a traversal that finds a dense cell searches the cell's points.
//
// Exactness under binary32 rounding.  Grid coordinates only decide which
// points share a cell; whether a cell is dense is decided on the cell's
// actual bounding box: dense <=> count >= T (T >= minPts) and
// sq_dist(box.lo, box.hi) <= e2.  For p, q in the box, |fl(p_a - q_a)| <=
// fl(hi_a - lo_a) (rounding is monotone) and squares and sums are monotone
// too, so every pair in a dense cell passes the predicate.  The same
// argument gives the two shortcuts below: the farthest corner of a box from
// a point (or from another box) bounds sq_dist from above for every point
// of the box, and the nearest one (box_sq_dist) from below.
//
// Cross pairs are handled once each by a pair traversal over primitives
// (section 4.2.3 applied to the mixed tree): point-point as in FDBSCAN;
// point-cell: a core point joins the cell's cluster on the first cell point
// within eps, a non-core point takes the smallest-input-index cell point
// within eps as its border candidate; cell-cell: skipped when both cells
// are already in one cluster, else joined on the first pair within eps.
#include <algorithm>

#include "pipeline.hpp"

namespace dbx {

namespace {

constexpr int32_t CELL_BIT = int32_t(0x80000000u);
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
constexpr uint32_t ST_AGG = 1u << 30;
constexpr uint32_t ST_INC = 2u << 30;
constexpr uint32_t ST_VAL = (1u << 30) - 1;
constexpr uint32_t SPIN_LIMIT = 1u << 22;

// Cell key: Morton code of the cell coordinates, so sorting by it orders
// the cells along the Z-curve.  Side max(h, extent / 2^21) per axis.
__global__ __launch_bounds__(256) void k_cell_keys(const float* __restrict__ pts, uint32_t n,
                                                  const uint32_t* __restrict__ bounds, float inv_h,
                                                  uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ hist) {
  __shared__ uint32_t sh[SORT_PASSES * RADIX];
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x) sh[t] = 0;
  float lo[3], s[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = ord2f(bounds[a]);
    const float ext = ord2f(bounds[3 + a]) - lo[a];
    s[a] = fminf(inv_h, float(1u << MORTON_BITS) / ext);  // ext = 0 gives inv_h
  }
  __syncthreads();
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    uint32_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float t = (pts[size_t(3) * i + a] - lo[a]) * s[a];
      t = fminf(fmaxf(floorf(t), 0.0f), float((1u << MORTON_BITS) - 1));  // NaN -> 0
      c[a] = uint32_t(t);
    }
    const uint64_t code = (spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]);
    keys[i] = code;
#pragma unroll
    for (int q = 0; q < SORT_PASSES; ++q)
      atomicAdd(&sh[q * RADIX + ((code >> (8 * q)) & 0xff)], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x)
    if (sh[t]) atomicAdd(&hist[t], sh[t]);
}

__global__ __launch_bounds__(256) void k_cell_heads(const uint64_t* __restrict__ keys, uint32_t n,
                                                   uint32_t* __restrict__ head) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// Exclusive prefix sum of u32 with the total, one pass: tiles take ids from
// a counter and find their offset by decoupled look-back (bounded waits).
__global__ __launch_bounds__(SCAN_THREADS) void k_scan(const uint32_t* __restrict__ in,
                                                      uint32_t* __restrict__ out, uint32_t n,
                                                      uint32_t* __restrict__ total,
                                                      uint32_t* __restrict__ status,
                                                      uint32_t* __restrict__ tile_ctr,
                                                      uint32_t* __restrict__ err) {
  __shared__ uint32_t s_tile, s_prefix;
  __shared__ uint32_t s_tmp[SCAN_THREADS / 64];
  if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint32_t base = tile * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? in[base + k] : 0u;
    sum += v[k];
  }
  // block exclusive scan of the thread sums
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  uint32_t wadd = 0, agg = 0;
  for (int w = 0; w < SCAN_THREADS / 64; ++w) {
    if (w < wave) wadd += s_tmp[w];
    agg += s_tmp[w];
  }
  const uint32_t texcl = x - sum + wadd;
  if (threadIdx.x == 0) {
    uint32_t excl = 0;
    uint32_t* st = status + tile;
    if (tile == 0) {
      st_agent(st, ST_INC | agg);
    } else {
      st_agent(st, ST_AGG | agg);
      int32_t j = int32_t(tile) - 1;
      uint32_t spins = 0;
      while (j >= 0) {
        const uint32_t w = ld_agent(status + j);
        const uint32_t f = w & ~ST_VAL;
        if (f == 0) {
          if (++spins > SPIN_LIMIT) { atomicOr(err, STATUS_SORT_STALL); break; }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += w & ST_VAL;
        if (f == ST_INC) break;
        --j;
      }
      st_agent(st, ST_INC | ((excl + agg) & ST_VAL));
    }
    s_prefix = excl;
    if ((tile + 1) * uint32_t(SCAN_TILE) >= n) *total = excl + agg;
  }
  __syncthreads();
  uint32_t run = s_prefix + texcl;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

// cid[i] = cell of sorted point i; cell_start[c] = first point of cell c,
// cell_start[ncells] = n.
__global__ __launch_bounds__(256) void k_cell_start(const uint32_t* __restrict__ head,
                                                   uint32_t* __restrict__ cid, uint32_t n,
                                                   const uint32_t* __restrict__ ncells,
                                                   uint32_t* __restrict__ cell_start) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t h = head[i];
  const uint32_t c = cid[i] + h - 1;  // exclusive count of heads before i, plus own
  cid[i] = c;
  if (h) cell_start[c] = i;
  if (i == 0) cell_start[*ncells] = n;
}

// Per cell: box, denseness, smallest (input index, position) over its
// points, and how many primitives it contributes (1 if dense, else one per
// point).  Threads past the last cell write a zero count.
__global__ __launch_bounds__(256) void k_cell_stats(
    const float4* __restrict__ pts, const uint32_t* __restrict__ perm, uint32_t n,
    const uint32_t* __restrict__ ncells_p, const uint32_t* __restrict__ cell_start, float e2,
    int32_t thresh, float4* __restrict__ cell_lo, float4* __restrict__ cell_hi,
    unsigned long long* __restrict__ cell_minorig, uint8_t* __restrict__ cell_dense,
    uint32_t* __restrict__ prim_count) {
  const uint32_t ncells = *ncells_p;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    if (c >= ncells) { prim_count[c] = 0; continue; }
    const uint32_t b = cell_start[c], e = cell_start[c + 1];
    float4 lo = pts[b], hi = lo;
    unsigned long long mo = (static_cast<unsigned long long>(perm[b]) << 32) | b;
    for (uint32_t i = b + 1; i < e; ++i) {
      const float4 p = pts[i];
      lo.x = fminf(lo.x, p.x); lo.y = fminf(lo.y, p.y); lo.z = fminf(lo.z, p.z);
      hi.x = fmaxf(hi.x, p.x); hi.y = fmaxf(hi.y, p.y); hi.z = fmaxf(hi.z, p.z);
      const unsigned long long o = (static_cast<unsigned long long>(perm[i]) << 32) | i;
      mo = o < mo ? o : mo;
    }
    const uint32_t cnt = e - b;
    const bool dense =
        int64_t(cnt) >= thresh && sq_dist(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z) <= e2;
    cell_lo[c] = lo;
    cell_hi[c] = hi;
    if (cell_minorig) cell_minorig[c] = mo;
    cell_dense[c] = dense;
    prim_count[c] = dense ? 1u : cnt;
  }
}

// Primitive records (Node layout: box, payload in `left`), their keys for
// the build, and the state of dense-cell points: joined to the cell's first
// point, marked core (or member, for minPts <= 2).
__global__ __launch_bounds__(256) void k_make_prims(
    const float4* __restrict__ pts, const uint64_t* __restrict__ keys, uint32_t n,
    const uint32_t* __restrict__ cid, const uint32_t* __restrict__ cell_start,
    const uint32_t* __restrict__ prim_start, const uint8_t* __restrict__ cell_dense,
    const float4* __restrict__ cell_lo, const float4* __restrict__ cell_hi,
    Node* __restrict__ prims, uint64_t* __restrict__ pkey, int32_t* __restrict__ parent,
    uint8_t* __restrict__ flag) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = cid[i];
  const uint32_t b = cell_start[c];
  float4* out;
  if (cell_dense[c]) {
    parent[i] = int32_t(b);
    flag[i] = 1;
    if (i != b) return;
    const uint32_t j = prim_start[c];
    out = reinterpret_cast<float4*>(prims + j);
    const float4 lo = cell_lo[c], hi = cell_hi[c];
    out[0] = make_float4(lo.x, lo.y, lo.z, __int_as_float(int32_t(c) | CELL_BIT));
    out[1] = make_float4(hi.x, hi.y, hi.z, __int_as_float(SENTINEL));
    pkey[j] = keys[i];
  } else {
    const uint32_t j = prim_start[c] + (i - b);
    out = reinterpret_cast<float4*>(prims + j);
    const float4 p = pts[i];
    out[0] = make_float4(p.x, p.y, p.z, __int_as_float(int32_t(i)));
    out[1] = make_float4(p.x, p.y, p.z, __int_as_float(SENTINEL));
    pkey[j] = keys[i];
  }
}

// ---- traversal helpers ------------------------------------------------------

__device__ __forceinline__ Node load_node(const Node* __restrict__ nodes, int32_t k) {
  const float4* p = reinterpret_cast<const float4*>(nodes + k);
  const float4 a = p[0], b = p[1];
  Node nd;
  nd.lox = a.x; nd.loy = a.y; nd.loz = a.z; nd.left = __float_as_int(a.w);
  nd.hix = b.x; nd.hiy = b.y; nd.hiz = b.z; nd.rope = __float_as_int(b.w);
  return nd;
}

// lower bound of sq_dist between any point of box a and any point of box b
__device__ __forceinline__ float box_box_near(const Node& a, const Node& b) {
#pragma clang fp contract(off)
  const float gx = fmaxf(fmaxf(b.lox - a.hix, a.lox - b.hix), 0.0f);
  const float gy = fmaxf(fmaxf(b.loy - a.hiy, a.loy - b.hiy), 0.0f);
  const float gz = fmaxf(fmaxf(b.loz - a.hiz, a.loz - b.hiz), 0.0f);
  const float xx = gx * gx, yy = gy * gy, zz = gz * gz;
  const float s = xx + yy;
  return s + zz;
}

// upper bound of sq_dist between any point of box a and any point of box b
// (a point is a box with lo = hi)
__device__ __forceinline__ float box_box_far(const Node& a, const Node& b) {
#pragma clang fp contract(off)
  const float dx = fmaxf(fabsf(a.hix - b.lox), fabsf(b.hix - a.lox));
  const float dy = fmaxf(fabsf(a.hiy - b.loy), fabsf(b.hiy - a.loy));
  const float dz = fmaxf(fabsf(a.hiz - b.loz), fabsf(b.hiz - a.loz));
  const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
  const float s = xx + yy;
  return s + zz;
}

__device__ __forceinline__ bool bad_ref(int32_t node, uint32_t n, uint32_t& steps) {
  if (++steps > 2 * n) return true;
  return is_leaf(node) ? uint32_t(leaf_index(node)) >= n : uint32_t(node) >= n - 1;
}

__device__ __forceinline__ uint32_t query_index() {
  return xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

// Counting (minPts > 2) for the points outside dense cells (theirs are core
// already): a full walk from the root, early exit at minPts.
__global__ void k_count_db(const Node* __restrict__ nodes, const Node* __restrict__ prims,
                           uint32_t nprims, const float4* __restrict__ pts, uint32_t n,
                           const uint32_t* __restrict__ cell_start, const int32_t* __restrict__ root,
                           float e2, int32_t min_pts, uint8_t* __restrict__ flag,
                           uint32_t* __restrict__ err) {
  const uint32_t i = query_index();
  if (i >= n || flag[i]) return;
  const float4 q4 = pts[i];
  Node q;
  q.lox = q.hix = q4.x; q.loy = q.hiy = q4.y; q.loz = q.hiz = q4.z;
  int32_t cnt = 0;
  int32_t node = *root;
  uint32_t steps = 0;
  while (node != SENTINEL && cnt < min_pts) {
    if (bad_ref(node, nprims, steps)) { atomicOr(err, STATUS_TREE); break; }
    if (!is_leaf(node)) {
      const Node nd = load_node(nodes, node);
      node = box_box_near(q, nd) <= e2 ? nd.left : nd.rope;
      continue;
    }
    const Node pr = load_node(prims, leaf_index(node));
    node = pr.rope;
    if (box_box_near(q, pr) > e2) continue;
    if (pr.left >= 0) {  // a point: its box is the point
      cnt += 1;
    } else {
      const uint32_t c = uint32_t(pr.left & 0x7fffffff);
      const uint32_t b = cell_start[c], e = cell_start[c + 1];
      if (box_box_far(q, pr) <= e2) {
        cnt += int32_t(e - b);
      } else {
        for (uint32_t k = b; k < e && cnt < min_pts; ++k) {
          const float4 p = pts[k];
          cnt += sq_dist(q.lox, q.loy, q.loz, p.x, p.y, p.z) <= e2;
        }
      }
    }
  }
  flag[i] = cnt >= min_pts;
}

struct DbArgs {
  const Node* nodes;
  const Node* prims;
  uint32_t nprims;
  const float4* pts;
  uint32_t n;
  const uint32_t* cell_start;
  const uint32_t* perm;
  const unsigned long long* cell_minorig;
  float e2;
  bool core_mode;     // minPts > 2
  int32_t* parent;
  uint8_t* flag;      // core (minPts > 2) or member (minPts <= 2)
  unsigned long long* bestcore;
  uint32_t* err;
};

__device__ __forceinline__ unsigned long long orig_key(const DbArgs& A, uint32_t pos) {
  return (static_cast<unsigned long long>(A.perm[pos]) << 32) | pos;
}

// Point x (sorted position xp, coordinates in box form) against dense cell c.
__device__ void point_cell(const DbArgs& A, uint32_t xp, const Node& xb, const Node& cb,
                           uint32_t c) {
  const uint32_t b = A.cell_start[c], e = A.cell_start[c + 1];
  const bool all_in = box_box_far(xb, cb) <= A.e2;
  const bool x_core = !A.core_mode || A.flag[xp];
  if (x_core) {
    bool hit = all_in;
    for (uint32_t k = b; k < e && !hit; ++k) {
      const float4 p = A.pts[k];
      hit = sq_dist(xb.lox, xb.loy, xb.loz, p.x, p.y, p.z) <= A.e2;
    }
    if (hit) {
      uf_union(A.parent, int32_t(xp), int32_t(b));
      if (!A.core_mode) A.flag[xp] = 1;
    }
  } else {  // border candidate: smallest input index among cell points in range
    unsigned long long best = ~0ull;
    if (all_in) {
      best = A.cell_minorig[c];
    } else {
      for (uint32_t k = b; k < e; ++k) {
        const float4 p = A.pts[k];
        if (sq_dist(xb.lox, xb.loy, xb.loz, p.x, p.y, p.z) <= A.e2) {
          const unsigned long long o = orig_key(A, k);
          best = o < best ? o : best;
        }
      }
    }
    if (best != ~0ull) atomicMin(A.bestcore + xp, best);
  }
}

__device__ void cell_cell(const DbArgs& A, const Node& ab, uint32_t ca, const Node& bb,
                          uint32_t cbi) {
  const uint32_t ra = A.cell_start[ca], rb = A.cell_start[cbi];
  if (uf_find(A.parent, int32_t(ra)) == uf_find(A.parent, int32_t(rb))) return;
  bool hit = box_box_far(ab, bb) <= A.e2;
  const uint32_t ea = A.cell_start[ca + 1], eb = A.cell_start[cbi + 1];
  for (uint32_t i = ra; i < ea && !hit; ++i) {
    const float4 p = A.pts[i];
    for (uint32_t k = rb; k < eb && !hit; ++k) {
      const float4 q = A.pts[k];
      hit = sq_dist(p.x, p.y, p.z, q.x, q.y, q.z) <= A.e2;
    }
  }
  if (hit) uf_union(A.parent, int32_t(ra), int32_t(rb));
}

__device__ void point_point(const DbArgs& A, uint32_t ip, const Node& ib, uint32_t jp,
                            const Node& jb, bool& found) {
  if (sq_dist(ib.lox, ib.loy, ib.loz, jb.lox, jb.loy, jb.loz) > A.e2) return;
  found = true;
  if (!A.core_mode) {
    uf_union(A.parent, int32_t(ip), int32_t(jp));
    A.flag[jp] = 1;
    return;
  }
  const bool ci = A.flag[ip] != 0, cj = A.flag[jp] != 0;
  if (ci && cj) uf_union(A.parent, int32_t(ip), int32_t(jp));
  else if (ci) atomicMin(A.bestcore + jp, orig_key(A, ip));
  else if (cj) atomicMin(A.bestcore + ip, orig_key(A, jp));
}

// Pair traversal over primitives: lane i starts at its primitive's rope and
// sees every primitive j > i whose box is within eps of its own.
__global__ void k_pairs_db(DbArgs A) {
  const uint32_t i = query_index();
  if (i >= A.nprims) return;
  const Node me = load_node(A.prims, int32_t(i));
  const bool me_cell = me.left < 0;
  const uint32_t me_idx = uint32_t(me.left & 0x7fffffff);
  bool found = false;
  int32_t node = me.rope;
  uint32_t steps = 0;
  while (node != SENTINEL) {
    if (bad_ref(node, A.nprims, steps)) { atomicOr(A.err, STATUS_TREE); break; }
    if (!is_leaf(node)) {
      const Node nd = load_node(A.nodes, node);
      node = box_box_near(me, nd) <= A.e2 ? nd.left : nd.rope;
      continue;
    }
    const Node pr = load_node(A.prims, leaf_index(node));
    node = pr.rope;
    if (box_box_near(me, pr) > A.e2) continue;
    const bool pr_cell = pr.left < 0;
    const uint32_t pr_idx = uint32_t(pr.left & 0x7fffffff);
    if (!me_cell && !pr_cell) point_point(A, me_idx, me, pr_idx, pr, found);
    else if (!me_cell) point_cell(A, me_idx, me, pr, pr_idx);
    else if (!pr_cell) point_cell(A, pr_idx, pr, me, me_idx);
    else cell_cell(A, me, me_idx, pr, pr_idx);
  }
  if (!A.core_mode && !me_cell && found) A.flag[me_idx] = 1;
}

}  // namespace

void launch_cell_keys(const float* pts, uint32_t n, const uint32_t* bounds, float inv_h,
                      uint64_t* keys, uint32_t* hist, hipStream_t s) {
  if (n == 0) return;
  const uint32_t blocks = std::max(1u, std::min((n + 255) / 256, 4096u));
  hipLaunchKernelGGL(k_cell_keys, dim3(blocks), dim3(256), 0, s, pts, n, bounds, inv_h, keys, hist);
}

size_t scan_status_words(uint32_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

void launch_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total,
                 uint32_t* status, uint32_t* tile_ctr, uint32_t* err, hipStream_t s) {
  if (n == 0) return;
  const uint32_t tiles = uint32_t(scan_status_words(n));
  hipLaunchKernelGGL(k_scan, dim3(tiles), dim3(SCAN_THREADS), 0, s, in, out, n, total, status,
                     tile_ctr, err);
}

void launch_cells(const uint64_t* sorted_keys, uint32_t n, uint32_t* head, uint32_t* cid,
                  uint32_t* ncells, uint32_t* cell_start, uint32_t* scan_status,
                  uint32_t* scan_ctr, uint32_t* err, hipStream_t s) {
  if (n == 0) return;
  const uint32_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_cell_heads, dim3(g), dim3(256), 0, s, sorted_keys, n, head);
  launch_scan(head, cid, n, ncells, scan_status, scan_ctr, err, s);
  hipLaunchKernelGGL(k_cell_start, dim3(g), dim3(256), 0, s, head, cid, n, ncells, cell_start);
}

void launch_cell_stats(const float4* pts, const uint32_t* perm, uint32_t n,
                       const uint32_t* ncells, const uint32_t* cell_start, float e2,
                       int32_t thresh, float4* cell_lo, float4* cell_hi,
                       unsigned long long* cell_minorig, uint8_t* cell_dense,
                       uint32_t* prim_count, hipStream_t s) {
  if (n == 0) return;
  const uint32_t blocks = std::max(1u, std::min((n + 255) / 256, 8192u));
  hipLaunchKernelGGL(k_cell_stats, dim3(blocks), dim3(256), 0, s, pts, perm, n, ncells,
                     cell_start, e2, thresh, cell_lo, cell_hi, cell_minorig, cell_dense,
                     prim_count);
}

void launch_make_prims(const float4* pts, const uint64_t* keys, uint32_t n, const uint32_t* cid,
                       const uint32_t* cell_start, const uint32_t* prim_start,
                       const uint8_t* cell_dense, const float4* cell_lo, const float4* cell_hi,
                       Node* prims, uint64_t* pkey, int32_t* parent, uint8_t* flag,
                       hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_make_prims, dim3((n + 255) / 256), dim3(256), 0, s, pts, keys, n, cid,
                     cell_start, prim_start, cell_dense, cell_lo, cell_hi, prims, pkey, parent,
                     flag);
}

void launch_count_db(const Node* nodes, const Node* prims, uint32_t nprims, const float4* pts,
                     uint32_t n, const uint32_t* cell_start, const int32_t* root, float e2,
                     int32_t min_pts, uint8_t* flag, uint32_t* err, int block, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_count_db, dim3((n + block - 1) / block), dim3(block), 0, s, nodes, prims,
                     nprims, pts, n, cell_start, root, e2, min_pts, flag, err);
}

void launch_pairs_db(const Node* nodes, const Node* prims, uint32_t nprims, const float4* pts,
                     uint32_t n, const uint32_t* cell_start, const uint32_t* perm,
                     const unsigned long long* cell_minorig, float e2, bool core_mode,
                     int32_t* parent, uint8_t* flag, unsigned long long* bestcore, uint32_t* err,
                     int block, hipStream_t s) {
  if (nprims == 0) return;
  DbArgs A{nodes, prims, nprims, pts, n, cell_start, perm, cell_minorig, e2, core_mode,
           parent, flag, bestcore, err};
  hipLaunchKernelGGL(k_pairs_db, dim3((nprims + block - 1) / block), dim3(block), 0, s, A);
}

}  // namespace dbx
