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

#include "walk.hpp"

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
// the cells along the Z-curve.  Side max(h, extent / 2^21) per axis.  The
// grid goes to *grid for the walks' early end.
__global__ __launch_bounds__(256) void k_cell_keys(const float* __restrict__ pts, uint32_t n,
                                                  const uint32_t* __restrict__ bounds, float inv_h,
                                                  uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ hist,
                                                  MortonGrid* __restrict__ grid) {
  __shared__ uint32_t sh[SORT_PASSES * RADIX];
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x) sh[t] = 0;
  MortonGrid g;
  g.maxc = float((1u << MORTON_BITS) - 1);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = ord2f(bounds[a]);
    const float ext = ord2f(bounds[3 + a]) - g.lo[a];
    g.s[a] = ext > 0.0f ? fminf(inv_h, float(1u << MORTON_BITS) / ext) : 0.0f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *grid = g;
  __syncthreads();
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float* p = pts + size_t(3) * i;
    const uint64_t code = g.code(p[0], p[1], p[2]);
    keys[i] = code;
    count_digits_wave(sh, code, SORT_PASSES);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x)
    if (sh[t]) atomicAdd(&hist[t], sh[t]);
}

// What the scan below sums and where it puts the result.
// A plain exclusive prefix sum of u32 values:
struct ValueScan {
  const uint32_t* in;
  uint32_t* out;
  __device__ uint32_t load(uint32_t i) const { return in[i]; }
  __device__ void store(uint32_t i, uint32_t excl, uint32_t) const { out[i] = excl; }
  __device__ void finish(uint32_t, uint32_t) const {}
};
// The cells of the sorted cell keys: point i starts a cell where its key
// differs from point i-1's; cid[i] = its cell, cell_start[c] = the cell's
// first point, cell_start[ncells] = n (run heads, their scan and the starts
// in one pass).
struct CellScan {
  const uint64_t* keys;
  uint32_t* cid;
  uint32_t* cell_start;
  __device__ uint32_t load(uint32_t i) const {
    return (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
  }
  __device__ void store(uint32_t i, uint32_t excl, uint32_t head) const {
    const uint32_t c = excl + head - 1;  // heads before i, plus its own
    cid[i] = c;
    if (head) cell_start[c] = i;
  }
  __device__ void finish(uint32_t total, uint32_t n) const { cell_start[total] = n; }
};

// Exclusive prefix sum with the total, one pass: tiles take ids from a
// counter and find their offset by decoupled look-back (bounded waits).
template <class P>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan(P sc, uint32_t n,
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
    v[k] = base + k < n ? sc.load(base + k) : 0u;
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
    if ((tile + 1) * uint32_t(SCAN_TILE) >= n) {
      *total = excl + agg;
      sc.finish(excl + agg, n);
    }
  }
  __syncthreads();
  uint32_t run = s_prefix + texcl;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) sc.store(base + k, run, v[k]);
    run += v[k];
  }
}

// Per cell: box, denseness (its set's eps and threshold), smallest (input
// index, position) over its points, and how many primitives it contributes
// (1 if dense, else one per point).  Threads past the last cell write a zero
// count.
__global__ __launch_bounds__(256) void k_cell_stats(
    const float4* __restrict__ pts, const uint32_t* __restrict__ perm,
    const uint64_t* __restrict__ keys, uint32_t n, const uint32_t* __restrict__ ncells_p,
    const uint32_t* __restrict__ cell_start, DbSets S, float4* __restrict__ cell_lo,
    float4* __restrict__ cell_hi, unsigned long long* __restrict__ cell_minorig,
    uint8_t* __restrict__ cell_dense, uint32_t* __restrict__ prim_count) {
  const uint32_t ncells = *ncells_p;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    if (c >= ncells) { prim_count[c] = 0; continue; }
    const uint32_t b = cell_start[c], e = cell_start[c + 1];
    const uint32_t cnt = e - b;
    const uint32_t set = S.shift < 64 ? uint32_t(keys[b] >> S.shift) : 0u;
    if (int64_t(cnt) < S.thresh[set]) {  // too few points: its points are primitives
      cell_dense[c] = 0;
      prim_count[c] = cnt;
      continue;
    }
    float4 lo = pts[b], hi = lo;
    unsigned long long mo = (static_cast<unsigned long long>(perm[b]) << 32) | b;
    for (uint32_t i = b + 1; i < e; ++i) {
      const float4 p = pts[i];
      lo.x = fminf(lo.x, p.x); lo.y = fminf(lo.y, p.y); lo.z = fminf(lo.z, p.z);
      hi.x = fmaxf(hi.x, p.x); hi.y = fmaxf(hi.y, p.y); hi.z = fmaxf(hi.z, p.z);
      const unsigned long long o = (static_cast<unsigned long long>(perm[i]) << 32) | i;
      mo = o < mo ? o : mo;
    }
    const bool dense = sq_dist(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z) <= S.e2[set];
    cell_lo[c] = lo;
    cell_hi[c] = hi;
    cell_minorig[c] = mo;
    cell_dense[c] = dense;
    prim_count[c] = dense ? 1u : cnt;
  }
}

// Primitive records (Node layout: box, payload in `left`), their keys for
// the build, and the state of dense-cell points: joined to the cell's
// representative (its point with the smallest input index, which keeps the
// union-find's key order), marked core (or member, for minPts <= 2).
__global__ __launch_bounds__(256) void k_make_prims(
    const float4* __restrict__ pts, const uint64_t* __restrict__ keys, uint32_t n,
    const uint32_t* __restrict__ cid, const uint32_t* __restrict__ cell_start,
    const uint32_t* __restrict__ prim_start, const uint8_t* __restrict__ cell_dense,
    const float4* __restrict__ cell_lo, const float4* __restrict__ cell_hi,
    const unsigned long long* __restrict__ cell_minorig, Node* __restrict__ prims,
    uint64_t* __restrict__ pkey, int32_t* __restrict__ parent, uint8_t* __restrict__ flag,
    uint32_t* __restrict__ deg) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (deg) deg[i] = 0;  // pair counts start here (core flags by pair traversal)
  const uint32_t c = cid[i];
  const uint32_t b = cell_start[c];
  float4* out;
  if (cell_dense[c]) {
    parent[i] = int32_t(uint32_t(cell_minorig[c]));
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

// ---- the DenseBox walk --------------------------------------------------------
// The walk of walk.hpp over a tree whose leaves are primitives (32-byte
// records: box, payload, rope) and whose query is a box (a point is the box
// [p, p]; for two points the box bound is exactly the predicate's sq_dist,
// since fl(q - p) = -fl(p - q)).  Work that needs a scan of a dense cell's
// points is not done by the lane that meets it: the lane queues it in its
// wave's LDS queue, and the wave drains the queue together, 64 lanes over
// the cell's points, once it holds 64 entries and before the wave ends.  A
// lane queues at most one entry per step, so 128 slots never overflow.

constexpr uint32_t QCAP = 128;
constexpr int32_t Q_JOIN = 0;    // core point vs cell: join on the first hit
constexpr int32_t Q_BORDER = 1;  // non-core point vs cell: smallest core hit
constexpr int32_t Q_CELLS = 2;   // cell vs cell: join on the first close pair
constexpr int32_t Q_COUNT = 3;   // point vs cell: count hits for the owner lane
constexpr int32_t Q_DEG = 4;     // point vs cell: add the hits to the point's count
constexpr int32_t Q_MARK = 1 << 10;  // Q_JOIN: mark the point a member on a hit
constexpr uint32_t Q_ALL = 0xffffu;  // Q_COUNT: no early stop

// lower bound of sq_dist between a point of box [al, ah] and one of [bl, bh]
__device__ __forceinline__ float box_box_near4(const float4& al, const float4& ah,
                                               const float4& bl, const float4& bh) {
#pragma clang fp contract(off)
  const float gx = fmaxf(fmaxf(bl.x - ah.x, al.x - bh.x), 0.0f);
  const float gy = fmaxf(fmaxf(bl.y - ah.y, al.y - bh.y), 0.0f);
  const float gz = fmaxf(fmaxf(bl.z - ah.z, al.z - bh.z), 0.0f);
  const float xx = gx * gx, yy = gy * gy, zz = gz * gz;
  const float s = xx + yy;
  return s + zz;
}

// upper bound of the same (farthest corners)
__device__ __forceinline__ float box_box_far4(const float4& al, const float4& ah,
                                              const float4& bl, const float4& bh) {
#pragma clang fp contract(off)
  const float dx = fmaxf(fabsf(ah.x - bl.x), fabsf(bh.x - al.x));
  const float dy = fmaxf(fabsf(ah.y - bl.y), fabsf(bh.y - al.y));
  const float dz = fmaxf(fabsf(ah.z - bl.z), fabsf(bh.z - al.z));
  const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
  const float s = xx + yy;
  return s + zz;
}

__device__ __forceinline__ float sq_dist4(const float4& a, const float4& b) {
  return sq_dist(a.x, a.y, a.z, b.x, b.y, b.z);
}

__device__ __forceinline__ uint32_t set_id(const DbSets& S, uint64_t key) {
  return S.shift < 64 ? uint32_t(key >> S.shift) : 0u;
}

// the early-end bound of a query box of set `set`: every primitive within
// eps of the box has a cell key at most this (cell coordinates are monotone
// in the position, and a cell's box corner is one of its points)
__device__ __forceinline__ uint64_t set_upper(const DbSets& S, uint32_t set, const float4& hi,
                                              float e2) {
  const uint64_t tag = S.shift < 64 ? uint64_t(set) << S.shift : 0ull;
  return tag | S.grid[set].upper_code(hi, e2);
}

// What a queue drain reads and writes.
struct DbData {
  const float4* pts;  // points in cell order
  const uint32_t* cell_start;
  const uint32_t* perm;
  const unsigned long long* cell_minorig;
  const float4* cell_lo;
  const float4* cell_hi;
  int32_t* parent;
  uint8_t* flag;
  unsigned long long* bestcore;
  uint32_t* deg;  // neighbour counts (core flags by pair traversal), else null
};

// One wave's queue in LDS.
struct DbQueue {
  int4* q;
  uint32_t* n;
  __device__ void push(int32_t meta, int32_t a, int32_t b, float e2) const {
    const uint32_t k = atomicAdd(n, 1u);
    q[k] = make_int4(meta | ((threadIdx.x & 63) << 4), a, b, __float_as_int(e2));
  }
  __device__ uint32_t size() const {
    return __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT));
  }
};

// a dense cell's union-find representative (its smallest input index)
__device__ __forceinline__ int32_t cell_rep(const DbData& D, uint32_t c) {
  return int32_t(uint32_t(D.cell_minorig[c]));
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(v, o, 64);
    v = t < v ? t : v;
  }
  return v;
}

// Drain the wave's queue; every lane of the wave calls it.  Returns the
// points counted for this lane's Q_COUNT entries.
__device__ uint32_t drain(const DbData& D, const DbQueue& Q) {
  const int lane = threadIdx.x & 63;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the lanes' pushes are in
  __builtin_amdgcn_wave_barrier();
  const uint32_t m = Q.size();
  uint32_t added = 0;
  for (uint32_t e = 0; e < m; ++e) {
    const int4 en = Q.q[e];
    const int32_t meta = __builtin_amdgcn_readfirstlane(en.x);
    const int32_t a = __builtin_amdgcn_readfirstlane(en.y);
    const int32_t b = __builtin_amdgcn_readfirstlane(en.z);
    const float e2 = __int_as_float(__builtin_amdgcn_readfirstlane(en.w));
    const int32_t kind = meta & 15;
    if (kind == Q_CELLS) {
      const int32_t ra = cell_rep(D, uint32_t(a)), rb = cell_rep(D, uint32_t(b));
      if (uf_find(D.parent, ra) == uf_find(D.parent, rb)) continue;
      // lanes over the larger cell's points (only those near the smaller
      // cell's box), the smaller cell's points in turn for all lanes
      const uint32_t na = D.cell_start[a + 1] - D.cell_start[a];
      const uint32_t nb = D.cell_start[b + 1] - D.cell_start[b];
      const int32_t co = na >= nb ? a : b, ci = na >= nb ? b : a;
      const uint32_t os = D.cell_start[co], oe = D.cell_start[co + 1];
      const uint32_t is = D.cell_start[ci], ie = D.cell_start[ci + 1];
      const float4 ilo = D.cell_lo[ci], ihi = D.cell_hi[ci];
      bool hit = false;
      for (uint32_t o0 = os; o0 < oe && !hit; o0 += 64) {
        const uint32_t k = o0 + uint32_t(lane);
        const float4 p = D.pts[k < oe ? k : os];
        const bool act = k < oe && box_sq_dist4(p, ilo, ihi) <= e2;
        if (__ballot(act) == 0ull) continue;
        for (uint32_t j = is; j < ie; ++j) {
          const float4 r = D.pts[j];
          if (__ballot(act && sq_dist4(p, r) <= e2) != 0ull) { hit = true; break; }
        }
      }
      if (hit && lane == 0) uf_union(D.parent, D.perm, ra, rb);
      continue;
    }
    const float4 p = D.pts[a];
    const uint32_t cb = D.cell_start[b], ce = D.cell_start[b + 1];
    if (kind == Q_JOIN) {
      const int32_t rep = cell_rep(D, uint32_t(b));
      if (uf_find(D.parent, a) == uf_find(D.parent, rep)) continue;
      bool hit = false;
      for (uint32_t k0 = cb; k0 < ce && !hit; k0 += 64) {
        const uint32_t k = k0 + uint32_t(lane);
        hit = __ballot(k < ce && sq_dist4(p, D.pts[k < ce ? k : cb]) <= e2) != 0ull;
      }
      if (hit && lane == 0) {
        uf_union(D.parent, D.perm, a, rep);
        if (meta & Q_MARK) D.flag[a] = 1;
      }
    } else if (kind == Q_BORDER) {
      if (D.bestcore[a] <= D.cell_minorig[b]) continue;  // no point here can lower it
      unsigned long long best = ~0ull;
      for (uint32_t k = cb + uint32_t(lane); k < ce; k += 64) {
        if (sq_dist4(p, D.pts[k]) <= e2) {
          const unsigned long long o = (static_cast<unsigned long long>(D.perm[k]) << 32) | k;
          best = o < best ? o : best;
        }
      }
      best = wave_min_u64(best);
      if (lane == 0 && best != ~0ull) atomicMin(D.bestcore + a, best);
    } else if (kind == Q_DEG) {
      const uint32_t need = uint32_t(meta) >> 16;
      uint32_t tot = 0;
      for (uint32_t k0 = cb; k0 < ce && tot < need; k0 += 64) {
        const uint32_t k = k0 + uint32_t(lane);
        tot += uint32_t(__popcll(__ballot(k < ce && sq_dist4(p, D.pts[k < ce ? k : cb]) <= e2)));
      }
      if (lane == 0 && tot) atomicAdd(D.deg + a, tot);
    } else {  // Q_COUNT
      const uint32_t need = uint32_t(meta) >> 16;
      uint32_t tot = 0;
      for (uint32_t k0 = cb; k0 < ce && (need == Q_ALL || tot < need); k0 += 64) {
        const uint32_t k = k0 + uint32_t(lane);
        tot += uint32_t(__popcll(__ballot(k < ce && sq_dist4(p, D.pts[k < ce ? k : cb]) <= e2)));
      }
      if (lane == ((meta >> 4) & 63)) added += tot;
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) *Q.n = 0;
  __builtin_amdgcn_wave_barrier();
  return added;
}

// The walks of one wave (the chunk scheme of wave_walks in walk.hpp).  The
// visitor V gives kStartIsRope and kDrainBeforeEnd (drain the queue before a
// lane's end(), so that queued counts are in), and
//   int32_t begin(uint32_t i, const float4& lo, const float4& hi)
//   uint64_t khi() const, float e2() const
//   bool hit(int32_t j, const float4& lo, const float4& hi)   true: walk over
//   bool drain()                                              true: walk over
//   void end()
template <class V, bool PERSIST>
__device__ __forceinline__ void db_walks(const Node* __restrict__ nodes,
                                         const Node* __restrict__ prims,
                                         const uint64_t* __restrict__ pkey, uint32_t np,
                                         WalkCfg wc, V& v, const DbQueue& Q, uint32_t* err) {
  uint32_t c0, c1;
  uint32_t home = blockIdx.x & 7u;
  bool drained = !PERSIST;  // no span left to take (static: the wave's one chunk)
  if (PERSIST) {
    if (!next_chunk(wc, np, home, c0, c1)) { c0 = c1 = np; drained = true; }
  } else {
    walk_chunk(np, wc.chunk, c0, c1);
  }
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t head = c0, i = 0, steps = 0;
  bool have = false, by_rope = false;
  int32_t node = SENTINEL;
  float4 ql = make_float4(0.f, 0.f, 0.f, 0.f), qh = ql;
  for (;;) {
    if (PERSIST && head >= c1 && !drained) {  // the next span
      if (next_chunk(wc, np, home, c0, c1)) head = c0;
      else drained = true;
    }
    if (V::kDrainBeforeEnd && v.drain()) node = SENTINEL;
    const bool need = node == SENTINEL;
    const uint64_t m = __ballot(need);
    if (need) {
      if (have) { v.end(); have = false; }
      const uint32_t idx = head + uint32_t(__popcll(m & lt));
      if (idx < c1) {
        i = idx;
        have = true;
        const float4* r = reinterpret_cast<const float4*>(prims + i);
        ql = r[0];
        qh = r[1];
        node = v.begin(i, ql, qh);
        steps = 0;
        by_rope = V::kStartIsRope;
      }
    }
    const uint32_t h = head + uint32_t(__popcll(m));
    head = h < c1 ? h : c1;
    if (__ballot(node != SENTINEL) == 0) {
      if (head >= c1 && (!PERSIST || drained)) break;
      continue;
    }
    for (;;) {
      bool act = node != SENTINEL;
      const bool lf = is_leaf(node);
      const uint32_t idx = lf ? uint32_t(leaf_index(node)) : uint32_t(node);
      steps += act ? 1u : 0u;  // bounds checked without a branch, as in wave_walks
      const bool bad = act && (steps > 2 * np || idx >= (lf ? np : np - 1));
      if (__builtin_expect(__ballot(bad) != 0ull, 0)) {
        if (bad) atomicOr(err, STATUS_TREE);
        node = bad ? SENTINEL : node;
      }
      act = act && !bad;
      const Node* rec = !act ? prims : lf ? prims + idx : nodes + idx;
      const float4 a = reinterpret_cast<const float4*>(rec)[0];
      const float4 b = reinterpret_cast<const float4*>(rec)[1];
      // a rope target's number is its first leaf: past the bound, stop
      const uint64_t kf = pkey[act && by_rope ? idx : 0u];
      if (act && by_rope && kf > v.khi()) {
        node = SENTINEL;
        act = false;
      }
      if (act) {
        const bool near = box_box_near4(ql, qh, a, b) <= v.e2();
        const bool down = near && !lf;
        int32_t next = down ? __float_as_int(a.w) : __float_as_int(b.w);
        if (near && lf && v.hit(leaf_index(node), a, b)) next = SENTINEL;
        node = next;
        by_rope = !down;
      }
      if (Q.size() >= QCAP / 2 && v.drain()) node = SENTINEL;
      const uint32_t busy = uint32_t(__popcll(__ballot(node != SENTINEL)));
      if (busy == 0 || ((head < c1 || (PERSIST && !drained)) && busy < wc.refill_at)) break;
    }
  }
  v.drain();
  if (have) v.end();
}

// Counting (sets with minPts > 2) for the points outside dense cells (those
// inside are core already): a walk from the set's root, ended at minPts.
struct CountDb {
  static constexpr bool kStartIsRope = false;
  static constexpr bool kDrainBeforeEnd = true;
  DbSets S;
  DbData D;
  DbQueue Q;
  const uint64_t* pkey;
  float r2;
  int32_t mp, x;  // x: the query point (sorted position), -1: nothing to count
  uint32_t cnt;
  uint64_t hi;
  float4 qp;
  __device__ int32_t begin(uint32_t i, const float4& lo, const float4& h) {
    x = -1;
    const int32_t pay = __float_as_int(lo.w);
    if (pay < 0) return SENTINEL;  // a dense cell
    const uint32_t set = set_id(S, pkey[i]);
    mp = S.minpts[set];
    if (mp <= 2) return SENTINEL;
    x = pay;
    r2 = S.e2[set];
    cnt = 0;
    qp = lo;
    hi = set_upper(S, set, h, r2);
    return S.root[set];
  }
  __device__ uint64_t khi() const { return hi; }
  __device__ float e2() const { return r2; }
  __device__ bool hit(int32_t, const float4& a, const float4& b) {
    const int32_t pay = __float_as_int(a.w);
    if (pay >= 0) return ++cnt >= uint32_t(mp);
    const uint32_t c = uint32_t(pay & 0x7fffffff);
    if (box_box_far4(qp, qp, a, b) <= r2) {
      cnt += D.cell_start[c + 1] - D.cell_start[c];
      return cnt >= uint32_t(mp);
    }
    const uint32_t need = mp < int32_t(Q_ALL) ? uint32_t(mp) : Q_ALL;
    Q.push(Q_COUNT | int32_t(need << 16), x, int32_t(c), r2);
    return false;
  }
  __device__ bool drain() {
    cnt += dbx::drain(D, Q);
    return x >= 0 && cnt >= uint32_t(mp);
  }
  __device__ void end() {
    if (x >= 0) D.flag[x] = cnt >= uint32_t(mp);
  }
};

// Counting by pair traversal (an option, sets with minPts > 2): lane i
// starts at primitive i's rope, so every pair of primitives within eps is
// met once, from the lower one, and adds to the counts of the points in it:
// two points, one to each; a point and a dense cell, the cell's points
// within eps of the point, to the point (a dense cell's own points are core
// and need no count; two cells add nothing).  No early exit at minPts, but
// no walk from the set's root either, which is most of the counting walk's
// cost where points have few neighbours.  The counts go to deg[], and
// k_degree_flags_db sets the flags once every walk is over.  A point only
// needs minPts - 1 neighbours, so a scan of a cell's points stops once the
// point's count (as far as it is known: deg[] only grows, so a stale read
// is smaller and the scan at most longer) reaches that; then deg[x] >=
// min(true count, minPts - 1), which gives the same flag.
struct PairCountDb {
  static constexpr bool kStartIsRope = true;
  static constexpr bool kDrainBeforeEnd = true;  // queued counts are this lane's
  DbSets S;
  DbData D;
  DbQueue Q;
  const uint64_t* pkey;
  float r2;
  int32_t me;    // payload: sorted position of a point, or cell | CELL_BIT
  bool live;     // a query of a set with minPts > 2
  uint32_t cnt;  // this point's neighbours met so far (itself excluded)
  uint32_t want; // minPts - 1 of the query's set: neighbours a point needs
  uint64_t hi;
  float4 ql, qh;
  __device__ int32_t begin(uint32_t i, const float4& lo, const float4& h) {
    me = __float_as_int(lo.w);
    const uint32_t set = set_id(S, pkey[i]);
    live = S.minpts[set] > 2;
    if (!live) return SENTINEL;
    want = uint32_t(S.minpts[set]) - 1u;
    r2 = S.e2[set];
    cnt = 0;
    ql = lo;
    qh = h;
    hi = set_upper(S, set, h, r2);
    return __float_as_int(h.w);
  }
  __device__ uint64_t khi() const { return hi; }
  __device__ float e2() const { return r2; }
  __device__ bool hit(int32_t, const float4& a, const float4& b) {
    const int32_t pr = __float_as_int(a.w);
    if (me >= 0 && pr >= 0) {  // two points: the box bound was the predicate
      ++cnt;
      atomicAdd(D.deg + pr, 1u);
      return false;
    }
    if (me < 0 && pr < 0) return false;  // two dense cells
    const bool all_in = box_box_far4(ql, qh, a, b) <= r2;
    const int32_t c = (me >= 0 ? pr : me) & 0x7fffffff;
    const uint32_t size = D.cell_start[c + 1] - D.cell_start[c];
    if (me >= 0) {  // this point against a cell
      if (all_in) {
        cnt += size;
      } else {
        const uint32_t have = cnt + ld_wg(D.deg + me);
        if (have < want) Q.push(Q_COUNT | int32_t(min(want - have, Q_ALL - 1u) << 16), me, c, r2);
      }
    } else if (all_in) {  // this cell against a point
      atomicAdd(D.deg + pr, size);
    } else {
      const uint32_t have = ld_wg(D.deg + pr);
      if (have < want) Q.push(Q_DEG | int32_t(min(want - have, Q_ALL - 1u) << 16), pr, c, r2);
    }
    return false;
  }
  __device__ bool drain() {
    cnt += dbx::drain(D, Q);
    return false;
  }
  __device__ void end() {
    if (live && me >= 0 && cnt) atomicAdd(D.deg + me, cnt);  // others add to it too
  }
};

// Pair traversal over primitives: lane i starts at primitive i's rope and
// meets every primitive j > i of its set whose box is within eps of its own.
struct PairDb {
  static constexpr bool kStartIsRope = true;
  static constexpr bool kDrainBeforeEnd = false;
  DbSets S;
  DbData D;
  DbQueue Q;
  const uint64_t* pkey;
  float r2;
  bool core_mode, me_core;
  int32_t me;  // payload: sorted position of a point, or cell | CELL_BIT
  int32_t ri;  // an ancestor of the query (its point or its cell's representative)
               // in the union-find forest: a union returns one, and the next
               // union's find starts there instead of at the bottom again
  uint64_t hi;
  float4 ql, qh;
  __device__ int32_t begin(uint32_t i, const float4& lo, const float4& h) {
    me = __float_as_int(lo.w);
    ri = me >= 0 ? me : cell_rep(D, uint32_t(me & 0x7fffffff));
    const uint32_t set = set_id(S, pkey[i]);
    r2 = S.e2[set];
    core_mode = S.minpts[set] > 2;
    me_core = me < 0 || !core_mode || D.flag[me] != 0;  // dense cells are core
    ql = lo;
    qh = h;
    hi = set_upper(S, set, h, r2);
    return __float_as_int(h.w);
  }
  __device__ uint64_t khi() const { return hi; }
  __device__ float e2() const { return r2; }
  __device__ unsigned long long okey(int32_t p) const {
    return (static_cast<unsigned long long>(D.perm[p]) << 32) | uint32_t(p);
  }
  __device__ bool hit(int32_t, const float4& a, const float4& b) {
    const int32_t pr = __float_as_int(a.w);
    if (me >= 0 && pr >= 0) {  // two points: the box bound was the predicate
      if (!core_mode) {
        ri = uf_union(D.parent, D.perm, ri, pr);
        D.flag[me] = 1;
        D.flag[pr] = 1;
        return false;
      }
      const bool cj = D.flag[pr] != 0;
      if (me_core && cj) ri = uf_union(D.parent, D.perm, ri, pr);
      else if (me_core) atomicMin(D.bestcore + pr, okey(me));
      else if (cj) atomicMin(D.bestcore + me, okey(pr));
      return false;
    }
    const bool all_in = box_box_far4(ql, qh, a, b) <= r2;
    if (me < 0 && pr < 0) {  // two dense cells
      const int32_t ca = me & 0x7fffffff, cb = pr & 0x7fffffff;
      if (all_in) ri = uf_union(D.parent, D.perm, ri, cell_rep(D, uint32_t(cb)));
      else Q.push(Q_CELLS, ca, cb, r2);
      return false;
    }
    const int32_t x = me >= 0 ? me : pr;
    const int32_t c = (me >= 0 ? pr : me) & 0x7fffffff;
    const bool x_core = me >= 0 ? me_core : (!core_mode || D.flag[x] != 0);
    if (x_core) {
      if (all_in) {
        // ri is an ancestor of the query: the point x, or the cell c
        ri = me >= 0 ? uf_union(D.parent, D.perm, ri, cell_rep(D, uint32_t(c)))
                     : uf_union(D.parent, D.perm, x, ri);
        if (!core_mode) D.flag[x] = 1;
      } else {
        Q.push(Q_JOIN | (core_mode ? 0 : Q_MARK), x, c, r2);
      }
    } else if (all_in) {
      atomicMin(D.bestcore + x, D.cell_minorig[c]);
    } else {
      Q.push(Q_BORDER, x, c, r2);
    }
    return false;
  }
  __device__ bool drain() {
    dbx::drain(D, Q);
    return false;
  }
  __device__ void end() {}
};

// the wave's queue in dynamic LDS: QCAP entries per wave, then the counts
__device__ __forceinline__ DbQueue wave_queue() {
  extern __shared__ int4 s_dyn[];
  const uint32_t waves = blockDim.x / 64, w = threadIdx.x / 64;
  DbQueue Q{s_dyn + size_t(w) * QCAP, reinterpret_cast<uint32_t*>(s_dyn + waves * QCAP) + w};
  if ((threadIdx.x & 63) == 0) *Q.n = 0;
  __builtin_amdgcn_wave_barrier();
  return Q;
}

template <bool PERSIST>
__global__ void k_count_db(const Node* __restrict__ nodes, const Node* __restrict__ prims,
                           const uint64_t* __restrict__ pkey, uint32_t np_bound,
                           const uint32_t* __restrict__ np_dev, WalkCfg wc, DbSets S, DbData D,
                           uint32_t* __restrict__ err) {
  const uint32_t np = min(*np_dev, np_bound);
  const DbQueue Q = wave_queue();
  CountDb v{S, D, Q, pkey, 0.f, 0, -1, 0u, 0ull, make_float4(0.f, 0.f, 0.f, 0.f)};
  db_walks<decltype(v), PERSIST>(nodes, prims, pkey, np, wc, v, Q, err);
}

template <bool PERSIST>
__global__ void k_count_pairs_db(const Node* __restrict__ nodes, const Node* __restrict__ prims,
                                 const uint64_t* __restrict__ pkey, uint32_t np_bound,
                                 const uint32_t* __restrict__ np_dev, WalkCfg wc, DbSets S,
                                 DbData D, uint32_t* __restrict__ err) {
  const uint32_t np = min(*np_dev, np_bound);
  const DbQueue Q = wave_queue();
  PairCountDb v{S, D, Q, pkey, 0.f, 0, false, 0u, 0u, 0ull, make_float4(0.f, 0.f, 0.f, 0.f),
                make_float4(0.f, 0.f, 0.f, 0.f)};
  db_walks<decltype(v), PERSIST>(nodes, prims, pkey, np, wc, v, Q, err);
}

// core flags of the points outside dense cells from their pair counts (the
// point itself counts too), in sets with minPts > 2
__global__ __launch_bounds__(256) void k_degree_flags_db(const Node* __restrict__ prims,
                                                        const uint64_t* __restrict__ pkey,
                                                        uint32_t np_bound,
                                                        const uint32_t* __restrict__ np_dev,
                                                        DbSets S, const uint32_t* __restrict__ deg,
                                                        uint8_t* __restrict__ flag) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= min(*np_dev, np_bound)) return;
  const int32_t x = prims[j].left;
  if (x < 0) return;  // a dense cell
  const int32_t mp = S.minpts[set_id(S, pkey[j])];
  if (mp > 2) flag[x] = int64_t(deg[x]) + 1 >= int64_t(mp);
}

template <bool PERSIST>
__global__ void k_pairs_db(const Node* __restrict__ nodes, const Node* __restrict__ prims,
                           const uint64_t* __restrict__ pkey, uint32_t np_bound,
                           const uint32_t* __restrict__ np_dev, WalkCfg wc, DbSets S, DbData D,
                           uint32_t* __restrict__ err) {
  const uint32_t np = min(*np_dev, np_bound);
  const DbQueue Q = wave_queue();
  PairDb v{S, D, Q, pkey, 0.f, false, false, 0, 0, 0ull, make_float4(0.f, 0.f, 0.f, 0.f),
           make_float4(0.f, 0.f, 0.f, 0.f)};
  db_walks<decltype(v), PERSIST>(nodes, prims, pkey, np, wc, v, Q, err);
}

__global__ void k_one_set(float e2, int32_t min_pts, int32_t thresh, float* __restrict__ e2o,
                          int32_t* __restrict__ mpo, int32_t* __restrict__ tho) {
  *e2o = e2;
  *mpo = min_pts;
  *tho = thresh;
}

}  // namespace

void launch_cell_keys(const float* pts, uint32_t n, const uint32_t* bounds, float inv_h,
                      uint64_t* keys, uint32_t* hist, MortonGrid* grid, hipStream_t s) {
  if (n == 0) return;
  const uint32_t blocks = std::max(1u, std::min((n + 255) / 256, 4096u));
  hipLaunchKernelGGL(k_cell_keys, dim3(blocks), dim3(256), 0, s, pts, n, bounds, inv_h, keys, hist,
                     grid);
}

size_t scan_status_words(uint32_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

void launch_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total,
                 uint32_t* status, uint32_t* tile_ctr, uint32_t* err, hipStream_t s) {
  if (n == 0) return;
  const uint32_t tiles = uint32_t(scan_status_words(n));
  hipLaunchKernelGGL(k_scan<ValueScan>, dim3(tiles), dim3(SCAN_THREADS), 0, s,
                     ValueScan{in, out}, n, total, status, tile_ctr, err);
}

void launch_cells(const uint64_t* sorted_keys, uint32_t n, uint32_t* cid, uint32_t* ncells,
                  uint32_t* cell_start, uint32_t* scan_status, uint32_t* scan_ctr, uint32_t* err,
                  hipStream_t s) {
  if (n == 0) return;
  const uint32_t tiles = uint32_t(scan_status_words(n));
  hipLaunchKernelGGL(k_scan<CellScan>, dim3(tiles), dim3(SCAN_THREADS), 0, s,
                     CellScan{sorted_keys, cid, cell_start}, n, ncells, scan_status, scan_ctr,
                     err);
}

void launch_cell_stats(const float4* pts, const uint32_t* perm, const uint64_t* keys, uint32_t n,
                       const uint32_t* ncells, const uint32_t* cell_start, const DbSets& sets,
                       float4* cell_lo, float4* cell_hi, unsigned long long* cell_minorig,
                       uint8_t* cell_dense, uint32_t* prim_count, hipStream_t s) {
  if (n == 0) return;
  const uint32_t blocks = std::max(1u, std::min((n + 255) / 256, 8192u));
  hipLaunchKernelGGL(k_cell_stats, dim3(blocks), dim3(256), 0, s, pts, perm, keys, n, ncells,
                     cell_start, sets, cell_lo, cell_hi, cell_minorig, cell_dense, prim_count);
}

void launch_make_prims(const float4* pts, const uint64_t* keys, uint32_t n, const uint32_t* cid,
                       const uint32_t* cell_start, const uint32_t* prim_start,
                       const uint8_t* cell_dense, const float4* cell_lo, const float4* cell_hi,
                       const unsigned long long* cell_minorig, Node* prims, uint64_t* pkey,
                       int32_t* parent, uint8_t* flag, uint32_t* deg, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_make_prims, dim3((n + 255) / 256), dim3(256), 0, s, pts, keys, n, cid,
                     cell_start, prim_start, cell_dense, cell_lo, cell_hi, cell_minorig, prims,
                     pkey, parent, flag, deg);
}

void launch_one_set(float e2, int32_t min_pts, int32_t thresh, float* e2o, int32_t* mpo,
                    int32_t* tho, hipStream_t s) {
  hipLaunchKernelGGL(k_one_set, dim3(1), dim3(1), 0, s, e2, min_pts, thresh, e2o, mpo, tho);
}

// Which DenseBox walks run persistently by default (see walk.hpp): the pair
// walk of batched calls, whose sets differ most in cost per query (on the
// 4,096 sub-halo sets 47 against 60 ms); the plain pair walk and the
// counting walks are faster with static chunks (on the 2^24 field the
// plain pair walk took 1.6 ms persistent, 0.96 ms static: 65k counter
// increments on eight addresses).
constexpr bool DB_PERSIST_COUNT = false;

static size_t queue_lds(int block) {
  const size_t waves = size_t(block) / 64;
  return waves * QCAP * sizeof(int4) + waves * sizeof(uint32_t);
}

void launch_count_db(const Node* nodes, const Node* prims, const uint64_t* pkey,
                     uint32_t np_bound, const uint32_t* np_dev, const DbSets& sets,
                     const DbTables& t, uint32_t* queue, uint32_t* err, int block,
                     hipStream_t s) {
  if (np_bound == 0) return;
  const DbData D{t.pts, t.cell_start, t.perm, t.cell_minorig, t.cell_lo, t.cell_hi, t.parent,
                 t.flag, t.bestcore};
  if (DB_PERSIST_COUNT) {
    const uint32_t grid = persistent_blocks(reinterpret_cast<const void*>(&k_count_db<true>), block,
                                            queue_lds(block), walk_grid(np_bound, block));
    hipLaunchKernelGGL(k_count_db<true>, dim3(grid), dim3(block), queue_lds(block), s, nodes, prims,
                       pkey, np_bound, np_dev, walk_cfg(np_bound, queue), sets, D, err);
  } else {
    hipLaunchKernelGGL(k_count_db<false>, dim3(walk_grid(np_bound, block)), dim3(block),
                       queue_lds(block), s, nodes, prims, pkey, np_bound, np_dev,
                       walk_cfg(np_bound), sets, D, err);
  }
}

void launch_count_pairs_db(const Node* nodes, const Node* prims, const uint64_t* pkey,
                           uint32_t np_bound, const uint32_t* np_dev, const DbSets& sets,
                           const DbTables& t, uint32_t* deg, uint32_t* queue, uint32_t* err,
                           int block, hipStream_t s) {
  if (np_bound == 0) return;
  const DbData D{t.pts, t.cell_start, t.perm, t.cell_minorig, t.cell_lo, t.cell_hi, t.parent,
                 t.flag, t.bestcore, deg};
  if (sets.shift < 64) {  // batched: the sets differ in cost per query, as in the pair walk
    const uint32_t grid = persistent_blocks(reinterpret_cast<const void*>(&k_count_pairs_db<true>),
                                            block, queue_lds(block), walk_grid(np_bound, block));
    hipLaunchKernelGGL(k_count_pairs_db<true>, dim3(grid), dim3(block), queue_lds(block), s, nodes,
                       prims, pkey, np_bound, np_dev, walk_cfg(np_bound, queue), sets, D, err);
  } else {
    hipLaunchKernelGGL(k_count_pairs_db<false>, dim3(walk_grid(np_bound, block)), dim3(block),
                       queue_lds(block), s, nodes, prims, pkey, np_bound, np_dev,
                       walk_cfg(np_bound), sets, D, err);
  }
  hipLaunchKernelGGL(k_degree_flags_db, dim3((np_bound + 255) / 256), dim3(256), 0, s, prims, pkey,
                     np_bound, np_dev, sets, deg, t.flag);
}

void launch_pairs_db(const Node* nodes, const Node* prims, const uint64_t* pkey,
                     uint32_t np_bound, const uint32_t* np_dev, const DbSets& sets,
                     const DbTables& t, uint32_t* queue, uint32_t* err, int block,
                     hipStream_t s) {
  if (np_bound == 0) return;
  const DbData D{t.pts, t.cell_start, t.perm, t.cell_minorig, t.cell_lo, t.cell_hi, t.parent,
                 t.flag, t.bestcore};
  if (sets.shift < 64) {  // batched
    const uint32_t grid = persistent_blocks(reinterpret_cast<const void*>(&k_pairs_db<true>), block,
                                            queue_lds(block), walk_grid(np_bound, block));
    hipLaunchKernelGGL(k_pairs_db<true>, dim3(grid), dim3(block), queue_lds(block), s, nodes, prims,
                       pkey, np_bound, np_dev, walk_cfg(np_bound, queue), sets, D, err);
  } else {
    hipLaunchKernelGGL(k_pairs_db<false>, dim3(walk_grid(np_bound, block)), dim3(block),
                       queue_lds(block), s, nodes, prims, pkey, np_bound, np_dev,
                       walk_cfg(np_bound), sets, D, err);
  }
}

}  // namespace dbx
