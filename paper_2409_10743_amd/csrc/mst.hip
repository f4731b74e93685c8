// Minimum spanning trees over the linear BVH: the Euclidean tree (one of
// ArborX's algorithms, section 3.2) and the tree of HDBSCAN*'s mutual
// reachability graph (section 5), whose edges weigh
//     w(i, j) = max(c_i, c_j, D(i, j)),
// D the binary32 squared distance of the DBSCAN predicate and c the squared
// core distances (all zero for the Euclidean tree).  Edges are ordered by
// (w, lo, hi), lo < hi the input indices of the ends; under that strict
// order the tree is unique.
//
// Borůvka rounds.  Every component takes the least edge leaving it; those
// edges are all in the tree (the cut property), at least half the
// components merge, and there are at most log2(n) rounds.  A round:
//
//  * runs of equal components.  Positions are the Morton-sorted leaves, so
//    a subtree covers a range [f, l] of them; the range is inside one
//    component exactly when the run of equal components that starts at f
//    reaches l.  run_end comes from one scan of the run ends per round.
//  * one walk per point (the stackless rope walk of the other traversals,
//    left-first from the root): a subtree whose range lies in the point's
//    own component is skipped whole, a subtree whose box bound (raised to
//    the point's core distance) exceeds the best edge found so far, the
//    point's own or its component's, is pruned, and a leaf of another
//    component is a candidate edge.  The point's best edge of the previous
//    round and the nearest positions of other components in Morton order
//    (just past either end of its run) seed the bound.
//  * per component, the least (w, lo) by a 64-bit atomicMin, then the least
//    hi among the points that reached it: one edge per component, found by
//    exactly one of its points.
//  * the edges are written (an edge two components both chose once) and
//    their ends unioned in the lock-free union-find of the clustering;
//    every point then takes its root as its component.
//
// The walk tracks the range of the node it is at: the root covers [0, n-1];
// a left child starts where its parent does; a node reached through a rope
// is a right child or a leaf, and its number is its first leaf; the rope of
// a node leads to the leaf or node just past its last leaf (or is the
// sentinel at the end), so the record read in the step gives the range's
// end.
#include "walk.hpp"

namespace dbx {

namespace {

constexpr unsigned long long NO_EDGE = ~0ull;

// atomicMin into a component's minimum, skipped when the value read there
// is already no larger (minima only fall, so a skipped key could not have
// lowered it): in the last rounds millions of points share a few minima
__device__ __forceinline__ void min_into(unsigned long long* at, unsigned long long key) {
  if (key < __hip_atomic_load(at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(at, key);
}

// first position of the range a rope leads past: the node's last leaf + 1
__device__ __forceinline__ uint32_t past_end(int32_t rope, uint32_t n) {
  return rope == SENTINEL ? n : uint32_t(rope < -1 ? leaf_index(rope) : rope);
}

__device__ __forceinline__ bool edge_before(float w, uint32_t lo, uint32_t hi, float bw,
                                            uint32_t blo, uint32_t bhi) {
  return w < bw || (w == bw && (lo < blo || (lo == blo && hi < bhi)));
}

__device__ __forceinline__ unsigned long long wlo_key(float w, uint32_t lo) {
  return (static_cast<unsigned long long>(__float_as_uint(w)) << 32) | lo;
}

__global__ __launch_bounds__(256) void k_mst_init(uint32_t n, int32_t* comp,
                                                  unsigned long long* comp_best,
                                                  uint32_t* comp_hi, int32_t* seed, float* lb,
                                                  int2* comp_edge) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  comp[i] = int32_t(i);
  comp_best[i] = NO_EDGE;
  comp_hi[i] = ~0u;
  seed[i] = -1;
  lb[i] = 0.0f;
  comp_edge[i] = make_int2(-1, -1);
}

// the last position of each run of equal components
__global__ __launch_bounds__(256) void k_mst_run_flags(uint32_t n, const int32_t* __restrict__ comp,
                                                       uint32_t* __restrict__ flag) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i + 1 == n || comp[i] != comp[i + 1]) ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_mst_run_ends(uint32_t n, const uint32_t* __restrict__ flag,
                                                      const uint32_t* __restrict__ run,
                                                      uint32_t* __restrict__ ends) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) ends[run[i]] = i;
}

__global__ __launch_bounds__(256) void k_mst_records(
    uint32_t n, const int32_t* __restrict__ comp, const uint32_t* __restrict__ run,
    const uint32_t* __restrict__ ends, const float* __restrict__ core_in,
    const uint32_t* __restrict__ perm, MstRec* __restrict__ rec) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t o = perm[i];
  MstRec r;
  r.run_end = ends[run[i]];
  r.comp = comp[i];
  r.core = core_in ? core_in[o] : 0.0f;
  r.orig = o;
  rec[i] = r;
}

// the seeds of a point: last round's edge and the positions just past
// either end of its run (its own position where there is none)
__device__ __forceinline__ void seeds_of(uint32_t i, uint32_t n, const MstRec& r,
                                         const int32_t* __restrict__ seed,
                                         const uint32_t* __restrict__ run,
                                         const uint32_t* __restrict__ ends, uint32_t sj[3]) {
  const int32_t s0 = seed[i];
  const uint32_t ri = run[i];
  sj[0] = s0 >= 0 ? uint32_t(s0) : i;
  sj[1] = r.run_end + 1 < n ? r.run_end + 1 : i;
  sj[2] = ri > 0 ? ends[ri - 1] : i;
}

// Before the walks: every point's best seed edge goes into its component's
// minimum, so that every walk starts with a bound for its whole component
// (and may find that it cannot beat it, below).  In the last rounds a few
// components hold millions of points: the keys of a block whose points
// share one component are combined first (one atomic per block).
__global__ __launch_bounds__(256) void k_mst_seed(uint32_t n, const float4* __restrict__ leaf,
                                                  const MstRec* __restrict__ rec,
                                                  const int32_t* __restrict__ seed,
                                                  const uint32_t* __restrict__ run,
                                                  const uint32_t* __restrict__ ends,
                                                  unsigned long long* comp_best) {
  __shared__ unsigned long long s_min[4];
  __shared__ int32_t s_comp[4];
  __shared__ int s_mixed;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n;
  const uint32_t k = in ? i : blockIdx.x * blockDim.x;  // the block's first point: in range
  const MstRec r = rec[k];
  const float4 q = leaf[k];
  uint32_t sj[3];
  seeds_of(k, n, r, seed, run, ends, sj);
  unsigned long long best = NO_EDGE;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const MstRec rs = rec[sj[t]];
    const float4 p = leaf[sj[t]];
    if (rs.comp != r.comp) {
      const float w = fmaxf(fmaxf(r.core, rs.core), sq_dist(q.x, q.y, q.z, p.x, p.y, p.z));
      const unsigned long long key = wlo_key(w, min(r.orig, rs.orig));
      best = key < best ? key : best;
    }
  }
  if (!in) best = NO_EDGE;
  if (threadIdx.x == 0) s_mixed = 0;
  __syncthreads();
  const int32_t c0 = __builtin_amdgcn_readfirstlane(r.comp);
  const bool wave_one = __ballot(r.comp != c0) == 0ull;  // out-of-range lanes hold the first point
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long x = __shfl_xor(best, o, 64);
    best = x < best ? x : best;
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_min[w] = best;
    s_comp[w] = c0;
    if (!wave_one) s_mixed = 1;
  }
  __syncthreads();
  if (s_mixed) {  // per point, as found
    unsigned long long mine = NO_EDGE;
    if (in) {
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const MstRec rs = rec[sj[t]];
        const float4 p = leaf[sj[t]];
        if (rs.comp != r.comp) {
          const float ww = fmaxf(fmaxf(r.core, rs.core), sq_dist(q.x, q.y, q.z, p.x, p.y, p.z));
          const unsigned long long key = wlo_key(ww, min(r.orig, rs.orig));
          mine = key < mine ? key : mine;
        }
      }
    }
    if (mine != NO_EDGE) min_into(comp_best + r.comp, mine);
    return;
  }
  if (threadIdx.x == 0) {
    unsigned long long m = s_min[0];
    bool one = true;
    for (int t = 1; t < int(blockDim.x >> 6); ++t) {
      m = s_min[t] < m ? s_min[t] : m;
      one = one && s_comp[t] == s_comp[0];
    }
    if (one) {
      if (m != NO_EDGE) min_into(comp_best + s_comp[0], m);
    } else {
      for (int t = 0; t < int(blockDim.x >> 6); ++t)
        if (s_min[t] != NO_EDGE) min_into(comp_best + s_comp[t], s_min[t]);
    }
  }
}

// The least edge from each point to another component (see the file
// comment).  One lane per point at a time, the chunk scheme of wave_walks.
__global__ __launch_bounds__(256) void k_mst_walk(
    const Node* __restrict__ nodes, const float4* __restrict__ leaf,
    const MstRec* __restrict__ rec, const uint32_t* __restrict__ run,
    const uint32_t* __restrict__ ends, uint32_t n, WalkCfg wc, const int32_t* __restrict__ root_p,
    unsigned long long* comp_best, float* __restrict__ best_w, int32_t* __restrict__ best_j,
    int32_t* __restrict__ seed, float* __restrict__ lb, uint32_t* err) {
  uint32_t c0, c1;
  walk_chunk(n, wc.chunk, c0, c1);
  const int32_t root = *root_p;
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t head = c0, i = 0, steps = 0, f = 0;
  bool have = false;
  int32_t node = SENTINEL;
  float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
  int32_t mycomp = 0;
  float mycore = 0.f, bw = INFINITY, cw = INFINITY;
  uint32_t me = 0, blo = ~0u, bhi = ~0u;
  int32_t bj = -1;
  // candidate j (position) with record r and point p
  auto offer = [&](uint32_t j, const MstRec& r, const float4& p) {
    const float d = sq_dist(q.x, q.y, q.z, p.x, p.y, p.z);
    const float w = fmaxf(fmaxf(mycore, r.core), d);
    const uint32_t lo = min(me, r.orig), hi = max(me, r.orig);
    if (edge_before(w, lo, hi, bw, blo, bhi)) {
      bw = w;
      blo = lo;
      bhi = hi;
      bj = int32_t(j);
    }
  };
  for (;;) {
    const bool need = node == SENTINEL;
    const uint64_t m = __ballot(need);
    if (need) {
      if (have) {
        best_w[i] = bw;
        best_j[i] = bj;
        if (bj >= 0) seed[i] = bj;
        lb[i] = fminf(bw, cw);
        if (bj >= 0) min_into(comp_best + mycomp, wlo_key(bw, blo));
        have = false;
      }
      const uint32_t idx = head + uint32_t(__popcll(m & lt));
      if (idx < c1) {
        i = idx;
        have = true;
        q = leaf[i];
        const MstRec r = rec[i];
        mycomp = r.comp;
        mycore = r.core;
        me = r.orig;
        bw = INFINITY;
        blo = bhi = ~0u;
        bj = -1;
        const unsigned long long cb = comp_best[mycomp];
        cw = cb == NO_EDGE ? INFINITY : __uint_as_float(uint32_t(cb >> 32));
        node = n > 1 ? root : SENTINEL;
        if (lb[i] > cw) {
          // every edge of this point weighs at least lb (other components
          // only merge, and the last walk saw every edge up to lb), more
          // than an edge its component already has: nothing to find
          node = SENTINEL;
          best_j[i] = -1;
          have = false;
        } else {
          // seeds: last round's edge (if it still leaves the component) and
          // the nearest positions of other components in Morton order, just
          // past either end of the point's run
          uint32_t sj[3];
          seeds_of(i, n, r, seed, run, ends, sj);
#pragma unroll
          for (int t = 0; t < 3; ++t) {
            const MstRec rs = rec[sj[t]];
            const float4 ps = leaf[sj[t]];
            if (rs.comp != mycomp) offer(sj[t], rs, ps);
          }
        }
        f = 0;
        steps = 0;
      }
    }
    const uint32_t h = head + uint32_t(__popcll(m));
    head = h < c1 ? h : c1;
    if (__ballot(node != SENTINEL) == 0) {
      if (head >= c1) break;
      continue;
    }
    for (;;) {
      bool act = node != SENTINEL;
      const bool lf = is_leaf(node);
      const uint32_t idx = lf ? uint32_t(leaf_index(node)) : uint32_t(node);
      steps += act ? 1u : 0u;
      const bool bad = act && (steps > 2 * n || idx >= (lf ? n : n - 1) || f >= n);
      if (__builtin_expect(__ballot(bad) != 0ull, 0)) {
        if (bad) atomicOr(err, STATUS_TREE);
        node = bad ? SENTINEL : node;
      }
      act = act && !bad;
      const float4* p = !act ? leaf
                        : lf ? leaf + idx
                             : reinterpret_cast<const float4*>(nodes + idx);
      const float4 a = p[0], b = p[1];
      const MstRec rf = rec[act ? f : 0u];  // the range's first position
      if (act) {
        int32_t next;
        bool down = false;
        if (lf) {
          if (rf.comp != mycomp && fmaxf(mycore, rf.core) <= fminf(bw, cw)) offer(idx, rf, a);
          next = __float_as_int(a.w);
        } else {
          const int32_t rope = __float_as_int(b.w);
          const bool own = rf.comp == mycomp && rf.run_end + 1 >= past_end(rope, n);
          const float bound = fmaxf(mycore, box_sq_dist4(q, a, b));
          down = !own && bound <= fminf(bw, cw);
          next = down ? __float_as_int(a.w) : rope;
        }
        node = next;
        // a left child starts where its parent does; a rope target's
        // number is its first leaf
        f = down ? f : (next == SENTINEL ? 0u : (is_leaf(next) ? uint32_t(leaf_index(next))
                                                               : uint32_t(next)));
      }
      const uint32_t busy = uint32_t(__popcll(__ballot(node != SENTINEL)));
      if (busy == 0 || (head < c1 && busy < wc.refill_at)) break;
    }
  }
  if (have) {
    best_w[i] = bw;
    best_j[i] = bj;
    if (bj >= 0) seed[i] = bj;
    lb[i] = fminf(bw, cw);
    if (bj >= 0) min_into(comp_best + mycomp, wlo_key(bw, blo));
  }
}

// the least hi among the points whose edge reached their component's (w, lo)
__global__ __launch_bounds__(256) void k_mst_hi(uint32_t n, const MstRec* __restrict__ rec,
                                                const float* __restrict__ best_w,
                                                const int32_t* __restrict__ best_j,
                                                const unsigned long long* __restrict__ comp_best,
                                                uint32_t* comp_hi) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t j = best_j[i];
  if (j < 0) return;
  const MstRec ri = rec[i];
  const uint32_t oj = rec[j].orig;
  if (wlo_key(best_w[i], min(ri.orig, oj)) == comp_best[ri.comp])
    atomicMin(comp_hi + ri.comp, max(ri.orig, oj));
}

// the one point of each component that found its edge records it
__global__ __launch_bounds__(256) void k_mst_pick(uint32_t n, const MstRec* __restrict__ rec,
                                                  const float* __restrict__ best_w,
                                                  const int32_t* __restrict__ best_j,
                                                  const unsigned long long* __restrict__ comp_best,
                                                  const uint32_t* __restrict__ comp_hi,
                                                  int2* __restrict__ comp_edge) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t j = best_j[i];
  if (j < 0) return;
  const MstRec ri = rec[i];
  const uint32_t oj = rec[j].orig;
  if (wlo_key(best_w[i], min(ri.orig, oj)) == comp_best[ri.comp] &&
      max(ri.orig, oj) == comp_hi[ri.comp])
    comp_edge[ri.comp] = make_int2(int32_t(i), j);
}

// write each chosen edge once and union its ends
__global__ __launch_bounds__(256) void k_mst_merge(
    uint32_t n, const MstRec* __restrict__ rec, const float* __restrict__ best_w,
    const unsigned long long* __restrict__ comp_best, const int2* __restrict__ comp_edge,
    const uint32_t* __restrict__ perm, int32_t* parent, uint32_t* count, uint32_t* out_lo,
    uint32_t* out_hi, float* out_w, uint32_t* err) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  if (rec[c].comp != int32_t(c) || comp_best[c] == NO_EDGE) return;
  const int2 e = comp_edge[c];
  if (e.x < 0 || e.y < 0 || uint32_t(e.x) >= n || uint32_t(e.y) >= n) {
    atomicOr(err, STATUS_TREE);
    return;
  }
  const MstRec ri = rec[e.x], rj = rec[e.y];
  const int2 o = comp_edge[rj.comp];
  const bool mutual = o.x == e.y && o.y == e.x;
  if (!mutual || ri.orig < rj.orig) {
    const uint32_t slot = atomicAdd(count, 1u);
    if (slot + 1 < n) {
      out_lo[slot] = min(ri.orig, rj.orig);
      out_hi[slot] = max(ri.orig, rj.orig);
      out_w[slot] = best_w[e.x];
    } else {
      atomicOr(err, STATUS_TREE);
    }
  }
  uf_union(parent, perm, e.x, e.y);
}

// every point takes its root as its component; clear the round's minima
__global__ __launch_bounds__(256) void k_mst_settle(uint32_t n, int32_t* parent, int32_t* comp,
                                                    unsigned long long* comp_best,
                                                    uint32_t* comp_hi, int2* comp_edge) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t r = uf_find(parent, int32_t(i));
  parent[i] = r;
  comp[i] = r;
  comp_best[i] = NO_EDGE;
  comp_hi[i] = ~0u;
  comp_edge[i] = make_int2(-1, -1);
}

// sort keys of the edges: first by hi (in the top word), then by (w, lo)
__global__ __launch_bounds__(256) void k_mst_key_hi(uint32_t m, const uint32_t* __restrict__ hi,
                                                    uint64_t* __restrict__ key) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) key[k] = uint64_t(hi[k]) << 32;
}
__global__ __launch_bounds__(256) void k_mst_key_wlo(uint32_t m, const uint32_t* __restrict__ order,
                                                     const uint32_t* __restrict__ lo,
                                                     const float* __restrict__ w,
                                                     uint64_t* __restrict__ key,
                                                     uint32_t* __restrict__ val) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const uint32_t e = order[k];
  key[k] = wlo_key(w[e], lo[e]);
  val[k] = e;
}
__global__ __launch_bounds__(256) void k_mst_out(uint32_t m, const uint32_t* __restrict__ order,
                                                 const uint32_t* __restrict__ lo,
                                                 const uint32_t* __restrict__ hi,
                                                 const float* __restrict__ w,
                                                 int32_t* __restrict__ edges,
                                                 float* __restrict__ weights) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const uint32_t e = order[k];
  edges[2 * size_t(k)] = int32_t(lo[e]);
  edges[2 * size_t(k) + 1] = int32_t(hi[e]);
  weights[k] = w[e];
}

inline dim3 grid_of(uint32_t n) { return dim3((n + 255) / 256); }

}  // namespace

void launch_mst_init(uint32_t n, int32_t* comp, unsigned long long* comp_best, uint32_t* comp_hi,
                     int32_t* seed, float* lb, int2* comp_edge, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_mst_init, grid_of(n), dim3(256), 0, s, n, comp, comp_best, comp_hi, seed, lb,
                     comp_edge);
}

void launch_mst_runs(uint32_t n, const int32_t* comp, uint32_t* flag, uint32_t* run,
                     uint32_t* ends, uint32_t* total, uint32_t* scan_status, uint32_t* scan_ctr,
                     uint32_t* err, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_mst_run_flags, grid_of(n), dim3(256), 0, s, n, comp, flag);
  launch_scan(flag, run, n, total, scan_status, scan_ctr, err, s);
  hipLaunchKernelGGL(k_mst_run_ends, grid_of(n), dim3(256), 0, s, n, flag, run, ends);
}

void launch_mst_records(uint32_t n, const int32_t* comp, const uint32_t* run, const uint32_t* ends,
                        const float* core_in, const uint32_t* perm, MstRec* rec, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_mst_records, grid_of(n), dim3(256), 0, s, n, comp, run, ends, core_in,
                     perm, rec);
}

void launch_mst_round(const Node* nodes, const float4* leaf, const MstRec* rec,
                      const uint32_t* run, const uint32_t* ends, uint32_t n,
                      const int32_t* root, const uint32_t* perm, int32_t* parent,
                      unsigned long long* comp_best, uint32_t* comp_hi, int2* comp_edge,
                      float* best_w, int32_t* best_j, int32_t* seed, float* lb, uint32_t* count,
                      uint32_t* out_lo, uint32_t* out_hi, float* out_w, uint32_t* err,
                      hipStream_t s) {
  if (n < 2) return;
  hipLaunchKernelGGL(k_mst_seed, grid_of(n), dim3(256), 0, s, n, leaf, rec, seed, run, ends,
                     comp_best);
  hipLaunchKernelGGL(k_mst_walk, dim3(walk_grid(n, 256)), dim3(256), 0, s, nodes, leaf, rec, run,
                     ends, n, walk_cfg(n), root, comp_best, best_w, best_j, seed, lb, err);
  hipLaunchKernelGGL(k_mst_hi, grid_of(n), dim3(256), 0, s, n, rec, best_w, best_j, comp_best,
                     comp_hi);
  hipLaunchKernelGGL(k_mst_pick, grid_of(n), dim3(256), 0, s, n, rec, best_w, best_j, comp_best,
                     comp_hi, comp_edge);
  hipLaunchKernelGGL(k_mst_merge, grid_of(n), dim3(256), 0, s, n, rec, best_w, comp_best,
                     comp_edge, perm, parent, count, out_lo, out_hi, out_w, err);
}

void launch_mst_settle(uint32_t n, int32_t* parent, int32_t* comp, unsigned long long* comp_best,
                       uint32_t* comp_hi, int2* comp_edge, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_mst_settle, grid_of(n), dim3(256), 0, s, n, parent, comp, comp_best,
                     comp_hi, comp_edge);
}

void launch_mst_sort_keys_hi(uint32_t m, const uint32_t* hi, uint64_t* key, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_mst_key_hi, grid_of(m), dim3(256), 0, s, m, hi, key);
}

void launch_mst_sort_keys_wlo(uint32_t m, const uint32_t* order, const uint32_t* lo,
                              const float* w, uint64_t* key, uint32_t* val, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_mst_key_wlo, grid_of(m), dim3(256), 0, s, m, order, lo, w, key, val);
}

void launch_mst_out(uint32_t m, const uint32_t* order, const uint32_t* lo, const uint32_t* hi,
                    const float* w, int32_t* edges, float* weights, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_mst_out, grid_of(m), dim3(256), 0, s, m, order, lo, hi, w, edges, weights);
}

}  // namespace dbx
