/*
 * mst_oracle.c -- plain, slow, obviously-correct CPU minimum spanning trees.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests and the benchmark's CPU leg do.  It shares
 * no code with the GPU path.
 *
 * What it computes.  The paper lists the Euclidean minimum spanning tree
 * among ArborX's algorithms (section 3.2) and names HDBSCAN* as the next
 * clustering algorithm (section 5); HDBSCAN* clusters from the minimum
 * spanning tree of the mutual reachability graph.  Both are the minimum
 * spanning tree of the complete graph on the n points with edge weights
 *
 *     w(i, j) = max(c_i, c_j, D(i, j))
 *
 * where D is the squared distance of the DBSCAN predicate (binary32,
 * ((dx*dx + dy*dy) + dz*dz), every operation rounded, no fused
 * multiply-add) and c_i is point i's squared core distance (the squared
 * distance to its minPts-th nearest point, itself counted; c = 0 for
 * minPts <= 1, which makes w = D and the tree the Euclidean one).  Squares
 * keep the order of the distances, so the tree is the same as with the
 * distances themselves, and max(c_i, c_j, D) is exactly the square of the
 * mutual reachability distance.
 *
 * Ties.  Edges are ordered by (w, lo, hi), lo < hi the two input indices,
 * lexicographically.  Under this strict total order the minimum spanning
 * tree is unique.
 *
 * How: Prim's algorithm on the complete graph, O(n^2) time, O(n) memory.
 * The tree grows from point 0; every point outside it keeps the best edge
 * (under the order above) joining it to the tree; each step adds the best
 * of those and updates the others with the new point's edges.  The n-1
 * edges are then listed in increasing (w, lo, hi) order.
 *
 * Parity status: pinned by tests/test_oracle_mst_pins.py (brute force over
 * every spanning tree of tiny inputs, scipy's minimum spanning tree on
 * tie-free inputs, the cycle property on every non-tree edge, closed forms,
 * planted mistakes).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define MO_OK 0
#define MO_EINVAL (-1)
#define MO_ENONFINITE (-2)
#define MO_ENOMEM (-3)

/* MST_MUTANT_* macros plant deliberate mistakes; only the test that checks
 * the pins' sensitivity defines them, in its own separate build. */

static float sq_dist3(const float *a, const float *b)
{
    float dx = a[0] - b[0];
    float dy = a[1] - b[1];
    float dz = a[2] - b[2];
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

typedef struct {
    float w;
    int32_t lo, hi;
} Edge;

/* (w, lo, hi) of a comes before that of b */
static int edge_before(const Edge *a, const Edge *b)
{
    if (a->w != b->w) return a->w < b->w;
#ifdef MST_MUTANT_TIE_HI_FIRST
    if (a->hi != b->hi) return a->hi < b->hi;
    return a->lo < b->lo;
#else
    if (a->lo != b->lo) return a->lo < b->lo;
    return a->hi < b->hi;
#endif
}

static int edge_cmp(const void *x, const void *y)
{
    const Edge *a = (const Edge *)x, *b = (const Edge *)y;
    if (edge_before(a, b)) return -1;
    if (edge_before(b, a)) return 1;
    return 0;
}

static Edge make_edge(const float *pts, const float *core, int64_t i, int64_t j)
{
    Edge e;
    float w = sq_dist3(pts + 3 * i, pts + 3 * j);
#ifndef MST_MUTANT_NO_CORE
    if (core) {
        if (core[i] > w) w = core[i];
#ifndef MST_MUTANT_ONE_CORE
        if (core[j] > w) w = core[j];
#endif
    }
#endif
    e.w = w;
    e.lo = (int32_t)(i < j ? i : j);
    e.hi = (int32_t)(i < j ? j : i);
    return e;
}

/* core: n squared core distances, or NULL for all zero (the Euclidean
 * tree).  lo, hi, w: n-1 entries each, in increasing (w, lo, hi) order. */
int oracle_mst(const float *pts, int64_t n, const float *core, int32_t *lo, int32_t *hi,
               float *w)
{
    if (n < 0 || n > 2147483647LL) return MO_EINVAL;
    if (n > 0 && !pts) return MO_EINVAL;
    if (n > 1 && (!lo || !hi || !w)) return MO_EINVAL;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(pts[i])) return MO_ENONFINITE;
    for (int64_t i = 0; core && i < n; ++i)
        if (!(core[i] >= 0.0f)) return MO_EINVAL;
    if (n < 2) return MO_OK;
    char *in_tree = calloc((size_t)n, 1);
    Edge *best = malloc((size_t)n * sizeof(Edge));
    Edge *out = malloc((size_t)(n - 1) * sizeof(Edge));
    if (!in_tree || !best || !out) {
        free(in_tree);
        free(best);
        free(out);
        return MO_ENOMEM;
    }
    in_tree[0] = 1;
    for (int64_t v = 1; v < n; ++v) best[v] = make_edge(pts, core, 0, v);
    for (int64_t step = 0; step < n - 1; ++step) {
        int64_t pick = -1;
        for (int64_t v = 0; v < n; ++v)
            if (!in_tree[v] && (pick < 0 || edge_before(&best[v], &best[pick]))) pick = v;
        out[step] = best[pick];
        in_tree[pick] = 1;
        for (int64_t v = 0; v < n; ++v) {
            if (in_tree[v]) continue;
            Edge e = make_edge(pts, core, pick, v);
            if (edge_before(&e, &best[v])) best[v] = e;
        }
    }
    qsort(out, (size_t)(n - 1), sizeof(Edge), edge_cmp);
    for (int64_t k = 0; k < n - 1; ++k) {
        lo[k] = out[k].lo;
        hi[k] = out[k].hi;
        w[k] = out[k].w;
    }
    free(in_tree);
    free(best);
    free(out);
    return MO_OK;
}
