/*
 * knn_oracle.c -- plain, slow, obviously-correct CPU k-nearest neighbours.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests and the benchmark's CPU leg do.  It shares
 * no code with the GPU path.
 *
 * What it computes (paper, section 3.2: the nearest search, which finds a
 * given number of the closest objects to a query whatever their distance;
 * HDBSCAN*, named in section 5 as the next algorithm, uses the distance to
 * the minPts-th nearest neighbour as a point's core distance):
 *   for a query point i, its k nearest neighbours are the k points j of the
 *   set, i itself included, with the smallest pairs (D(i,j), j) in
 *   lexicographic order, where D is the squared distance of the DBSCAN
 *   predicate: binary32 ((dx*dx + dy*dy) + dz*dz), every operation rounded,
 *   no fused multiply-add, subnormals kept.  Ties in D go to the smaller
 *   index, so the answer is unique.  Listed in that order; past n the
 *   entries are index -1 and D = +inf.
 *
 * How: every query scans every point (no index structure) and keeps its k
 * best in a sorted array by insertion.  Queries are independent and may be
 * spread over host threads (knn_set_threads); the result does not depend
 * on it.
 *
 * Parity status: pinned by tests/test_oracle_knn_pins.py (hand cases, ties,
 * duplicates, k > n, a numpy brute force, scipy's k-d tree on tie-free
 * inputs, exact metamorphic relations, the DBSCAN oracle's neighbour counts,
 * planted mistakes).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define KO_OK 0
#define KO_EINVAL (-1)
#define KO_ENONFINITE (-2)

/* KNN_MUTANT_* macros plant deliberate mistakes; only the test that checks
 * the pins' sensitivity defines them, in its own separate build. */

static float sq_dist(const float *a, const float *b)
{
    float dx = a[0] - b[0];
    float dy = a[1] - b[1];
    float dz = a[2] - b[2];
#ifdef KNN_MUTANT_FMA
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
#else
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
#ifdef KNN_MUTANT_NO_DZ
    (void)zz;
    return s;
#else
    return s + zz;
#endif
#endif
}

/* (d, j) comes before (e, k) */
static int before(float d, int64_t j, float e, int64_t k)
{
#ifdef KNN_MUTANT_TIE_LARGER
    return d < e || (d == e && j > k);
#else
    return d < e || (d == e && j < k);
#endif
}

static int g_threads = 1;

int knn_set_threads(int t)
{
    g_threads = t < 1 ? 1 : t;
    return g_threads;
}

/* queries: nq query point indices, or NULL for all n points (nq = n).
 * idx, d2: int32 / float [nq][k], written row by row. */
int oracle_knn(const float *pts, int64_t n, const int64_t *queries, int64_t nq, int32_t k,
               int32_t *idx, float *d2)
{
    if (n < 0 || nq < 0 || k < 1 || n > 2147483647LL) return KO_EINVAL;
    if ((n > 0 && !pts) || (nq > 0 && (!idx || !d2))) return KO_EINVAL;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(pts[i])) return KO_ENONFINITE;
    for (int64_t q = 0; queries && q < nq; ++q)
        if (queries[q] < 0 || queries[q] >= n) return KO_EINVAL;
#pragma omp parallel for schedule(dynamic, 16) num_threads(g_threads)
    for (int64_t q = 0; q < nq; ++q) {
        const int64_t i = queries ? queries[q] : q;
        int32_t *bi = idx + q * (int64_t)k;
        float *bd = d2 + q * (int64_t)k;
        for (int32_t t = 0; t < k; ++t) {
            bi[t] = -1;
            bd[t] = INFINITY;
        }
        int32_t have = 0;
        for (int64_t j = 0; j < n; ++j) {
#ifdef KNN_MUTANT_NO_SELF
            if (j == i) continue;
#endif
            const float d = sq_dist(pts + 3 * i, pts + 3 * j);
            if (have == k && !before(d, j, bd[k - 1], bi[k - 1])) continue;
            /* insert (d, j) at its place, dropping the last if full */
            int32_t t = have < k ? have : k - 1;
            while (t > 0 && before(d, j, bd[t - 1], bi[t - 1])) {
                bd[t] = bd[t - 1];
                bi[t] = bi[t - 1];
                --t;
            }
            bd[t] = d;
            bi[t] = (int32_t)j;
            if (have < k) ++have;
        }
    }
    return KO_OK;
}
