/*
 * dbscan_oracle.c -- plain, slow, obviously-correct CPU DBSCAN.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the GPU path.
 *
 * What it computes (paper, section 3.1 "DBSCAN algorithm"):
 *   N_eps(x) = { y in X : dist(x,y) <= eps }   (x itself included)
 *   x is core        <=> |N_eps(x)| >= minPts
 *   clusters         =  connected components of the core points under the
 *                       eps relation, plus the border points attached to them
 *   border           =  non-core point with at least one core point in N_eps
 *   noise            =  everything else, label -1
 *
 * Readings where the paper is silent (they make the result unique):
 *   - dist is evaluated in IEEE binary32 as ((dx*dx + dy*dy) + dz*dz) with
 *     every operation rounded to nearest-even, no fused multiply-add, no
 *     flushing of subnormals, and compared with e2 = fl32(eps*eps) by "<=".
 *     Build with -ffp-contract=off and without -ffast-math.
 *   - a border point joins the cluster of its core neighbour with the
 *     smallest input index (the paper's parallel algorithm uses a
 *     first-come critical section, which is not deterministic).
 *   - a cluster's label is the smallest input index among all its members,
 *     core and border.
 *
 * How (section 4.3, the disjoint-set DBSCAN of Algorithm 1, sequential):
 *   neighbour lists come from a uniform grid whose cell side is at least the
 *   largest separation that can pass the float predicate, so every
 *   eps-neighbour lies in one of the 27 surrounding cells; core points found
 *   neighbours of each other are merged with a sequential union-find.
 *
 * Threads.  Counting neighbours and attaching border points read shared
 * data and write one entry per point, so they may run on several host
 * threads (OpenMP, oracle_set_threads); the union-find merge always runs
 * sequentially.  The result does not depend on the thread count.
 *
 * Parity status: pinned by the CPU tests (O(N^2) brute force with
 * scipy connected components, hand-built boundary cases, exact
 * metamorphic relations, the minPts = 2 / connected-components reduction).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENONFINITE (-2)
#define OR_ENOMEM (-3)

/* ---- the predicate ------------------------------------------------------ */

/* ORACLE_MUTANT_* macros plant deliberate mistakes; only the test that
 * checks the pins' sensitivity defines them, in its own separate build. */

static float sq_dist(const float *a, const float *b)
{
    float dx = a[0] - b[0];
    float dy = a[1] - b[1];
#ifdef ORACLE_MUTANT_INDEX
    float dz = a[2] - b[1];
#else
    float dz = a[2] - b[2];
#endif
#ifdef ORACLE_MUTANT_FMA
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
#else
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
#ifdef ORACLE_MUTANT_NO_DZ
    (void)zz;
    return s;
#else
    return s + zz;
#endif
#endif
}

static int is_neighbour(const float *a, const float *b, float e2)
{
#ifdef ORACLE_MUTANT_STRICT
    return sq_dist(a, b) < e2;
#else
    return sq_dist(a, b) <= e2;
#endif
}

/* ---- argument checks (same rules as the library's boundary) ------------- */

static int check_args(const float *pts, int64_t n, float eps, int32_t min_pts,
                      const void *out)
{
    if (n < 0 || n > 2147483647LL) return OR_EINVAL;
    if (n > 0 && (pts == NULL || out == NULL)) return OR_EINVAL;
    if (!(eps >= 0.0f) || isinf(eps)) return OR_EINVAL; /* NaN fails >= */
    float e2 = eps * eps;
    if (isinf(e2)) return OR_EINVAL;
    if (min_pts < 1) return OR_EINVAL;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(pts[i])) return OR_ENONFINITE;
    return OR_OK;
}

/* ---- uniform grid -------------------------------------------------------- */

typedef struct {
    uint64_t key;
    int64_t idx;
} keyed_t;

typedef struct {
    int64_t n;
    keyed_t *order;      /* points sorted by (cell key, index) */
    int64_t ncells;
    uint64_t *cell_key;  /* per occupied cell, increasing */
    int64_t *cell_start; /* per cell, into order[]; cell_start[ncells] = n */
} grid_t;

static int cmp_keyed(const void *pa, const void *pb)
{
    const keyed_t *a = (const keyed_t *)pa, *b = (const keyed_t *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* cell key: x, y, z cell coordinates (< 2^21 each) packed so that numeric
 * order is lexicographic (x, y, z) order */
static uint64_t cell_pack(uint64_t cx, uint64_t cy, uint64_t cz)
{
    return (cx << 42) | (cy << 21) | cz;
}

static void grid_free(grid_t *g)
{
    free(g->order);
    free(g->cell_key);
    free(g->cell_start);
}

static int grid_build(grid_t *g, const float *pts, int64_t n, float eps)
{
    memset(g, 0, sizeof(*g));
    g->n = n;
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = pts[a];
    for (int64_t i = 1; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = pts[3 * i + a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    double ext = 0.0;
    for (int a = 0; a < 3; ++a)
        if (hi[a] - lo[a] > ext) ext = hi[a] - lo[a];
    /* any side >= the largest separation passing the float predicate is
     * correct; the slack covers rounding and squares underflowing to 0.
     * At most 2^20 + 1 cells per axis, so a coordinate fits in 21 bits. */
    double side = (double)eps * (1.0 + 1e-5);
    if (side < 1e-20) side = 1e-20;
    if (side < ext / 1048576.0) side = ext / 1048576.0;

    g->order = (keyed_t *)malloc((size_t)n * sizeof(keyed_t));
    if (!g->order) return OR_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t c[3];
        for (int a = 0; a < 3; ++a)
            c[a] = (uint64_t)floor(((double)pts[3 * i + a] - lo[a]) / side);
        g->order[i].key = cell_pack(c[0], c[1], c[2]);
        g->order[i].idx = i;
    }
    qsort(g->order, (size_t)n, sizeof(keyed_t), cmp_keyed);

    int64_t nc = 0;
    for (int64_t k = 0; k < n; ++k)
        if (k == 0 || g->order[k].key != g->order[k - 1].key) ++nc;
    g->ncells = nc;
    g->cell_key = (uint64_t *)malloc((size_t)(nc + 1) * sizeof(uint64_t));
    g->cell_start = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
    if (!g->cell_key || !g->cell_start) return OR_ENOMEM;
    int64_t c = -1;
    for (int64_t k = 0; k < n; ++k)
        if (k == 0 || g->order[k].key != g->order[k - 1].key) {
            ++c;
            g->cell_key[c] = g->order[k].key;
            g->cell_start[c] = k;
        }
    g->cell_start[nc] = n;
    return OR_OK;
}

/* Neighbourhood of cell c: the 3x3 columns (x+dx, y+dy) over z-1..z+1.
 * Within a column those cells are consecutive in key order, so each column
 * is one range of order[].  Cells are visited in increasing key order, which
 * makes every column's lower bound increase too: one cursor per column
 * (cur[9], zero before the first cell) only ever moves forward. */
typedef struct {
    int64_t begin[9], end[9];
    int m;
} nbhd_t;

static void neighbourhood(const grid_t *g, int64_t c, int64_t cur[9], nbhd_t *nb)
{
    uint64_t key = g->cell_key[c];
    int64_t cx = (int64_t)(key >> 42), cy = (int64_t)((key >> 21) & 0x1FFFFF),
            cz = (int64_t)(key & 0x1FFFFF);
    nb->m = 0;
    int col = 0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy, ++col) {
            if (cx + dx < 0 || cy + dy < 0) continue;
            uint64_t lo = cell_pack((uint64_t)(cx + dx), (uint64_t)(cy + dy),
                                    (uint64_t)(cz > 0 ? cz - 1 : 0));
            uint64_t hi = cell_pack((uint64_t)(cx + dx), (uint64_t)(cy + dy),
                                    (uint64_t)(cz + 1));
            int64_t p = cur[col];
            while (p < g->ncells && g->cell_key[p] < lo) ++p;
            cur[col] = p;
            int64_t q = p;
            while (q < g->ncells && g->cell_key[q] <= hi) ++q;
            if (q > p) {
                nb->begin[nb->m] = g->cell_start[p];
                nb->end[nb->m] = g->cell_start[q];
                nb->m++;
            }
        }
}

/* Column cursors for a walk over the cells that starts at cell c: each one
 * at the first cell whose key is not below its column's lowest key (binary
 * search), where neighbourhood() would have left it after cells 0..c-1. */
static void cursors_at(const grid_t *g, int64_t c, int64_t cur[9])
{
    uint64_t key = g->cell_key[c];
    int64_t cx = (int64_t)(key >> 42), cy = (int64_t)((key >> 21) & 0x1FFFFF),
            cz = (int64_t)(key & 0x1FFFFF);
    int col = 0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy, ++col) {
            cur[col] = 0;
            if (cx + dx < 0 || cy + dy < 0) continue;
            uint64_t lo = cell_pack((uint64_t)(cx + dx), (uint64_t)(cy + dy),
                                    (uint64_t)(cz > 0 ? cz - 1 : 0));
            int64_t a = 0, b = g->ncells; /* first index with key >= lo */
            while (a < b) {
                int64_t m = a + (b - a) / 2;
                if (g->cell_key[m] < lo) a = m + 1;
                else b = m;
            }
            cur[col] = a;
        }
}

/* ---- sequential union-find (Tarjan), section 4.3 -------------------------- */

static int64_t uf_find(int64_t *parent, int64_t x)
{
    int64_t r = x;
    while (parent[r] != r) r = parent[r];
    while (parent[x] != r) { /* full path compression */
        int64_t nx = parent[x];
        parent[x] = r;
        x = nx;
    }
    return r;
}

static void uf_union(int64_t *parent, int64_t a, int64_t b)
{
    int64_t ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb) return;
    if (ra < rb) parent[rb] = ra;
    else parent[ra] = rb;
}

/* ---- the clustering ------------------------------------------------------ */

/* Cells are handed to threads in contiguous blocks; each block sets its own
 * column cursors at its first cell (cursors_at). */
#define CELL_BLOCK 4096

/* threads of the counting and border steps, for every calling thread */
static int g_threads = 1;

/* Neighbour counts |N_eps(i)| (self included) for every point. */
static void count_neighbours(const grid_t *g, const float *pts, float e2,
                             int64_t *cnt)
{
    const int64_t nblocks = (g->ncells + CELL_BLOCK - 1) / CELL_BLOCK;
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
    for (int64_t b = 0; b < nblocks; ++b) {
        int64_t cur[9];
        cursors_at(g, b * CELL_BLOCK, cur);
        const int64_t c1 = (b + 1) * CELL_BLOCK < g->ncells ? (b + 1) * CELL_BLOCK : g->ncells;
        for (int64_t c = b * CELL_BLOCK; c < c1; ++c) {
            nbhd_t nb;
            neighbourhood(g, c, cur, &nb);
            for (int64_t k = g->cell_start[c]; k < g->cell_start[c + 1]; ++k) {
                int64_t i = g->order[k].idx;
                int64_t s = 0;
                for (int t = 0; t < nb.m; ++t)
                    for (int64_t q = nb.begin[t]; q < nb.end[t]; ++q)
                        s += is_neighbour(pts + 3 * i, pts + 3 * g->order[q].idx, e2);
#ifdef ORACLE_MUTANT_NOSELF
                s -= 1;
#endif
                cnt[i] = s;
            }
        }
    }
}

int oracle_neighbour_counts(const float *pts, int64_t n, float eps,
                            int64_t *cnt)
{
    int st = check_args(pts, n, eps, 1, cnt);
    if (st != OR_OK || n == 0) return st;
    grid_t g;
    st = grid_build(&g, pts, n, eps);
    if (st == OR_OK) count_neighbours(&g, pts, eps * eps, cnt);
    grid_free(&g);
    return st;
}

/* Number of unordered pairs {i, j}, i != j, that pass the predicate. */
int oracle_pair_count(const float *pts, int64_t n, float eps, int64_t *out)
{
    int st = check_args(pts, n, eps, 1, out);
    if (st != OR_OK) return st;
    *out = 0;
    if (n == 0) return OR_OK;
    int64_t *cnt = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!cnt) return OR_ENOMEM;
    st = oracle_neighbour_counts(pts, n, eps, cnt);
    int64_t s = 0;
    for (int64_t i = 0; i < n; ++i) s += cnt[i] - 1;
    *out = s / 2;
    free(cnt);
    return st;
}

int oracle_dbscan(const float *pts, int64_t n, float eps, int32_t min_pts,
                  int32_t *labels, uint8_t *core_out)
{
    int st = check_args(pts, n, eps, min_pts, labels);
    if (st != OR_OK || n == 0) return st;
    const float e2 = eps * eps;

    grid_t g;
    int64_t *cnt = NULL, *parent = NULL, *attach = NULL, *minidx = NULL;
    uint8_t *core = NULL;
    st = grid_build(&g, pts, n, eps);
    if (st != OR_OK) goto done;
    cnt = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    parent = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    attach = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    minidx = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    core = (uint8_t *)malloc((size_t)n);
    if (!cnt || !parent || !attach || !minidx || !core) {
        st = OR_ENOMEM;
        goto done;
    }

    /* 1. core points: |N_eps(x)| >= minPts */
    count_neighbours(&g, pts, e2, cnt);
    for (int64_t i = 0; i < n; ++i) core[i] = cnt[i] >= min_pts;

    /* 2. merge core points that are eps-neighbours (union-find, sequential) */
    for (int64_t i = 0; i < n; ++i) parent[i] = i;
    int64_t cur[9] = {0};
    for (int64_t c = 0; c < g.ncells; ++c) {
        nbhd_t nb;
        neighbourhood(&g, c, cur, &nb);
        for (int64_t k = g.cell_start[c]; k < g.cell_start[c + 1]; ++k) {
            int64_t i = g.order[k].idx;
            if (!core[i]) continue;
            for (int t = 0; t < nb.m; ++t)
                for (int64_t q = nb.begin[t]; q < nb.end[t]; ++q) {
                    int64_t j = g.order[q].idx;
                    if (j > i && core[j] && is_neighbour(pts + 3 * i, pts + 3 * j, e2))
                        uf_union(parent, i, j);
                }
        }
    }

    /* 3. attach every non-core point to its smallest-index core neighbour */
    const int64_t nblocks = (g.ncells + CELL_BLOCK - 1) / CELL_BLOCK;
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
    for (int64_t b = 0; b < nblocks; ++b) {
        int64_t bcur[9];
        cursors_at(&g, b * CELL_BLOCK, bcur);
        const int64_t c1 = (b + 1) * CELL_BLOCK < g.ncells ? (b + 1) * CELL_BLOCK : g.ncells;
        for (int64_t c = b * CELL_BLOCK; c < c1; ++c) {
            nbhd_t nb;
            neighbourhood(&g, c, bcur, &nb);
            for (int64_t k = g.cell_start[c]; k < g.cell_start[c + 1]; ++k) {
                int64_t i = g.order[k].idx;
                attach[i] = -1;
                if (core[i]) continue;
                for (int t = 0; t < nb.m; ++t)
                    for (int64_t q = nb.begin[t]; q < nb.end[t]; ++q) {
                        int64_t j = g.order[q].idx;
                        if (!core[j] || !is_neighbour(pts + 3 * i, pts + 3 * j, e2))
                            continue;
#ifdef ORACLE_MUTANT_BORDER_MAX
                        if (attach[i] < 0 || j > attach[i])
#else
                        if (attach[i] < 0 || j < attach[i])
#endif
                            attach[i] = j;
                    }
            }
        }
    }

    /* 4. label = smallest index over all members of the cluster */
    for (int64_t i = 0; i < n; ++i) minidx[i] = INT64_MAX;
    for (int64_t i = 0; i < n; ++i) {
        int64_t r = core[i] ? uf_find(parent, i)
                  : attach[i] >= 0 ? uf_find(parent, attach[i]) : -1;
        attach[i] = r; /* reuse: the cluster root, or -1 for noise */
#ifdef ORACLE_MUTANT_LABEL_CORE
        if (r >= 0 && core[i] && i < minidx[r]) minidx[r] = i;
#else
        if (r >= 0 && i < minidx[r]) minidx[r] = i;
#endif
    }
    for (int64_t i = 0; i < n; ++i)
        labels[i] = attach[i] < 0 ? -1 : (int32_t)minidx[attach[i]];
    if (core_out)
        for (int64_t i = 0; i < n; ++i) core_out[i] = core[i];

done:
    grid_free(&g);
    free(cnt);
    free(parent);
    free(attach);
    free(minidx);
    free(core);
    return st;
}

/* Host threads for the counting and border steps (1 = sequential; values
 * below 1 are taken as 1).  Returns the number in effect. */
int oracle_set_threads(int t)
{
    if (t < 1) t = 1;
#ifdef _OPENMP
    g_threads = t;
    return t;
#else
    return 1;
#endif
}

const char *oracle_version(void)
{
    return "dbscan-oracle 1";
}
