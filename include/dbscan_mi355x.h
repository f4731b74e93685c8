/*
 * dbscan_mi355x.h -- C ABI of the MI355X (gfx950) DBSCAN library.
 *
 * The operation (Prokopenko et al., "Advances in ArborX to support exascale
 * applications", section 3.1): given n points X in 3D, eps and minPts,
 *   N_eps(x) = { y in X : |x - y| <= eps }   (x itself included),
 *   x is a core point iff |N_eps(x)| >= minPts,
 *   clusters are the sets of core points connected through eps-neighbours,
 *   together with the non-core points within eps of one of their cores
 *   (border points); all other points are noise.
 * It is computed as in section 4.3.3 (FDBSCAN: a linear BVH over the points
 * with tree traversal fused with union-find) or section 4.3.4
 * (FDBSCAN-DenseBox: dense grid cells of side eps/sqrt(3) taken whole).
 *
 * Exact results.  The distance test is the binary32 evaluation of
 * ((dx*dx + dy*dy) + dz*dz) <= fl(eps*eps), every operation rounded to
 * nearest even, no fused multiply-add, subnormals kept.  A border point
 * belongs to the cluster of its core neighbour with the smallest input
 * index; a cluster is labelled with the smallest input index among its
 * members (core and border); noise is -1.  Labels are therefore unique and
 * identical across algorithms, block sizes and runs.
 *
 * Conventions for every call below:
 *   - points are float32, row-major [n][3] (x0,y0,z0,x1,...), 4-byte aligned;
 *     labels are int32[n]; "device" pointers are HIP device memory of the
 *     current device, "host" pointers ordinary host memory;
 *   - the caller owns every buffer; the library keeps no pointer after a
 *     call returns;
 *   - `stream` is a hipStream_t; NULL means the context's own stream (made
 *     with default flags, so it is ordered with the null stream).  Work is
 *     enqueued on it and the call returns once it has completed, so every
 *     status is synchronous;
 *   - the return value is a status code (DBSCAN_OK or a negative error),
 *     never an exception; dbscan_last_error() gives a message for the
 *     calling thread's last failure.
 */
#ifndef DBSCAN_MI355X_H
#define DBSCAN_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
#define DBSCAN_OK 0
#define DBSCAN_EINVAL (-1)     /* bad argument: null pointer with n > 0, n < 0,
                                  n >= 2^30 (the radix sort's look-back words
                                  hold a 30-bit count), eps NaN/inf/negative,
                                  eps*eps not finite, min_pts < 1, bad
                                  option; labels untouched */
#define DBSCAN_ENONFINITE (-2) /* a coordinate is NaN or infinite; labels unspecified */
#define DBSCAN_ENOMEM (-3)     /* device memory allocation failed */
#define DBSCAN_EDEVICE (-4)    /* HIP runtime error or a kernel-side failure */
#define DBSCAN_ETOOBIG (-5)    /* the job needs more device memory than the
                                  context's budget allows */

/* ---- algorithms and options -------------------------------------------------- */
/* AUTO picks per call: a density probe (a few thousand sampled points per
 * call, at most 256 per set of a batch; one small kernel and one 8-byte
 * read-back, kept for later calls on the same points, sizes, eps and minPts)
 * estimates the mean number of eps-neighbours per point; DenseBox when it is
 * at least 4 times minPts (point-weighted over sets), FDBSCAN otherwise;
 * with min_pts > 2 the core points come from the pair traversal
 * (DBSCAN_FLAG_PAIR_COUNT) with DenseBox, and with plain FDBSCAN when the
 * mean is below min_pts.
 * Labels do not depend on the pick. */
#define DBSCAN_ALGO_AUTO 0
#define DBSCAN_ALGO_FDBSCAN 1   /* section 4.3.3 */
#define DBSCAN_ALGO_DENSEBOX 2  /* section 4.3.4 */

#define DBSCAN_FLAG_TIMING 1u   /* record per-phase times (dbscan_phase_times) */
/* Enqueue the call's work as a HIP graph: captured on first use, replayed by
 * later calls of the same shape (same point and label buffers, sizes, eps
 * and minPts for a plain call; same sets count and total for a batched one,
 * whose per-set values are re-read at each replay) while the context's
 * scratch has not moved.  A context keeps up to 4 graphs.  Both algorithms
 * (DenseBox keeps its primitive count on the device).  Ignored when the
 * stream argument is NULL; no timing in this mode. */
#define DBSCAN_FLAG_GRAPH 2u
/* With min_pts > 2 (plain FDBSCAN, and DenseBox plain or batched): find
 * the core points by pair traversal (every pair adds one to both points'
 * neighbour counts; section 4.2.3 applied to counting; with DenseBox a point
 * and a dense cell add the cell's points within eps to the point) instead
 * of a walk per point from the root (of its set) that stops at min_pts
 * (section 4.1.2).  Faster where points have few neighbours (no walk from
 * the root), slower in dense regions (no early exit); labels are the same.
 * With plain FDBSCAN the counts also spare the main phase: it walks only
 * from points whose counting walk found a pair, and not at all when no
 * point is core.  The autotuners try both.  Ignored otherwise (batched
 * FDBSCAN). */
#define DBSCAN_FLAG_PAIR_COUNT 4u

typedef struct dbscan_options {
  int32_t algorithm;        /* DBSCAN_ALGO_* */
  int32_t dense_threshold;  /* DenseBox: points that make a cell dense;
                               0 = min_pts; values below min_pts are EINVAL */
  int32_t block_size;       /* traversal workgroup size: 0 = default, else a
                               multiple of 64 in [64, 1024] */
  uint32_t flags;           /* DBSCAN_FLAG_* */
  int32_t sort_tile;        /* keys per workgroup of each radix-sort pass:
                               0 = default (4096), else 2048, 3072 or 4096;
                               other values are EINVAL.  Smaller tiles put
                               more workgroups on small inputs.  (The digit
                               is always 8 bits: 256 look-back words per
                               tile and pass.) */
} dbscan_options;

/* A context owns device scratch memory (grown on demand up to its budget and
 * reused by later calls) and per-phase timing events.  Not thread-safe: use
 * one context per host thread. */
typedef struct dbscan_ctx dbscan_ctx;

/* Create a context on HIP device `device`; `hbm_budget_bytes` caps its
 * scratch memory (0 = no cap).  Returns DBSCAN_OK and sets *out. */
int dbscan_ctx_create(int device, uint64_t hbm_budget_bytes, dbscan_ctx** out);
/* Release a context and its device memory (NULL is ignored). */
int dbscan_ctx_destroy(dbscan_ctx* ctx);
/* Bytes of scratch a job of n points needs (what admission checks). */
uint64_t dbscan_scratch_bytes(int64_t n, int32_t min_pts, int32_t algorithm);

/* Cluster n device-resident points; labels (device) in input order.
 * Uses a per-device default context without a budget. */
int dbscan_cluster(const float* points, int64_t n, float eps, int32_t min_pts,
                   int32_t* labels, void* stream);

/* As dbscan_cluster, with an explicit context and options (NULL = defaults). */
int dbscan_cluster_ex(dbscan_ctx* ctx, const float* points, int64_t n, float eps,
                      int32_t min_pts, int32_t* labels, void* stream,
                      const dbscan_options* opts);

/* Batched: num_sets independent sets, set k = points[offsets[k] .. offsets[k+1])
 * (offsets: host int64[num_sets + 1], offsets[0] = 0, non-decreasing,
 * offsets[num_sets] < 2^30), each clustered with its own eps[k] and
 * min_pts[k] (host arrays) in one pass of the whole path: one sort, one
 * build in which every set is a subtree, one traversal.  labels (device
 * int32[offsets[num_sets]]) are set-local: -1 or the smallest index within
 * the set of the point's cluster, exactly what dbscan_cluster returns for
 * that set alone.  Both algorithms: with DENSEBOX every set gets its own
 * grid of cells (side eps[k]/sqrt(3)) and dense threshold
 * (opts->dense_threshold, 0 = each set's min_pts; below any set's min_pts is
 * EINVAL).  num_sets <= 2^20. */
int dbscan_cluster_batched(dbscan_ctx* ctx, const float* points, const int64_t* offsets,
                           int32_t num_sets, const float* eps, const int32_t* min_pts,
                           int32_t* labels, void* stream, const dbscan_options* opts);

/* Host buffers: copies points to the device, clusters, copies labels back. */
int dbscan_cluster_host(const float* host_points, int64_t n, float eps,
                        int32_t min_pts, int32_t* host_labels);

/* ---- an entry point that allocates nothing ----------------------------------- */
/* For callers that cannot allocate device memory: code that runs while
 * another part of the process captures a HIP graph, tight serving loops,
 * harnesses that forbid hipMalloc.  dbscan_cluster with every scratch buffer
 * in one fixed device array of the library, DBSCAN_NOALLOC_SCRATCH_BYTES
 * long; each GPU gets its own copy of the array when the library first runs
 * on it and keeps it until the process ends.  The call itself allocates no
 * device or pinned host memory and creates no stream, event or context.
 *   points, labels: device pointers as for dbscan_cluster (the caller still
 *     owns and passes both);
 *   n <= DBSCAN_NOALLOC_MAX_POINTS; a larger n is DBSCAN_ETOOBIG and the
 *     labels are untouched;
 *   FDBSCAN with the default options, on the current device;
 *   stream: a hipStream_t, NULL = the null stream; the call returns once its
 *     work has completed (a D2H copy of a status word to pageable memory).
 * Every call on one GPU uses that GPU's one array and leaves its last
 * contents there (the call clears what must start at zero itself), so two
 * calls that overlapped on one GPU would race: the library serialises the
 * calls of one process per device with a host lock.
 * Labels and errors are exactly those of dbscan_cluster. */
#define DBSCAN_NOALLOC_MAX_POINTS 1048576
#define DBSCAN_NOALLOC_SCRATCH_BYTES 102760448  /* 98 MiB: 97.1 B per point at the maximum */
int dbscan_cluster_noalloc(const float* points, int64_t n, float eps, int32_t min_pts,
                           int32_t* labels, void* stream);

/* Per-phase device times (ms) of the context's last call made with
 * DBSCAN_FLAG_TIMING, in the order of dbscan_phase_name(); returns how many
 * were written (at most max). */
int dbscan_phase_times(const dbscan_ctx* ctx, float* ms, int32_t max);
/* Name of timing slot k (one per kernel launch of a run: "prep", "bounds",
 * "morton", "sort0".."sort7", "gather", "cells", "build_frame", "build_levels",
 * "count", "pairs", "final_roots", "final_labels"; a slot a run does not use
 * reads 0 ms: FDBSCAN gathers inside "build_frame", only DenseBox has
 * "gather" and "cells", and the whole label pass is timed as
 * "final_labels"), NULL past the last. */
const char* dbscan_phase_name(int32_t k);

/* Sort passes the context's last plain clustering call ran: 8 minus the
 * low-digit passes it skipped because eps does not need those code bits
 * (the skipped passes are the first ones, "sort0".., and launch a kernel
 * that returns at once).  -1 for a null context. */
int dbscan_sort_passes(const dbscan_ctx* ctx);

/* ---- autotuning ---------------------------------------------------------------- */
/* Run the call on the given input once per candidate option set (traversal
 * workgroup sizes 64/128/256/512; for DenseBox also dense thresholds minPts,
 * 2*minPts, 4*minPts), time each (best of two after a warm-up, HIP events on
 * `stream`) and return the fastest in *best (its time in *best_ms); then
 * time the fastest again with sort tiles of 3072 and 2048 keys and keep
 * the sort tile that wins (sort_tile 0 when the default does).  The
 * candidates cannot change the labels, which end in `labels` (device).
 * For FDBSCAN with min_pts > 2 each size is also tried with
 * DBSCAN_FLAG_PAIR_COUNT (returned in best->flags).  The batched tuner tries
 * both algorithms: FDBSCAN at each workgroup size, and DenseBox at each
 * workgroup size with thresholds 0 (each set's minPts), 2 and 4 times the
 * largest minPts.  A DenseBox pick with min_pts > 2 (the largest, for a
 * batch) is then timed again with DBSCAN_FLAG_PAIR_COUNT toggled. */
int dbscan_autotune(dbscan_ctx* ctx, const float* points, int64_t n, float eps,
                    int32_t min_pts, int32_t algorithm, int32_t* labels,
                    dbscan_options* best, float* best_ms, void* stream);
int dbscan_autotune_batched(dbscan_ctx* ctx, const float* points, const int64_t* offsets,
                            int32_t num_sets, const float* eps, const int32_t* min_pts,
                            int32_t* labels, dbscan_options* best, float* best_ms,
                            void* stream);

/* ---- serving: continuous batching of arriving jobs -------------------------- */
/* A server runs jobs that arrive one at a time (host buffers) on one GPU.
 * Work of several jobs is on the device at once (`slots` worker threads, each
 * with its own stream and resident device arena); small jobs (n < batch_cut)
 * waiting in the queue are clustered together in one batched call (the
 * batched entry point above).  hbm_budget_bytes bounds the device memory the
 * slots hold, which they keep between jobs: a job starts on a slot only if
 * that slot's memory after the job fits next to what the other slots hold
 * (idle slots give theirs back first); a job that could never fit fails with
 * DBSCAN_ETOOBIG.  Results are identical to dbscan_cluster on each job
 * alone.  Thread-safe. */
typedef struct dbscan_server dbscan_server;

typedef struct dbscan_server_options {
  int32_t device;            /* HIP device */
  int32_t slots;             /* concurrent jobs or batches, 0 = 4 (max 64) */
  uint64_t hbm_budget_bytes; /* cap on device bytes of jobs in flight, 0 = none */
  int64_t batch_cut;         /* jobs with fewer points are batched, 0 = 2^18 */
  int64_t batch_max_points;  /* points per batched call, 0 = 2^24 */
  int32_t batch_max_jobs;    /* jobs per batched call, 0 = 1024 */
  int32_t fake_executor;     /* 1: no GPU; a job "runs" for fake_us_per_mpoint
                                microseconds per million points and returns all
                                labels -1 (scheduler tests on the CPU) */
  double fake_us_per_mpoint;
} dbscan_server_options;

typedef struct dbscan_serving_stats {
  uint64_t submitted, completed, failed, points;
  uint64_t batches, batched_jobs;   /* batched calls made, jobs they held */
  uint64_t peak_in_flight_bytes;    /* most device bytes the slots held (arenas and
                                       I/O buffers, kept between jobs) or had reserved */
  double p50_ms, p99_ms, mean_ms, max_ms;  /* latency: completion - submit */
  double mpoints_per_s;             /* points / (last completion - first submit) */
} dbscan_serving_stats;

int dbscan_server_create(const dbscan_server_options* opts, dbscan_server** out);
/* Queue a job; host_pts float32[n][3] and host_labels int32[n] must stay
 * valid until the job is done.  Invalid arguments fail here (EINVAL) and
 * nothing is queued.  *ticket identifies the job. */
int dbscan_server_submit(dbscan_server* srv, const float* host_pts, int64_t n, float eps,
                         int32_t min_pts, int32_t* host_labels, uint64_t* ticket);
/* 1 and *job_status = the job's status when done, 0 while pending. */
int dbscan_server_poll(dbscan_server* srv, uint64_t ticket, int32_t* job_status);
/* As poll, blocking up to timeout_s seconds (negative = no limit). */
int dbscan_server_wait(dbscan_server* srv, uint64_t ticket, double timeout_s,
                       int32_t* job_status);
/* Submit and completion times (seconds, steady clock) of a finished job. */
int dbscan_server_job_times(dbscan_server* srv, uint64_t ticket, double* submit_s,
                            double* done_s);
int dbscan_server_stats(dbscan_server* srv, dbscan_serving_stats* out);
/* Finishes the queued jobs, then stops the workers and frees the server. */
int dbscan_server_destroy(dbscan_server* srv);

/* ---- stages of the path, exposed for testing ------------------------------- */

/* 63-bit Morton codes of n device points (section 4.2.2): per-axis grid
 * coordinate min(floor((p - lo) * (2^21 / (hi - lo))), 2^21 - 1) in binary32
 * (0 for a zero extent), lo/hi the per-axis min/max; bit b of x, y, z goes to
 * bit 3b+2, 3b+1, 3b.  codes: device uint64[n]. */
int dbscan_morton_codes(dbscan_ctx* ctx, const float* points, int64_t n,
                        uint64_t* codes, void* stream);

/* Stable LSD radix sort of device (keys, vals) in place by all 64 key bits;
 * vals is a permutation carried along. */
int dbscan_sort_pairs(dbscan_ctx* ctx, uint64_t* keys, uint32_t* vals, int64_t n,
                      void* stream);

/* Build the linear BVH of n device points inside the context and copy it out
 * (section 3.2, 4.2.1).  All outputs are device buffers:
 *   perm   uint32[n]      input index of the leaf at each sorted position
 *   leaf   float[n][4]    x, y, z and the leaf's rope (int bits)
 *   nodes  float[n-1][8]  lo xyz, left (int bits), hi xyz, rope (int bits)
 *   root   int32[1]       root reference
 * References: k >= 0 internal node k, (j | 0x80000000) leaf j, -1 sentinel. */
int dbscan_build_tree(dbscan_ctx* ctx, const float* points, int64_t n,
                      uint32_t* perm, float* leaf, float* nodes, int32_t* root,
                      void* stream);

/* Core flags |N_eps(x)| >= min_pts (device uint8[n], input order), computed
 * by the early-terminating counting traversal (sections 4.1.2, 4.3.2). */
int dbscan_core_flags(dbscan_ctx* ctx, const float* points, int64_t n, float eps,
                      int32_t min_pts, uint8_t* core, void* stream);

/* Number of unordered pairs {i, j}, i != j, within eps, found by the pair
 * traversal (section 4.2.3), which reports each pair exactly once.
 * count: host pointer. */
int dbscan_pair_count(dbscan_ctx* ctx, const float* points, int64_t n, float eps,
                      int64_t* count, void* stream);
/* The same traversal with counters, summed over all queries (host int64[4]):
 * out4[0] pairs, out4[1] internal-node visits, out4[2] of those whose box
 * was within eps (the walk descended), out4[3] leaf tests. */
int dbscan_traversal_stats(dbscan_ctx* ctx, const float* points, int64_t n, float eps,
                           int64_t* out4, void* stream);

/* ---- nearest neighbours and core distances ---------------------------------- */
/* The k nearest neighbours of every point (section 3.2, the nearest search:
 * a given number of the closest points, whatever their distance), the point
 * itself included, over the same linear BVH (built with full 63-bit codes).
 * Neighbours are ranked by (D, input index), D the binary32 squared distance
 * of the clustering predicate ((dx*dx + dy*dy) + dz*dz, no fused
 * multiply-add), so the answer is unique.  1 <= k <= 32, else EINVAL.
 *   indices  device int32[n][k], row i = point i's neighbours in rank order,
 *            -1 past the n-th;
 *   sq_dists device float[n][k], their D (+inf past the n-th).
 * Errors as for dbscan_cluster_ex (non-finite coordinates: ENONFINITE). */
int dbscan_knn(dbscan_ctx* ctx, const float* points, int64_t n, int32_t k,
               int32_t* indices, float* sq_dists, void* stream);
/* HDBSCAN*'s core distance of every point (section 5 names HDBSCAN* as the
 * next algorithm on this tree), squared: D to the min_pts-th nearest
 * neighbour, the point itself counted (+inf when n < min_pts); sq_dists:
 * device float[n], input order.  1 <= min_pts <= 32. */
int dbscan_core_distances(dbscan_ctx* ctx, const float* points, int64_t n, int32_t min_pts,
                          float* sq_dists, void* stream);

/* Minimum spanning tree of the points over the same linear BVH: with
 * min_pts <= 1 the Euclidean tree (one of ArborX's algorithms, section 3.2);
 * with min_pts >= 2 the tree of HDBSCAN*'s mutual reachability graph
 * (section 5), the graph HDBSCAN* clusters from.  An edge {i, j} weighs
 *     w = max(c_i, c_j, D(i, j)),
 * D the binary32 squared distance of the clustering predicate and c the
 * squared core distances of dbscan_core_distances at min_pts (zero for
 * min_pts = 1), so w is the square of the mutual reachability distance.
 * Edges are ordered by (w, lo, hi), lo < hi the input indices of the ends;
 * under that strict order the tree is unique, and it is returned in that
 * order (the order single-linkage merges them).
 *   edges      device int32[n-1][2]: (lo, hi) of each edge;
 *   sq_weights device float[n-1]: w of each edge.
 * 1 <= min_pts <= 32, else EINVAL; n < 2: nothing is written.  Errors as
 * for dbscan_cluster_ex; EDEVICE if the Borůvka rounds stop adding edges
 * (a malformed tree).  The context keeps a device buffer of about 120
 * bytes per point for the rounds, on top of its arena. */
int dbscan_mst(dbscan_ctx* ctx, const float* points, int64_t n, int32_t min_pts,
               int32_t* edges, float* sq_weights, void* stream);

/* ---- diagnostics ------------------------------------------------------------ */
const char* dbscan_strerror(int status);
const char* dbscan_last_error(void);
const char* dbscan_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DBSCAN_MI355X_H */
