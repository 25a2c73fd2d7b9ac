/*
 * snaps.h -- C ABI of the MI355X similarity self-join library (libsnaps.so).
 *
 * The library computes, for one population of objects and one feature
 * subspace at a time (or for thousands of such jobs in one call), the two
 * similarity self-joins of the SNAPS population outlier detector and their
 * four per-object outlier metrics and rankings:
 *
 *   - the eps-range self-join ("distance similarity self-join", paper
 *     Sec. 3.5): every other object within Euclidean distance eps.  Metrics:
 *     the neighbour count (Sec. 3.5.1, distance-oblivious; fewest = most
 *     outlying) and the mean neighbour distance (distance-aware; largest =
 *     most outlying; 0 and most outlying when there is no neighbour,
 *     Sec. 3.7 / Tab. 2 point 10);
 *   - the k-nearest-neighbour self-join (Sec. 3.6): the k nearest other
 *     objects of every object (Fig. 1b).  Metrics: the in-degree of the kNN
 *     graph (Sec. 3.6.1, distance-oblivious; fewest = most outlying) and the
 *     mean distance to the k neighbours (distance-aware; largest = most
 *     outlying);
 *   - dense 0-based rankings of the four metrics, rank 0 = most outlying,
 *     equal values sharing a rank (Sec. 3.4, Tab. 2).
 *
 * Conventions shared by every entry point
 *   Memory:   every array argument is DEVICE memory owned by the caller
 *             (allocate it with hipMalloc or a framework allocator).  The
 *             library allocates no device memory of its own: scratch space
 *             comes from the caller's workspace (`ws`, `ws_bytes`), sized with
 *             the matching *_workspace_bytes query.  Structs passed by
 *             pointer (populations, jobs, tuning) live in HOST memory and are
 *             read during the call only.
 *   Layout:   a population is feature-major: value of feature f of object i
 *             at cols[f * ld + i], ld >= n.  Features are min-max normalised
 *             to [0, 1] and finite (Sec. 3.3); the library does not check.
 *   Spaces:   a subspace is a bit mask over the population's features (bit f
 *             = feature f); it needs 2..16 set bits, all < n_features.
 *   Ids:      objects are identified by their row index i (int32, n < 2^31).
 *   Ties:     the k-th neighbour is chosen in ascending (distance, id) order,
 *             so equal distances go to the lower id; the eps ball is closed
 *             (distance <= eps).  Objects never count as their own neighbour.
 *   Streams:  `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *             asynchronous on it; argument errors are reported by the return
 *             code immediately, device faults surface at the next call or
 *             synchronisation as SNAPS_EDEVICE.
 *   Errors:   functions return a snaps_status; snaps_last_error() gives a
 *             message for the last non-OK return of the calling thread.
 *   Numerics: distances are evaluated in float32 in the direct form
 *             sum_f (x_f - y_f)^2; eps sums are accumulated in float64.
 *   Limits:   2 <= n <= 2^30 objects per job (larger n returns
 *             SNAPS_EUNSUPPORTED); 1 <= k <= n - 1.  Up to k = 32 the kNN
 *             side runs inside the fused join (per-lane top-k lists); above,
 *             a selection kernel finds each object's k-th (distance, id) key
 *             exactly by radix selection over recomputed distances, and
 *             writes sorted kNN lists for k <= 4096 (lists above that are
 *             refused with SNAPS_EUNSUPPORTED; the scores take any k).  Jobs
 *             with n <= 32768 are indexed and ranked inside one workgroup's
 *             LDS, larger ones through a device-wide radix sort.
 */
#ifndef SNAPS_H
#define SNAPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SNAPS_OK = 0,
    SNAPS_EINVAL = -1,       /* invalid argument (message via snaps_last_error) */
    SNAPS_ENOMEM = -2,       /* workspace too small */
    SNAPS_EDEVICE = -3,      /* HIP runtime or device error */
    SNAPS_EUNSUPPORTED = -4  /* valid request outside this version's limits */
} snaps_status;

/* A population: n objects with n_features normalised features (device). */
typedef struct {
    const float* cols;      /* [n_features][ld] device array */
    int64_t ld;             /* leading dimension, >= n */
    int64_t n;              /* number of objects, >= 2 */
    int32_t n_features;     /* 2..32 */
} snaps_population;

/* Per-object metric outputs of one job (device arrays of length n, indexed
 * by object id). */
typedef struct {
    int32_t* eps_count;     /* neighbours within eps (Sec. 3.5.1 distance-oblivious) */
    float* eps_mean;        /* their mean distance, 0 if none (Sec. 3.5.1 distance-aware) */
    int32_t* indeg;         /* kNN-graph in-degree (Sec. 3.6.1 distance-oblivious) */
    float* knn_mean;        /* mean distance to the k neighbours (Sec. 3.6.1 distance-aware) */
} snaps_scores;

/* One (population, subspace) job. */
typedef struct {
    const snaps_population* pop;
    uint32_t mask;          /* subspace */
    int32_t k;              /* neighbours per object */
    float eps;              /* range radius, > 0 and finite */
    snaps_scores out;       /* required */
    int32_t* rank;          /* [4][n] device or NULL: dense ranks of (eps_count, eps_mean,
                               indeg, knn_mean), 0 = most outlying */
    float* ensemble;        /* [n] device or NULL (needs rank): the mean of the object's four
                               ranks, the average over the four methods that Sec. 5 suggests
                               for objects outlying in several of them; lower = more outlying */
    int32_t mode;           /* 0: the call's snaps_tuning.mode; else this job's (1 brute force,
                               2 box pruning) -- per-job choices such as an autotuner's */
    int32_t index_dims;     /* 0: the call's snaps_tuning.index_dims; else this job's, 1..6
                               (capped at d) */
    int32_t* knn_ids;       /* [n][k] device or NULL: each object's k neighbours (Sec. 3.6,
                               Fig. 1b) in ascending (distance, id) order -- the lists the
                               in-degree of this call was counted from */
    float* knn_dist;        /* [n][k] device or NULL: their Euclidean distances */
    int32_t tile_shape;     /* 0: the call's snaps_tuning.tile_shape; else this job's (1, 2 or 3) */
    int32_t reserved;       /* must be 0 */
} snaps_job;

/* Passes of snaps_outlier_scores (snaps_tuning.passes). */
#define SNAPS_PASS_INDEX 1   /* per-job index: sort by cell key, reorder into tiles, tile boxes */
#define SNAPS_PASS_JOIN 2    /* fused kNN + eps join and the four metrics */
#define SNAPS_PASS_RANK 4    /* dense rankings */

/* Optional tuning (NULL or zero fields = automatic). */
typedef struct {
    int32_t mode;           /* 0 auto (2 up to d = 14, else 1), 1 brute force over every candidate
                               tile, 2 skip candidate tiles whose bounding box is provably out of reach */
    int32_t split;          /* 0 auto (1, the matrix-core kernel, when it applies and the call
                               has at least 48 query tiles; else enough wavefronts per SIMD
                               for the vector-ALU kernel), else waves sharing one query
                               tile: 1, 2, 4 or 8 */
    int32_t index_dims;     /* 0 auto (min(d, 4): the autotuner's usual choice; Sec. 3.8.1 uses
                               min(d, 6), which serving states keep), else 1..min(d, 6) */
    int32_t filter;         /* 0 auto (3), 1 direct distance form only,
                               2 expanded-form prefilter on the vector ALU with exact direct
                               recheck, 3 the same prefilter as a dense contraction on the
                               matrix cores (fp16 MFMA over each coordinate split into two
                               fp16 pieces, limit widened by the split and accumulation
                               bounds), exact direct recheck; with split or mq
                               above 1 the vector-ALU prefilter runs instead.  All give
                               identical results. */
    int32_t passes;         /* 0 = all; else a mask of SNAPS_PASS_*.  A call that runs the join
                               or rank pass without the index pass must follow a call with the
                               same jobs and workspace that ran the earlier passes. */
    int32_t mq;             /* 0 auto, else waves per workgroup that take consecutive query tiles
                               of one job and walk the same candidate tiles in lockstep: 1, 2,
                               4 or 8 (1 = off).  Used only when split is 1. */
    int32_t index_sort;     /* 0 auto (2), 1 object id packed under the cell key in 32 bits and
                               sorted in one workgroup's LDS (coarser cells; jobs with n above
                               32,768 always use 2), 2 device-wide radix sort of full 32-bit
                               cell keys with the id as payload.  Results do not depend on it
                               beyond the summation order of the eps means. */
    int32_t tile_shape;     /* how the matrix-core join walks the candidate tiles of a pruned job;
                               results do not depend on it.  0 auto (3 for jobs of at least
                               65,536 objects, else 1); 1: tiles in order of index distance, a
                               64-query x 64-candidate tile pair screened when the candidate
                               tile's bounding box is in reach (the leanest kernel); 2: as 3, and
                               each candidate tile taken as two 32-object halves with boxes of
                               their own, so a half out of reach of a 32-query block is not
                               contracted (more box tests, fewer pairs); 3: as 1, with each run
                               of 64 tiles culled as a whole by its box first (large jobs) */
    uint64_t* stats;        /* optional device uint64[4], accumulated (never cleared) by the
                               join pass: [0] query-candidate pairs evaluated, [1] candidate
                               tiles scanned, [2] candidate tiles skipped, [3] pairs evaluated
                               times the subspace dimensionality (3x this is the float32
                               operation count of the distance evaluations) */
} snaps_tuning;

/* Operation codes of snaps_workspace_bytes. */
#define SNAPS_OP_KNN 0
#define SNAPS_OP_EPS 1
#define SNAPS_OP_SCORES 2
#define SNAPS_OP_RANK 3

/* Message of the last non-OK return on this thread ("" if none).  The
 * pointer stays valid until the next library call on the same thread. */
const char* snaps_last_error(void);

/* Library version string. */
const char* snaps_version(void);

/* Workspace bytes needed by one call of the given operation on one job of n
 * objects in a d-dimensional subspace with k neighbours (k is ignored by
 * SNAPS_OP_EPS and SNAPS_OP_RANK, d by SNAPS_OP_RANK).  SNAPS_OP_SCORES
 * includes the scratch of the rank pass.  Returns 0 for invalid arguments
 * (and for SNAPS_OP_RANK with n <= 32768, which needs no workspace).  Pure
 * host function. */
size_t snaps_workspace_bytes(int32_t op, int64_t n, int32_t d, int32_t k);

/* Workspace bytes needed by snaps_outlier_scores for this list of jobs.
 * Returns 0 for invalid arguments.  Pure host function. */
size_t snaps_outlier_scores_workspace(const snaps_job* jobs, int32_t n_jobs,
                                      const snaps_tuning* tune);

/* kNN self-join (Sec. 3.6, Fig. 1b): for every object i of population P in
 * subspace `mask`, its k nearest other objects in ascending (distance, id)
 * order.
 *   ids   [n][k] int32 device, output: neighbour ids, row i = object i
 *   dist  [n][k] float device, output: their Euclidean distances (or NULL)
 * Returns SNAPS_EINVAL for k < 1, k > n-1, a bad mask or population, and
 * SNAPS_EUNSUPPORTED for k > 4096.  Above k = 32 no workspace is used (ws may
 * be NULL). */
int snaps_knn_selfjoin(const snaps_population* P, uint32_t mask, int32_t k,
                       int32_t* ids, float* dist,
                       void* ws, size_t ws_bytes, void* stream);

/* eps-range self-join (Sec. 3.5): for every object, the number of other
 * objects at Euclidean distance <= eps and their mean distance, and
 * optionally the pair list (the result set A without the self-pairs) in CSR
 * form.
 *   count      [n] int32 device, output
 *   mean_dist  [n] float device, output (0 where count is 0)
 *   pair_off   [n + 1] int64 device output, or NULL (no pair list):
 *              pair_off[i] is where object i's row starts, pair_off[n] the
 *              total number of pairs
 *   pairs      [pair_cap] int32 device output, or NULL: row i holds the ids
 *              of object i's neighbours in an unspecified order that repeats
 *              from call to call; an entry whose position is >= pair_cap is
 *              not written, so a caller compares pair_off[n] with pair_cap
 *              (and may size pairs from a first call with pair_cap = 0)
 * With a pair list the join runs twice (counts, then rows) and the workspace
 * of snaps_workspace_bytes(SNAPS_OP_EPS, ...) is required even for small n.
 * Returns SNAPS_EINVAL for eps <= 0 or non-finite, a bad mask or population,
 * pair_cap < 0, or pairs / pair_cap > 0 without pair_off. */
int snaps_eps_selfjoin(const snaps_population* P, uint32_t mask, float eps,
                       int32_t* count, float* mean_dist,
                       int64_t* pair_off, int32_t* pairs, int64_t pair_cap,
                       void* ws, size_t ws_bytes, void* stream);

/* Both joins, the four metrics (Sec. 3.5.1, 3.6.1) and, where job.rank is
 * not NULL, the four dense rankings (Sec. 3.4) for n_jobs independent jobs
 * in one call.  Jobs may share populations; their outputs must not overlap.
 * With n_jobs > 1 the job table is uploaded to the workspace by a copy from
 * host memory, which may wait for earlier work on `stream`.
 * Returns SNAPS_EINVAL for any invalid job (nothing is launched),
 * SNAPS_ENOMEM if ws_bytes < snaps_outlier_scores_workspace(...). */
int snaps_outlier_scores(const snaps_job* jobs, int32_t n_jobs, const snaps_tuning* tune,
                         void* ws, size_t ws_bytes, void* stream);

/* Batched form as a replayable HIP graph.  snaps_plan_create validates the
 * jobs, uploads their table into `ws` once (waiting for `stream`), and
 * captures the launches of the selected passes (tune->passes, all by
 * default) into a graph; snaps_plan_launch replays it on a stream.  Every
 * replay recomputes the same jobs into the same outputs; the jobs' inputs,
 * outputs and `ws` must stay allocated while the plan exists, and replays
 * that overlap on different streams race.  Several plans of different
 * passes may share jobs and workspace (run them in pass order). */
typedef struct snaps_plan snaps_plan;
int snaps_plan_create(const snaps_job* jobs, int32_t n_jobs, const snaps_tuning* tune,
                      void* ws, size_t ws_bytes, void* stream, snaps_plan** plan);
int snaps_plan_launch(const snaps_plan* plan, void* stream);
void snaps_plan_destroy(snaps_plan* plan);

/* snaps_outlier_scores without a workspace argument and without any device
 * allocation, for callers that cannot allocate device memory: code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc.
 * The scratch space is a fixed array of SNAPS_STATIC_SCRATCH_BYTES inside
 * the library, one per device, held until the process ends (its address is
 * looked up once per device, on the first call with that device current).
 * Same jobs, tuning, outputs and results as snaps_outlier_scores (the same
 * kernels run); inputs and outputs remain caller memory.
 *   Returns SNAPS_ENOMEM (nothing launched) when the jobs need more scratch
 *   than SNAPS_STATIC_SCRATCH_BYTES, i.e. when
 *   snaps_outlier_scores_workspace(jobs, n_jobs, tune) exceeds it (about
 *   2.8 MB per job of 31,693 objects at d = 15; one job of up to ~700,000
 *   objects at d = 15).
 *   Every call on a device shares that device's array and leaves its
 *   contents behind; the kernels initialise what they read.  Calls that
 *   overlap on one device (other streams, other threads) race on the array:
 *   serialise them.  As with snaps_outlier_scores, the job table is copied
 *   from host memory (into the array), which may wait for earlier work on
 *   `stream`. */
#define SNAPS_STATIC_SCRATCH_BYTES (64u << 20)
int snaps_outlier_scores_static(const snaps_job* jobs, int32_t n_jobs, const snaps_tuning* tune,
                                void* stream);

/* Dense rankings of the four metrics of one job (Sec. 3.4, Tab. 2): rank 0
 * is the most outlying; eps_count and indeg rank ascending, eps_mean and
 * knn_mean descending, and objects with eps_count == 0 rank first on
 * eps_mean whatever their stored mean.
 *   rank  [4][n] int32 device, output, rows in the order
 *         (eps_count, eps_mean, indeg, knn_mean)
 *   ws    workspace of snaps_workspace_bytes(SNAPS_OP_RANK, n, 0, 0) bytes
 *         (none needed for n <= 32768; NULL then allowed)
 * eps_count and indeg values must be non-negative. */
int snaps_rank(const int32_t* eps_count, const float* eps_mean, const int32_t* indeg,
               const float* knn_mean, int64_t n, int32_t* rank,
               void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- serving
 *
 * Scoring new objects ("alerts") against a resident population in one
 * subspace.  The paper has no serving path; an alert is scored as one extra
 * object that changes nothing in the population and sees no other alert:
 * its k nearest population objects and their mean distance, its population
 * neighbours within eps (count and mean distance), its in-degree (the number
 * of population objects whose own k-th neighbour distance is strictly larger
 * than their distance to the alert), and on each metric the number of
 * distinct population values strictly more outlying than its own (its dense
 * rank position).  Results therefore do not depend on which other alerts
 * share a call. */

/* Device bytes of the resident state of (P, mask, k); 0 for invalid input. */
size_t snaps_serve_state_bytes(const snaps_population* P, uint32_t mask, int32_t k);

/* Build the resident state into caller-owned device memory `state`: runs the
 * full self-join of P in `mask` (index, both joins, metrics, ranks) and keeps
 * what alert scoring needs.  The state refers to P->cols, which must stay
 * allocated and unchanged while the state is used.  Asynchronous on stream. */
int snaps_serve_state_build(const snaps_population* P, uint32_t mask, int32_t k, float eps,
                            void* state, size_t state_bytes, void* stream);

/* Device pointers, inside a built state, of the population's own four
 * metrics ([n] each) and ranks ([4][n]).  Pure host function. */
int snaps_serve_state_outputs(const void* state, int64_t n, int32_t d, int32_t k,
                              const int32_t** eps_count, const float** eps_mean,
                              const int32_t** indeg, const float** knn_mean,
                              const int32_t** rank);

/* One batch of alerts for one built state (all device pointers). */
typedef struct {
    const void* state;      /* built by snaps_serve_state_build */
    const float* alerts;    /* [m][d] row-major, the subspace's columns in ascending
                               feature order, normalised with the population's bounds */
    int32_t m;              /* number of alerts (0 allowed) */
    int32_t method;         /* 0 automatic, 1 one wavefront per alert, 2 matrix-core
                               cross-join of 64-alert groups (see snaps_alerts_score) */
    int32_t* eps_count;     /* [m] outputs */
    float* eps_mean;
    int32_t* indeg;
    float* knn_mean;
    int32_t* rank;          /* [4][m] or NULL */
} snaps_alert_job;

/* Score n_jobs alert batches whose states all have dimensionality d and the
 * same k (the job list is host memory, read during the call).  Jobs may use
 * different states and populations.  Two kernels compute the same scores:
 *   method 1: one wavefront per alert walks the population's index;
 *   method 2: a cross-join of groups of 64 alerts against the population's
 *             tiles, screened on the matrix cores (the half-precision
 *             contraction of the join, widened so that a pair passes if the
 *             alert may list the object or the object may count the alert)
 *             with every passing pair re-evaluated exactly; the population
 *             is cut into slices whose partial results are merged in a
 *             fixed order;
 *   method 0: 2 for d >= 6 and for d = 5 with at most 512 alerts, else 1.
 * Both give identical eps counts, in-degrees, kNN means and their rank
 * positions; the eps mean (a float64 sum taken in another order) may differ
 * in the last float bit.  A job's kernel and slicing depend only on its own
 * method, d and m, so the results of an alert do not depend on the other
 * alerts or jobs of the call.
 *   ws   device workspace of snaps_alerts_workspace_bytes(jobs, n_jobs, d, k)
 *        bytes (0, and NULL allowed, when no job runs method 2); it must not
 *        be used by anything else until the call's work on stream is done.
 *        A NULL ws that is needed, or a method outside 0..2, is SNAPS_EINVAL;
 *        a smaller ws_bytes is SNAPS_ENOMEM; both before any device work.
 * The state header lives in device memory, so a mismatch is found on the
 * device: an alert whose state has another dimensionality than d, or a k
 * above the top-k capacity chosen for k, is not scored (eps_count and indeg
 * are set to -1, the means to NaN, ranks are left untouched).  At most 2^31
 * alerts per call.  Asynchronous on stream. */
int snaps_alerts_score(const snaps_alert_job* jobs, int32_t n_jobs, int32_t d, int32_t k,
                       void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes snaps_alerts_score needs for these jobs: the partial
 * results of the method-2 jobs' slices and one k-th distance bound per alert
 * of those jobs (rounded up to 64 per job); 0 for invalid arguments or when
 * no job runs method 2.  Pure host function. */
size_t snaps_alerts_workspace_bytes(const snaps_alert_job* jobs, int32_t n_jobs, int32_t d, int32_t k);

/* ------------------------------------------------------------------------
 * Sampled-distance search radius (paper Sec. 3.5.3).  The paper picks the
 * radii eps_min and eps_max of its eps grid -- the radii at which the mean
 * number of neighbours per object (the selectivity s) reaches about 0.1 % and
 * 15 % of the population -- by sampling: the distances of a sample of objects
 * to every other object give the relation between a radius and the mean
 * neighbour count.  For each target count T this computes the midpoint
 * between the r-th smallest of the sample's m (n - 1) Euclidean distances,
 * r = round(T m) (ties to even), and the next one: the radius at which the
 * sample's mean neighbour count reaches T.  Distances are float32 (direct
 * form); the selection over them is exact.  The sample is an input: the
 * caller draws it (distinct object ids). */
#define SNAPS_MAX_EPS_TARGETS 8
typedef struct {
    const snaps_population* pop;
    uint32_t mask;              /* subspace */
    int32_t m;                  /* sample size, 1..n */
    const int32_t* sample;      /* [m] device: distinct object ids in [0, n); ids outside are
                                   ignored (the radius is NaN if too few distances remain) */
    int32_t n_targets;          /* 1..SNAPS_MAX_EPS_TARGETS */
    float target[SNAPS_MAX_EPS_TARGETS];   /* mean neighbour counts, with 1 <= round(T m)
                                              <= m (n - 1) - 1 */
    float* eps;                 /* [n_targets] device output */
} snaps_eps_job;

/* Workspace bytes of snaps_eps_sample for these jobs (0 if a job is invalid). */
size_t snaps_eps_sample_workspace(const snaps_eps_job* jobs, int32_t n_jobs);
/* Radii of every job (any mix of populations and subspaces; m (n - 1) < 2^32
 * per job, at most 2^31 - 1 sample objects per call).  The job list is host
 * memory, read during the call.  Asynchronous on stream. */
int snaps_eps_sample(const snaps_eps_job* jobs, int32_t n_jobs, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Radius between under- and overfitting (paper Sec. 3.5.2, Eq. 2-3).  For an
 * ascending grid of radii eps_1 .. eps_g (the paper spaces them evenly from
 * eps_min to eps_max, which snaps_eps_sample finds): the neighbour count and
 * mean neighbour distance of every object at every radius (one range join at
 * eps_g; the result sets of smaller radii are subsets of it, Sec. 3.5.3), the
 * rankings of both metrics at every radius, the similarity (Eq. 2) of each
 * ranking's top n (in rank, then id order) to those of eps_1 (U^min) and eps_g
 * (U^max), and the index of the radius minimising |U^min - U^max| (Eq. 3, the
 * first of equal gaps).  Metric 0 is the number of neighbours, metric 1 the
 * mean neighbour distance (Sec. 3.5.1). */
#define SNAPS_MAX_GRID 16
typedef struct {
    const snaps_population* pop;   /* columns 16-byte aligned and ld a multiple of 4: this pass
                                      reads whole 4-object groups, up to index ld - 1 of a column */
    uint32_t mask;                 /* subspace */
    int32_t n_grid;                /* 2..SNAPS_MAX_GRID */
    float eps[SNAPS_MAX_GRID];     /* strictly ascending radii, > 0 and finite */
    int32_t top_n;                 /* n of Eq. 2, 1..n (the paper: 1 % of the population) */
    int32_t* count;                /* [n_grid][n] device or NULL: neighbours per object and radius */
    float* mean;                   /* [n_grid][n] device or NULL: mean neighbour distance (0 if none) */
    float* similarity;             /* [2][2][n_grid] device: per metric, U^min then U^max */
    int32_t* select;               /* [2] device: selected grid index per metric */
} snaps_eps_grid_job;

/* Workspace bytes of snaps_eps_grid for these jobs (0 if a job is invalid). */
size_t snaps_eps_grid_workspace(const snaps_eps_grid_job* jobs, int32_t n_jobs);
/* Selection for every job (any mix of populations and subspaces).  The job
 * list is host memory, read during the call.  Asynchronous on stream. */
int snaps_eps_grid(const snaps_eps_grid_job* jobs, int32_t n_jobs, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * k between under- and overfitting (paper Sec. 3.6.2, with Eq. 2-3 as in
 * Sec. 3.5.2).  For an ascending grid k_1 < .. < k_g (the paper: k_min = 2 to
 * k_max = 4096, sampled finely at small k): the in-degree and the mean kNN
 * distance of every object at every k (from the k_g nearest neighbours of
 * every object, which hold those of every smaller k; ties of distance go to
 * the lower id), the rankings of both metrics at every k, the similarity
 * (Eq. 2) of each ranking's top n (in rank, then id order) to those of k_1
 * (U^min) and k_g (U^max), and the index of the k minimising |U^min - U^max|
 * (the first of equal gaps).  Metric 0 is the in-degree (ascending), metric 1
 * the mean kNN distance (descending) (Sec. 3.6.1). */
#define SNAPS_MAX_KGRID_K 4096       /* largest k of a k grid */
typedef struct {
    const snaps_population* pop;   /* columns 16-byte aligned and ld a multiple of 4, as for the eps grid;
                                      n >= 2 (each query's distances are held in registers up to
                                      32,768 objects and recomputed in every selection pass above) */
    uint32_t mask;                 /* subspace */
    int32_t n_grid;                /* 2..SNAPS_MAX_GRID */
    int32_t k[SNAPS_MAX_GRID];     /* strictly ascending, k_1 >= 1, k_g <= min(SNAPS_MAX_KGRID_K, n - 1) */
    int32_t top_n;                 /* n of Eq. 2, 1..n (the paper: 1 % of the population) */
    int32_t* indeg;                /* [n_grid][n] device or NULL: in-degree per object and k */
    float* knn_mean;               /* [n_grid][n] device or NULL: mean distance to the k nearest */
    float* similarity;             /* [2][2][n_grid] device: per metric, U^min then U^max */
    int32_t* select;               /* [2] device: selected grid index per metric */
} snaps_k_grid_job;

/* Workspace bytes of snaps_k_grid for these jobs (0 if a job is invalid). */
size_t snaps_k_grid_workspace(const snaps_k_grid_job* jobs, int32_t n_jobs);
/* Selection for every job (any mix of populations and subspaces).  The job
 * list is host memory, read during the call.  Asynchronous on stream. */
int snaps_k_grid(const snaps_k_grid_job* jobs, int32_t n_jobs, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SNAPS_H */
