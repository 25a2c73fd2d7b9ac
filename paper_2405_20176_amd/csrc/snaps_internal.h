// Internal declarations shared by the kernels and the C ABI of libsnaps.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace snaps {

constexpr int kTile = 64;            // objects per tile (= one wavefront of queries)
constexpr int kSuper = 64;           // tiles per super-tile (the join culls these first)
constexpr int kMaxD = 16;            // largest subspace dimensionality
constexpr int kMaxIndexDims = 6;     // c <= 6 indexed dimensions (paper Sec. 3.8.1)
constexpr int kLdsSortMax = 32768;   // largest n sorted inside one workgroup's LDS
constexpr int kMaxK = 32;            // largest k of the fused join (larger k: the selection kernel)
constexpr int kMaxListK = 4096;      // largest k whose sorted lists the selection kernel writes
constexpr int kSortThreads = 1024;
constexpr int kRadixChunk = 4096;    // elements per workgroup of the device-wide radix sort

// Row stride (floats) of the tile-ordered coordinate array for dimension d:
// d coordinates, the prefilter addend (scaled squared norm), the object id
// (as raw bits), padded to a multiple of 4 floats.
__host__ __device__ constexpr int row_stride(int d) { return ((d + 2 + 3) / 4) * 4; }

// One (population, subspace) job as the kernels see it.  Lives in device
// memory (the job table inside the caller's workspace).
// DevJob.flags: which jobs the device-wide radix sort indexes / ranks (the
// others are sorted inside one workgroup's LDS).
constexpr int kJobRadixIndex = 1;
constexpr int kJobRadixRank = 2;

struct DevJob {
    const float* cols;       // population, cols[f * ld + i]
    int64_t ld;
    int32_t n;               // objects
    int32_t d;               // subspace dimensionality
    int32_t k;               // neighbours (0: no kNN join)
    int32_t ntiles;          // ceil(n / 64)
    float eps2;              // eps^2 (< 0: no range join)
    int32_t c;               // indexed dimensions
    int32_t feat[kMaxD];     // population columns of the subspace, ascending
    int32_t idbits;          // bits of the packed sort key holding the object id
    int32_t bits;            // Morton bits per indexed dimension
    int32_t prune;           // 1: skip candidate tiles whose box is out of reach
    int32_t flags;           // kJobRadixIndex | kJobRadixRank: passes taken by the device-wide sort
    float* xs;               // [ntiles*64][row_stride(d)] coordinates in index order (+ norm)
    int32_t* perm;           // [ntiles*64] index position -> object id (pads: INT32_MAX)
                             // (the id is also stored in slot d + 1 of each xs row)
    float* boxes;            // [ntiles][2][row_stride(d)] per-tile lower / upper corners
    float* sboxes;           // [nsuper][2][row_stride(d)] corners of each run of kSuper tiles
    float* hboxes;           // [ntiles][2 halves][2][row_stride(d)] corners of objects 0-31 and 32-63 of each tile
    int32_t nsuper;          // ceil(ntiles / kSuper)
    int32_t halves;          // 1: the join culls 32-candidate halves of a tile by their own boxes
    int32_t hier;            // 1: joined by the walk with super-tile culls (kernel variant, host side)
    int32_t pad_h;
    int32_t* eps_count;      // outputs, [n], indexed by object id (may be null)
    float* eps_mean;
    int32_t* indeg;
    float* knn_mean;
    int32_t* rank;           // [4][n] or null
    float* ensemble;         // [n] mean of the four ranks, or null
    int32_t* knn_ids;        // [n][k] or null
    float* knn_dist;         // [n][k] or null
    float* knn_kth;          // [n] squared float32 distance of the k-th neighbour, or null
    int64_t* pair_off;       // eps-only jobs: [n + 1] start of each object's row in pairs, or null
    int32_t* pairs;          // eps-only jobs: neighbour ids, row by row (entries at >= pair_cap dropped)
    int64_t pair_cap;
};

// Small per-call metadata that lives next to the job table in the workspace.
struct Meta {
    DevJob* table;           // [n_jobs]
    int32_t* order;          // join processing order, grouped by kernel class
    int32_t* unit_prefix;    // per class: tiles prefix over that class's jobs (n+1 entries each)
    int32_t* tile_prefix;    // [n_jobs + 1] tiles prefix in table order
    int32_t* super_prefix;   // [n_jobs + 1] super-tiles prefix in table order
    int32_t* counters;       // [n_classes * kQueues] persistent work counters
    int32_t n_counters;
};

struct IndexArgs {
    Meta meta;
    int32_t n_jobs;
    int32_t seed;            // 1: single job passed by value, block 0 writes the metadata
    int32_t single_units;    // join work units of the single job
    int32_t single_tiles;    // tiles of the single job
    int32_t single_supers;   // super-tiles of the single job
    DevJob single;
};

// Work queues of one join launch: one per XCD (the MI355X has 8; workgroup b
// is dispatched to XCD b mod 8).  Queue q holds a share of the class's jobs
// (consecutive sub-lists of `order` / `unit_prefix`), so the candidate rows
// a queue's workgroups stream stay in that XCD's L2; an empty queue steals.
constexpr int kQueues = 8;

struct JoinArgs {
    const DevJob* table;
    const int32_t* order;        // this class's job ids, queue by queue
    const int32_t* unit_prefix;  // per queue: [q_jobs + 1] unit prefix
    int32_t q_order_off[kQueues];
    int32_t q_prefix_off[kQueues];
    int32_t q_jobs[kQueues];
    int32_t q_units[kQueues];
    int32_t* counter;            // [kQueues]
    int32_t split;               // waves per workgroup sharing a query tile
    int32_t mq;                  // waves per workgroup, each with its own query tile, scanning the
                                 // same candidate tiles in lockstep (1: off)
    unsigned long long* stats;   // optional [4] counters (see snaps_tuning.stats)
};

// One segment of the device-wide radix sort: ping-pong key (and optional
// payload) buffers, result in buffer 0 after an even number of passes.
struct SortSeg {
    uint32_t* key[2];
    uint32_t* val[2];        // null: keys only
    int32_t* hist;           // [256][nchunks] scratch
    int64_t n;
    int32_t nchunks;
    int32_t pad0;
};

// Index build of a job too large for the LDS sort: statistics accumulators,
// the chosen index dimensions and the key buffer of its sort segment.
struct LargeIndex {
    int32_t job;             // index into the job table
    int32_t nchunks;
    double* acc;             // [2][kMaxD] sums and sums of squares
    int32_t* sel_col;        // [kMaxIndexDims] population columns of the index dims
    float* sel_lo;           // [kMaxIndexDims]
    float* sel_scale;        // [kMaxIndexDims]
    uint32_t* keys;          // [ntiles*64] Morton keys (sort buffer 0)
    uint32_t* vals;          // [ntiles*64] object ids (sort buffer 0 payload = perm)
};

// Rank of a job too large for the LDS sort: per metric, the sort segment
// holding its keys and the number of distinct values found.
struct LargeRank {
    int32_t job;
    int32_t nchunks;
    uint32_t* keys[4];       // sorted keys of each metric (buffer 0)
    uint32_t* distinct[4];   // distinct sorted keys (buffer 1 is reused)
    int32_t* n_distinct;     // [4]
};

// Sampled-distance radius selection (one job = one subspace and sample).
constexpr int kMaxEpsTargets = 8;
struct EpsState {
    uint32_t prefix;         // bits of the squared distance found so far
    uint32_t rem;            // remaining 1-based rank among values with that prefix
    uint32_t eq;             // values in the last chosen bucket
    uint32_t next;           // smallest squared-distance bits above the r-th (atomic min)
    uint32_t need_next;      // the (r + 1)-th is not a tie of the r-th
    uint32_t bad;            // fewer distances than the rank
};
struct EpsJob {
    const float* cols;
    int64_t ld;
    int32_t n, d;
    int32_t feat[kMaxD];
    const int32_t* sample;   // [m] object ids
    int32_t m, n_targets;
    uint32_t rank[kMaxEpsTargets];   // r = round(target m), 1-based
    float* eps;              // [n_targets] output
    uint32_t* hist;          // [n_targets][256] scratch
    EpsState* state;         // [n_targets] scratch
};

// Radius selection on a grid of radii (one job = one subspace and grid).
constexpr int kMaxGrid = 16;
struct GridJob {
    const float* cols;       // 16-byte aligned columns, ld a multiple of 4
    int64_t ld;
    int32_t n, d;
    int32_t feat[kMaxD];
    int32_t g;               // radii in the grid
    int32_t top_n;           // n of Eq. 2
    float e2[kMaxGrid];      // squared radii as the joins compare them (float32 of the exact square)
    int32_t* count;          // [g][n] neighbours per object and radius
    float* mean;             // [g][n] mean neighbour distance
    uint32_t* member;        // [2][g][words] top-n bit sets (scratch)
    int32_t words;           // ceil(n / 32)
    int32_t knn;             // 1: k grid (count = in-degree, mean = mean kNN distance, ranked without
                             // the no-neighbour rule of the range join)
    float* similarity;       // [2][2][g] U^min, U^max per metric
    int32_t* select;         // [2] selected radius index per metric
};

// k selection on a grid of k (one job = one subspace and grid).
constexpr int kMaxKGridN = 32768;     // distances of one query held in registers (larger: recomputed per pass)
constexpr int kMaxKGridK = 4096;
struct KGridJob {
    const float* cols;       // 16-byte aligned columns, ld a multiple of 4
    int64_t ld;
    int32_t n, d;
    int32_t feat[kMaxD];
    int32_t g;
    int32_t pad0;
    int32_t k[kMaxGrid];     // strictly ascending, k[g - 1] < n
    uint64_t* thr;           // [n][kMaxGrid] (distance bits << 32 | id) of the k_j-th neighbour of each object
    float* kmean;            // [g][n] mean distance to the k_j nearest
    int32_t* indeg;          // [g][n]
};

// kNN metrics (and lists) of one job with k above kMaxK, by selection.
struct BigKJob {
    const float* cols;       // population columns, cols[f * ld + i]
    int64_t ld;
    int32_t n, k;
    int32_t feat[kMaxD];     // population columns of the subspace, ascending
    int32_t* indeg;          // [n] added to (atomics), or null
    float* knn_mean;         // [n] or null
    int32_t* ids;            // [n][k] or null (k <= kMaxListK)
    float* dist;             // [n][k] or null
};
struct BigKArgs {
    const BigKJob* table;    // jobs of one (d, lists) class
    const int64_t* prefix;   // [n_jobs + 1] queries before each job
    int32_t n_jobs;
    int32_t use_single;      // 1: the single job below, blocks = its queries
    BigKJob single;
};

struct RankArgs {
    const DevJob* table;
    int32_t n_jobs;
};

// Queries per lane of the join instantiation for top-k capacity kc: one
// (two per lane coarsened the tile pruning more than it saved in loads).
__host__ __device__ constexpr int join_ql(int kc) { return kc < 0 ? 2 : 1; }

// Launchers (each returns the HIP status of the launch).
hipError_t launch_index_sort(const IndexArgs& a, int grid, hipStream_t s);
hipError_t launch_reorder(const Meta& m, int32_t n_jobs, int32_t total_tiles, hipStream_t s);
// Corners of every super-tile of every job (after the reorder).
hipError_t launch_super_boxes(const Meta& m, int32_t n_jobs, int32_t total_supers, hipStream_t s);
hipError_t launch_rank(const RankArgs& a, hipStream_t s);
hipError_t launch_grid_join(const GridJob* jobs, const int32_t* tile_prefix, int n_jobs, int total_tiles, int d,
                            hipStream_t s);
hipError_t launch_grid_select(const GridJob* jobs, int n_jobs, hipStream_t s);
// k grid: per-query thresholds and means, then in-degrees; jobs of one d,
// query_prefix / group_prefix [n_jobs + 1] by queries and by groups of
// kgrid_tiles_per_group() 64-object tiles.
int kgrid_tiles_per_group();
hipError_t launch_kgrid(const KGridJob* jobs, const int32_t* query_prefix, const int32_t* group_prefix, int n_jobs,
                        int total_queries, int total_groups, int d, bool stream, hipStream_t s);
hipError_t launch_eps_sample(const EpsJob* jobs, const int32_t* prefix, int n_jobs, int total_blocks, int d,
                             hipStream_t s);
// Mean of the four ranks of every object of every job with an ensemble
// output (after both rank paths); tile_prefix as in Meta.
hipError_t launch_ensemble(const DevJob* table, int n_jobs, const int32_t* tile_prefix, int total_tiles,
                           hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t n, int32_t v, hipStream_t s);
// Selection kernel for k above kMaxK: one workgroup per query of the jobs of
// one dimensionality D; lists: the jobs write sorted kNN lists.
hipError_t launch_bigk(int D, bool lists, const BigKArgs& a, int64_t queries, hipStream_t s);
// Zero the in-degree output of every job of a call (start of the join pass).
hipError_t launch_zero_indeg(const Meta& m, int32_t n_jobs, int32_t total_tiles, hipStream_t s);
// off[0] = 0, off[i + 1] = off[i] + count[i] (int64), i < n; scratch holds
// pair_scan_scratch(n) bytes.
size_t pair_scan_scratch(int64_t n);
hipError_t launch_pair_offsets(const int32_t* count, int64_t n, int64_t* off, void* scratch, hipStream_t s);
hipError_t launch_radix_sort(const SortSeg* segs, const int32_t* chunk_prefix, int n_segs, int total_chunks,
                             int passes, hipStream_t s);
// Large-n index build (before k_reorder) and rank, over every large job of a call.
hipError_t launch_large_index(const DevJob* table, const LargeIndex* li, int n_large, const int32_t* chunk_prefix,
                              int total_chunks, const SortSeg* segs, hipStream_t s);
hipError_t launch_large_rank(const DevJob* table, const LargeRank* lr, int n_large, const int32_t* chunk_prefix,
                             int total_chunks, const SortSeg* segs, const int32_t* seg_chunk_prefix,
                             int total_seg_chunks, hipStream_t s);
// Join kernel for dimensionality D, top-k capacity class kc, filter
// flavour xf and walk (hier: super-tile and candidate-half culls of the
// matrix-core kernel); grid == 0 asks for a persistent grid filling the device.
hipError_t launch_join(int D, int kc, int xf, int hier, const JoinArgs& a, int grid, hipStream_t s);
int join_blocks_per_cu(int D, int kc, int xf, int hier, int split, int mq);
int kc_class(int k);              // top-k capacity used for a k (0 for no kNN)
size_t join_lds_bytes(int kc, int split);

}  // namespace snaps
