// Internal declarations shared by the kernels and the C ABI of libsnaps.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace snaps {

constexpr int kTile = 64;            // objects per tile (= one wavefront of queries)
constexpr int kMaxD = 16;            // largest subspace dimensionality
constexpr int kMaxIndexDims = 6;     // c <= 6 indexed dimensions (paper Sec. 3.8.1)
constexpr int kLdsSortMax = 32768;   // largest n sorted inside one workgroup's LDS
constexpr int kMaxK = 32;            // largest k
constexpr int kSortThreads = 1024;

// Row stride (floats) of the tile-ordered coordinate array for dimension d:
// d coordinates, the squared norm, padded to a multiple of 4 floats.
__host__ __device__ constexpr int row_stride(int d) { return ((d + 1 + 3) / 4) * 4; }

// One (population, subspace) job as the kernels see it.  Lives in device
// memory (the job table inside the caller's workspace).
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
    int32_t pad0;
    float* xs;               // [ntiles*64][row_stride(d)] coordinates in index order (+ norm)
    int32_t* perm;           // [ntiles*64] index position -> object id (pads: INT32_MAX)
    float* boxes;            // [ntiles][2][row_stride(d)] per-tile lower / upper corners
    int32_t* eps_count;      // outputs, [n], indexed by object id (may be null)
    float* eps_mean;
    int32_t* indeg;
    float* knn_mean;
    int32_t* rank;           // [4][n] or null
    int32_t* knn_ids;        // [n][k] or null
    float* knn_dist;         // [n][k] or null
};

// Small per-call metadata that lives next to the job table in the workspace.
struct Meta {
    DevJob* table;           // [n_jobs]
    int32_t* order;          // join processing order, grouped by kernel class
    int32_t* unit_prefix;    // per class: tiles prefix over that class's jobs (n+1 entries each)
    int32_t* tile_prefix;    // [n_jobs + 1] tiles prefix in table order
    int32_t* counters;       // [n_classes] persistent work counters
    int32_t n_counters;
};

struct IndexArgs {
    Meta meta;
    int32_t n_jobs;
    int32_t seed;            // 1: single job passed by value, block 0 writes the metadata
    int32_t single_units;    // tiles of the single job
    DevJob single;
};

struct JoinArgs {
    const DevJob* table;
    const int32_t* order;        // this class's job ids in processing order
    const int32_t* unit_prefix;  // [n_class_jobs + 1]
    int32_t n_class_jobs;
    int32_t total_units;
    int32_t* counter;
    int32_t split;               // waves per workgroup sharing a query tile
    unsigned long long* stats;   // optional [4] counters (see snaps_tuning.stats)
};

struct RankArgs {
    const DevJob* table;
    int32_t n_jobs;
};

// Launchers (each returns the HIP status of the launch).
hipError_t launch_index_sort(const IndexArgs& a, int grid, hipStream_t s);
hipError_t launch_reorder(const Meta& m, int32_t n_jobs, int32_t total_tiles, hipStream_t s);
hipError_t launch_rank(const RankArgs& a, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t n, int32_t v, hipStream_t s);
// Join kernel for dimensionality D, top-k capacity class kc and filter
// flavour xf; grid == 0 asks for a persistent grid filling the device.
hipError_t launch_join(int D, int kc, int xf, const JoinArgs& a, int grid, hipStream_t s);
int join_blocks_per_cu(int D, int kc, int xf, int split);
int kc_class(int k);              // top-k capacity used for a k (0 for no kNN)
size_t join_lds_bytes(int kc, int split);

}  // namespace snaps
