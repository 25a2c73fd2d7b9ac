// Serving (alert scoring) declarations shared by the library's host code
// and the alert kernels; kept apart from snaps_internal.h, which the join
// kernels include.
#pragma once

#include "snaps_internal.h"

namespace snaps {

// Resident scoring state of one (population, subspace), kept in device
// memory for serving: the index (tile rows and boxes), every object's k-th
// neighbour dd in index order, per-tile maxima of it, the Morton key of each
// tile's first object, and the sorted distinct keys of the four metrics.
struct ServeState {
    int32_t n, d, k, ntiles;
    float eps2;
    int32_t c, bits, pad0;
    const float* cols;
    int64_t ld;
    int32_t feat[kMaxD];
    const float* xs;
    const float* boxes;
    const float* rk2;          // [ntiles*64] k-th neighbour dd at each index position (pads: -inf)
    const float* tmax;         // [ntiles]
    const uint32_t* tkey;      // [ntiles] non-decreasing
    const float* sbox;         // [nsuper][2][DP] union of the boxes of tiles 64 S .. 64 S + 63
    const float* smax;         // [nsuper] max of tmax over the same tiles
    int32_t nsuper, pad1;
    const int32_t* sel_col;    // index dimensions and their cell grids
    const float* sel_lo;
    const float* sel_scale;
    const uint32_t* distinct[4];
    const int32_t* n_distinct;  // [4]
};

// Alert scoring launch: up to kAlertJobs jobs passed by value; one
// wavefront per alert, kAlertWaves wavefronts per workgroup.
constexpr int kAlertJobs = 32;
constexpr int kAlertWaves = 4;
struct AlertJob {
    const ServeState* st;
    const float* alerts;       // [m][d] row-major
    int32_t m;
    int32_t pad0;
    int32_t* eps_count;
    float* eps_mean;
    int32_t* indeg;
    float* knn_mean;
    int32_t* rank;             // [4][m] or null
};
struct AlertArgs {
    AlertJob jobs[kAlertJobs];
    int32_t alert_prefix[kAlertJobs + 1];      // alerts of jobs before each job
    // Matrix-core kernel: workgroups (64-alert groups x slices) and groups
    // of the jobs before each job, each job's slice count, and its partial
    // results' offset (floats) in `part`.
    int32_t group_prefix[kAlertJobs + 1];
    int32_t merge_prefix[kAlertJobs + 1];
    int32_t slices[kAlertJobs];
    int64_t part_off[kAlertJobs];
    float* part;
    // k-th distance bound per alert slot (float bits, +inf at the start),
    // shared by the slices of a group; each job's first slot in `bounds`.
    int64_t bound_off[kAlertJobs];
    uint32_t* bounds;
    int32_t n_jobs, d;
};
static_assert(sizeof(AlertArgs) <= 4096, "alert launches pass AlertArgs by value as kernel arguments");
// Matrix-core alert scoring: the population of a job is cut into `slices`
// contiguous runs of tiles; one workgroup of alert_mfma_waves(d) wavefronts
// per (group of 64 alerts, slice) splits the slice among its wavefronts and
// writes the slice's partial results; one wavefront per group then merges
// them in slice order.  The slice count depends only on the job's alert
// count and d, so the scores of a job do not depend on the other jobs of a
// call.  (Measured on 10^6-object states, d = 6..15: eight wavefronts per
// workgroup and about 8,192 wavefronts per job; at d = 15-16, where the two
// tile buffers of eight wavefronts leave room for one workgroup per compute
// unit, four wavefronts per workgroup, 1.2-1.4x faster on 4,096-10^4-alert
// requests.  Sixteen wavefronts, or 4,096 per job, were up to 25 % slower.)
__host__ __device__ constexpr int alert_mfma_waves(int d) { return row_stride(d) > 16 ? 4 : 8; }
constexpr int kAlertTargetWaves = 8192;
inline int alert_slices(int m, int d) {
    const int w = alert_mfma_waves(d);
    const int groups = (m + kTile - 1) / kTile;
    const int s = (kAlertTargetWaves / w + groups - 1) / groups;
    const int cap = 512 / w;
    return s < 1 ? 1 : (s > cap ? cap : s);
}
// Floats of one partial result: KS kNN slots, count, in-degree, float64 sum, for 64 lanes.
__host__ __device__ constexpr int64_t alert_part_floats(int kc) { return (int64_t)(kc + 4) * kTile; }

hipError_t launch_serve_finish(const DevJob& j, const LargeIndex& li, float* rk2, float* tmax, uint32_t* tkey,
                               const float* kth, hipStream_t s);
hipError_t launch_serve_super(int ntiles, int dp, const float* boxes, const float* tmax, float* sbox, float* smax,
                              hipStream_t s);
hipError_t launch_alerts(int D, int kc, const AlertArgs& a, hipStream_t s);
hipError_t launch_alerts_mfma(int D, int kc, const AlertArgs& a, hipStream_t s);   // both kernels
using AlertKernel = void (*)(AlertArgs);
AlertKernel alert_mfma_pick_group0(int D, int kc);   // matrix-core alert kernels, d 2..8
AlertKernel alert_mfma_pick_group1(int D, int kc);   // d 9..16

}  // namespace snaps
