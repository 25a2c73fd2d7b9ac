// Index build of one (population, subspace) job: the grid index of the
// paper (Sec. 3.8.1: objects indexed in c = min(d, 6) of the d dimensions),
// laid out for a GPU that scans whole tiles of candidates.
//
//   1. k_index_sort (one workgroup per job): per-dimension mean and spread of
//      the job's d columns; the c most spread dimensions are cut into 2^bits
//      cells over mean +/- 3 sigma; every object gets the Morton (Z-order)
//      interleaving of its c cell coordinates, packed above its id into one
//      32-bit key; the keys are sorted in LDS.  Sorted position -> id is the
//      permutation `perm`.
//   2. k_reorder (one wavefront per tile of 64 positions): gathers the d
//      subspace columns of every object in sorted order into a row-major
//      array (plus a scaled squared norm and the object id), pads the last
//      tile with NaN rows, and
//      records each tile's bounding box in all d dimensions.
//
// Any order of the objects gives the same join results (the join prunes a
// tile only when its box is provably out of reach); the index order only
// decides how much the join can skip.
#include "snaps_internal.h"
#include "common.cuh"
#include "keys.cuh"

#include <climits>

namespace snaps {

__global__ __launch_bounds__(kSortThreads) void k_index_sort(IndexArgs A) {
    __shared__ uint32_t buf[kLdsSortMax];
    __shared__ float red[2][16][kMaxD];     // per-wave partial sums / sums of squares
    __shared__ int s_col[kMaxIndexDims];
    __shared__ float s_lo[kMaxIndexDims];
    __shared__ float s_scale[kMaxIndexDims];

    DevJob J;
    if (A.seed) {
        J = A.single;
        if (threadIdx.x == 0) {
            *A.meta.table = A.single;
            A.meta.order[0] = 0;
            A.meta.unit_prefix[0] = 0;
            A.meta.unit_prefix[1] = A.single_units;
            A.meta.tile_prefix[0] = 0;
            A.meta.tile_prefix[1] = A.single_tiles;
            A.meta.super_prefix[0] = 0;
            A.meta.super_prefix[1] = A.single_supers;
        }
    } else {
        J = A.meta.table[blockIdx.x];
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < A.meta.n_counters) A.meta.counters[threadIdx.x] = 0;
    if (J.flags & kJobRadixIndex) return;    // indexed by the device-wide path

    const int n = J.n;
    const int d = J.d;
    const int c = J.c;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    // Mean and spread of every dimension of the subspace.
    float s[kMaxD], ss[kMaxD];
#pragma unroll
    for (int f = 0; f < kMaxD; ++f) { s[f] = 0.f; ss[f] = 0.f; }
    for (int i = tid; i < n; i += blockDim.x) {
#pragma unroll
        for (int f = 0; f < kMaxD; ++f) {
            if (f < d) {
                const float v = J.cols[(int64_t)J.feat[f] * J.ld + i];
                s[f] += v;
                ss[f] = fmaf(v, v, ss[f]);
            }
        }
    }
#pragma unroll
    for (int f = 0; f < kMaxD; ++f) {
        if (f < d) {
            const float a = wave_sum(s[f]);
            const float b = wave_sum(ss[f]);
            if (lane == 0) { red[0][wave][f] = a; red[1][wave][f] = b; }
        }
    }
    __syncthreads();
    if (tid == 0) {
        float mean[kMaxD], sd[kMaxD];
        const int nw = blockDim.x >> 6;
        for (int f = 0; f < d; ++f) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < nw; ++w) { a += red[0][w][f]; b += red[1][w][f]; }
            const double m = a / n;
            const double var = b / n - m * m;
            mean[f] = (float)m;
            sd[f] = var > 0.0 ? (float)sqrt(var) : 0.f;
        }
        choose_index_dims(J, mean, sd, s_col, s_lo, s_scale);
    }
    __syncthreads();

    const int P = next_pow2(n < 2 ? 2 : n);
    for (int i = tid; i < P; i += blockDim.x) {
        uint32_t packed = 0xFFFFFFFFu;
        if (i < n) packed = (morton_key(J, s_col, s_lo, s_scale, i) << J.idbits) | (uint32_t)i;
        buf[i] = packed;
    }
    __syncthreads();
    bitonic_sort_lds(buf, P);
    const uint32_t idmask = (J.idbits >= 32) ? 0xFFFFFFFFu : ((1u << J.idbits) - 1u);
    for (int i = tid; i < n; i += blockDim.x) J.perm[i] = (int32_t)(buf[i] & idmask);
}

__global__ __launch_bounds__(64) void k_reorder(Meta m, int32_t n_jobs) {
    const int u = blockIdx.x;
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (m.tile_prefix[mid] <= u) lo = mid; else hi = mid;
    }
    const DevJob J = m.table[lo];
    const int t = u - m.tile_prefix[lo];
    const int lane = threadIdx.x;
    const int pos = t * kTile + lane;
    const int n = J.n;
    const int d = J.d;
    const int dp = row_stride(d);
    const bool valid = pos < n;
    // The tile's 64 rows are one contiguous span of xs.  Each lane builds its
    // row in LDS and the wave then stores the span with consecutive lanes on
    // consecutive words: stored straight from the lanes, every store would
    // touch 64 cache lines at a stride of dp words, and the partial-line
    // writes cost several times the row bytes in HBM writes.
    __shared__ float s_tile[kTile * row_stride(kMaxD)];
    float* row = s_tile + lane * dp;
    float* box = J.boxes + (int64_t)t * 2 * dp;
    float* hbox = J.hboxes + (int64_t)t * 4 * dp;
    int id = INT32_MAX;
    if (valid) id = J.perm[pos];
    else J.perm[pos] = INT32_MAX;
    const float qnan = __int_as_float(0x7fc00000);
    float norm = 0.f;
#pragma unroll
    for (int f = 0; f < kMaxD + 4; ++f) {
        if (f < dp) {
            float v;
            if (f < d) {
                v = valid ? J.cols[(int64_t)J.feat[f] * J.ld + id] : qnan;
                if (valid) norm = fmaf(v, v, norm);
                // corners of each 32-object half, then of the whole tile
                const float hmn = half_min(valid ? v : INFINITY);
                const float hmx = half_max(valid ? v : -INFINITY);
                const float mn = fminf(hmn, __shfl_xor(hmn, 32, 64));
                const float mx = fmaxf(hmx, __shfl_xor(hmx, 32, 64));
                if (lane == 0) { box[f] = mn; box[dp + f] = mx; }
                if ((lane & 31) == 0) { hbox[(lane >> 5) * 2 * dp + f] = hmn; hbox[(lane >> 5) * 2 * dp + dp + f] = hmx; }
            } else {
                v = 0.f;
                if (lane == 0) { box[f] = 0.f; box[dp + f] = 0.f; }
                if ((lane & 31) == 0) { hbox[(lane >> 5) * 2 * dp + f] = 0.f; hbox[(lane >> 5) * 2 * dp + dp + f] = 0.f; }
            }
            row[f] = v;
        }
    }
    // Slot d: -pn (1 - c0) / 2, the addend of the join's expanded-form
    // prefilter (c0 = (8d + 24) 2^-24, see the join kernel).
    const float c0 = (float)(8 * d + 24) * 5.9604644775390625e-8f;
    row[d] = valid ? -0.5f * (norm * (1.0f - c0)) : qnan;
    // Slot d + 1: the object id, so the join reads it with the coordinates.
    row[d + 1] = __int_as_float(id);
    __syncthreads();
    float* span = J.xs + (int64_t)t * kTile * dp;
    for (int i = lane; i < kTile * dp; i += kTile) span[i] = s_tile[i];
}

// Corners of each super-tile (kSuper consecutive tiles of one job): one
// wavefront per super-tile, one lane per tile, after k_reorder.
__global__ __launch_bounds__(64) void k_super_boxes(Meta m, int32_t n_jobs) {
    const int u = blockIdx.x;
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (m.super_prefix[mid] <= u) lo = mid; else hi = mid;
    }
    const DevJob J = m.table[lo];
    const int S = u - m.super_prefix[lo];
    const int t = S * kSuper + (int)threadIdx.x;
    const bool valid = t < J.ntiles;
    const int dp = row_stride(J.d);
    for (int f = 0; f < dp; ++f) {
        const float l = wave_min(valid ? J.boxes[((int64_t)t * 2) * dp + f] : INFINITY);
        const float h = wave_max(valid ? J.boxes[((int64_t)t * 2 + 1) * dp + f] : -INFINITY);
        if (threadIdx.x == 0) {
            J.sboxes[((int64_t)S * 2) * dp + f] = l;
            J.sboxes[((int64_t)S * 2 + 1) * dp + f] = h;
        }
    }
}

hipError_t launch_super_boxes(const Meta& m, int32_t n_jobs, int32_t total_supers, hipStream_t s) {
    if (total_supers <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_super_boxes, dim3(total_supers), dim3(64), 0, s, m, n_jobs);
    return hipGetLastError();
}

// Clears the in-degree outputs of every job (four 64-object tiles per
// workgroup) at the start of the join pass, which adds to them atomically:
// a replay of the join pass alone recomputes the same in-degrees.
__global__ __launch_bounds__(256) void k_zero_indeg(Meta m, int32_t n_jobs, int32_t total_tiles) {
    const int u = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (u >= total_tiles) return;
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (m.tile_prefix[mid] <= u) lo = mid; else hi = mid;
    }
    int32_t* indeg = m.table[lo].indeg;
    const int64_t i = (int64_t)(u - m.tile_prefix[lo]) * kTile + (threadIdx.x & 63);
    if (indeg && i < m.table[lo].n) indeg[i] = 0;
}

hipError_t launch_zero_indeg(const Meta& m, int32_t n_jobs, int32_t total_tiles, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_indeg, dim3((total_tiles + 3) / 4), dim3(256), 0, s, m, n_jobs, total_tiles);
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int32_t n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_index_sort(const IndexArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_index_sort, dim3(grid), dim3(kSortThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reorder(const Meta& m, int32_t n_jobs, int32_t total_tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_reorder, dim3(total_tiles), dim3(64), 0, s, m, n_jobs);
    return hipGetLastError();
}

}  // namespace snaps
