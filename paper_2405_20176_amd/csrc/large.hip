// Index build and ranks of jobs whose n exceeds one workgroup's LDS sort.
//
// Index (before k_reorder, which is shared with small jobs):
//   k_large_zero / k_large_stats: per-dimension sums and sums of squares over
//     the job's d columns (float per chunk, float64 atomics across chunks);
//   k_large_select: mean and spread -> the c most spread dimensions and their
//     cell grids (same rule as the LDS path);
//   k_large_keys: Morton key of every object (32 bits) and its id;
//   device-wide stable radix sort of (key, id): ids in key order = perm.
// Ranks (after the join):
//   k_large_rank_keys: order-preserving key of every object on each metric;
//   device-wide radix sort of every (job, metric) key segment;
//   k_large_rank_distinct: one workgroup per segment compacts the sorted keys
//     to their distinct values;
//   k_large_rank_lookup: rank = position of the object's key among them.
#include "snaps_internal.h"
#include "common.cuh"
#include "keys.cuh"

namespace snaps {

namespace {

__device__ __forceinline__ int find_seg(const int32_t* prefix, int n, int b) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace

__global__ void k_large_zero(const LargeIndex* li) {
    const LargeIndex L = li[blockIdx.x];
    if (threadIdx.x < 2 * kMaxD) L.acc[threadIdx.x] = 0.0;
}

__global__ __launch_bounds__(256) void k_large_stats(const DevJob* table, const LargeIndex* li, const int32_t* prefix,
                                                      int n_large) {
    __shared__ float red[2][4][kMaxD];
    const int b = blockIdx.x;
    const int s = find_seg(prefix, n_large, b);
    const LargeIndex L = li[s];
    const DevJob J = table[L.job];
    const int64_t c = b - prefix[s];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float sm[kMaxD], sq[kMaxD];
#pragma unroll
    for (int f = 0; f < kMaxD; ++f) { sm[f] = 0.f; sq[f] = 0.f; }
    for (int r = 0; r < kRadixChunk / 256; ++r) {
        const int64_t i = c * kRadixChunk + r * 256 + tid;
        if (i < J.n) {
#pragma unroll
            for (int f = 0; f < kMaxD; ++f) {
                if (f < J.d) {
                    const float v = J.cols[(int64_t)J.feat[f] * J.ld + i];
                    sm[f] += v;
                    sq[f] = fmaf(v, v, sq[f]);
                }
            }
        }
    }
#pragma unroll
    for (int f = 0; f < kMaxD; ++f) {
        const float a = wave_sum(sm[f]);
        const float q = wave_sum(sq[f]);
        if (lane == 0) { red[0][wave][f] = a; red[1][wave][f] = q; }
    }
    __syncthreads();
    if (tid < 2 * kMaxD) {
        const int which = tid / kMaxD, f = tid % kMaxD;
        if (f < J.d) {
            const float v = red[which][0][f] + red[which][1][f] + red[which][2][f] + red[which][3][f];
            atomicAdd(L.acc + which * kMaxD + f, (double)v);
        }
    }
}

__global__ void k_large_select(const DevJob* table, const LargeIndex* li) {
    const LargeIndex L = li[blockIdx.x];
    const DevJob J = table[L.job];
    if (threadIdx.x != 0) return;
    float mean[kMaxD], sd[kMaxD];
    for (int f = 0; f < J.d; ++f) {
        const double m = L.acc[f] / J.n;
        const double var = L.acc[kMaxD + f] / J.n - m * m;
        mean[f] = (float)m;
        sd[f] = var > 0.0 ? (float)sqrt(var) : 0.f;
    }
    choose_index_dims(J, mean, sd, L.sel_col, L.sel_lo, L.sel_scale);
}

__global__ __launch_bounds__(256) void k_large_keys(const DevJob* table, const LargeIndex* li, const int32_t* prefix,
                                                     int n_large) {
    __shared__ int col[kMaxIndexDims];
    __shared__ float lo[kMaxIndexDims], sc[kMaxIndexDims];
    const int b = blockIdx.x;
    const int s = find_seg(prefix, n_large, b);
    const LargeIndex L = li[s];
    const DevJob J = table[L.job];
    if (threadIdx.x < kMaxIndexDims) {
        col[threadIdx.x] = L.sel_col[threadIdx.x];
        lo[threadIdx.x] = L.sel_lo[threadIdx.x];
        sc[threadIdx.x] = L.sel_scale[threadIdx.x];
    }
    __syncthreads();
    const int64_t c = b - prefix[s];
    for (int r = 0; r < kRadixChunk / 256; ++r) {
        const int64_t i = c * kRadixChunk + r * 256 + threadIdx.x;
        if (i < J.n) {
            L.keys[i] = morton_key(J, col, lo, sc, i);
            L.vals[i] = (uint32_t)i;
        }
    }
}

hipError_t launch_large_index(const DevJob* table, const LargeIndex* li, int n_large, const int32_t* chunk_prefix,
                              int total_chunks, const SortSeg* segs, hipStream_t s) {
    if (n_large == 0) return hipSuccess;
    hipLaunchKernelGGL(k_large_zero, dim3(n_large), dim3(64), 0, s, li);
    hipLaunchKernelGGL(k_large_stats, dim3(total_chunks), dim3(256), 0, s, table, li, chunk_prefix, n_large);
    hipLaunchKernelGGL(k_large_select, dim3(n_large), dim3(64), 0, s, table, li);
    hipLaunchKernelGGL(k_large_keys, dim3(total_chunks), dim3(256), 0, s, table, li, chunk_prefix, n_large);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_radix_sort(segs, chunk_prefix, n_large, total_chunks, 4, s);
}

__global__ __launch_bounds__(256) void k_large_rank_keys(const DevJob* table, const LargeRank* lr,
                                                          const int32_t* prefix, int n_large) {
    const int b = blockIdx.x;
    const int m = blockIdx.y;
    const int s = find_seg(prefix, n_large, b);
    const LargeRank L = lr[s];
    const DevJob J = table[L.job];
    const int64_t c = b - prefix[s];
    for (int r = 0; r < kRadixChunk / 256; ++r) {
        const int64_t i = c * kRadixChunk + r * 256 + threadIdx.x;
        if (i < J.n) L.keys[m][i] = metric_key(J, m, i);
    }
}

__global__ __launch_bounds__(1024) void k_large_rank_distinct(const DevJob* table, const LargeRank* lr) {
    __shared__ int tmp[17];
    const int s = blockIdx.x >> 2;
    const int m = blockIdx.x & 3;
    const LargeRank L = lr[s];
    const int64_t n = table[L.job].n;
    const uint32_t* key = L.keys[m];
    uint32_t* out = L.distinct[m];
    const int64_t per = (n + blockDim.x - 1) / blockDim.x;
    const int64_t b0 = per * threadIdx.x;
    const int64_t b1 = b0 + per < n ? b0 + per : n;
    int local = 0;
    for (int64_t i = b0; i < b1; ++i) local += (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
    int total = 0;
    int pos = block_exclusive_scan(local, tmp, &total);
    for (int64_t i = b0; i < b1; ++i)
        if (i == 0 || key[i] != key[i - 1]) out[pos++] = key[i];
    if (threadIdx.x == 0) L.n_distinct[m] = total;
}

__global__ __launch_bounds__(256) void k_large_rank_lookup(const DevJob* table, const LargeRank* lr,
                                                            const int32_t* prefix, int n_large) {
    const int b = blockIdx.x;
    const int m = blockIdx.y;
    const int s = find_seg(prefix, n_large, b);
    const LargeRank L = lr[s];
    const DevJob J = table[L.job];
    const int64_t c = b - prefix[s];
    const uint32_t* dv = L.distinct[m];
    const int nd = L.n_distinct[m];
    int32_t* out = J.rank + (int64_t)m * J.n;
    for (int r = 0; r < kRadixChunk / 256; ++r) {
        const int64_t i = c * kRadixChunk + r * 256 + threadIdx.x;
        if (i < J.n) {
            const uint32_t key = metric_key(J, m, i);
            int lo = 0, hi = nd;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (dv[mid] < key) lo = mid + 1; else hi = mid;
            }
            out[i] = lo;
        }
    }
}

hipError_t launch_large_rank(const DevJob* table, const LargeRank* lr, int n_large, const int32_t* chunk_prefix,
                             int total_chunks, const SortSeg* segs, const int32_t* seg_chunk_prefix,
                             int total_seg_chunks, hipStream_t s) {
    if (n_large == 0) return hipSuccess;
    hipLaunchKernelGGL(k_large_rank_keys, dim3(total_chunks, 4), dim3(256), 0, s, table, lr, chunk_prefix, n_large);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_radix_sort(segs, seg_chunk_prefix, 4 * n_large, total_seg_chunks, 4, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_large_rank_distinct, dim3(4 * n_large), dim3(1024), 0, s, table, lr);
    hipLaunchKernelGGL(k_large_rank_lookup, dim3(total_chunks, 4), dim3(256), 0, s, table, lr, chunk_prefix,
                       n_large);
    return hipGetLastError();
}

}  // namespace snaps
