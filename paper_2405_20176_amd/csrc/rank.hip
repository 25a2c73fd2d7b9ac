// Dense per-space rankings of the four outlier metrics (paper Sec. 3.4,
// Tab. 2): r_i = the number of distinct metric values strictly more
// outlying than object i's value, so rank 0 is the most outlying object and
// equal values share a rank.
//
// One workgroup per (job, metric).  Each metric is mapped to a 32-bit key
// whose ascending order is "more outlying first":
//   eps_count, indeg   ascending integers, the value itself;
//   eps_mean           descending, objects without any eps neighbour first;
//   knn_mean           descending.
// The float metrics' keys are sorted in LDS, compacted to their distinct
// values, and every object's rank is the position of its key among the
// distinct values (binary search).  The integer metrics (values below
// 32,768 here) need no sort: a bitmap in LDS marks the values present, and
// an object's rank is the number of marked values below its own (a scan of
// the words' popcounts, then one popcount within the word).
#include "snaps_internal.h"
#include "common.cuh"
#include "keys.cuh"

namespace snaps {

struct RankLaunch {
    RankArgs a;
    int32_t seed;
    DevJob single;
};

__global__ __launch_bounds__(kSortThreads) void k_rank(RankLaunch L) {
    __shared__ uint32_t buf[kLdsSortMax];
    __shared__ int tmp[17];
    const DevJob J = L.seed ? L.single : L.a.table[blockIdx.x];
    if (J.rank == nullptr || (J.flags & kJobRadixRank)) return;   // ranked by the device-wide path
    const int metric = blockIdx.y;
    const int n = J.n;
    const int tid = threadIdx.x;
    const int P = next_pow2(n < 2 ? 2 : n);

    bool small_ints = false;
    if (metric == 0 || metric == 2) {
        // integer metric: the bitmap path when every value is below
        // kLdsSortMax (always for the join's counts and in-degrees here, as
        // n <= kLdsSortMax; values from a caller of snaps_rank may not be)
        uint32_t mx = 0u;
        for (int i = tid; i < n; i += blockDim.x) mx = max(mx, metric_key(J, metric, i));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
        if ((tid & 63) == 0) tmp[tid >> 6] = (int)mx;
        __syncthreads();
        if (tid == 0) {
            uint32_t m = 0u;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = max(m, (uint32_t)tmp[w]);
            tmp[16] = m < (uint32_t)kLdsSortMax ? 1 : 0;
        }
        __syncthreads();
        small_ints = tmp[16] != 0;
        __syncthreads();
    }
    if (small_ints) {
        constexpr int kWords = kLdsSortMax / 32;
        uint32_t* bm = buf;                      // presence bitmap
        uint32_t* pre = buf + kWords;            // marked values below each word
        for (int w = tid; w < kWords; w += blockDim.x) bm[w] = 0u;
        __syncthreads();
        for (int i = tid; i < n; i += blockDim.x) {
            const uint32_t v = metric_key(J, metric, i);
            atomicOr(&bm[v >> 5], 1u << (v & 31u));
        }
        __syncthreads();
        static_assert(kWords == kSortThreads, "one bitmap word per thread");
        int total = 0;
        const int below = block_exclusive_scan(__popc(bm[tid]), tmp, &total);
        pre[tid] = (uint32_t)below;
        __syncthreads();
        int32_t* out = J.rank + (int64_t)metric * n;
        for (int i = tid; i < n; i += blockDim.x) {
            const uint32_t v = metric_key(J, metric, i);
            out[i] = (int32_t)(pre[v >> 5] + __popc(bm[v >> 5] & ((1u << (v & 31u)) - 1u)));
        }
        return;
    }

    for (int i = tid; i < P; i += blockDim.x) buf[i] = i < n ? metric_key(J, metric, i) : 0xFFFFFFFFu;
    __syncthreads();
    bitonic_sort_lds(buf, P);

    // Compact the sorted keys to their distinct values, in place: every thread
    // first reads its block of E consecutive keys (and the key before it) into
    // registers, then the blocks are written at their scanned offsets.
    constexpr int kMaxE = kLdsSortMax / kSortThreads;
    const int E = P >= (int)blockDim.x ? P / (int)blockDim.x : 1;
    const int b0 = tid * E;
    uint32_t vals[kMaxE];
    bool flag[kMaxE];
    int nflag = 0;
    uint32_t prev = (b0 > 0 && b0 - 1 < P) ? buf[b0 - 1] : 0u;
#pragma unroll
    for (int e = 0; e < kMaxE; ++e) {
        vals[e] = 0u;
        flag[e] = false;
        if (e < E) {
            const int i = b0 + e;
            if (i < n) {
                vals[e] = buf[i];
                flag[e] = (i == 0) || (vals[e] != prev);
                prev = vals[e];
                nflag += flag[e] ? 1 : 0;
            }
        }
    }
    int total = 0;
    int pos = block_exclusive_scan(nflag, tmp, &total);
#pragma unroll
    for (int e = 0; e < kMaxE; ++e) {
        if (flag[e]) buf[pos++] = vals[e];
    }
    __syncthreads();

    int32_t* out = J.rank + (int64_t)metric * n;
    for (int i = tid; i < n; i += blockDim.x) {
        const uint32_t key = metric_key(J, metric, i);
        int lo = 0, hi = total;          // first distinct value >= key
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (buf[mid] < key) lo = mid + 1; else hi = mid;
        }
        out[i] = lo;
    }
}

// One 64-object tile of one job per workgroup: ensemble[i] = the mean of
// the object's four dense ranks (rounded once, from the exact integer sum).
__global__ __launch_bounds__(64) void k_ensemble(const DevJob* table, int n_jobs, const int32_t* tile_prefix) {
    const int b = blockIdx.x;
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_prefix[mid] <= b) lo = mid; else hi = mid;
    }
    const DevJob& J = table[lo];
    if (J.ensemble == nullptr || J.rank == nullptr) return;
    const int64_t i = (int64_t)(b - tile_prefix[lo]) * kTile + threadIdx.x;
    if (i >= J.n) return;
    const int64_t n = J.n;
    const int64_t sum = (int64_t)J.rank[i] + J.rank[n + i] + J.rank[2 * n + i] + J.rank[3 * n + i];
    J.ensemble[i] = (float)((double)sum * 0.25);
}

hipError_t launch_ensemble(const DevJob* table, int n_jobs, const int32_t* tile_prefix, int total_tiles,
                           hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ensemble, dim3(total_tiles), dim3(64), 0, s, table, n_jobs, tile_prefix);
    return hipGetLastError();
}

hipError_t launch_rank(const RankArgs& a, hipStream_t s) {
    RankLaunch L{};
    L.a = a;
    L.seed = 0;
    hipLaunchKernelGGL(k_rank, dim3(a.n_jobs, 4), dim3(kSortThreads), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_rank_single(const DevJob& j, hipStream_t s) {
    RankLaunch L{};
    L.a.table = nullptr;
    L.a.n_jobs = 1;
    L.seed = 1;
    L.single = j;
    hipLaunchKernelGGL(k_rank, dim3(1, 4), dim3(kSortThreads), 0, s, L);
    return hipGetLastError();
}

}  // namespace snaps
