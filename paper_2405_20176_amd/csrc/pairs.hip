// Row starts of the eps pair list (the result set A of Sec. 3.5 without the
// self-pairs): off[0] = 0 and off[i + 1] = off[i] + count[i] in int64, by a
// three-kernel scan -- chunk sums, a scan of the chunk sums in one
// workgroup, then each chunk's prefix from its start.
#include "snaps_internal.h"

namespace snaps {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;                             // counts per thread and chunk
constexpr int64_t kScanChunk = (int64_t)kScanThreads * kScanPer;

__device__ __forceinline__ long long wave_scan64(long long v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}

// Exclusive scan over the workgroup; *total gets the sum.
__device__ long long block_scan64(long long v, long long* tmp, long long* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const long long inc = wave_scan64(v);
    if (lane == 63) tmp[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        const long long w = lane < nw ? tmp[lane] : 0;
        const long long wi = wave_scan64(w);
        if (lane < nw) tmp[lane] = wi - w;
        if (lane == nw - 1) tmp[16] = wi;
    }
    __syncthreads();
    const long long out = inc - v + tmp[wave];
    *total = tmp[16];
    __syncthreads();
    return out;
}

__global__ __launch_bounds__(kScanThreads) void k_pair_chunk_sums(const int32_t* count, int64_t n, long long* sums) {
    __shared__ long long tmp[17];
    const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
    long long v = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int64_t i = c0 + (int64_t)j * kScanThreads + threadIdx.x;
        if (i < n) v += count[i];
    }
    long long total;
    block_scan64(v, tmp, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the chunk sums in place.
__global__ __launch_bounds__(kScanThreads) void k_pair_scan_sums(long long* sums, int nb) {
    __shared__ long long tmp[17];
    const int per = (nb + kScanThreads - 1) / kScanThreads;
    const int b0 = threadIdx.x * per;
    long long v = 0;
    for (int b = 0; b < per; ++b)
        if (b0 + b < nb) v += sums[b0 + b];
    long long total;
    long long run = block_scan64(v, tmp, &total);
    for (int b = 0; b < per; ++b) {
        if (b0 + b < nb) {
            const long long x = sums[b0 + b];
            sums[b0 + b] = run;
            run += x;
        }
    }
}

// Each thread scans its kScanPer consecutive counts of the chunk.
__global__ __launch_bounds__(kScanThreads) void k_pair_offsets(const int32_t* count, int64_t n, const long long* sums,
                                                               int64_t* off) {
    __shared__ long long tmp[17];
    const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    int32_t c[kScanPer];
    long long v = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        c[j] = i0 + j < n ? count[i0 + j] : 0;
        v += c[j];
    }
    long long total;
    long long run = sums[blockIdx.x] + block_scan64(v, tmp, &total);
    if (blockIdx.x == 0 && threadIdx.x == 0) off[0] = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        run += c[j];
        if (i0 + j < n) off[i0 + j + 1] = run;
    }
}

}  // namespace

size_t pair_scan_scratch(int64_t n) {
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    return (size_t)nb * sizeof(long long);
}

hipError_t launch_pair_offsets(const int32_t* count, int64_t n, int64_t* off, void* scratch, hipStream_t s) {
    if (n < 1) return hipSuccess;
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    long long* sums = static_cast<long long*>(scratch);
    hipLaunchKernelGGL(k_pair_chunk_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, s, count, n, sums);
    hipLaunchKernelGGL(k_pair_scan_sums, dim3(1), dim3(kScanThreads), 0, s, sums, (int)nb);
    hipLaunchKernelGGL(k_pair_offsets, dim3((unsigned)nb), dim3(kScanThreads), 0, s, count, n,
                       (const long long*)sums, off);
    return hipGetLastError();
}

}  // namespace snaps
