// Segmented, stable LSD radix sort of 32-bit keys (optionally with a 32-bit
// payload) in device memory, for segments too large for one workgroup's LDS.
//
// Each segment is cut into chunks of 4096 elements; one workgroup handles one
// chunk of one segment.  One pass over 8 key bits:
//   1. k_radix_hist:    per-chunk histogram of the 256 digit values (LDS atomics)
//   2. k_radix_scan:    per segment (one workgroup), exclusive scan of the
//                       histograms in digit-major order -> each chunk's first
//                       output slot for each digit
//   3. k_radix_scatter: per chunk, the elements are taken in their input order
//                       in rounds of 256; inside a round every wavefront ranks
//                       its 64 elements among equal digits with 8 ballots, the
//                       wavefronts' counts are scanned in LDS, so every element
//                       gets its place among the chunk's equal digits: the pass
//                       is stable.  The chunk is first laid out in LDS in digit
//                       order, then stored with consecutive threads on
//                       consecutive elements, so each digit's run of the chunk
//                       goes out as one contiguous span (stored straight from
//                       the rounds, each round's elements would land on up to
//                       256 runs, a few bytes per cache line).
// Four passes sort 32-bit keys; an even number of passes leaves the result in
// buffer 0.
#include "snaps_internal.h"
#include "common.cuh"

namespace snaps {

constexpr int kRadixThreads = 256;
constexpr int kRadixRounds = kRadixChunk / kRadixThreads;

namespace {

__device__ __forceinline__ int find_segment(const int32_t* chunk_prefix, int n_segs, int b) {
    int lo = 0, hi = n_segs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (chunk_prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const SortSeg* segs, const int32_t* chunk_prefix,
                                                               int n_segs, int shift, int src) {
    __shared__ int h[256];
    const int b = blockIdx.x;
    const int s = find_segment(chunk_prefix, n_segs, b);
    const SortSeg g = segs[s];
    const int c = b - chunk_prefix[s];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint32_t* key = g.key[src];
    const int64_t base = (int64_t)c * kRadixChunk;
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t i = base + r * kRadixThreads + tid;
        if (i < g.n) atomicAdd(&h[(key[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    g.hist[(int64_t)tid * g.nchunks + c] = h[tid];
}

__global__ __launch_bounds__(1024) void k_radix_scan(const SortSeg* segs) {
    __shared__ int tmp[17];
    const SortSeg g = segs[blockIdx.x];
    const int64_t total = 256 * (int64_t)g.nchunks;
    const int64_t per = (total + blockDim.x - 1) / blockDim.x;
    const int64_t b0 = per * threadIdx.x;
    const int64_t b1 = b0 + per < total ? b0 + per : total;
    int local = 0;
    for (int64_t i = b0; i < b1; ++i) local += g.hist[i];
    int tot = 0;
    int run = block_exclusive_scan(local, tmp, &tot);
    for (int64_t i = b0; i < b1; ++i) {
        const int v = g.hist[i];
        g.hist[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const SortSeg* segs, const int32_t* chunk_prefix,
                                                                  int n_segs, int shift, int src) {
    __shared__ int off[256];                     // chunk-local start of each digit's run
    __shared__ int goff[256];                    // global start of each digit's run of this chunk
    __shared__ int wcnt[kRadixThreads / 64][256];
    __shared__ int tmp[17];
    __shared__ uint32_t s_key[kRadixChunk];
    __shared__ uint32_t s_val[kRadixChunk];
    const int b = blockIdx.x;
    const int s = find_segment(chunk_prefix, n_segs, b);
    const SortSeg g = segs[s];
    const int c = b - chunk_prefix[s];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const uint32_t* kin = g.key[src];
    uint32_t* kout = g.key[src ^ 1];
    const uint32_t* vin = g.val[src];
    uint32_t* vout = g.val[src ^ 1];
    const int64_t base = (int64_t)c * kRadixChunk;
    const int m = (int)min((int64_t)kRadixChunk, g.n - base);    // elements of this chunk
    // The chunk's histogram (for the local run starts), from this pass's keys.
    off[tid] = 0;
    __syncthreads();
    for (int r = 0; r < kRadixRounds; ++r) {
        const int e = r * kRadixThreads + tid;
        if (e < m) atomicAdd(&off[(kin[base + e] >> shift) & 255u], 1);
    }
    __syncthreads();
    {
        int total;
        const int cnt = off[tid];
        const int start = block_exclusive_scan(cnt, tmp, &total);
        goff[tid] = g.hist[(int64_t)tid * g.nchunks + c] - start;   // global position = goff + local
        off[tid] = start;
    }
    __syncthreads();
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kRadixRounds; ++r) {
#pragma unroll
        for (int w = 0; w < kRadixThreads / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int e = r * kRadixThreads + tid;
        const bool valid = e < m;
        const uint32_t key = valid ? kin[base + e] : 0u;
        const uint32_t digit = (key >> shift) & 255u;
        unsigned long long match = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const unsigned long long bb = __ballot((digit >> bit) & 1u);
            match &= ((digit >> bit) & 1u) ? bb : ~bb;
        }
        const int rank = __popcll(match & below);
        if (valid && rank == 0) wcnt[wave][digit] = __popcll(match);
        __syncthreads();
        {
            int run = off[tid];
#pragma unroll
            for (int w = 0; w < kRadixThreads / 64; ++w) {
                const int cw = wcnt[w][tid];
                wcnt[w][tid] = run;
                run += cw;
            }
            off[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const int at = wcnt[wave][digit] + rank;   // chunk-local position in digit order
            s_key[at] = key;
            if (vin) s_val[at] = vin[base + e];
        }
        __syncthreads();
    }
    // Digit-ordered chunk out: local position p of digit d goes to goff[d] + p.
    for (int p = tid; p < m; p += kRadixThreads) {
        const uint32_t key = s_key[p];
        const int dst = goff[(key >> shift) & 255u] + p;
        kout[dst] = key;
        if (vin) vout[dst] = s_val[p];
    }
}

hipError_t launch_radix_sort(const SortSeg* segs, const int32_t* chunk_prefix, int n_segs, int total_chunks,
                             int passes, hipStream_t s) {
    if (n_segs == 0 || total_chunks == 0) return hipSuccess;
    for (int p = 0; p < passes; ++p) {
        const int src = p & 1;
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(total_chunks), dim3(kRadixThreads), 0, s, segs, chunk_prefix, n_segs,
                           shift, src);
        hipLaunchKernelGGL(k_radix_scan, dim3(n_segs), dim3(1024), 0, s, segs);
        hipLaunchKernelGGL(k_radix_scatter, dim3(total_chunks), dim3(kRadixThreads), 0, s, segs, chunk_prefix,
                           n_segs, shift, src);
    }
    return hipGetLastError();
}

}  // namespace snaps
