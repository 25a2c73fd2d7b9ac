// Sampled-distance choice of the search radius (paper Sec. 3.5.3): for a
// sample of m objects, the distances to every other object of the subspace,
// and the radius at which the sample's mean neighbour count reaches a target
// selectivity -- the midpoint between the r-th smallest of those m (n - 1)
// distances (r = round(target m)) and the next one.  The paper uses it to
// find eps_min and eps_max of the eps grid (selectivities 0.1 % and 15 % of
// the population).
//
// The r-th smallest is found exactly, without storing the distances: a
// radix selection over the bits of the float32 squared distances (all >= 0,
// so their bit patterns order like their values), 8 bits per pass, each
// pass recomputing the sample's distances and histogramming those that
// share the prefix found so far.  sqrt is monotone and correctly rounded,
// so the r-th smallest distance is the square root of the r-th smallest
// squared distance.  A last pass finds the smallest squared distance above
// it when the r-th is the last of its ties.
#include "snaps_internal.h"
#include "common.cuh"

namespace snaps {

namespace {

constexpr int kEpsThreads = 256;

// One block per (job, sample object).
__device__ __forceinline__ int eps_job_of(const int32_t* prefix, int n_jobs, int b) {
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Squared float32 distance of object i to the sample object's coordinates,
// in the direct form and feature order of the join.
template <int D>
__device__ __forceinline__ float sq_dist(const EpsJob& J, const float (&q)[kMaxD], int64_t i) {
    float dd = 0.f;
#pragma unroll
    for (int f = 0; f < kMaxD; ++f) {
        if (f < D) {
            const float tq = q[f] - J.cols[(int64_t)J.feat[f] * J.ld + i];
            dd = fmaf(tq, tq, dd);
        }
    }
    return dd;
}

template <int D>
__device__ void eps_hist_body(const EpsJob& J, int s, int pass) {
    __shared__ unsigned h[kMaxEpsTargets][256];
    for (int x = threadIdx.x; x < kMaxEpsTargets * 256; x += blockDim.x) h[x >> 8][x & 255] = 0u;
    __syncthreads();
    const int qid = J.sample[s];
    if (qid >= 0 && qid < J.n) {
        float q[kMaxD];
#pragma unroll
        for (int f = 0; f < kMaxD; ++f) q[f] = f < D ? J.cols[(int64_t)J.feat[f] * J.ld + qid] : 0.f;
        const int shift = 24 - 8 * pass;        // bits of this pass: [shift, shift + 8)
        for (int64_t i = threadIdx.x; i < J.n; i += blockDim.x) {
            if (i == qid) continue;
            const uint32_t bits = __float_as_uint(sq_dist<D>(J, q, i));
            for (int t = 0; t < J.n_targets; ++t) {
                const EpsState& st = J.state[t];
                if (pass > 0 && (bits >> (shift + 8)) != st.prefix) continue;
                atomicAdd(&h[t][(bits >> shift) & 255u], 1u);
            }
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < J.n_targets * 256; x += blockDim.x) {
        const unsigned c = h[x >> 8][x & 255];
        if (c) atomicAdd(J.hist + x, c);
    }
}

template <int D>
__device__ void eps_next_body(const EpsJob& J, int s) {
    __shared__ unsigned mn[kMaxEpsTargets];
    if (threadIdx.x < kMaxEpsTargets) mn[threadIdx.x] = 0xFFFFFFFFu;
    __syncthreads();
    const int qid = J.sample[s];
    if (qid >= 0 && qid < J.n) {
        float q[kMaxD];
#pragma unroll
        for (int f = 0; f < kMaxD; ++f) q[f] = f < D ? J.cols[(int64_t)J.feat[f] * J.ld + qid] : 0.f;
        for (int64_t i = threadIdx.x; i < J.n; i += blockDim.x) {
            if (i == qid) continue;
            const uint32_t bits = __float_as_uint(sq_dist<D>(J, q, i));
            for (int t = 0; t < J.n_targets; ++t) {
                const EpsState& st = J.state[t];
                if (st.need_next && bits > st.prefix) atomicMin(&mn[t], bits);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < J.n_targets && mn[threadIdx.x] != 0xFFFFFFFFu)
        atomicMin(&J.state[threadIdx.x].next, mn[threadIdx.x]);
}

template <int D>
__global__ __launch_bounds__(kEpsThreads) void k_eps_hist(const EpsJob* jobs, const int32_t* prefix, int n_jobs,
                                                          int pass, int block0) {
    const int b = block0 + (int)blockIdx.x;
    const int j = eps_job_of(prefix, n_jobs, b);
    eps_hist_body<D>(jobs[j], b - prefix[j], pass);
}

template <int D>
__global__ __launch_bounds__(kEpsThreads) void k_eps_next(const EpsJob* jobs, const int32_t* prefix, int n_jobs,
                                                          int block0) {
    const int b = block0 + (int)blockIdx.x;
    const int j = eps_job_of(prefix, n_jobs, b);
    eps_next_body<D>(jobs[j], b - prefix[j]);
}

__global__ void k_eps_init(const EpsJob* jobs, int n_jobs) {
    const int j = blockIdx.x;
    if (j >= n_jobs) return;
    const EpsJob& J = jobs[j];
    for (int x = threadIdx.x; x < J.n_targets * 256; x += blockDim.x) J.hist[x] = 0u;
    if (threadIdx.x < J.n_targets) {
        EpsState& st = J.state[threadIdx.x];
        st.prefix = 0u;
        st.rem = J.rank[threadIdx.x];
        st.eq = 0u;
        st.next = 0xFFFFFFFFu;
        st.need_next = 0u;
        st.bad = 0u;
    }
}

// After a histogram pass: the bucket holding the remaining rank becomes the
// next 8 bits of the prefix; the histogram is cleared for the next pass.
__global__ void k_eps_pick(const EpsJob* jobs, int n_jobs, int pass) {
    const int j = blockIdx.x;
    if (j >= n_jobs) return;
    const EpsJob& J = jobs[j];
    if (threadIdx.x < J.n_targets) {
        const int t = threadIdx.x;
        EpsState& st = J.state[t];
        unsigned* h = J.hist + t * 256;
        unsigned cum = 0u;
        int b = -1;
        for (int x = 0; x < 256; ++x) {
            if (b < 0 && cum + h[x] >= st.rem) b = x;
            else if (b < 0) cum += h[x];
        }
        if (b < 0) {
            st.bad = 1u;                          // fewer distances than the rank (ids outside [0, n))
            b = 255;
        } else {
            st.rem -= cum;
            st.eq = h[b];
        }
        st.prefix = (st.prefix << 8) | (unsigned)b;
        if (pass == 3) st.need_next = (st.rem + 1u > st.eq) ? 1u : 0u;
    }
    __syncthreads();
    for (int x = threadIdx.x; x < J.n_targets * 256; x += blockDim.x) J.hist[x] = 0u;
}

__global__ void k_eps_finish(const EpsJob* jobs, int n_jobs) {
    const int j = blockIdx.x;
    if (j >= n_jobs) return;
    const EpsJob& J = jobs[j];
    if (threadIdx.x < J.n_targets) {
        const EpsState& st = J.state[threadIdx.x];
        const unsigned nb = st.need_next ? st.next : st.prefix;
        float e;
        if (st.bad || nb == 0xFFFFFFFFu) {
            e = NAN;
        } else {
            const float a = sqrtf(__uint_as_float(st.prefix));
            const float b = sqrtf(__uint_as_float(nb));
            e = 0.5f * (a + b);
        }
        J.eps[threadIdx.x] = e;
    }
}

using EpsFn = void (*)(const EpsJob*, const int32_t*, int, int, int);
using EpsNextFn = void (*)(const EpsJob*, const int32_t*, int, int);

template <int D>
void eps_fns(EpsFn* h, EpsNextFn* nx) {
    *h = k_eps_hist<D>;
    *nx = k_eps_next<D>;
}

bool eps_pick_d(int d, EpsFn* h, EpsNextFn* nx) {
    switch (d) {
        case 2: eps_fns<2>(h, nx); return true;
        case 3: eps_fns<3>(h, nx); return true;
        case 4: eps_fns<4>(h, nx); return true;
        case 5: eps_fns<5>(h, nx); return true;
        case 6: eps_fns<6>(h, nx); return true;
        case 7: eps_fns<7>(h, nx); return true;
        case 8: eps_fns<8>(h, nx); return true;
        case 9: eps_fns<9>(h, nx); return true;
        case 10: eps_fns<10>(h, nx); return true;
        case 11: eps_fns<11>(h, nx); return true;
        case 12: eps_fns<12>(h, nx); return true;
        case 13: eps_fns<13>(h, nx); return true;
        case 14: eps_fns<14>(h, nx); return true;
        case 15: eps_fns<15>(h, nx); return true;
        case 16: eps_fns<16>(h, nx); return true;
    }
    return false;
}

}  // namespace

// jobs: device table of one dimensionality d; prefix[n_jobs + 1]: sample
// prefix (blocks per job = m).
hipError_t launch_eps_sample(const EpsJob* jobs, const int32_t* prefix, int n_jobs, int total_blocks, int d,
                             hipStream_t s) {
    EpsFn hist;
    EpsNextFn next;
    if (!eps_pick_d(d, &hist, &next)) return hipErrorInvalidValue;
    if (n_jobs <= 0 || total_blocks <= 0) return hipSuccess;
    // A dispatch counts its work-items in 32 bits: launches of at most 2^22
    // workgroups of 256.
    constexpr int kMaxBlocks = 1 << 22;
    hipLaunchKernelGGL(k_eps_init, dim3(n_jobs), dim3(256), 0, s, jobs, n_jobs);
    for (int pass = 0; pass < 4; ++pass) {
        for (int b0 = 0; b0 < total_blocks; b0 += kMaxBlocks)
            hipLaunchKernelGGL(hist, dim3(min(kMaxBlocks, total_blocks - b0)), dim3(kEpsThreads), 0, s, jobs, prefix,
                               n_jobs, pass, b0);
        hipLaunchKernelGGL(k_eps_pick, dim3(n_jobs), dim3(256), 0, s, jobs, n_jobs, pass);
    }
    for (int b0 = 0; b0 < total_blocks; b0 += kMaxBlocks)
        hipLaunchKernelGGL(next, dim3(min(kMaxBlocks, total_blocks - b0)), dim3(kEpsThreads), 0, s, jobs, prefix, n_jobs,
                           b0);
    hipLaunchKernelGGL(k_eps_finish, dim3(n_jobs), dim3(64), 0, s, jobs, n_jobs);
    return hipGetLastError();
}

}  // namespace snaps
