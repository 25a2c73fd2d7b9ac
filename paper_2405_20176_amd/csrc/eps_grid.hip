// Selection of the search radius between under- and overfitting (paper
// Sec. 3.5.2, Eq. 2-3).  For a grid of radii eps_1 < ... < eps_g of one
// subspace:
//   k_grid_join: one range self-join at the largest radius whose neighbours
//     are binned by the smallest grid radius that holds them, so that the
//     result sets of every smaller radius follow by accumulation (Sec. 3.5.3:
//     they are subsets of the largest one).  Per object and radius: the
//     neighbour count and the mean neighbour distance.
//   k_grid_top: for every radius and both metrics (count ascending, mean
//     descending with neighbourless objects first -- the order of the dense
//     rankings), the top n most outlying objects in (rank, id) order, found
//     by an exact radix selection of the n-th smallest key and an id-order
//     scan of the ties at it; stored as a bit set.
//   k_grid_select: Eq. 2 similarities of every radius's top n to those of
//     the smallest (U^min) and largest (U^max) radius, and Eq. 3: the radius
//     minimising |U^min - U^max| (the first of equal gaps).
#include "snaps_internal.h"
#include "common.cuh"
#include "keys.cuh"

namespace snaps {

namespace {

constexpr int kTopThreads = 1024;

__device__ __forceinline__ int job_of_prefix(const int32_t* prefix, int n_jobs, int b) {
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// One 64-query tile of one job per workgroup (one wavefront).  Candidates in
// groups of four consecutive objects, read as one 16-byte scalar load per
// feature column (the columns are 16-byte aligned, ld a multiple of 4).
template <int D>
__global__ __launch_bounds__(64) void k_grid_join(const GridJob* jobs, const int32_t* tile_prefix, int n_jobs) {
    __shared__ unsigned cnt[kMaxGrid][64];
    __shared__ double sm[kMaxGrid][64];
    const int jb = job_of_prefix(tile_prefix, n_jobs, blockIdx.x);
    const GridJob& J = jobs[jb];
    const int lane = threadIdx.x;
    const int n = J.n;
    const int g = J.g;
    const int i = (blockIdx.x - tile_prefix[jb]) * kTile + lane;
    const bool valid = i < n;
    const int qi = valid ? i : n - 1;
    for (int j = 0; j < kMaxGrid; ++j) {
        cnt[j][lane] = 0u;
        sm[j][lane] = 0.0;
    }
    float q[D];
#pragma unroll
    for (int f = 0; f < D; ++f) q[f] = J.cols[(int64_t)J.feat[f] * J.ld + qi];
    // The radii (padded with the largest) in vector registers: compares
    // with a scalar-register operand issue at a lower rate.
    float e2[kMaxGrid];
#pragma unroll
    for (int r = 0; r < kMaxGrid; ++r) {
        e2[r] = J.e2[r];
        asm volatile("" : "+v"(e2[r]));
    }
    const float emax2 = J.e2[g - 1];
    typedef float f4 __attribute__((ext_vector_type(4)));
    for (int c0 = 0; c0 < n; c0 += 4) {
        f4 p[D];
#pragma unroll
        for (int f = 0; f < D; ++f) p[f] = *(cptr<f4>)as_const(J.cols + (int64_t)J.feat[f] * J.ld + c0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u;
            float dd = 0.f;
#pragma unroll
            for (int f = 0; f < D; ++f) {
                const float tq = q[f] - p[f][u];
                dd = fmaf(tq, tq, dd);
            }
            if (dd <= emax2 && c < n && c != qi && valid) {
                int j = 0;                                 // the smallest radius that holds it
#pragma unroll
                for (int r = 0; r < kMaxGrid - 1; ++r) j += dd > e2[r] ? 1 : 0;   // padded: never past g - 1
                cnt[j][lane] += 1u;
                sm[j][lane] += (double)__builtin_amdgcn_sqrtf(dd);   // hardware sqrt, <= 1 ulp
            }
        }
    }
    if (!valid) return;
    unsigned c = 0u;
    double s = 0.0;
    for (int j = 0; j < g; ++j) {
        c += cnt[j][lane];
        s += sm[j][lane];
        J.count[(int64_t)j * n + i] = (int32_t)c;
        J.mean[(int64_t)j * n + i] = c > 0u ? (float)(s / (double)c) : 0.f;
    }
}

__device__ __forceinline__ uint32_t grid_key(const GridJob& J, int metric, int j, int64_t i) {
    const int32_t c = J.count[(int64_t)j * J.n + i];
    if (metric == 0) return (uint32_t)c;
    return ~asc_key(c > 0 || J.knn ? J.mean[(int64_t)j * J.n + i] : INFINITY);
}

// Top n of one (job, radius, metric): radix selection of the n-th smallest
// key, then the objects below it and the first ties at it in id order.
__global__ __launch_bounds__(kTopThreads) void k_grid_top(const GridJob* jobs) {
    __shared__ unsigned hist[256];
    __shared__ unsigned s_prefix, s_rem;
    __shared__ int tmp[17];
    __shared__ int s_total;
    const GridJob& J = jobs[blockIdx.x];
    const int j = blockIdx.y >> 1;
    const int metric = blockIdx.y & 1;
    if (j >= J.g) return;
    const int n = J.n;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_prefix = 0u;
        s_rem = (unsigned)J.top_n;
    }
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int x = tid; x < 256; x += blockDim.x) hist[x] = 0u;
        __syncthreads();
        const unsigned pre = s_prefix;
        for (int64_t base = 0; base < n; base += blockDim.x) {     // same trip count in every lane
            const int64_t i = base + tid;
            uint32_t k = 0u;
            bool on = i < n;
            if (on) {
                k = grid_key(J, metric, j, i);
                on = pass == 0 || (k >> (shift + 8)) == pre;
            }
            wave_hist_add(hist, (k >> shift) & 255u, on);
        }
        __syncthreads();
        if (tid == 0) {
            unsigned cum = 0u, rem = s_rem;
            int b = 0;
            for (; b < 256; ++b) {
                if (cum + hist[b] >= rem) break;
                cum += hist[b];
            }
            s_rem = rem - cum;
            s_prefix = (pre << 8) | (unsigned)b;
        }
        __syncthreads();
    }
    const uint32_t T = s_prefix;
    const int take = (int)s_rem;                       // ties at T that belong to the top n
    uint32_t* bits = J.member + ((int64_t)metric * J.g + j) * J.words;
    int ties_before = 0;
    for (int64_t base = 0; base < n; base += blockDim.x) {
        const int64_t i = base + tid;
        uint32_t k = 0xFFFFFFFFu;
        bool in = false, tie = false;
        if (i < n) {
            k = grid_key(J, metric, j, i);
            tie = k == T;
            in = k < T;
        }
        const int rank_tie = block_exclusive_scan(tie ? 1 : 0, tmp, &s_total) + ties_before;
        in = in || (tie && rank_tie < take);
        const unsigned long long bal = __ballot(in);
        if ((tid & 63) == 0 && i < n) {
            const int64_t w = i >> 5;                  // i is a multiple of 64
            bits[w] = (uint32_t)bal;
            if (w + 1 < J.words) bits[w + 1] = (uint32_t)(bal >> 32);
        }
        ties_before += s_total;
        __syncthreads();
    }
}

// Eq. 2 against the smallest and largest radius, and Eq. 3.
__global__ __launch_bounds__(256) void k_grid_select(const GridJob* jobs) {
    __shared__ int red[2][256];
    const GridJob& J = jobs[blockIdx.x];
    const int metric = blockIdx.y;
    const int g = J.g;
    const uint32_t* base = J.member + (int64_t)metric * g * J.words;
    const uint32_t* first = base;
    const uint32_t* last = base + (int64_t)(g - 1) * J.words;
    __shared__ int both_min[kMaxGrid], both_max[kMaxGrid];
    for (int j = 0; j < g; ++j) {
        const uint32_t* cur = base + (int64_t)j * J.words;
        int a = 0, b = 0;
        for (int w = threadIdx.x; w < J.words; w += blockDim.x) {
            a += __popc(first[w] & cur[w]);
            b += __popc(last[w] & cur[w]);
        }
        red[0][threadIdx.x] = a;
        red[1][threadIdx.x] = b;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) {
                red[0][threadIdx.x] += red[0][threadIdx.x + o];
                red[1][threadIdx.x] += red[1][threadIdx.x + o];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            both_min[j] = red[0][0];
            both_max[j] = red[1][0];
            J.similarity[((int64_t)metric * 2 + 0) * g + j] = (float)red[0][0] / (float)J.top_n;
            J.similarity[((int64_t)metric * 2 + 1) * g + j] = (float)red[1][0] / (float)J.top_n;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int best = 0, gap = abs(both_min[0] - both_max[0]);
        for (int j = 1; j < g; ++j) {
            const int d = abs(both_min[j] - both_max[j]);
            if (d < gap) {
                gap = d;
                best = j;
            }
        }
        J.select[metric] = best;
    }
}

using GridJoinFn = void (*)(const GridJob*, const int32_t*, int);

template <int D>
GridJoinFn grid_fn() {
    return k_grid_join<D>;
}

GridJoinFn grid_pick(int d) {
    switch (d) {
        case 2: return grid_fn<2>();
        case 3: return grid_fn<3>();
        case 4: return grid_fn<4>();
        case 5: return grid_fn<5>();
        case 6: return grid_fn<6>();
        case 7: return grid_fn<7>();
        case 8: return grid_fn<8>();
        case 9: return grid_fn<9>();
        case 10: return grid_fn<10>();
        case 11: return grid_fn<11>();
        case 12: return grid_fn<12>();
        case 13: return grid_fn<13>();
        case 14: return grid_fn<14>();
        case 15: return grid_fn<15>();
        case 16: return grid_fn<16>();
    }
    return nullptr;
}

}  // namespace

hipError_t launch_grid_join(const GridJob* jobs, const int32_t* tile_prefix, int n_jobs, int total_tiles, int d,
                            hipStream_t s) {
    GridJoinFn fn = grid_pick(d);
    if (!fn) return hipErrorInvalidValue;
    if (n_jobs <= 0 || total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(fn, dim3(total_tiles), dim3(64), 0, s, jobs, tile_prefix, n_jobs);
    return hipGetLastError();
}

hipError_t launch_grid_select(const GridJob* jobs, int n_jobs, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grid_top, dim3(n_jobs, 2 * kMaxGrid), dim3(kTopThreads), 0, s, jobs);
    hipLaunchKernelGGL(k_grid_select, dim3(n_jobs, 2), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

}  // namespace snaps
