// Selection of k between under- and overfitting (paper Sec. 3.6.2): for a
// grid k_1 < ... < k_g (the paper: from k_min = 2 to k_max = 4096), the
// in-degree and the mean kNN distance of every object at every k, from the
// k_max nearest neighbours, which hold those of every smaller k.
//   k_kgrid_thresh: one workgroup per query.  Its distances to every object
//     go to LDS; a radix selection finds the k_max-th smallest (distance, id)
//     -- ties in id order -- and the k_max nearest are compacted and sorted
//     by (distance, id), which gives, for every k_j, the key of the k_j-th
//     neighbour and the sum of the k_j smallest distances.
//   k_kgrid_indeg: one lane per object p scans every query q: p is among the
//     k_j nearest of q exactly when (distance, id of p) is at most q's k_j-th
//     (distance, id), so p's in-degree at every k needs no global atomics.
// The rankings, Eq. 2 similarities and the Eq. 3 choice are those of the
// radius grid (eps_grid.hip) with in-degree for the neighbour count and the
// mean kNN distance for the mean.
#include "snaps_internal.h"
#include "common.cuh"

namespace snaps {

namespace {

constexpr int kThreshThreads = 512;

__device__ __forceinline__ int kjob_of(const int32_t* prefix, int n_jobs, int b) {
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Radix selection over the keys v[0, m) in LDS of the r-th smallest
// (1-based, r <= m) by the whole workgroup, in digits of 12, 10 and 10 bits
// (the top digit spans the exponent, where distances crowd).  Returns its
// value; *rem is its rank among the keys equal to it.  hist holds 4096 bins.
__device__ uint32_t lds_select(const uint32_t* v, int m, unsigned r, unsigned* hist, int* tmp, unsigned* s_sel,
                               unsigned* rem) {
    const int tid = threadIdx.x;
    unsigned pre = 0u;
    for (int pass = 0; pass < 3; ++pass) {
        const int bits = pass == 0 ? 12 : 10;
        const int shift = pass == 0 ? 20 : (pass == 1 ? 10 : 0);
        const int nb = 1 << bits;
        for (int x = tid; x < nb; x += blockDim.x) hist[x] = 0u;
        __syncthreads();
        for (int e = tid; e < m; e += blockDim.x) {
            const uint32_t x = v[e];
            if (pass == 0 || (x >> (shift + bits)) == pre) atomicAdd(&hist[(x >> shift) & (unsigned)(nb - 1)], 1u);
        }
        __syncthreads();
        // Bins per thread; the one thread whose bins reach rank r picks the bin.
        const int per = nb / (int)blockDim.x;
        unsigned local = 0u;
        for (int b = 0; b < per; ++b) local += hist[tid * per + b];
        int total;
        const unsigned before = (unsigned)block_exclusive_scan((int)local, tmp, &total);
        if (before < r && before + local >= r) {
            unsigned cum = before;
            int b = tid * per;
            while (cum + hist[b] < r) cum += hist[b++];
            s_sel[0] = (pre << bits) | (unsigned)b;
            s_sel[1] = r - cum;
        }
        __syncthreads();
        pre = s_sel[0];
        r = s_sel[1];
        __syncthreads();
    }
    *rem = r;
    return pre;
}

template <int D>
__global__ __launch_bounds__(kThreshThreads) void k_kgrid_thresh(const KGridJob* jobs, const int32_t* prefix,
                                                                  int n_jobs) {
    // dist: distance bits by object id; then the k_max nearest in id order
    // ([0, k_max)), and their 64-bit (distance, id) keys, sorted, from
    // uint32 offset kMaxKGridK.
    __shared__ __align__(16) uint32_t dist[kMaxKGridN];
    __shared__ uint16_t lid[kMaxKGridK];
    __shared__ unsigned hist[4096];
    __shared__ double s_part[kThreshThreads / 64][kMaxGrid];
    __shared__ int tmp[17];
    __shared__ unsigned s_sel[2];
    const int jb = kjob_of(prefix, n_jobs, blockIdx.x);
    const KGridJob& J = jobs[jb];
    const int qid = blockIdx.x - prefix[jb];
    const int n = J.n;
    const int g = J.g;
    const int tid = threadIdx.x;
    float q[D];
#pragma unroll
    for (int f = 0; f < D; ++f) q[f] = J.cols[(int64_t)J.feat[f] * J.ld + qid];
    for (int i = tid; i < n; i += blockDim.x) {
        float dd = 0.f;
#pragma unroll
        for (int f = 0; f < D; ++f) {
            const float tq = q[f] - J.cols[(int64_t)J.feat[f] * J.ld + i];     // query minus object
            dd = fmaf(tq, tq, dd);
        }
        dist[i] = i == qid ? 0x7F800000u : __float_as_uint(dd);              // self: +inf, never chosen
    }
    __syncthreads();

    // The k_max nearest: every distance below the k_max-th value, then the
    // first ties at it in id order; compacted in place in id order.
    const int kmax = J.k[g - 1];
    unsigned take;
    const uint32_t vmax = lds_select(dist, n, (unsigned)kmax, hist, tmp, s_sel, &take);
    int placed = 0, ties = 0;
    for (int base = 0; base < n; base += blockDim.x) {
        const int i = base + tid;
        const uint32_t v = i < n ? dist[i] : 0xFFFFFFFFu;
        const bool tie = i < n && v == vmax;
        int nt, np;
        const int tie_rank = block_exclusive_scan(tie ? 1 : 0, tmp, &nt) + ties;
        const bool in = i < n && (v < vmax || (tie && tie_rank < (int)take));
        const int pos = block_exclusive_scan(in ? 1 : 0, tmp, &np) + placed;
        if (in) {                                   // pos <= i, and every read of this round is done
            dist[pos] = v;
            lid[pos] = (uint16_t)i;
        }
        ties += nt;
        placed += np;
        __syncthreads();
    }

    // Sort the list by (distance, id): the k_j-th key and the k_j smallest
    // distances of every grid point follow.
    uint64_t* key = reinterpret_cast<uint64_t*>(dist + kMaxKGridK);
    const int P = next_pow2(kmax);
    for (int e = tid; e < P; e += blockDim.x)
        key[e] = e < kmax ? (((uint64_t)dist[e] << 32) | (uint64_t)lid[e]) : ~0ull;
    __syncthreads();
    bitonic_sort_lds(key, P);
    double part[kMaxGrid];
#pragma unroll
    for (int t = 0; t < kMaxGrid; ++t) part[t] = 0.0;
    for (int e = tid; e < kmax; e += blockDim.x) {
        const double dv = (double)sqrtf(__uint_as_float((uint32_t)(key[e] >> 32)));
#pragma unroll
        for (int t = 0; t < kMaxGrid; ++t)
            if (t < g && e < J.k[t]) part[t] += dv;
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int t = 0; t < kMaxGrid; ++t) {
        double v = part[t];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) s_part[wave][t] = v;
    }
    __syncthreads();
    if (tid < g) {
        double sum = 0.0;
        for (int w = 0; w < kThreshThreads / 64; ++w) sum += s_part[w][tid];
        const int kt = J.k[tid];
        J.kmean[(int64_t)tid * n + qid] = (float)(sum / (double)kt);
        J.thr[(int64_t)qid * kMaxGrid + tid] = key[kt - 1];
    }
}

// One 64-object tile per workgroup (one wavefront), lane = object p: every
// query q in groups of four (one 16-byte scalar load per feature column);
// p is among the k_j nearest of q when its (distance, id) key is at most q's
// j-th threshold.  Lanes count each q at the smallest such j; prefix sums
// over j give the in-degrees.
template <int D>
__global__ __launch_bounds__(64) void k_kgrid_indeg(const KGridJob* jobs, const int32_t* tile_prefix, int n_jobs) {
    __shared__ unsigned cnt[kMaxGrid][64];
    const int jb = kjob_of(tile_prefix, n_jobs, blockIdx.x);
    const KGridJob& J = jobs[jb];
    const int lane = threadIdx.x;
    const int n = J.n;
    const int g = J.g;
    const int p = (blockIdx.x - tile_prefix[jb]) * kTile + lane;
    const bool valid = p < n;
    const int pr = valid ? p : n - 1;
    for (int j = 0; j < kMaxGrid; ++j) cnt[j][lane] = 0u;
    float pc[D];
#pragma unroll
    for (int f = 0; f < D; ++f) pc[f] = J.cols[(int64_t)J.feat[f] * J.ld + pr];
    cptr<uint64_t> thr = as_const(J.thr);
    typedef float f4 __attribute__((ext_vector_type(4)));
    for (int c0 = 0; c0 < n; c0 += 4) {
        f4 qc[D];
#pragma unroll
        for (int f = 0; f < D; ++f) qc[f] = *(cptr<f4>)as_const(J.cols + (int64_t)J.feat[f] * J.ld + c0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u;
            if (c >= n) break;
            float dd = 0.f;
#pragma unroll
            for (int f = 0; f < D; ++f) {
                const float tq = qc[f][u] - pc[f];                              // query minus object
                dd = fmaf(tq, tq, dd);
            }
            const uint64_t key = ((uint64_t)__float_as_uint(dd) << 32) | (uint64_t)(uint32_t)p;
            cptr<uint64_t> tc = thr + (int64_t)c * kMaxGrid;
            const bool near = valid && p != c && key <= tc[g - 1];
            if (!__any(near)) continue;
            if (near) {
                int j0 = 0;                                                     // thresholds below the key
                for (int t = 0; t < g - 1; ++t) j0 += key > tc[t] ? 1 : 0;
                cnt[j0][lane] += 1u;
            }
        }
    }
    if (!valid) return;
    unsigned c = 0u;
    for (int j = 0; j < g; ++j) {
        c += cnt[j][lane];
        J.indeg[(int64_t)j * n + p] = (int32_t)c;
    }
}

using KThreshFn = void (*)(const KGridJob*, const int32_t*, int);

template <int D>
void kgrid_fns(KThreshFn* a, KThreshFn* b) {
    *a = k_kgrid_thresh<D>;
    *b = k_kgrid_indeg<D>;
}

bool kgrid_pick(int d, KThreshFn* a, KThreshFn* b) {
    switch (d) {
        case 2: kgrid_fns<2>(a, b); return true;
        case 3: kgrid_fns<3>(a, b); return true;
        case 4: kgrid_fns<4>(a, b); return true;
        case 5: kgrid_fns<5>(a, b); return true;
        case 6: kgrid_fns<6>(a, b); return true;
        case 7: kgrid_fns<7>(a, b); return true;
        case 8: kgrid_fns<8>(a, b); return true;
        case 9: kgrid_fns<9>(a, b); return true;
        case 10: kgrid_fns<10>(a, b); return true;
        case 11: kgrid_fns<11>(a, b); return true;
        case 12: kgrid_fns<12>(a, b); return true;
        case 13: kgrid_fns<13>(a, b); return true;
        case 14: kgrid_fns<14>(a, b); return true;
        case 15: kgrid_fns<15>(a, b); return true;
        case 16: kgrid_fns<16>(a, b); return true;
    }
    return false;
}

}  // namespace

hipError_t launch_kgrid(const KGridJob* jobs, const int32_t* query_prefix, const int32_t* tile_prefix, int n_jobs,
                        int total_queries, int total_tiles, int d, hipStream_t s) {
    KThreshFn thresh, indeg;
    if (!kgrid_pick(d, &thresh, &indeg)) return hipErrorInvalidValue;
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(thresh, dim3(total_queries), dim3(kThreshThreads), 0, s, jobs, query_prefix, n_jobs);
    hipLaunchKernelGGL(indeg, dim3(total_tiles), dim3(64), 0, s, jobs, tile_prefix, n_jobs);
    return hipGetLastError();
}

}  // namespace snaps
