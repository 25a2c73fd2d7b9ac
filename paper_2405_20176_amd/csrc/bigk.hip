// k-nearest-neighbour metrics for k above the fused join's register lists
// (paper Sec. 3.6: the in-degree of the kNN graph and the mean distance to
// the k nearest neighbours, Sec. 3.6.1; the kNN lists of Fig. 1b).
//
// One workgroup per query.  The k nearest other objects in ascending
// (distance, id) order are exactly the objects whose key (float32 squared
// distance, id) is at most the k-th smallest key, so the query first finds
// that key by radix selection: three passes over the candidates build
// histograms of the squared distance's bits (11, 11 and 10 bits, the
// candidates that still share the chosen prefix), and only if objects at
// exactly the k-th distance straddle the boundary, three more passes over
// their ids (10 bits each).  Distances are recomputed in every pass from the
// population's feature columns (direct form, the same operations as the
// fused join), so nothing is stored per pair.  A last pass takes the
// members: it adds one in-degree per neighbour (integer atomics), sums the
// neighbours' distances in float64 (per thread in candidate order, then a
// fixed reduction tree: deterministic), and, when lists are asked for,
// appends (distance, id) keys to an LDS list that is then sorted.
#include "snaps_internal.h"
#include "common.cuh"

namespace snaps {

namespace {

constexpr int kBigKThreads = 256;

__device__ __forceinline__ int64_t job_of_qprefix(const int64_t* prefix, int n, int64_t b) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// The bin of hist[0, nb) that holds the need-th (1-based) counted value:
// out[0] = bin, out[1] = values in lower bins, out[2] = values in the bin.
__device__ __forceinline__ void find_bin(const uint32_t* hist, int nb, uint32_t need, int* tmp, uint32_t* out) {
    const int per = nb / kBigKThreads;
    const int b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int j = 0; j < per; ++j) s += hist[b0 + j];
    int total;
    const uint32_t base = (uint32_t)block_exclusive_scan((int)s, tmp, &total);
    if (base < need && need <= base + s) {
        uint32_t c = base;
        for (int j = 0; j < per; ++j) {
            const uint32_t h = hist[b0 + j];
            if (need <= c + h) {
                out[0] = (uint32_t)(b0 + j);
                out[1] = c;
                out[2] = h;
                break;
            }
            c += h;
        }
    }
    __syncthreads();
}

template <int D, bool LISTS>
__global__ __launch_bounds__(kBigKThreads) void k_bigk(BigKArgs A) {
    __shared__ uint32_t hist[2048];
    __shared__ int tmp[17];
    __shared__ uint32_t s_bin[3];
    __shared__ double s_red[kBigKThreads / 64];
    __shared__ uint32_t s_count;
    __shared__ uint64_t list[LISTS ? kMaxListK : 1];

    const int64_t b = blockIdx.x;
    int jn = 0;
    BigKJob J;
    if (A.use_single) {
        J = A.single;
    } else {
        jn = (int)job_of_qprefix(A.prefix, A.n_jobs, b);
        J = A.table[jn];
    }
    const int64_t qid = A.use_single ? b : b - A.prefix[jn];
    const int n = J.n;
    const int k = J.k;
    const int tid = threadIdx.x;

    const float* col[D];
    float q[D];
#pragma unroll
    for (int f = 0; f < D; ++f) {
        col[f] = J.cols + (int64_t)J.feat[f] * J.ld;
        q[f] = col[f][qid];
    }
    auto dist2 = [&](int64_t i) {
        float dd = 0.f;
#pragma unroll
        for (int f = 0; f < D; ++f) {
            const float t = q[f] - col[f][i];
            dd = fmaf(t, t, dd);
        }
        return dd;
    };

    // The k-th smallest squared distance (its bits, most significant digit
    // first) and the rank `need` of the k-th neighbour among the objects at
    // exactly that distance.
    uint32_t pre = 0, need = (uint32_t)k, eq = 0;
#pragma unroll 1
    for (int p = 0; p < 3; ++p) {
        const int shift = p == 0 ? 21 : (p == 1 ? 10 : 0);
        const int nb = p == 2 ? 1024 : 2048;
        const uint32_t himask = p == 0 ? 0u : (0xFFFFFFFFu << (p == 1 ? 21 : 10));
        for (int i = tid; i < nb; i += kBigKThreads) hist[i] = 0u;
        __syncthreads();
        for (int64_t i = tid; i < n; i += kBigKThreads) {
            if (i == qid) continue;
            const uint32_t key = __float_as_uint(dist2(i));
            if ((key & himask) == pre) atomicAdd(&hist[(key >> shift) & (uint32_t)(nb - 1)], 1u);
        }
        __syncthreads();
        find_bin(hist, nb, need, tmp, s_bin);
        pre |= s_bin[0] << shift;
        need -= s_bin[1];
        eq = s_bin[2];
        __syncthreads();
    }
    // Ties at the k-th distance: the need-th smallest id among them.
    uint32_t idb = 0xFFFFFFFFu;
    if (need < eq) {
        uint32_t ipre = 0;
#pragma unroll 1
        for (int p = 0; p < 3; ++p) {
            const int shift = 20 - 10 * p;
            const uint32_t himask = p == 0 ? 0u : (0xFFFFFFFFu << (shift + 10));
            for (int i = tid; i < 1024; i += kBigKThreads) hist[i] = 0u;
            __syncthreads();
            for (int64_t i = tid; i < n; i += kBigKThreads) {
                if (i == qid) continue;
                if (__float_as_uint(dist2(i)) != pre) continue;
                const uint32_t u = (uint32_t)i;
                if ((u & himask) == ipre) atomicAdd(&hist[(u >> shift) & 1023u], 1u);
            }
            __syncthreads();
            find_bin(hist, 1024, need, tmp, s_bin);
            ipre |= s_bin[0] << shift;
            need -= s_bin[1];
            __syncthreads();
        }
        idb = ipre;
    }

    // Members: key below the bound.
    if (LISTS && tid == 0) s_count = 0u;
    __syncthreads();
    double sum = 0.0;
    int32_t* indeg = J.indeg;
    for (int64_t i = tid; i < n; i += kBigKThreads) {
        if (i == qid) continue;
        const float dd = dist2(i);
        const uint32_t key = __float_as_uint(dd);
        if (key < pre || (key == pre && (uint32_t)i <= idb)) {
            sum += (double)sqrtf(dd);
            if (indeg) atomicAdd(indeg + i, 1);
            if constexpr (LISTS) {
                const uint32_t at = atomicAdd(&s_count, 1u);
                list[at] = ((uint64_t)key << 32) | (uint32_t)i;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if ((tid & 63) == 0) s_red[tid >> 6] = sum;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int w = 0; w < kBigKThreads / 64; ++w) tot += s_red[w];
        if (J.knn_mean) J.knn_mean[qid] = (float)(tot / (double)k);
    }
    if constexpr (LISTS) {
        if (J.ids) {
            const int P = next_pow2(k);
            for (int i = k + tid; i < P; i += kBigKThreads) list[i] = ~0ull;
            __syncthreads();
            bitonic_sort_lds(list, P);
            for (int j = tid; j < k; j += kBigKThreads) {
                const uint64_t v = list[j];
                J.ids[qid * k + j] = (int32_t)(uint32_t)v;
                if (J.dist) J.dist[qid * k + j] = sqrtf(__uint_as_float((uint32_t)(v >> 32)));
            }
        }
    }
}

template <int D>
void* bigk_pick_lists(bool lists) {
    return lists ? reinterpret_cast<void*>(k_bigk<D, true>) : reinterpret_cast<void*>(k_bigk<D, false>);
}

void* bigk_pick(int D, bool lists) {
    switch (D) {
        case 2: return bigk_pick_lists<2>(lists);
        case 3: return bigk_pick_lists<3>(lists);
        case 4: return bigk_pick_lists<4>(lists);
        case 5: return bigk_pick_lists<5>(lists);
        case 6: return bigk_pick_lists<6>(lists);
        case 7: return bigk_pick_lists<7>(lists);
        case 8: return bigk_pick_lists<8>(lists);
        case 9: return bigk_pick_lists<9>(lists);
        case 10: return bigk_pick_lists<10>(lists);
        case 11: return bigk_pick_lists<11>(lists);
        case 12: return bigk_pick_lists<12>(lists);
        case 13: return bigk_pick_lists<13>(lists);
        case 14: return bigk_pick_lists<14>(lists);
        case 15: return bigk_pick_lists<15>(lists);
        case 16: return bigk_pick_lists<16>(lists);
    }
    return nullptr;
}

}  // namespace

hipError_t launch_bigk(int D, bool lists, const BigKArgs& a, int64_t queries, hipStream_t s) {
    if (queries <= 0) return hipSuccess;
    if (queries > INT32_MAX) return hipErrorInvalidValue;
    void* fn = bigk_pick(D, lists);
    if (!fn) return hipErrorInvalidValue;
    BigKArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(fn, dim3((unsigned)queries), dim3(kBigKThreads), args, 0, s);
}

}  // namespace snaps
