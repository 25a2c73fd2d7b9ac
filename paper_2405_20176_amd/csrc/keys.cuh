// Device helpers shared by the LDS-resident and device-wide index and rank
// passes: the choice of indexed dimensions, the Morton cell key, and the
// order-preserving keys of the four metrics.
#pragma once

#include "snaps_internal.h"

namespace snaps {

// The c dimensions of the subspace with the largest spread (lower index on
// ties), each cut into 2^bits cells over mean +/- 3 sigma (values outside
// fall into the edge cells).
__device__ inline void choose_index_dims(const DevJob& J, const float* mean, const float* sd, int* col, float* lo,
                                         float* scale) {
    unsigned used = 0;
    for (int e = 0; e < J.c; ++e) {
        int best = -1;
        for (int f = 0; f < J.d; ++f) {
            if ((used >> f) & 1u) continue;
            if (best < 0 || sd[f] > sd[best]) best = f;
        }
        used |= 1u << best;
        const float sg = sd[best];
        const float l = sg > 0.f ? mean[best] - 3.f * sg : mean[best] - 0.5f;
        const float h = sg > 0.f ? mean[best] + 3.f * sg : mean[best] + 0.5f;
        col[e] = J.feat[best];
        lo[e] = l;
        scale[e] = (float)(1ull << J.bits) / (h - l);
    }
}

// Morton (Z-order) interleaving of object i's cell coordinates, most
// significant bits first.
__device__ inline uint32_t morton_key(const DevJob& J, const int* col, const float* lo, const float* scale,
                                      int64_t i) {
    const int c = J.c;
    const int bits = J.bits;
    const uint32_t qmax = (bits >= 32) ? 0xFFFFFFFFu : ((1u << bits) - 1u);
    uint32_t qv[kMaxIndexDims];
#pragma unroll
    for (int e = 0; e < kMaxIndexDims; ++e) {
        qv[e] = 0;
        if (e < c) {
            const float v = J.cols[(int64_t)col[e] * J.ld + i];
            float t = (v - lo[e]) * scale[e];
            t = fminf(fmaxf(t, 0.f), (float)qmax);
            qv[e] = (uint32_t)t;
        }
    }
    uint32_t key = 0;
    for (int b = bits - 1; b >= 0; --b) {
#pragma unroll
        for (int e = 0; e < kMaxIndexDims; ++e)
            if (e < c) key = (key << 1) | ((qv[e] >> b) & 1u);
    }
    return key;
}

// Monotone map of a float to an unsigned key (ascending float order).
__device__ __forceinline__ uint32_t asc_key(float x) {
    const uint32_t b = __float_as_uint(x);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Key of object i on metric m, ascending = more outlying (paper Sec. 3.5.1,
// 3.6.1, Tab. 2): eps_count and indeg ascending; eps_mean descending with
// objects that have no eps neighbour first; knn_mean descending.
__device__ __forceinline__ uint32_t metric_key(const DevJob& J, int metric, int64_t i) {
    switch (metric) {
        case 0: return (uint32_t)J.eps_count[i];
        case 1: return ~asc_key(J.eps_count[i] > 0 ? J.eps_mean[i] : INFINITY);
        case 2: return (uint32_t)J.indeg[i];
        default: return ~asc_key(J.knn_mean[i]);
    }
}

}  // namespace snaps
