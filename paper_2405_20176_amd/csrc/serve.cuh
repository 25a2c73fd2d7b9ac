// Helpers shared by the two alert scoring kernels.
#pragma once

#include "common.cuh"

namespace snaps {

namespace alert_detail {

// Squared float32 distance from q to the box [lo, hi] (0 inside), computed
// with the same operations in the same order as a point distance, so it
// never exceeds the float32 distance of any point in the box.
template <int D, int DP>
__device__ __forceinline__ float box_dist2(const float (&q)[D], const float* b) {
    float lb = 0.f;
#pragma unroll
    for (int f = 0; f < D; ++f) {
        const float g = fmaxf(fmaxf(b[f] - q[f], q[f] - b[DP + f]), 0.f);
        lb = fmaf(g, g, lb);
    }
    return lb;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Number of keys of the ascending distinct list dv[0..nd) strictly below
// key: an alert's dense rank position on one metric.
__device__ __forceinline__ int distinct_below(const uint32_t* dv, int nd, uint32_t key) {
    int a = 0, b = nd;
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (dv[mid] < key) a = mid + 1; else b = mid;
    }
    return a;
}

}  // namespace alert_detail

}  // namespace snaps
