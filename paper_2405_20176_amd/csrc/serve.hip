// Serving: scoring new objects ("alerts") against a resident population in
// one subspace.  The paper has no serving path; the reading used here scores
// an alert as one extra object that changes nothing in the population and
// sees no other alert:
//   - its k nearest population objects (ascending distance, then id) and their
//     mean distance;
//   - its population neighbours within eps (closed ball), count and mean;
//   - its in-degree: the number of population objects p whose own k-th
//     neighbour distance exceeds their distance to the alert (strictly), i.e.
//     the objects that would list the alert among their k nearest;
//   - on each metric, the number of distinct population values strictly more
//     outlying than the alert's value (its dense rank position).
// The state is built once by the ordinary self-join pipeline (k_serve_finish
// adds the index-order k-th distances, their per-tile maxima and per-tile
// Morton keys).  One lane scores one alert; every wavefront walks the
// population tiles outward from the tile where its first alert's Morton key
// falls, skipping tiles whose box is out of reach of every lane's kNN, eps and
// in-degree thresholds.
#include "snaps_internal.h"
#include "common.cuh"
#include "keys.cuh"
#include "join_kernel.cuh"

#include <climits>

namespace snaps {

__global__ __launch_bounds__(64) void k_serve_finish(DevJob J, LargeIndex L, float* rk2, float* tmax, uint32_t* tkey,
                                                      const float* kth) {
    const int t = blockIdx.x;
    const int lane = threadIdx.x;
    const int pos = t * kTile + lane;
    const bool valid = pos < J.n;
    float v = -INFINITY;
    if (valid) v = kth[J.perm[pos]];
    rk2[pos] = v;
    const float mx = wave_max(v);
    if (lane == 0) {
        tmax[t] = mx;
        tkey[t] = morton_key(J, L.sel_col, L.sel_lo, L.sel_scale, J.perm[t * kTile]);
    }
}

hipError_t launch_serve_finish(const DevJob& j, const LargeIndex& li, float* rk2, float* tmax, uint32_t* tkey,
                               const float* kth, hipStream_t s) {
    hipLaunchKernelGGL(k_serve_finish, dim3(j.ntiles), dim3(64), 0, s, j, li, rk2, tmax, tkey, kth);
    return hipGetLastError();
}

template <int D, int KC>
__global__ __launch_bounds__(64) void k_alerts(AlertArgs A) {
    constexpr int DP = row_stride(D);
    constexpr int KS = KC > 0 ? KC : 1;
    constexpr int GS = Group<DP>::G;
    constexpr int NV = Group<DP>::NV;
    const int u = blockIdx.x;
    const int lane = threadIdx.x;
    int lo = 0, hi = A.n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (A.tile_prefix[mid] <= u) lo = mid; else hi = mid;
    }
    const AlertJob& J = A.jobs[lo];
    const ServeState* St = J.st;
    const int n = St->n;
    const int nt = St->ntiles;
    const int k = St->k;
    const float eps2 = St->eps2;
    cptr<float> xs = as_const(St->xs);
    cptr<float> boxes = as_const(St->boxes);
    cptr<float> rk2 = as_const(St->rk2);
    cptr<float> tmax = as_const(St->tmax);
    const int m = J.m;
    const int ai = (u - A.tile_prefix[lo]) * kTile + lane;
    const bool valid = ai < m;
    const int row = valid ? ai : m - 1;
    float q[D];
#pragma unroll
    for (int f = 0; f < D; ++f) q[f] = J.alerts[(int64_t)row * D + f];

    // Morton key of the alert in the population's cell grid -> start tile.
    uint32_t qv[kMaxIndexDims];
    const int c = St->c;
    const int bits = St->bits;
    const uint32_t qmax = (bits >= 32) ? 0xFFFFFFFFu : ((1u << bits) - 1u);
#pragma unroll
    for (int e = 0; e < kMaxIndexDims; ++e) {
        qv[e] = 0;
        if (e < c) {
            const int col = St->sel_col[e];
            float v = 0.f;
#pragma unroll
            for (int f = 0; f < D; ++f) v = (St->feat[f] == col) ? q[f] : v;
            float t = (v - St->sel_lo[e]) * St->sel_scale[e];
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
    int tl = 0, th = nt;                          // first tile whose key exceeds the alert's
    while (tl < th) {
        const int mid = (tl + th) >> 1;
        if (St->tkey[mid] <= key) tl = mid + 1; else th = mid;
    }
    const int tc = __builtin_amdgcn_readfirstlane(tl > 0 ? tl - 1 : 0);

    float kd[KS];
    int kid[KS];
#pragma unroll
    for (int j = 0; j < KS; ++j) {
        const bool dummy = j < KS - k;
        kd[j] = dummy ? -INFINITY : INFINITY;
        kid[j] = dummy ? -1 : INT_MAX;
    }
    int cnt = 0, deg = 0;
    double sum = 0.0;
    float thr = fmaxf(kd[KS - 1], eps2);

    for (int s = 0; s < nt; ++s) {
        const int t = spiral(tc, s, nt);
        cptr<float> bx = boxes + (int64_t)t * 2 * DP;
        float lb = 0.f;
#pragma unroll
        for (int f = 0; f < D; ++f) {
            const float g = fmaxf(fmaxf(bx[f] - q[f], q[f] - bx[DP + f]), 0.f);
            lb = fmaf(g, g, lb);
        }
        const float tm = tmax[t];
        if (!__any(lb <= thr || lb < tm)) continue;
        const int cbase = t * kTile;
#pragma unroll 1
        for (int g = 0; g < kTile; g += GS) {
            const int c0 = cbase + g;
            cptr<f4v> pv = (cptr<f4v>)(xs + (int64_t)c0 * DP);
            f4v blk[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) blk[v] = pv[v];
            float rk[GS];
#pragma unroll
            for (int j = 0; j < GS; ++j) rk[j] = rk2[c0 + j];
#define PV(j, f) blk[((j) * DP + (f)) >> 2][((j) * DP + (f)) & 3]
            float dd[GS];
#pragma unroll
            for (int j = 0; j < GS; ++j) {
                float acc = 0.f;
#pragma unroll
                for (int f = 0; f < D; ++f) {
                    const float tq = q[f] - PV(j, f);
                    acc = fmaf(tq, tq, acc);
                }
                dd[j] = acc;
                deg += (acc < rk[j]) ? 1 : 0;
            }
            float mn = dd[0];
#pragma unroll
            for (int j = 1; j < GS; ++j) mn = fminf(mn, dd[j]);
            if (mn <= thr) {
#pragma unroll
                for (int j = 0; j < GS; ++j) {
                    if (dd[j] <= thr) {
                        if (dd[j] <= eps2) {
                            cnt += 1;
                            sum += (double)__builtin_amdgcn_sqrtf(dd[j]);   // hardware sqrt, <= 1 ulp
                        }
                        if (KC > 0) {
                            const int cid = __float_as_int(PV(j, D + 1));
                            if (before(dd[j], cid, kd[KS - 1], kid[KS - 1])) topk_insert<KS>(kd, kid, dd[j], cid);
                            thr = fmaxf(kd[KS - 1], eps2);
                        }
                    }
                }
            }
#undef PV
        }
    }
    (void)n;
    if (!valid) return;
    const float mean = cnt > 0 ? (float)(sum / (double)cnt) : 0.f;
    float accm = 0.f;
#pragma unroll
    for (int j = 0; j < KS; ++j)
        if (j >= KS - k) accm += sqrtf(kd[j]);
    const float kmean = accm / (float)k;
    J.eps_count[ai] = cnt;
    J.eps_mean[ai] = mean;
    J.indeg[ai] = deg;
    J.knn_mean[ai] = kmean;
    if (J.rank) {
        const uint32_t keys[4] = {(uint32_t)cnt, ~asc_key(cnt > 0 ? mean : INFINITY), (uint32_t)deg,
                                  ~asc_key(kmean)};
#pragma unroll
        for (int mtr = 0; mtr < 4; ++mtr) {
            const uint32_t* dv = St->distinct[mtr];
            int a = 0, b = St->n_distinct[mtr];
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (dv[mid] < keys[mtr]) a = mid + 1; else b = mid;
            }
            J.rank[(int64_t)mtr * m + ai] = a;
        }
    }
}

namespace {

using AlertFn = void (*)(AlertArgs);

template <int D>
AlertFn alert_kc(int kc) {
    switch (kc) {
        case 5: return k_alerts<D, 5>;
        case 10: return k_alerts<D, 10>;
        case 20: return k_alerts<D, 20>;
        case 32: return k_alerts<D, 32>;
    }
    return nullptr;
}

AlertFn alert_pick(int D, int kc) {
    switch (D) {
        case 2: return alert_kc<2>(kc);
        case 3: return alert_kc<3>(kc);
        case 4: return alert_kc<4>(kc);
        case 5: return alert_kc<5>(kc);
        case 6: return alert_kc<6>(kc);
        case 7: return alert_kc<7>(kc);
        case 8: return alert_kc<8>(kc);
        case 9: return alert_kc<9>(kc);
        case 10: return alert_kc<10>(kc);
        case 11: return alert_kc<11>(kc);
        case 12: return alert_kc<12>(kc);
        case 13: return alert_kc<13>(kc);
        case 14: return alert_kc<14>(kc);
        case 15: return alert_kc<15>(kc);
        case 16: return alert_kc<16>(kc);
    }
    return nullptr;
}

}  // namespace

hipError_t launch_alerts(int D, int kc, const AlertArgs& a, int total_tiles, hipStream_t s) {
    AlertFn fn = alert_pick(D, kc);
    if (!fn) return hipErrorInvalidValue;
    if (total_tiles <= 0) return hipSuccess;
    AlertArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(total_tiles), dim3(64), args, 0, s);
}

}  // namespace snaps
