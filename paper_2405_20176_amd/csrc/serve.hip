// Serving: scoring new objects ("alerts") against a resident population in
// one subspace.  The paper has no serving path; the reading used here scores
// an alert as one extra object that changes nothing in the population and
// sees no other alert:
//   - its k nearest population objects and their mean distance;
//   - its population neighbours within eps (closed ball), count and mean;
//   - its in-degree: the number of population objects p whose own k-th
//     neighbour distance exceeds their distance to the alert (strictly), i.e.
//     the objects that would list the alert among their k nearest;
//   - on each metric, the number of distinct population values strictly more
//     outlying than the alert's value (its dense rank position).
// The state is built once by the ordinary self-join pipeline; k_serve_finish
// adds the index-order k-th distances, their per-tile maxima and per-tile
// Morton keys, and k_serve_super the boxes and maxima of super-tiles of 64
// tiles.
//
// One wavefront scores one alert, its lanes spread over the 64 objects of a
// population tile.  The walk starts at the tiles around the alert's Morton
// key (a good first k-th distance), then culls the rest hierarchically: the
// lanes test 64 super-tile boxes at once, then the 64 tile boxes of each
// super-tile that may matter, and only tiles that may hold a kNN candidate,
// an eps neighbour or an object that would count the alert are read.  The
// k best distances are kept sorted across lanes 0..KC-1; eps hits and
// in-degree are wavefront ballots, the eps distance sum a float64 reduction.
#include "serve_internal.h"
#include "common.cuh"
#include "keys.cuh"
#include "join_kernel.cuh"
#include "serve.cuh"
#include "serve_mfma.cuh"

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

// Super-tile S covers tiles [64 S, 64 S + 64): the union of their boxes and
// the maximum of their k-th distances.
__global__ __launch_bounds__(64) void k_serve_super(int ntiles, int dp, const float* boxes, const float* tmax,
                                                     float* sbox, float* smax) {
    const int S = blockIdx.x;
    const int t = S * 64 + (int)threadIdx.x;
    const bool valid = t < ntiles;
    const float tm = wave_max(valid ? tmax[t] : -INFINITY);
    for (int f = 0; f < dp; ++f) {
        const float lo = wave_min(valid ? boxes[((int64_t)t * 2) * dp + f] : INFINITY);
        const float hi = wave_max(valid ? boxes[((int64_t)t * 2 + 1) * dp + f] : -INFINITY);
        if (threadIdx.x == 0) {
            sbox[((int64_t)S * 2) * dp + f] = lo;
            sbox[((int64_t)S * 2 + 1) * dp + f] = hi;
        }
    }
    if (threadIdx.x == 0) smax[S] = tm;
}

hipError_t launch_serve_super(int ntiles, int dp, const float* boxes, const float* tmax, float* sbox, float* smax,
                              hipStream_t s) {
    const int nst = (ntiles + 63) / 64;
    hipLaunchKernelGGL(k_serve_super, dim3(nst), dim3(64), 0, s, ntiles, dp, boxes, tmax, sbox, smax);
    return hipGetLastError();
}


template <int D, int KC>
__global__ __launch_bounds__(64 * kAlertWaves) void k_alerts(AlertArgs A) {
    using namespace alert_detail;
    constexpr int DP = row_stride(D);
    constexpr int KS = KC > 0 ? KC : 1;
    const int lane = threadIdx.x & 63;
    const int g = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kAlertWaves + (threadIdx.x >> 6)));
    if (g >= A.alert_prefix[A.n_jobs]) return;
    int lo = 0, hi = A.n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (A.alert_prefix[mid] <= g) lo = mid; else hi = mid;
    }
    const AlertJob& J = A.jobs[lo];
    const int ai = g - A.alert_prefix[lo];
    const ServeState* St = J.st;
    const int nt = St->ntiles;
    const int nst = St->nsuper;
    const int k = St->k;
    if (St->d != D || k < 1 || k > KS) {         // state of another shape: flag the alert, read nothing
        if (lane == 0) {
            J.eps_count[ai] = -1;
            J.indeg[ai] = -1;
            J.eps_mean[ai] = NAN;
            J.knn_mean[ai] = NAN;
        }
        return;
    }
    const float eps2 = St->eps2;
    const float* xs = St->xs;
    const float* boxes = St->boxes;
    const float* sbox = St->sbox;
    const float* rk2 = St->rk2;
    const float* tmaxp = St->tmax;
    const float* smaxp = St->smax;

    float q[D];
#pragma unroll
    for (int f = 0; f < D; ++f) q[f] = J.alerts[(int64_t)ai * D + f];

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
    const int w0 = max(0, tc - 1), w1 = min(nt, tc + 3);   // start window, read first

    // k best squared distances, ascending over lanes 0..KS-1; the KS - k
    // slots in front hold -inf so that slot KS-1 is always the k-th.
    float kd = (lane < KS - k) ? -INFINITY : INFINITY;
    float kth = INFINITY;
    int cnt = 0, deg = 0;
    double sum = 0.0;

    auto scan_tile = [&](int t) {
        const int pos = t * kTile + lane;
        const float* row = xs + (int64_t)pos * DP;
        float p[DP];
#pragma unroll
        for (int v = 0; v < DP / 4; ++v) {
            const float4 r4 = *reinterpret_cast<const float4*>(row + 4 * v);
            p[4 * v] = r4.x; p[4 * v + 1] = r4.y; p[4 * v + 2] = r4.z; p[4 * v + 3] = r4.w;
        }
        const float rk = rk2[pos];
        float dd = 0.f;
#pragma unroll
        for (int f = 0; f < D; ++f) {
            const float tq = q[f] - p[f];
            dd = fmaf(tq, tq, dd);
        }
        // pad rows hold NaN: every comparison below is false for them
        deg += __popcll(__ballot(dd < rk));
        const bool hit = dd <= eps2;
        const unsigned long long hm = __ballot(hit);
        if (hm) {
            cnt += __popcll(hm);
            sum += wave_sum_f64(hit ? (double)__builtin_amdgcn_sqrtf(dd) : 0.0);
        }
        unsigned long long cm = __ballot(dd < kth);
        while (cm) {
            const int b = __builtin_ctzll(cm);
            cm &= cm - 1;
            const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dd), b));
            if (v < kth) {
                const int at = __popcll(__ballot(lane < KS && kd <= v));
                const float up = __shfl_up(kd, 1, 64);
                kd = (lane == at) ? v : ((lane > at && lane < KS) ? up : kd);
                kth = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kd), KS - 1));
            }
        }
    };
    auto tile_matters = [&](int t) {
        const float lb = box_dist2<D, DP>(q, boxes + (int64_t)t * 2 * DP);
        return lb <= fmaxf(kth, eps2) || lb < tmaxp[t];
    };

    for (int t = w0; t < w1; ++t)
        if (tile_matters(t)) scan_tile(t);

    for (int s0 = 0; s0 < nst; s0 += 64) {
        const int S = s0 + lane;
        bool sm = false;
        if (S < nst) {
            const float lb = box_dist2<D, DP>(q, sbox + (int64_t)S * 2 * DP);
            sm = lb <= fmaxf(kth, eps2) || lb < smaxp[S];
        }
        unsigned long long smask = __ballot(sm);
        while (smask) {
            const int Sb = s0 + __builtin_ctzll(smask);
            smask &= smask - 1;
            const int t = Sb * 64 + lane;
            float lb = INFINITY, tm = -INFINITY;
            bool tmat = false;
            if (t < nt && (t < w0 || t >= w1)) {         // the start window is done
                lb = box_dist2<D, DP>(q, boxes + (int64_t)t * 2 * DP);
                tm = tmaxp[t];
                tmat = lb <= fmaxf(kth, eps2) || lb < tm;
            }
            unsigned long long tmask = __ballot(tmat);
            while (tmask) {
                const int b = __builtin_ctzll(tmask);
                tmask &= tmask - 1;
                // re-test with the k-th distance found so far
                const float lbt = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lb), b));
                const float tmt = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tm), b));
                if (lbt <= fmaxf(kth, eps2) || lbt < tmt) scan_tile(Sb * 64 + b);
            }
        }
    }

    // kNN mean over the k real slots (ascending order, fixed reduction tree)
    const float kv = (lane >= KS - k && lane < KS) ? __builtin_amdgcn_sqrtf(kd) : 0.f;
    const float ksum = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum(kv)), 0));
    const float kmean = ksum / (float)k;
    // the butterfly leaves each lane its own rounding of the sum: take lane 0's
    const long long sb = __double_as_longlong(sum);
    const unsigned s_lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(sb & 0xffffffffLL), 0);
    const unsigned s_hi = (unsigned)__builtin_amdgcn_readlane((int)(sb >> 32), 0);
    const double sum0 = __longlong_as_double((long long)(((unsigned long long)s_hi << 32) | s_lo));
    const float mean = cnt > 0 ? (float)(sum0 / (double)cnt) : 0.f;
    if (lane == 0) {
        J.eps_count[ai] = cnt;
        J.eps_mean[ai] = mean;
        J.indeg[ai] = deg;
        J.knn_mean[ai] = kmean;
    }
    if (J.rank && lane < 4) {
        const int mtr = lane;
        const uint32_t key_m = mtr == 0 ? (uint32_t)cnt
                             : mtr == 1 ? ~asc_key(cnt > 0 ? mean : INFINITY)
                             : mtr == 2 ? (uint32_t)deg
                                        : ~asc_key(kmean);
        J.rank[(int64_t)mtr * J.m + ai] = distinct_below(St->distinct[mtr], St->n_distinct[mtr], key_m);
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

hipError_t launch_alerts(int D, int kc, const AlertArgs& a, hipStream_t s) {
    AlertFn fn = alert_pick(D, kc);
    if (!fn) return hipErrorInvalidValue;
    const int total = a.alert_prefix[a.n_jobs];
    if (total <= 0) return hipSuccess;
    AlertArgs copy = a;
    void* args[] = {&copy};
    const int grid = (total + kAlertWaves - 1) / kAlertWaves;
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(grid), dim3(64 * kAlertWaves), args, 0, s);
}

// Merges the slices' partial results of one group of 64 alerts (one lane
// per alert) and writes the scores and rank positions exactly as k_alerts
// does: the k nearest distances are the k smallest of the slices' lists, and
// the kNN mean is lane 0's result of k_alerts' wavefront sum (each lane i of
// the first 32 holding slot i, the others 0), step by step.  Wavefront w of
// the kMergeWaves takes the slices w, w + kMergeWaves, ... in order, the
// next slice's values loaded while the current one is merged; wavefront 0
// then adds the others' results in wavefront order, so the float64 eps sum
// is taken in a fixed order for a given slice count.
constexpr int kMergeWaves = 4;

template <int KC>
__global__ __launch_bounds__(64 * kMergeWaves) void k_alerts_merge(AlertArgs A) {
    using namespace alert_detail;
    constexpr int KS = KC;
    constexpr int NV = KS + 4;                   // values of one partial result per lane
    static_assert(KS <= 32, "the kNN mean's reduction order assumes at most 32 slots");
    __shared__ float s_part[kMergeWaves - 1][NV][kTile];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int g = blockIdx.x;
    if (g >= A.merge_prefix[A.n_jobs]) return;
    int lo = 0, hi = A.n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (A.merge_prefix[mid] <= g) lo = mid; else hi = mid;
    }
    const AlertJob& J = A.jobs[lo];
    const int gi = g - A.merge_prefix[lo];
    const int ai = gi * kTile + lane;
    const bool live = ai < J.m;
    const ServeState* St = J.st;
    const int k = St->k;
    if (St->d != A.d || k < 1 || k > KS) {       // state of another shape: flag the alert
        if (wv == 0 && live) {
            J.eps_count[ai] = -1;
            J.indeg[ai] = -1;
            J.eps_mean[ai] = NAN;
            J.knn_mean[ai] = NAN;
        }
        return;
    }
    const int nsl = A.slices[lo];
    const float* part = A.part + A.part_off[lo] + (int64_t)gi * nsl * alert_part_floats(KS);
    float kd[KS];
#pragma unroll
    for (int j = 0; j < KS; ++j) kd[j] = j < KS - k ? -INFINITY : INFINITY;
    int cnt = 0, deg = 0;
    double sum = 0.0;
    auto fetch = [&](int sl, float (&v)[NV]) {
        const float* ps = part + (int64_t)sl * alert_part_floats(KS) + lane;
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = ps[j * kTile];
    };
    auto merge = [&](const float (&v)[NV]) {
#pragma unroll
        for (int j = 0; j < KS; ++j)
            if (j >= KS - k && v[j] < kd[KS - 1]) alert_mfma_detail::dist_insert<KS>(kd, v[j]);
        cnt += __float_as_int(v[KS]);
        deg += __float_as_int(v[KS + 1]);
        const unsigned long long lo32 = (unsigned)__float_as_int(v[KS + 2]);
        const unsigned long long hi32 = (unsigned)__float_as_int(v[KS + 3]);
        sum += __longlong_as_double((long long)((hi32 << 32) | lo32));
    };
    if (wv < nsl) {
        float cur[NV], nxt[NV];
        fetch(wv, cur);
        for (int sl = wv; sl < nsl; sl += kMergeWaves) {
            const bool more = sl + kMergeWaves < nsl;
            if (more) fetch(sl + kMergeWaves, nxt);
            merge(cur);
            if (more) {
#pragma unroll
                for (int j = 0; j < NV; ++j) cur[j] = nxt[j];
            }
        }
    }
    if (wv > 0) {
        const long long sb = __double_as_longlong(sum);
#pragma unroll
        for (int j = 0; j < KS; ++j) s_part[wv - 1][j][lane] = kd[j];
        s_part[wv - 1][KS][lane] = __int_as_float(cnt);
        s_part[wv - 1][KS + 1][lane] = __int_as_float(deg);
        s_part[wv - 1][KS + 2][lane] = __int_as_float((int)(unsigned)(sb & 0xffffffffLL));
        s_part[wv - 1][KS + 3][lane] = __int_as_float((int)(sb >> 32));
    }
    __syncthreads();
    if (wv != 0 || !live) return;
    for (int w = 1; w < kMergeWaves; ++w) {
        float v[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = s_part[w - 1][j][lane];
        merge(v);
    }
    float v[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = (i >= KS - k && i < KS) ? __builtin_amdgcn_sqrtf(kd[i]) : 0.f;
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
#pragma unroll
        for (int i = 0; i < o; ++i) v[i] += v[i + o];
    }
    const float kmean = v[0] / (float)k;
    const float mean = cnt > 0 ? (float)(sum / (double)cnt) : 0.f;
    J.eps_count[ai] = cnt;
    J.eps_mean[ai] = mean;
    J.indeg[ai] = deg;
    J.knn_mean[ai] = kmean;
    if (J.rank) {
        J.rank[ai] = distinct_below(St->distinct[0], St->n_distinct[0], (uint32_t)cnt);
        J.rank[(int64_t)J.m + ai] =
            distinct_below(St->distinct[1], St->n_distinct[1], ~asc_key(cnt > 0 ? mean : INFINITY));
        J.rank[(int64_t)2 * J.m + ai] = distinct_below(St->distinct[2], St->n_distinct[2], (uint32_t)deg);
        J.rank[(int64_t)3 * J.m + ai] = distinct_below(St->distinct[3], St->n_distinct[3], ~asc_key(kmean));
    }
}

hipError_t launch_alerts_mfma(int D, int kc, const AlertArgs& a, hipStream_t s) {
    AlertKernel fn = D <= 8 ? alert_mfma_pick_group0(D, kc) : alert_mfma_pick_group1(D, kc);
    AlertKernel mfn = kc == 5 ? k_alerts_merge<5> : kc == 10 ? k_alerts_merge<10> : kc == 20 ? k_alerts_merge<20>
                    : kc == 32 ? k_alerts_merge<32> : nullptr;
    if (!fn || !mfn) return hipErrorInvalidValue;
    const int blocks = a.group_prefix[a.n_jobs];
    if (blocks <= 0) return hipSuccess;
    AlertArgs copy = a;
    void* args[] = {&copy};
    hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(blocks), dim3(64 * alert_mfma_waves(D)),
                                   args, 0, s);
    if (e != hipSuccess) return e;
    return hipLaunchKernel(reinterpret_cast<const void*>(mfn), dim3(a.merge_prefix[a.n_jobs]), dim3(64 * kMergeWaves), args,
                           0, s);
}

}  // namespace snaps
