// Alert scoring on the matrix cores: the scores of k_alerts (serve.hip) as a
// cross-join of groups of 64 alerts against the population's tiles.
//
// A workgroup takes one group of 64 alerts of one job, one alert per lane in
// each of its W = alert_mfma_waves(d) wavefronts, and one slice (a run of
// consecutive tiles) of the population, which it splits among its
// wavefronts: wavefront w takes the slice's tiles w, w + W, w + 2 W, ...
// It tests the next 64 of its tiles at once, one per lane, with the group's
// box (the corners of its alerts) against each tile's box, and skips a tile
// that no alert of the group can reach: neither for its k nearest or its eps
// ball (box distance above the group's largest threshold) nor as an object
// that would count the alert (box distance at or above the tile's largest
// k-th neighbour distance).  Per dimension the boxes' gap is at most each
// pair's own difference (the same subtractions with the alert replaced by
// its box's near corner, and float rounding is monotone), so a skipped tile
// holds no pair that matters.  The wavefronts of a workgroup share, through
// LDS, the smallest k-th distance any of them has found for each alert, and
// the workgroups of a group through a slot per alert in global memory; each
// screens with the smallest it has seen (the final k-th distance is at most
// that).  A kept tile's rows and k-th distances are
// copied into LDS, and its 64 x 64 pairs are screened by the half-precision
// contraction of the matrix-core join (join_mfma.cuh), rows being alerts.
// A pair passes if it can matter to either side:
//   alert side:   q . p - L_q >= -h_p, with L_q the limit of the alert's
//                 threshold T_q = max(k-th distance so far, eps^2);
//   object side:  dd < rk_p (the object's own k-th neighbour dd) needs
//                 q . p - L_q >= -h_p + (L(qn, rk_p) - L_q), where the
//                 bracket is at least A_q + B_p with
//                 A_q = (1/2 + c16 - K u) T_q - 2 K u qn and
//                 B_p = -(1/2 + c16 + K u) rk_p - 4 u |h_p|
//                 (u = 2^-24, K = 64 NS + 32 with NS the K steps of the
//                 contraction: twice what the float32 evaluation of both
//                 limits, the half-precision pieces of both and the matrix
//                 core's accumulation loss on them, (16 NS + 1) 2^-22 of
//                 the summed magnitudes, can take).
// One block row of 32 alerts uses its smallest A_q, so the pass threshold
// of candidate column p is -h_p + min(0, A_min + B_p): a pair that passes
// neither test may pass, never the reverse.  Every passing pair is
// re-evaluated in the float32 direct form with the operations of k_alerts,
// so the in-degree, the eps count and the k nearest distances are exactly
// those of k_alerts, and so is the kNN mean (summed in the order of
// k_alerts' wavefront reduction).  At the end the wavefronts' partial
// results are merged through LDS in wavefront order and wavefront 0 writes
// the workgroup's partial result; k_alerts_merge (serve.hip) combines the
// slices of each group in slice order and writes the scores and rank
// positions.  The eps distance sum is thus taken in another order than in
// k_alerts (float64, per wavefront, then in wavefront order, then in slice
// order), so the eps mean may differ from k_alerts' in the last float bit.
#pragma once

#include "join_mfma.cuh"
#include "serve_internal.h"
#include "keys.cuh"
#include "serve.cuh"

namespace snaps {

namespace alert_mfma_detail {

constexpr float kU = 5.9604644775390625e-8f;   // 2^-24

// Inserts v into the ascending list kd (dropping the largest entry).
template <int KS>
__device__ __forceinline__ void dist_insert(float (&kd)[KS], float v) {
    bool b[KS];
#pragma unroll
    for (int j = 0; j < KS; ++j) b[j] = v < kd[j];
#pragma unroll
    for (int j = KS - 1; j > 0; --j) kd[j] = b[j - 1] ? kd[j - 1] : (b[j] ? v : kd[j]);
    kd[0] = b[0] ? v : kd[0];
}

}  // namespace alert_mfma_detail

template <int D, int KC>
__device__ __forceinline__ void alerts_mfma_body(const AlertArgs& A) {
    using namespace mfma_detail;
    using namespace alert_detail;
    using namespace alert_mfma_detail;
    constexpr int DP = row_stride(D);
    constexpr int KS = KC;
    using Sp = Split<D>;
    constexpr int M = Sp::M;
    constexpr int NS = Sp::NS;
    constexpr int W = alert_mfma_waves(D);
    constexpr int kRowShift = 26;                // walk entry: tile | block rows in reach << 26
    constexpr int kTileMask = (1 << kRowShift) - 1;
    constexpr float kSlack = (float)(64 * NS + 32) * kU;
    constexpr float ca = 0.5f + Sp::c16 - kSlack;
    constexpr float cr = 0.5f + Sp::c16 + kSlack;
    static_assert(KS <= 32, "the kNN mean's reduction order assumes at most 32 slots");

    // Per wavefront: the rows and k-th distances of two tiles (the one
    // screened and the next, copied in while the first is screened).  The
    // two buffers are separate arrays so that the compiler can tell a read
    // of one from the copy in flight into the other.
    __shared__ __align__(16) float s_rows0[W][kTile * DP];
    __shared__ __align__(16) float s_rows1[W][kTile * DP];
    __shared__ __align__(16) float s_rk0[W][kTile];
    __shared__ __align__(16) float s_rk1[W][kTile];
    __shared__ float s_part[KS + 4][kTile];      // one wavefront's partial results, for the merge
    // Smallest k-th distance any wavefront of the workgroup has found for
    // each alert (float bits; the values are >= 0, so integer order is float
    // order).  The final k-th distance is at most each of them, so every
    // wavefront may screen with the smallest.  The same bound is published,
    // by device-scope atomic minimum, to the group's slot in A.bounds, where
    // the workgroups of the group's other slices take it up.
    __shared__ unsigned s_kth[kTile];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int half = lane >> 5;
    const int col = lane & 31;
    const int grp = blockIdx.x;
    if (grp >= A.group_prefix[A.n_jobs]) return;
    int lo = 0, hi = A.n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (A.group_prefix[mid] <= grp) lo = mid; else hi = mid;
    }
    const AlertJob& J = A.jobs[lo];
    const int m = J.m;
    const int nsl = A.slices[lo];
    const int li = grp - A.group_prefix[lo];     // (group, slice) of this workgroup
    const int gi = li / nsl;
    const int sl = li - gi * nsl;
    const int a0 = gi * kTile;
    const int ai = a0 + lane;
    const bool qpad = ai >= m;                   // lane beyond the job's last alert
    const ServeState* St = J.st;
    const int k = St->k;
    if (St->d != D || k < 1 || k > KS) return;   // state of another shape: the merge flags the alerts
    if (wv == 0) s_kth[lane] = 0x7F800000u;      // +inf
    __syncthreads();
    unsigned* const gbound = A.bounds + A.bound_off[lo] + (int64_t)gi * kTile + lane;
    // This slice's run of tiles.
    const int per = (St->ntiles + nsl - 1) / nsl;
    const int t_lo = sl * per;
    const int nt = min(St->ntiles, t_lo + per);
    const float eps2 = St->eps2;
    const float* boxes = St->boxes;
    const float* tmaxp = St->tmax;

    float q[D];
    {
        const float* qa = J.alerts + (int64_t)(qpad ? m - 1 : ai) * D;
#pragma unroll
        for (int f = 0; f < D; ++f) q[f] = qa[f];
    }
    float kd[KS];                                // k nearest dd ascending; KS - k leading -inf
#pragma unroll
    for (int j = 0; j < KS; ++j) kd[j] = j < KS - k ? -INFINITY : INFINITY;
    int cnt = 0, deg = 0;
    double sum = 0.0;
    // kb: the smallest k-th distance known for the alert (this wavefront's
    // own or another's).  A pad lane has nothing in reach (-inf threshold:
    // its limit is +inf and its scores never pass; excluded from the culls
    // and from A_min).
    float kb = INFINITY;
    float thr = qpad ? -INFINITY : fmaxf(kb, eps2);
    float qn = 0.f;
#pragma unroll
    for (int f = 0; f < D; ++f) qn = fmaf(q[f], q[f], qn);
    float lim = f16_limit<D>(qn, thr);

    // A operands: alert rows 32 rb + col of the group (pad rows repeat the
    // last alert; their limit makes them fail), this lane half's
    // coordinates, then the limit pieces.  A group with a coordinate out of
    // the pieces' range is not screened (every pair is re-evaluated).
    u4v aw[2][NS];
    float rq[2];
    bool unit_all;
    {
        float amax = 0.f;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const float* rowp = J.alerts + (int64_t)min(a0 + 32 * rb + col, m - 1) * D + half * M;
            float v[M];
#pragma unroll
            for (int i = 0; i < M; ++i) {
                v[i] = (D % 2 == 1 && i == M - 1 && half) ? 0.f : rowp[i];
                amax = fmaxf(amax, fabsf(v[i]));
            }
            a_words<D>(v, aw[rb], rq[rb]);
        }
        unit_all = __any(amax > kF16Range);
    }
    float amin0 = INFINITY, amin1 = INFINITY;    // smallest A_q of each block row
    auto refresh = [&]() {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) limit_words<D>(__shfl(lim, 32 * rb + col, 64), half, rq[rb], aw[rb]);
        const float aq = qpad ? INFINITY : fmaf(ca, thr, -2.f * kSlack * qn);
        const float hm = half_min(aq);
        amin0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hm), 0));
        amin1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hm), 32));
    };
    refresh();

    // The group's box (corners of its alerts, in scalar registers) and its
    // block rows with an alert (a block row of pad lanes only is not
    // contracted).
    float glo[D], ghi[D];
#pragma unroll
    for (int f = 0; f < D; ++f) {
        glo[f] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_min(qpad ? INFINITY : q[f]))));
        ghi[f] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_max(qpad ? -INFINITY : q[f]))));
    }
    const unsigned long long live = __ballot(!qpad);
    const int rows_live = ((unsigned)live ? 1 : 0) | ((live >> 32) ? 2 : 0);

    // Next tile of this wavefront that an alert of the group may reach (-1
    // at the end), with the block rows to contract in bits 26-27.  Window:
    // this wavefront's tiles t_lo + wv + W (wb + j), j = 0..63, tested one
    // per lane.
    int wb = -64;
    unsigned long long wmask = 0ull;
    auto next_tile = [&]() -> int {
        for (;;) {
            if (wmask) {
                const int j = __builtin_ctzll(wmask);
                wmask &= wmask - 1;
                return (t_lo + wv + W * (wb + j)) | (rows_live << kRowShift);
            }
            wb += 64;
            if (t_lo + wv + W * wb >= nt) return -1;
            const float gthr = wave_max(qpad ? -INFINITY : thr);
            const int t = t_lo + wv + W * (wb + lane);
            bool keep = false;
            if (t < nt) {
                const float* b = boxes + (int64_t)t * 2 * DP;
                float lb = 0.f;
#pragma unroll
                for (int f = 0; f < D; ++f) {
                    const float g = fmaxf(fmaxf(b[f] - ghi[f], glo[f] - b[DP + f]), 0.f);
                    lb = fmaf(g, g, lb);
                }
                keep = lb <= gthr || lb < tmaxp[t];
            }
            wmask = __ballot(keep);
        }
    };

    typedef const __attribute__((address_space(1))) float* gfloat;
    const gfloat xg = (gfloat)St->xs;
    const gfloat rkg = (gfloat)St->rk2;
    // Tile t's 64 rows (DP / 4 copies of 16 bytes per lane) and k-th
    // distances (one copy of 4 bytes per lane), global memory to LDS without
    // registers, after the LDS reads of the buffer's previous tile.
    auto load_rows = [&](int tv, float* dst, float* rdst) {
        const int t = tv & kTileMask;
        const gfloat src = xg + (int64_t)t * kTile * DP + lane * 4;
        wait_lds();
#pragma unroll
        for (int i = 0; i < DP / 4; ++i)
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + i * 256),
                                             (__attribute__((address_space(3))) void*)(dst + i * 256), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(rkg + (int64_t)t * kTile + lane),
                                         (__attribute__((address_space(3))) void*)rdst, 4, 0, 0);
    };

    auto process = [&](int tv, const float* rows_l, const float* rk_l) {
        const int rows = tv >> kRowShift;
        // The bound the group's other slices have published, read now and
        // taken up after this tile (so the load's latency is hidden).
        const unsigned gb = __hip_atomic_load(gbound, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        {   // take up a smaller k-th distance found by another wavefront
            const float sk = __uint_as_float(s_kth[lane]);
            const bool tighter = !qpad && sk < kb;
            if (tighter) {
                kb = sk;
                thr = fmaxf(kb, eps2);
                lim = f16_limit<D>(qn, thr);
            }
            if (__any(tighter)) refresh();
        }
        bool hit = false, all = unit_all;
        unsigned mk[2] = {0u, 0u};
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            // This lane's candidate (row 32 cb + col): its half's
            // coordinates, h and k-th distance.
            const float* rowc = rows_l + (32 * cb + col) * DP;
            float v[M];
            float cmax = 0.f;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                v[i] = (D % 2 == 1 && i == M - 1 && half) ? 0.f : rowc[half * M + i];
                cmax = fmaxf(cmax, fabsf(v[i]));
            }
            if (__any(cmax > kF16Range)) {
                all = true;
                continue;
            }
            u4v bw[NS];
            b_words<D>(v, bw);
            const float hp = rowc[D];
            const float bp = fmaf(-cr, rk_l[32 * cb + col], -4.f * kU * fabsf(hp));
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                if (!((rows >> rb) & 1)) continue;
                // pass threshold of this lane's candidate column (pad rows:
                // NaN h, never passes)
                const float x = -hp + fminf(0.f, (rb ? amin1 : amin0) + bp);
                f16v acc = f16v{};
#pragma unroll
                for (int s2 = 0; s2 < NS; ++s2)
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(op(aw[rb][s2]), op(bw[s2]), acc, 0, 0, 0);
                float mx = -INFINITY;
#pragma unroll
                for (int r = 0; r < 16; ++r) mx = fmaxf(mx, acc[r]);
                if (!__any(mx >= x)) continue;
                hit = true;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const unsigned long long bm = __ballot(acc[r] >= x);
                    const int i0 = acc_row(rb, r, 0);
                    mk[cb] = (unsigned)lane_write((int)(unsigned)bm, i0, (int)mk[cb]);
                    mk[cb] = (unsigned)lane_write((int)(unsigned)(bm >> 32), i0 + 4, (int)mk[cb]);
                }
            }
        }
        bool moved = false;
        if (hit || all) {
            unsigned long long mine = all ? ~0ull : (((unsigned long long)mk[1] << 32) | mk[0]);
            if (qpad) mine = 0ull;
            while (mine) {
                const int j = __builtin_ctzll(mine);
                mine &= mine - 1;
                const float* row = rows_l + j * DP;
                float dd = 0.f;
#pragma unroll
                for (int f = 0; f < D; ++f) {
                    const float tq = q[f] - row[f];
                    dd = fmaf(tq, tq, dd);
                }
                // pad rows hold NaN: every comparison below is false for them
                deg += dd < rk_l[j];
                if (dd <= eps2) {
                    cnt += 1;
                    sum += (double)__builtin_amdgcn_sqrtf(dd);
                }
                if (dd < kd[KS - 1]) {
                    dist_insert<KS>(kd, dd);
                    moved = true;
                }
            }
            if (moved && kd[KS - 1] < kb) {
                kb = kd[KS - 1];
                thr = fmaxf(kb, eps2);
                lim = f16_limit<D>(qn, thr);
                atomicMin(&s_kth[lane], __float_as_uint(kb));
                __hip_atomic_fetch_min(gbound, __float_as_uint(kb), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        const bool from_group = !qpad && __uint_as_float(gb) < kb;
        if (from_group) {
            kb = __uint_as_float(gb);
            thr = fmaxf(kb, eps2);
            lim = f16_limit<D>(qn, thr);
            atomicMin(&s_kth[lane], gb);
        }
        if (__any(moved) || __any(from_group)) refresh();
    };

    float* const r0 = s_rows0[wv];
    float* const r1 = s_rows1[wv];
    float* const k0 = s_rk0[wv];
    float* const k1 = s_rk1[wv];
    int t = next_tile();
    if (t >= 0) load_rows(t, r0, k0);
    while (t >= 0) {
        const int tn = next_tile();
        if (tn >= 0) {
            load_rows(tn, r1, k1);
            wait_vmem<DP / 4 + 1>();
        } else {
            wait_vmem<0>();
        }
        process(t, r0, k0);
        if (tn < 0) break;
        t = next_tile();
        if (t >= 0) {
            load_rows(t, r0, k0);
            wait_vmem<DP / 4 + 1>();
        } else {
            wait_vmem<0>();
        }
        process(tn, r1, k1);
    }

    // Merge into wavefront 0, in wavefront order.
    for (int w = 1; w < W; ++w) {
        __syncthreads();
        if (wv == w) {
#pragma unroll
            for (int j = 0; j < KS; ++j) s_part[j][lane] = kd[j];
            const long long sb = __double_as_longlong(sum);
            s_part[KS][lane] = __int_as_float(cnt);
            s_part[KS + 1][lane] = __int_as_float(deg);
            s_part[KS + 2][lane] = __int_as_float((int)(unsigned)(sb & 0xffffffffLL));
            s_part[KS + 3][lane] = __int_as_float((int)(sb >> 32));
        }
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int j = 0; j < KS; ++j) {
                if (j >= KS - k) {
                    const float v = s_part[j][lane];
                    if (v < kd[KS - 1]) dist_insert<KS>(kd, v);
                }
            }
            cnt += __float_as_int(s_part[KS][lane]);
            deg += __float_as_int(s_part[KS + 1][lane]);
            const unsigned long long lo32 = (unsigned)__float_as_int(s_part[KS + 2][lane]);
            const unsigned long long hi32 = (unsigned)__float_as_int(s_part[KS + 3][lane]);
            sum += __longlong_as_double((long long)((hi32 << 32) | lo32));
        }
    }
    if (wv != 0) return;
    float* part = A.part + A.part_off[lo] + (int64_t)li * alert_part_floats(KS);
#pragma unroll
    for (int j = 0; j < KS; ++j) part[j * kTile + lane] = kd[j];
    const long long sb = __double_as_longlong(sum);
    part[KS * kTile + lane] = __int_as_float(cnt);
    part[(KS + 1) * kTile + lane] = __int_as_float(deg);
    part[(KS + 2) * kTile + lane] = __int_as_float((int)(unsigned)(sb & 0xffffffffLL));
    part[(KS + 3) * kTile + lane] = __int_as_float((int)(sb >> 32));
}

template <int D, int KC>
__global__ __launch_bounds__(64 * alert_mfma_waves(D)) void k_alerts_mfma(AlertArgs A) {
    alerts_mfma_body<D, KC>(A);
}

// The same kernel held to 128 VGPRs (four wavefronts per SIMD, two
// eight-wavefront workgroups per compute unit) for k <= 10 with eight
// wavefronts, where it needs at most a few more (d = 14: 129 VGPRs, three
// wavefronts per SIMD and one workgroup per compute unit otherwise).
template <int D, int KC>
__global__ __launch_bounds__(64 * alert_mfma_waves(D)) __attribute__((amdgpu_waves_per_eu(4))) void
k_alerts_mfma_o4(AlertArgs A) {
    alerts_mfma_body<D, KC>(A);
}

template <int D>
AlertKernel alert_mfma_kc(int kc) {
    switch (kc) {
        case 5:
            if constexpr (alert_mfma_waves(D) == 8) return k_alerts_mfma_o4<D, 5>;
            else return k_alerts_mfma<D, 5>;
        case 10:
            if constexpr (alert_mfma_waves(D) == 8) return k_alerts_mfma_o4<D, 10>;
            else return k_alerts_mfma<D, 10>;
        case 20: return k_alerts_mfma<D, 20>;
        case 32: return k_alerts_mfma<D, 32>;
    }
    return nullptr;
}

}  // namespace snaps
