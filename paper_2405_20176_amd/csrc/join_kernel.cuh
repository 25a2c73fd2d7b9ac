// Fused similarity self-join of one (population, subspace) job per work
// unit: the k-nearest-neighbour self-join (paper Sec. 3.6) and the eps-range
// self-join (Sec. 3.5) computed in one candidate pass, reduced on the fly to
// the four per-object metrics (Sec. 3.5.1, 3.6.1).
//
// Work unit = one block of 64*QL queries of one job per wavefront: every lane
// carries QL queries (rows lane, lane + 64, ... of the block).  Candidate
// tiles (64 objects each) are visited starting at the query block and moving
// outward in index order, so that near candidates tighten the k-th distance
// early.  Candidate rows are wavefront-uniform: they arrive by wide scalar
// loads into SGPRs and feed the vector ALU directly, with no LDS traffic in
// the distance loop.  Two workgroup shapes:
//   split: `split` wavefronts share one query block and divide the candidate
//     tiles between them (few units: one small job);
//   mq: `mq` wavefronts take consecutive query blocks of the same job and walk
//     the same candidate tiles in lockstep (one barrier per tile), so the row
//     that the first wavefront pulls into the CU's scalar cache is a cache
//     hit for the others (many units: batched jobs).
//
// Two flavours of the per-pair test (XF):
//   XF = 0, direct form: dd = sum_f (q_f - p_f)^2 in float32 (one subtract and
//     one fma per dimension), then dd <= thr with thr = max(k-th dd, eps^2).
//   XF = 1, expanded-form prefilter: one fma per dimension (see xf_limit);
//     only candidates that pass are re-evaluated in the direct form.  The
//     prefilter never rejects a candidate the direct form accepts, so both
//     flavours give bit-identical results.
// Candidates with dd <= thr count as eps hits (float64 sum of distances) when
// dd <= eps^2 and enter the per-query sorted top-k registers (order: dd, then
// object id) when they beat the current k-th.
//
// A candidate tile is skipped when, for every query of the wavefront, the
// float32 distance from the query to the tile's bounding box exceeds thr.
// That bound is computed with the same operations in the same order as dd,
// and float rounding is monotone, so it never exceeds the dd of any object in
// the box: skipping cannot change any result.
//
// The workgroup's wavefronts merge their top-k lists and eps partial sums in
// LDS; wavefront 0 writes the metrics by object id and adds the in-degree of
// the k neighbours with integer atomics (order-independent).
#pragma once

#include "snaps_internal.h"
#include "common.cuh"

#include <climits>

namespace snaps {

namespace join_detail {

// A kNN list entry as one 64-bit key: the float32 squared distance's bits
// (non-negative, so their order is the distances' order) above the object
// id, so that key order is (distance, id) order.  Empty slots hold the key
// of (+inf, INT_MAX); the slots in front of the k real ones hold 0.
typedef unsigned long long u64;
constexpr u64 kEmptyKey = (0x7F800000ull << 32) | 0x7FFFFFFFull;
__device__ __forceinline__ u64 knn_key(float dd, int id) {
    return ((u64)__float_as_uint(dd) << 32) | (unsigned)id;
}
__device__ __forceinline__ float key_dist(u64 key) {
    return __uint_as_float((unsigned)(key >> 32));
}

// Insert `key` into the ascending list kk of KC keys; the caller has checked
// that it goes before the last one.
template <int KC>
__device__ __forceinline__ void key_insert(u64 (&kk)[KC], u64 key) {
    bool b[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) b[j] = key < kk[j];
#pragma unroll
    for (int j = KC - 1; j > 0; --j) kk[j] = b[j - 1] ? kk[j - 1] : (b[j] ? key : kk[j]);
    kk[0] = b[0] ? key : kk[0];
}

// Lower limit of the expanded-form score of a candidate that can still
// matter to a query.  Each candidate row stores, after its d coordinates,
// h = -pn (1 - c0) / 2 with pn its float32 squared norm and c0 = (8d + 24) u
// (u = 2^-24).  The query computes acc = h + sum_f q_f p_f with one fma per
// dimension.  Expanding dd = qn + pn - 2 q.p and bounding the float32
// rounding of the direct form, of the norms and of the fma chain (each at
// most (d + 3) u times qn + pn), every candidate whose direct-form dd is <= thr
// has acc >= (qn - thr) / 2 - c0 qn; subtracting cq (qn + thr) with cq = 2 c0
// more than covers the rounding of this limit itself.  Candidates below the
// limit are skipped; the rest are re-evaluated in the direct form, so the
// results are identical to a direct-form-only scan.
__device__ __forceinline__ float xf_limit(float qn, float thr, float cq) {
    return fmaf(-cq, qn + thr, 0.5f * (qn - thr));
}

// Tile visited at step s of the candidate walk of query tile t0 over nt
// tiles: tiles in order of their index distance from t0, the higher one
// first at equal distance, and once one end is reached the other side alone
// (t0, t0+1, t0-1, t0+2, t0-2, ...).  A bijection of [0, nt).  The join on
// the matrix cores walks the same order as a merge of its two frontiers and
// can drop a whole super-tile of kSuper tiles when a frontier enters it, so
// the tiles it visits keep this relative order.
__device__ __forceinline__ int walk_tile(int t0, int s, int nt) {
    const int m = min(t0, nt - 1 - t0);
    if (s <= 2 * m) return t0 + ((s & 1) ? ((s + 1) >> 1) : -(s >> 1));
    return t0 < nt - 1 - t0 ? t0 + s - m : t0 + m - s;
}

// Candidates per group of the distance loop: the group's rows are loaded
// with wide scalar loads before any of them is used (one wait per group);
// 4 rows while they fit in 48 SGPRs, else 2.
template <int DP>
struct Group {
    static constexpr int G = (DP * 4 <= 48) ? 4 : 2;
    static constexpr int NV = DP * G / 4;     // 4-float vectors per group
};

typedef float f4v __attribute__((ext_vector_type(4)));

// Next work unit of a persistent join workgroup: thread 0 takes one from the
// workgroup's home queue (its XCD), or steals from the others once it is
// drained; every thread gets the unit u, its queue qu and the queue-local
// index lo of its job (prefix[lo] <= u < prefix[lo + 1]).  False when every
// queue is drained.  Contains two workgroup barriers.
__device__ __forceinline__ bool next_unit(const JoinArgs& A, int home, unsigned& drained, int& s_unit, int& s_queue,
                                          int& u, int& qu, int& lo) {
    if (threadIdx.x == 0) {
        int got = -1, gq = 0;
        for (int i = 0; i < kQueues && got < 0; ++i) {
            const int qq = (home + i) % kQueues;
            if ((drained >> qq) & 1u) continue;
            const int v = A.q_units[qq] > 0 ? atomicAdd(A.counter + qq, 1) : A.q_units[qq];
            if (v < A.q_units[qq]) { got = v; gq = qq; }
            else drained |= 1u << qq;
        }
        s_unit = got;
        s_queue = gq;
    }
    __syncthreads();
    u = __builtin_amdgcn_readfirstlane(s_unit);
    qu = __builtin_amdgcn_readfirstlane(s_queue);
    __syncthreads();
    if (u < 0) return false;
    const int32_t* prefix = A.unit_prefix + A.q_prefix_off[qu];
    int l = 0, h = A.q_jobs[qu];
    while (h - l > 1) {
        const int mid = (l + h) >> 1;
        if (prefix[mid] <= u) l = mid; else h = mid;
    }
    lo = l;
    return true;
}

}  // namespace join_detail

using namespace join_detail;

template <int D, int KC, int XF, int QL>
__global__ __launch_bounds__(512) void k_join(JoinArgs A) {
    constexpr int DP = row_stride(D);
    constexpr int KS = KC > 0 ? KC : 1;
    constexpr float cq = (float)(2 * (8 * D + 24)) * 5.9604644775390625e-8f;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_unit, s_queue;

    const int S = A.split;
    const int W = A.mq;
    // Wavefront-uniform values are passed through readfirstlane so that the
    // compiler keeps them (and every address derived from them) in SGPRs.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;

    const int home = blockIdx.x % kQueues;                   // this workgroup's XCD
    unsigned drained = 0;                                     // queues found empty (thread 0)
    for (;;) {
        int u, qu, lo;
        if (!next_unit(A, home, drained, s_unit, s_queue, u, qu, lo)) break;
        const int32_t* prefix = A.unit_prefix + A.q_prefix_off[qu];
        const int tu = (u - prefix[lo]) * QL * W;            // first query tile of the unit
        const int t0 = W > 1 ? tu + wave * QL : tu;          // this wavefront's first query tile
        const DevJob* Jp = A.table + A.order[A.q_order_off[qu] + lo];
        const int n = Jp->n;
        const int nt = Jp->ntiles;
        const int k = KC > 0 ? Jp->k : 0;
        const float eps2 = Jp->eps2;
        const int prune = Jp->prune;
        const float* xs_g = Jp->xs;
        cptr<float> xs = as_const(xs_g);
        cptr<float> boxes = as_const((const float*)Jp->boxes);

        int qpos[QL];
        float q[QL][D];
        u64 kk[QL][KS];
        int cnt[QL];
        double sum[QL];
        float thr[QL], qn[QL], lim[QL];
        int nq_total = 0;
#pragma unroll
        for (int r = 0; r < QL; ++r) {
            qpos[r] = (t0 + r) * kTile + lane;
            const int qrow = qpos[r] < n ? qpos[r] : (n - 1);
#pragma unroll
            for (int f = 0; f < D; ++f) q[r][f] = xs_g[(int64_t)qrow * DP + f];
#pragma unroll
            for (int j = 0; j < KS; ++j) kk[r][j] = j < KS - k ? 0ull : kEmptyKey;   // 0: slots in front of the k real ones
            cnt[r] = 0;
            sum[r] = 0.0;
            thr[r] = KC > 0 ? fmaxf(key_dist(kk[r][KS - 1]), eps2) : eps2;
            if (qpos[r] >= n) thr[r] = -INFINITY;             // no query (pad lane or missing tile): nothing in reach
            qn[r] = 0.f;
#pragma unroll
            for (int f = 0; f < D; ++f) qn[r] = fmaf(q[r][f], q[r][f], qn[r]);
            lim[r] = XF ? xf_limit(qn[r], thr[r], cq) : 0.f;
            nq_total += max(0, min(kTile, n - (t0 + r) * kTile));
        }
        // work counters (wavefront-uniform)
        long long pairs = 0;
        int scanned = 0, skipped = 0;

        // Relevant candidate c for query r: eps hit and / or top-k update.
        auto take = [&](int r, float dd, int cid) {
            if (dd <= eps2) {
                cnt[r] += 1;
                sum[r] += (double)__builtin_amdgcn_sqrtf(dd);   // hardware sqrt, <= 1 ulp
            }
            if (KC > 0) {
                const u64 key = knn_key(dd, cid);
                if (key < kk[r][KS - 1]) key_insert<KS>(kk[r], key);
                thr[r] = fmaxf(key_dist(kk[r][KS - 1]), eps2);
                if (XF) lim[r] = xf_limit(qn[r], thr[r], cq);
            }
        };

        for (int s = (W > 1 ? 0 : wave); s < nt; s += (W > 1 ? 1 : S)) {
            if (W > 1 && s > 0) __syncthreads();             // keep the wavefronts in lockstep
            const int t = walk_tile(W > 1 ? tu : t0, s, nt);
            if (prune) {
                cptr<float> bx = boxes + (int64_t)t * 2 * DP;
                bool near = false;
#pragma unroll
                for (int r = 0; r < QL; ++r) {
                    float lb = 0.f;
#pragma unroll
                    for (int f = 0; f < D; ++f) {
                        const float g = fmaxf(fmaxf(bx[f] - q[r][f], q[r][f] - bx[DP + f]), 0.f);
                        lb = fmaf(g, g, lb);
                    }
                    near = near || (lb <= thr[r]);
                }
                if (!__any(near)) {
                    ++skipped;
                    continue;
                }
            }
            ++scanned;
            pairs += (long long)nq_total * min(kTile, n - t * kTile);
            const int cbase = t * kTile;
            constexpr int GS = Group<DP>::G;
            constexpr int NV = Group<DP>::NV;
#pragma unroll 1
            for (int g = 0; g < kTile; g += GS) {
                const int c0 = cbase + g;
                cptr<f4v> pv = (cptr<f4v>)(xs + (int64_t)c0 * DP);
                f4v blk[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) blk[v] = pv[v];
#define PV(j, f) blk[((j) * DP + (f)) >> 2][((j) * DP + (f)) & 3]
                if (XF) {
                    float acc[QL][GS];
#pragma unroll
                    for (int j = 0; j < GS; ++j) {
#pragma unroll
                        for (int r = 0; r < QL; ++r) acc[r][j] = fmaf(q[r][0], PV(j, 0), PV(j, D));
#pragma unroll
                        for (int f = 1; f < D; ++f) {
#pragma unroll
                            for (int r = 0; r < QL; ++r) acc[r][j] = fmaf(q[r][f], PV(j, f), acc[r][j]);
                        }
                    }
                    bool pass = false;
#pragma unroll
                    for (int r = 0; r < QL; ++r) {
                        float m = acc[r][0];
#pragma unroll
                        for (int j = 1; j < GS; ++j) m = fmaxf(m, acc[r][j]);
                        pass = pass || (m >= lim[r]);
                    }
                    if (pass) {
#pragma unroll
                        for (int j = 0; j < GS; ++j) {
                            const int c = c0 + j;
#pragma unroll
                            for (int r = 0; r < QL; ++r) {
                                if (acc[r][j] >= lim[r] && c != qpos[r]) {
                                    float dd = 0.f;
#pragma unroll
                                    for (int f = 0; f < D; ++f) {
                                        const float tq = q[r][f] - PV(j, f);
                                        dd = fmaf(tq, tq, dd);
                                    }
                                    if (dd <= thr[r]) take(r, dd, __float_as_int(PV(j, D + 1)));
                                }
                            }
                        }
                    }
                } else {
                    float dd[QL][GS];
#pragma unroll
                    for (int j = 0; j < GS; ++j) {
#pragma unroll
                        for (int r = 0; r < QL; ++r) dd[r][j] = 0.f;
#pragma unroll
                        for (int f = 0; f < D; ++f) {
#pragma unroll
                            for (int r = 0; r < QL; ++r) {
                                const float tq = q[r][f] - PV(j, f);
                                dd[r][j] = fmaf(tq, tq, dd[r][j]);
                            }
                        }
                    }
                    bool pass = false;
#pragma unroll
                    for (int r = 0; r < QL; ++r) {
                        float m = dd[r][0];
#pragma unroll
                        for (int j = 1; j < GS; ++j) m = fminf(m, dd[r][j]);
                        pass = pass || (m <= thr[r]);
                    }
                    if (pass) {
#pragma unroll
                        for (int j = 0; j < GS; ++j) {
                            const int c = c0 + j;
#pragma unroll
                            for (int r = 0; r < QL; ++r)
                                if (dd[r][j] <= thr[r] && c != qpos[r]) take(r, dd[r][j], __float_as_int(PV(j, D + 1)));
                        }
                    }
                }
#undef PV
            }
        }

        if (A.stats && lane == 0) {
            atomicAdd(A.stats + 0, (unsigned long long)pairs);
            atomicAdd(A.stats + 1, (unsigned long long)scanned);
            atomicAdd(A.stats + 2, (unsigned long long)skipped);
            atomicAdd(A.stats + 3, (unsigned long long)pairs * D);
        }

        // Merge the split wavefronts' partial results into wavefront 0.
        // LDS layout per wavefront and query slot r: KS list keys (64 lanes
        // each), the eps count, then (after all of those) the float64 eps sums.
        if (S > 1) {
            u64* mkk = reinterpret_cast<u64*>(smem);
            int* mcnt = reinterpret_cast<int*>(mkk + S * QL * KS * 64);
            double* msum = reinterpret_cast<double*>(smem + (size_t)S * QL * (KS * 64 * 8 + 64 * 4));
            if (wave > 0) {
#pragma unroll
                for (int r = 0; r < QL; ++r) {
                    const int wr = wave * QL + r;
#pragma unroll
                    for (int j = 0; j < KS; ++j) mkk[(wr * KS + j) * 64 + lane] = kk[r][j];
                    mcnt[wr * 64 + lane] = cnt[r];
                    msum[wr * 64 + lane] = sum[r];
                }
            }
            __syncthreads();
            if (wave == 0) {
                for (int w = 1; w < S; ++w) {
#pragma unroll
                    for (int r = 0; r < QL; ++r) {
                        const int wr = w * QL + r;
                        cnt[r] += mcnt[wr * 64 + lane];
                        sum[r] += msum[wr * 64 + lane];
                        if (KC > 0) {
#pragma unroll
                            for (int j = 0; j < KS; ++j) {
                                if (j >= KS - k) {
                                    const u64 key = mkk[(wr * KS + j) * 64 + lane];
                                    if (key < kk[r][KS - 1]) key_insert<KS>(kk[r], key);
                                }
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }

        if (W > 1 || wave == 0) {
#pragma unroll
            for (int r = 0; r < QL; ++r) {
                if (qpos[r] >= n) continue;
                const int id = Jp->perm[qpos[r]];
                int32_t* eps_count = Jp->eps_count;
                if (eps_count) {
                    eps_count[id] = cnt[r];
                    Jp->eps_mean[id] = cnt[r] > 0 ? (float)(sum[r] / (double)cnt[r]) : 0.f;
                }
                if (KC > 0) {
                    int32_t* indeg = Jp->indeg;
                    int32_t* kids = Jp->knn_ids;
                    float* kdist = Jp->knn_dist;
                    float accm = 0.f;
#pragma unroll
                    for (int j = 0; j < KS; ++j) {
                        if (j >= KS - k) {
                            const float dj = sqrtf(key_dist(kk[r][j]));
                            const int kid = (int)(unsigned)kk[r][j];
                            accm += dj;
                            const int o = j - (KS - k);
                            if (kids) kids[(int64_t)id * k + o] = kid;
                            if (kdist) kdist[(int64_t)id * k + o] = dj;
                            if (indeg) atomicAdd(indeg + kid, 1);
                        }
                    }
                    float* kmean = Jp->knn_mean;
                    if (kmean) kmean[id] = accm / (float)k;
                    float* kth = Jp->knn_kth;
                    if (kth) kth[id] = key_dist(kk[r][KS - 1]);
                }
            }
        }
    }
}

using JoinFn = void (*)(JoinArgs);

template <int D, int XF>
JoinFn join_pick_kc(int kc) {
    switch (kc) {
        case 0: return k_join<D, 0, XF, join_ql(0)>;
        case 5: return k_join<D, 5, XF, join_ql(5)>;
        case 10: return k_join<D, 10, XF, join_ql(10)>;
        case 20: return k_join<D, 20, XF, join_ql(20)>;
        case 32: return k_join<D, 32, XF, join_ql(32)>;
    }
    return nullptr;
}

template <int D>
JoinFn join_pick_d(int kc, int xf) {
    return xf ? join_pick_kc<D, 1>(kc) : join_pick_kc<D, 0>(kc);
}

// Instantiation groups, one per translation unit (compiled in parallel).
JoinFn join_pick_group0(int D, int kc, int xf);
JoinFn join_pick_group1(int D, int kc, int xf);
JoinFn join_pick_group2(int D, int kc, int xf);
JoinFn join_pick_group3(int D, int kc, int xf);

}  // namespace snaps
