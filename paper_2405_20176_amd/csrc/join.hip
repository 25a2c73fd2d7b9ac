// Fused similarity self-join of one (population, subspace) job per work
// unit: the k-nearest-neighbour self-join (paper Sec. 3.6) and the eps-range
// self-join (Sec. 3.5) computed in one candidate pass, reduced on the fly to
// the four per-object metrics (Sec. 3.5.1, 3.6.1).
//
// Work unit = one tile of 64 queries of one job (one query per lane).  A
// workgroup of `split` wavefronts shares the unit; each wavefront scans its
// share of the candidate tiles, starting at the query tile and moving outward
// in index order, so that near candidates tighten the k-th distance early.
// Candidate coordinates are wavefront-uniform: they arrive by scalar loads
// into SGPRs and feed the vector ALU directly, with no LDS traffic in the
// distance loop.
//
// Per lane and candidate the common path is the float32 direct form
// dd = sum_f (q_f - p_f)^2 (one subtract and one fma per dimension) and one
// compare of min(dd over 4 candidates) against the lane's threshold
// thr = max(current k-th dd, eps^2).  Only candidates with dd <= thr take the
// branch that counts eps hits (float64 sum of distances) and inserts into the
// per-lane sorted top-k registers (order: dd, then object id).
//
// A candidate tile is skipped when, for every lane, the float32 distance from
// the query to the tile's bounding box exceeds thr.  That bound is computed
// with the same operations in the same order as dd, and float rounding is
// monotone, so it never exceeds the dd of any object in the box: skipping
// cannot change any result.
//
// The workgroup's wavefronts merge their top-k lists and eps partial sums in
// LDS; wavefront 0 writes the metrics by object id and adds the in-degree of
// the k neighbours with integer atomics (order-independent).
#include "snaps_internal.h"
#include "common.cuh"

#include <climits>

namespace snaps {

namespace {

__device__ __forceinline__ bool before(float d, int id, float bd, int bid) {
    return d < bd || (d == bd && id < bid);
}

// Insert (dn, idn) into the ascending list (kd, kid) of KC slots; the caller
// has checked that it goes before the last slot.
template <int KC>
__device__ __forceinline__ void topk_insert(float (&kd)[KC], int (&kid)[KC], float dn, int idn) {
    bool b[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) b[j] = before(dn, idn, kd[j], kid[j]);
#pragma unroll
    for (int j = KC - 1; j > 0; --j) {
        kd[j] = b[j - 1] ? kd[j - 1] : (b[j] ? dn : kd[j]);
        kid[j] = b[j - 1] ? kid[j - 1] : (b[j] ? idn : kid[j]);
    }
    kd[0] = b[0] ? dn : kd[0];
    kid[0] = b[0] ? idn : kid[0];
}

// Tile visited at step s of a walk that starts at t0 and alternates outward
// (t0, t0+1, t0-1, t0+2, ...) modulo nt: a bijection of [0, nt).
__device__ __forceinline__ int spiral(int t0, int s, int nt) {
    const int off = (s & 1) ? ((s + 1) >> 1) : -(s >> 1);
    int t = t0 + off;
    t %= nt;
    if (t < 0) t += nt;
    return t;
}

}  // namespace

template <int D, int KC, int XF>
__global__ __launch_bounds__(512) void k_join(JoinArgs A) {
    constexpr int DP = row_stride(D);
    constexpr int KS = KC > 0 ? KC : 1;
    extern __shared__ unsigned char smem[];
    __shared__ int s_unit;

    const int S = A.split;
    // Wavefront-uniform values are passed through readfirstlane so that the
    // compiler keeps them (and every address derived from them) in SGPRs.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;

    for (;;) {
        if (threadIdx.x == 0) s_unit = atomicAdd(A.counter, 1);
        __syncthreads();
        const int u = __builtin_amdgcn_readfirstlane(s_unit);
        __syncthreads();
        if (u >= A.total_units) break;

        // Locate the job of unit u: unit_prefix[j] <= u < unit_prefix[j+1].
        int lo = 0, hi = A.n_class_jobs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (A.unit_prefix[mid] <= u) lo = mid; else hi = mid;
        }
        const int t0 = u - A.unit_prefix[lo];
        const DevJob* Jp = A.table + A.order[lo];
        const int n = Jp->n;
        const int nt = Jp->ntiles;
        const int k = KC > 0 ? Jp->k : 0;
        const float eps2 = Jp->eps2;
        const int prune = Jp->prune;
        const float* xs_g = Jp->xs;
        cptr<float> xs = as_const(xs_g);
        cptr<int32_t> perm = as_const((const int32_t*)Jp->perm);
        cptr<float> boxes = as_const((const float*)Jp->boxes);

        const int qpos = t0 * kTile + lane;
        const bool qvalid = qpos < n;
        const int qrow = qvalid ? qpos : (n - 1);
        float q[D];
#pragma unroll
        for (int f = 0; f < D; ++f) q[f] = xs_g[(int64_t)qrow * DP + f];

        float kd[KS];
        int kid[KS];
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const bool dummy = j < KS - k;     // slots in front of the k real ones
            kd[j] = dummy ? -INFINITY : INFINITY;
            kid[j] = dummy ? -1 : INT_MAX;
        }
        int cnt = 0;
        double sum = 0.0;
        float thr = KC > 0 ? fmaxf(kd[KS - 1], eps2) : eps2;
        // work counters (wavefront-uniform)
        const int nq = min(kTile, n - t0 * kTile);
        long long pairs = 0;
        int scanned = 0, skipped = 0;

        for (int s = wave; s < nt; s += S) {
            const int t = spiral(t0, s, nt);
            if (prune) {
                cptr<float> bx = boxes + (int64_t)t * 2 * DP;
                float lb = 0.f;
#pragma unroll
                for (int f = 0; f < D; ++f) {
                    const float g = fmaxf(fmaxf(bx[f] - q[f], q[f] - bx[DP + f]), 0.f);
                    lb = fmaf(g, g, lb);
                }
                if (!__any(lb <= thr)) {
                    ++skipped;
                    continue;
                }
            }
            ++scanned;
            pairs += (long long)nq * min(kTile, n - t * kTile);
            const int cbase = t * kTile;
#pragma unroll 1
            for (int g = 0; g < kTile; g += 4) {
                const int c0 = cbase + g;
                cptr<float> p = xs + (int64_t)c0 * DP;
                float dd[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float acc = 0.f;
#pragma unroll
                    for (int f = 0; f < D; ++f) {
                        const float tq = q[f] - p[j * DP + f];
                        acc = fmaf(tq, tq, acc);
                    }
                    dd[j] = acc;
                }
                const float m = fminf(fminf(dd[0], dd[1]), fminf(dd[2], dd[3]));
                if (m <= thr) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int c = c0 + j;
                        const int cid = perm[c];
                        if (dd[j] <= thr && c != qpos) {
                            if (dd[j] <= eps2) {
                                cnt += 1;
                                sum += (double)sqrtf(dd[j]);
                            }
                            if (KC > 0) {
                                if (before(dd[j], cid, kd[KS - 1], kid[KS - 1])) topk_insert<KS>(kd, kid, dd[j], cid);
                                thr = fmaxf(kd[KS - 1], eps2);
                            }
                        }
                    }
                }
            }
        }

        if (A.stats && lane == 0) {
            atomicAdd(A.stats + 0, (unsigned long long)pairs);
            atomicAdd(A.stats + 1, (unsigned long long)scanned);
            atomicAdd(A.stats + 2, (unsigned long long)skipped);
            atomicAdd(A.stats + 3, (unsigned long long)pairs * D);
        }

        // Merge the split wavefronts' partial results into wavefront 0.
        if (S > 1) {
            float* mkd = reinterpret_cast<float*>(smem);
            int* mkid = reinterpret_cast<int*>(mkd + S * KS * 64);
            int* mcnt = mkid + S * KS * 64;
            double* msum = reinterpret_cast<double*>(smem + (size_t)S * (KS * 64 * 8 + 64 * 4));
            if (wave > 0) {
#pragma unroll
                for (int j = 0; j < KS; ++j) {
                    mkd[(wave * KS + j) * 64 + lane] = kd[j];
                    mkid[(wave * KS + j) * 64 + lane] = kid[j];
                }
                mcnt[wave * 64 + lane] = cnt;
                msum[wave * 64 + lane] = sum;
            }
            __syncthreads();
            if (wave == 0) {
                for (int w = 1; w < S; ++w) {
                    cnt += mcnt[w * 64 + lane];
                    sum += msum[w * 64 + lane];
                    if (KC > 0) {
#pragma unroll
                        for (int j = 0; j < KS; ++j) {
                            if (j >= KS - k) {
                                const float dn = mkd[(w * KS + j) * 64 + lane];
                                const int idn = mkid[(w * KS + j) * 64 + lane];
                                if (before(dn, idn, kd[KS - 1], kid[KS - 1])) topk_insert<KS>(kd, kid, dn, idn);
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }

        if (wave == 0 && qvalid) {
            const int id = Jp->perm[qpos];
            int32_t* eps_count = Jp->eps_count;
            if (eps_count) {
                eps_count[id] = cnt;
                Jp->eps_mean[id] = cnt > 0 ? (float)(sum / (double)cnt) : 0.f;
            }
            if (KC > 0) {
                int32_t* indeg = Jp->indeg;
                int32_t* kids = Jp->knn_ids;
                float* kdist = Jp->knn_dist;
                float acc = 0.f;
#pragma unroll
                for (int j = 0; j < KS; ++j) {
                    if (j >= KS - k) {
                        const float dj = sqrtf(kd[j]);
                        acc += dj;
                        const int o = j - (KS - k);
                        if (kids) kids[(int64_t)id * k + o] = kid[j];
                        if (kdist) kdist[(int64_t)id * k + o] = dj;
                        if (indeg) atomicAdd(indeg + kid[j], 1);
                    }
                }
                float* kmean = Jp->knn_mean;
                if (kmean) kmean[id] = acc / (float)k;
            }
        }
    }
}

int kc_class(int k) {
    if (k <= 0) return 0;
    if (k <= 5) return 5;
    if (k <= 10) return 10;
    if (k <= 20) return 20;
    return 32;
}

size_t join_lds_bytes(int kc, int split) {
    if (split <= 1) return 0;
    const int ks = kc > 0 ? kc : 1;
    // top-k distances and ids, eps counts, then the float64 eps sums (the
    // offset of the last block is a multiple of 256 bytes)
    return (size_t)split * (ks * 64 * 8 + 64 * 4 + 64 * 8);
}

namespace {

using JoinFn = void (*)(JoinArgs);

template <int D, int KC, int XF>
JoinFn pick_fn() { return k_join<D, KC, XF>; }

template <int D>
JoinFn pick_kc(int kc, int xf) {
    (void)xf;
    switch (kc) {
        case 0: return pick_fn<D, 0, 0>();
        case 5: return pick_fn<D, 5, 0>();
        case 10: return pick_fn<D, 10, 0>();
        case 20: return pick_fn<D, 20, 0>();
        case 32: return pick_fn<D, 32, 0>();
    }
    return nullptr;
}

JoinFn pick(int D, int kc, int xf) {
    switch (D) {
        case 2: return pick_kc<2>(kc, xf);
        case 3: return pick_kc<3>(kc, xf);
        case 4: return pick_kc<4>(kc, xf);
        case 5: return pick_kc<5>(kc, xf);
        case 6: return pick_kc<6>(kc, xf);
        case 7: return pick_kc<7>(kc, xf);
        case 8: return pick_kc<8>(kc, xf);
        case 9: return pick_kc<9>(kc, xf);
        case 10: return pick_kc<10>(kc, xf);
        case 11: return pick_kc<11>(kc, xf);
        case 12: return pick_kc<12>(kc, xf);
        case 13: return pick_kc<13>(kc, xf);
        case 14: return pick_kc<14>(kc, xf);
        case 15: return pick_kc<15>(kc, xf);
        case 16: return pick_kc<16>(kc, xf);
    }
    return nullptr;
}

}  // namespace

int join_blocks_per_cu(int D, int kc, int xf, int split) {
    JoinFn fn = pick(D, kc, xf);
    if (!fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn), split * 64,
                                                     join_lds_bytes(kc, split)) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_join(int D, int kc, int xf, const JoinArgs& a, int grid, hipStream_t s) {
    JoinFn fn = pick(D, kc, xf);
    if (!fn) return hipErrorInvalidValue;
    JoinArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(grid), dim3(a.split * 64), args,
                           join_lds_bytes(kc, a.split), s);
}

}  // namespace snaps
