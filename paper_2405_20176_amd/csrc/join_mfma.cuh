// Fused kNN + eps self-join with the expanded-form prefilter on the matrix
// cores.  Same work units, walk, pruning, per-query state and outputs as
// k_join with one wavefront per workgroup and one query per lane; what
// changes is how a (query tile, candidate tile) pair is screened.
//
// The prefilter test of query i and candidate j is h_j + q_i . p_j >= lim_i
// (h_j = -pn_j (1 - c0) / 2 stored in the candidate's row, lim_i from
// xf_limit).  For a 64 x 64 tile pair the scores h_j + q_i . p_j - lim_i are
// a dense contraction, computed by v_mfma_f32_32x32x2f32 in four 32 x 32
// blocks over ceil(d / 2) + 1 K-steps: the coordinates, then one step whose
// two K slots carry (-lim_i, 1) and (1, h_j).  A pair passes when its
// accumulator is >= 0.  For odd d the coordinate steps' pad slot carries
// (-lim_i, 1) instead and the test is accumulator >= -h_j.  The rounding of that accumulation, with |lim_i|
// among the summed magnitudes, stays inside the prefilter's margin (the
// margin also allows products and sums that round separately), so every
// candidate the exact direct form would accept still passes.
//
// Operand layouts (32 x 32 x 2, one block): lane l holds A[l % 32][l / 32]
// and B[l / 32][l % 32]; accumulator register r of lane l is element
// (8 (r / 4) + 4 (l / 32) + r % 4, l % 32).  Rows are queries, columns
// candidates.  Most tile pairs have no passing pair, which a per-lane
// maximum over the accumulators and one ballot establish.  Otherwise the
// ballot of each accumulator register gives, in its low and high 32 bits,
// the passing candidates of two queries in one candidate block; those bits
// are written into the owning lanes' per-query candidate masks.  The tile's
// candidate rows go from the operand registers into LDS, and each lane walks
// its own mask in ascending candidate order: it re-evaluates the exact
// direct-form distance of each candidate and updates its query's kNN list
// and eps sums exactly as k_join does, in the same order, so the results
// are identical to both k_join flavours.  (A wavefront-uniform walk over the
// union of the masks costs one iteration per distinct candidate; the
// per-lane walk costs the largest per-query count.)
//
// Two walks (template parameter H).  H = 0 visits the candidate tiles in the
// order of walk_tile and skips a tile whose box no query can reach; the
// contraction of a 32-query block row that no query of it can reach is
// skipped.  H = 1 adds two levels: a frontier of the walk that enters a new
// super-tile (kSuper tiles) first tests the super-tile's box and drops all
// of its tiles on that side if no query can reach it, and, for jobs that ask
// for it, each candidate tile is tested as two 32-object halves with boxes
// of their own, so each of the four 32 x 32 blocks of a tile pair is
// contracted only if a query of its row block may reach its half.  The tiles
// H = 1 visits keep the order of walk_tile.  Both give the same results; they
// differ in the work skipped and in register use (H = 0 keeps the leaner
// kernel for the jobs whose index gains nothing from the extra levels).
#pragma once

#include "join_kernel.cuh"

#include <type_traits>

namespace snaps {

namespace mfma_detail {

typedef float f16v __attribute__((ext_vector_type(16)));

// Row (within the 64-query tile) of accumulator register r of block row rb
// in lane half h.
__device__ __forceinline__ constexpr int acc_row(int rb, int r, int h) {
    return 32 * rb + 8 * (r >> 2) + 4 * h + (r & 3);
}


}  // namespace mfma_detail

template <int D, int KC, int H>
__device__ __forceinline__ void join_mfma_body(JoinArgs A) {
    using namespace mfma_detail;
    constexpr int DP = row_stride(D);
    constexpr int KS = KC > 0 ? KC : 1;
    constexpr int KSTEPS = (D + 1) / 2;      // coordinate steps
    // Even d: one more step carries (-lim_i, 1) and (1, h_j), and a pair
    // passes when its score is >= 0.  Odd d: the pad slot of the last
    // coordinate step carries (-lim_i, 1), and h_j moves into the comparison
    // (score >= -h_j, exact), which saves that step.
    constexpr bool kFold = D % 2 == 1;
    constexpr int NSTEP = kFold ? KSTEPS : KSTEPS + 1;
    constexpr float cq = (float)(2 * (8 * D + 24)) * 5.9604644775390625e-8f;
    __shared__ int s_unit, s_queue;
    __shared__ uint2 s_mask[64];            // per-query candidate masks of one tile pair
    __shared__ __align__(16) float s_cand[64][DP];   // candidate rows of a tile pair with passes
    // Walk entries: tile index | the 32 x 32 blocks (query block row rb,
    // candidate half cb) that may hold a pair in reach, bit rb + 2 cb, << 26
    // (H = 0 sets both halves of a block row together).
    constexpr int kRowShift = 26;
    constexpr int kTileMask = (1 << kRowShift) - 1;

    const int lane = threadIdx.x;
    const int half = lane >> 5;
    s_mask[lane] = make_uint2(0u, 0u);
    const int col = lane & 31;
    const int home = blockIdx.x % kQueues;
    unsigned drained = 0;
    for (;;) {
        int u, qu, lo;
        if (!next_unit(A, home, drained, s_unit, s_queue, u, qu, lo)) break;
        const int32_t* prefix = A.unit_prefix + A.q_prefix_off[qu];
        const int t0 = u - prefix[lo];
        const DevJob* Jp = A.table + A.order[A.q_order_off[qu] + lo];
        const int n = Jp->n;
        const int nt = Jp->ntiles;
        const int k = KC > 0 ? Jp->k : 0;
        const float eps2 = Jp->eps2;
        const int prune = Jp->prune;
        const float* xs_g = Jp->xs;
        cptr<float> xs = as_const(xs_g);
        cptr<float> boxes = as_const((const float*)Jp->boxes);

        // Per-lane query (lane = query row of the tile), as in k_join.
        const int qpos = t0 * kTile + lane;
        const int qrow = qpos < n ? qpos : (n - 1);
        float q[D];
#pragma unroll
        for (int f = 0; f < D; ++f) q[f] = xs_g[(int64_t)qrow * DP + f];
        float kd[KS];
        int kid[KS];
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const bool dummy = j < KS - k;
            kd[j] = dummy ? -INFINITY : INFINITY;
            kid[j] = dummy ? -1 : INT_MAX;
        }
        int cnt = 0;
        double sum = 0.0;
        float thr = KC > 0 ? fmaxf(kd[KS - 1], eps2) : eps2;
        float qn = 0.f;
#pragma unroll
        for (int f = 0; f < D; ++f) qn = fmaf(q[f], q[f], qn);
        float lim = xf_limit(qn, thr, cq);
        const int nq = max(0, min(kTile, n - t0 * kTile));
        long long pairs = 0;
        int scanned = 0, skipped = 0;

        // A operands: query rows 32 rb + col of the tile, dimensions 2 s + half
        // (pad rows beyond n hold NaN and never pass; a pad dimension is 0),
        // then (-lim, 1) of the same query.
        float av[2][KSTEPS + 1];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const float* rowp = xs_g + (int64_t)(t0 * kTile + 32 * rb + col) * DP + half;
#pragma unroll
            for (int s = 0; s < KSTEPS; ++s) {
                const float v = rowp[2 * s];
                av[rb][s] = (kFold && s == KSTEPS - 1 && half) ? 0.f : v;
            }
        }
        auto refresh_limits = [&]() {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const float l = __shfl(lim, 32 * rb + col, 64);
                if (kFold)
                    av[rb][KSTEPS - 1] = half ? -l : av[rb][KSTEPS - 1];
                else
                    av[rb][KSTEPS] = half ? 1.f : -l;
            }
        };
        refresh_limits();

        // An eps-only job may also list each query's hits: the query's row of
        // the pair list starts at pair_off[id]; hits are appended in the
        // order the walk meets them (pad lanes write nothing).
        int32_t* const prow = KC == 0 ? Jp->pairs : nullptr;
        int64_t poff = 0, pcap = 0;
        if (KC == 0 && prow && qpos < n) {
            poff = Jp->pair_off[Jp->perm[qpos]];
            pcap = Jp->pair_cap;
        }

        // Exact re-evaluation of one candidate (same operations as k_join).
        auto take = [&](float dd, int cid) {
            if (dd <= eps2) {
                if constexpr (KC == 0) {
                    if (prow) {
                        const int64_t at = poff + cnt;
                        if (at < pcap) prow[at] = cid;
                    }
                }
                cnt += 1;
                sum += (double)__builtin_amdgcn_sqrtf(dd);   // hardware sqrt, <= 1 ulp
            }
            if (KC > 0) {
                if (before(dd, cid, kd[KS - 1], kid[KS - 1])) topk_insert<KS>(kd, kid, dd, cid);
                const float nthr = fmaxf(kd[KS - 1], eps2);
                const bool moved = nthr != thr;
                thr = nthr;
                lim = xf_limit(qn, thr, cq);
                return moved;
            }
            return false;
        };

        // Next candidate tile of the walk whose box may hold a candidate (or
        // -1 at the end), in the order of walk_tile; bits 26-29 of the result
        // flag the 32 x 32 blocks with a query that may reach the candidates
        // (the other blocks' contractions are skipped).
        auto reach_of = [&](cptr<float> bx) -> unsigned long long {
            float lb = 0.f;
#pragma unroll
            for (int f = 0; f < D; ++f) {
                const float g = fmaxf(fmaxf(bx[f] - q[f], q[f] - bx[DP + f]), 0.f);
                lb = fmaf(g, g, lb);
            }
            return __ballot(lb <= thr);
        };
        int ws = 0;                                  // H = 0: walk step
        // H = 1: the walk as a merge of its two frontiers (the tile nearer to
        // t0, the right one on ties), each with the super-tile it is in.
        int wr = t0, wl = t0 - 1;
        int sr = t0 / kSuper, sl = t0 / kSuper;
        cptr<float> sboxes = as_const((const float*)Jp->sboxes);
        cptr<float> hboxes = as_const((const float*)Jp->hboxes);
        const int halves = H ? Jp->halves : 0;
        auto next_tile = [&]() -> int {
            if constexpr (H == 0) {
                while (ws < nt) {
                    const int t = walk_tile(t0, ws, nt);
                    ++ws;
                    if (!prune) return t | (15 << kRowShift);
                    const unsigned long long reach = reach_of(boxes + (int64_t)t * 2 * DP);
                    if (reach) {
                        const int rows = ((unsigned)reach ? 1 : 0) | ((reach >> 32) ? 2 : 0);
                        return t | ((rows | (rows << 2)) << kRowShift);
                    }
                    ++skipped;
                }
                return -1;
            } else {
                for (;;) {
                    const bool rv = wr < nt, lv = wl >= 0;
                    if (!rv && !lv) return -1;
                    int t;
                    if (rv && (!lv || wr - t0 <= t0 - wl)) {
                        if (prune && wr / kSuper != sr) {
                            sr = wr / kSuper;
                            if (!reach_of(sboxes + (int64_t)sr * 2 * DP)) {
                                const int e = min(nt, (sr + 1) * kSuper);
                                skipped += e - wr;
                                wr = e;
                                continue;
                            }
                        }
                        t = wr++;
                    } else {
                        if (prune && wl / kSuper != sl) {
                            sl = wl / kSuper;
                            if (!reach_of(sboxes + (int64_t)sl * 2 * DP)) {
                                skipped += wl - sl * kSuper + 1;
                                wl = sl * kSuper - 1;
                                continue;
                            }
                        }
                        t = wl--;
                    }
                    if (!prune) return t | (15 << kRowShift);
                    int blocks;
                    if (halves) {
                        const unsigned long long r0 = reach_of(hboxes + (int64_t)t * 4 * DP);
                        const unsigned long long r1 = reach_of(hboxes + (int64_t)t * 4 * DP + 2 * DP);
                        blocks = ((unsigned)r0 ? 1 : 0) | ((r0 >> 32) ? 2 : 0) | ((unsigned)r1 ? 4 : 0) |
                                 ((r1 >> 32) ? 8 : 0);
                    } else {
                        const unsigned long long r = reach_of(boxes + (int64_t)t * 2 * DP);
                        const int rows = ((unsigned)r ? 1 : 0) | ((r >> 32) ? 2 : 0);
                        blocks = rows | (rows << 2);
                    }
                    if (blocks) return t | (blocks << kRowShift);
                    ++skipped;
                }
            }
        };
        // Raw B operands of tile t (candidate rows 32 cb + col: lane half 0
        // reads the even dimensions, half 1 the odd ones, then h), loaded
        // through the global address space so that the loads are waited on
        // only where the values are used, one tile later.
        typedef const __attribute__((address_space(1))) float* gfloat;
        const gfloat xg = (gfloat)xs_g;
        // The candidate's id bits come along, so that the exact recheck can
        // stage whole candidate rows from these registers.
        auto load_b = [&](int tv, float (&br)[2][KSTEPS + 2]) {
            const int t = tv & kTileMask;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const gfloat rowc = xg + (int64_t)(t * kTile + 32 * cb + col) * DP + half;
#pragma unroll
                for (int s2 = 0; s2 < KSTEPS; ++s2) br[cb][s2] = rowc[2 * s2];
                br[cb][KSTEPS] = rowc[D - half];
                br[cb][KSTEPS + 1] = rowc[D + 1 - half];
            }
        };

        // Software pipeline: the next tile is chosen (with the threshold as
        // it stands, which only ever shrinks, so the choice is conservative)
        // and its operands requested before the current tile is screened.
        // Two operand buffers, used alternately (no copies between them, so a
        // tile's loads are waited on only when that tile is screened).
        auto process = [&](int tv, float (&br)[2][KSTEPS + 2]) {
            const int t = tv & kTileMask;
            const int blocks = tv >> kRowShift;
            const int rows = (blocks | (blocks >> 2)) & 3;
            ++scanned;
            if constexpr (H == 0) {
                pairs += (long long)((rows & 1 ? min(nq, 32) : 0) + (rows & 2 ? max(0, nq - 32) : 0)) *
                         min(kTile, n - t * kTile);
            } else {
                const int nq0 = min(nq, 32), nq1 = max(0, nq - 32);
                const int nc0 = max(0, min(32, n - t * kTile)), nc1 = max(0, min(32, n - t * kTile - 32));
                pairs += ((blocks & 1 ? nq0 : 0) + (blocks & 2 ? nq1 : 0)) * nc0 +
                         ((blocks & 4 ? nq0 : 0) + (blocks & 8 ? nq1 : 0)) * nc1;
            }
            const int cbase = t * kTile;

            // B operands in place: 0 in the pad slot of an odd d, then (1, h)
            // (the exact recheck reads only the coordinates and the id).
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                if (kFold)
                    br[cb][KSTEPS - 1] = half ? 1.f : br[cb][KSTEPS - 1];
                else
                    br[cb][KSTEPS] = half ? br[cb][KSTEPS] : 1.f;
            }
            // Pass threshold of this lane's candidate column in each block.
            const float nh0 = kFold ? -br[0][KSTEPS] : 0.f;
            const float nh1 = kFold ? -br[1][KSTEPS] : 0.f;
            // One block row of queries at a time (32 accumulators live): the
            // scores, a screen (most tile pairs have no passing pair), then the
            // ballots, whose low and high halves lane 0 writes into the owning
            // queries' rows of an LDS table of candidate masks.
            unsigned u_lo = 0, u_hi = 0;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                if (!((rows >> rb) & 1)) continue;
                // H = 1: a candidate half out of reach of this block row is
                // not contracted (both chains otherwise, interleaved on the
                // matrix pipe); its scores never pass.
                const bool act0 = H ? ((blocks >> rb) & 1) != 0 : true;
                const bool act1 = H ? ((blocks >> (rb + 2)) & 1) != 0 : true;
                f16v acc[2];
                if (act0 && act1) {
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        acc[cb] = f16v{};
#pragma unroll
                        for (int s2 = 0; s2 < NSTEP; ++s2)
                            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb][s2], br[cb][s2], acc[cb], 0, 0, 0);
                    }
                } else {
                    const int cb = act0 ? 0 : 1;
                    acc[0] = f16v{};
                    acc[1] = f16v{};
                    f16v a1 = f16v{};
#pragma unroll
                    for (int s2 = 0; s2 < NSTEP; ++s2)
                        a1 = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb][s2], cb ? br[1][s2] : br[0][s2], a1, 0, 0, 0);
                    if (cb) acc[1] = a1; else acc[0] = a1;
                }
                float mx0 = -INFINITY, mx1 = -INFINITY;     // NaN pads never pass
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    mx0 = fmaxf(mx0, acc[0][r]);
                    mx1 = fmaxf(mx1, acc[1][r]);
                }
                if (!act0) mx0 = -INFINITY;
                if (!act1) mx1 = -INFINITY;
                if (!__any(mx0 >= nh0 || mx1 >= nh1)) continue;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const unsigned long long b0 = act0 ? __ballot(acc[0][r] >= nh0) : 0ull;
                    const unsigned long long b1 = act1 ? __ballot(acc[1][r] >= nh1) : 0ull;
                    if (b0 | b1) {
                        const int i0 = acc_row(rb, r, 0);
                        if (lane == 0) {
                            s_mask[i0] = make_uint2((unsigned)b0, (unsigned)b1);
                            s_mask[i0 + 4] = make_uint2((unsigned)(b0 >> 32), (unsigned)(b1 >> 32));
                        }
                        u_lo |= (unsigned)b0 | (unsigned)(b0 >> 32);
                        u_hi |= (unsigned)b1 | (unsigned)(b1 >> 32);
                    }
                }
            }
            if (u_lo | u_hi) {
                const uint2 mine2 = s_mask[lane];
                s_mask[lane] = make_uint2(0u, 0u);
                // The tile's candidate rows into LDS (row 32 cb + col: this
                // lane's dimensions 2 s + half; the id from lane half 0), so
                // that each lane reads the rows of its own passing candidates.
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    float* row = &s_cand[32 * cb + col][0];
#pragma unroll
                    for (int s2 = 0; s2 < KSTEPS; ++s2)
                        if (2 * s2 + half < D) row[2 * s2 + half] = br[cb][s2];
                    if (!half) reinterpret_cast<int*>(row)[D] = __float_as_int(br[cb][KSTEPS + 1]);
                }
                bool moved = false;
                // This lane's passing candidates in ascending order (block 0,
                // then block 1): the order in which the direct form meets them.
                unsigned long long mine = ((unsigned long long)mine2.y << 32) | mine2.x;
                while (mine) {
                    const int j = __builtin_ctzll(mine);
                    mine &= mine - 1;
                    if (cbase + j == qpos) continue;
                    const float* row = &s_cand[j][0];
                    float dd = 0.f;
#pragma unroll
                    for (int f = 0; f < D; ++f) {
                        const float tq = q[f] - row[f];
                        dd = fmaf(tq, tq, dd);
                    }
                    if (dd <= thr) moved |= take(dd, reinterpret_cast<const int*>(row)[D]);
                }
                if (__any(moved)) refresh_limits();
            }
        };
        // The loads are issued unconditionally (the last prefetch re-reads the
        // current tile) so that every path waits on the same load count.
        // A scheduling barrier after each prefetch keeps the compiler from
        // hoisting the other buffer's uses (and their waits) above it.
        float ba[2][KSTEPS + 2], bb[2][KSTEPS + 2];
        int t = next_tile();
        load_b(t >= 0 ? t : t0, ba);
        while (t >= 0) {
            const int tn = next_tile();
            load_b(tn >= 0 ? tn : t, bb);
            __builtin_amdgcn_sched_barrier(0);
            process(t, ba);
            if (tn < 0) break;
            t = next_tile();
            load_b(t >= 0 ? t : tn, ba);
            __builtin_amdgcn_sched_barrier(0);
            process(tn, bb);
        }

        if (A.stats && lane == 0) {
            atomicAdd(A.stats + 0, (unsigned long long)pairs);
            atomicAdd(A.stats + 1, (unsigned long long)scanned);
            atomicAdd(A.stats + 2, (unsigned long long)skipped);
            atomicAdd(A.stats + 3, (unsigned long long)pairs * D);
        }

        if (qpos < n) {
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
                float accm = 0.f;
#pragma unroll
                for (int j = 0; j < KS; ++j) {
                    if (j >= KS - k) {
                        const float dj = sqrtf(kd[j]);
                        accm += dj;
                        const int o = j - (KS - k);
                        if (kids) kids[(int64_t)id * k + o] = kid[j];
                        if (kdist) kdist[(int64_t)id * k + o] = dj;
                        if (indeg) atomicAdd(indeg + kid[j], 1);
                    }
                }
                float* kmean = Jp->knn_mean;
                if (kmean) kmean[id] = accm / (float)k;
                float* kth = Jp->knn_kth;
                if (kth) kth[id] = kd[KS - 1];
            }
        }
    }
}

template <int D, int KC, int H>
__global__ __launch_bounds__(64) void k_join_mfma(JoinArgs A) {
    join_mfma_body<D, KC, H>(A);
}

// The same kernel held to 128 VGPRs, four wavefronts per SIMD instead of
// three.  It spills a few registers; for d = 7..10 with k <= 10 it is still
// 2-10 % faster (measured per d over 1,024 SNAPShot1-shaped subspaces), at
// d >= 11 it is slower.
template <int D, int KC, int H>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_join_mfma_w4(JoinArgs A) {
    join_mfma_body<D, KC, H>(A);
}

template <int D, int H>
JoinFn join_mfma_pick_kc(int kc) {
    // Four waves per SIMD: d = 7..10 (k <= 10), and the hierarchical walk at
    // d <= 6, whose extra state would otherwise leave it three.
    constexpr bool w4 = (D >= 7 && D <= 10) || (H && D <= 6);
    switch (kc) {
        case 0: return k_join_mfma<D, 0, H>;
        case 5: return w4 ? k_join_mfma_w4<D, 5, H> : k_join_mfma<D, 5, H>;
        case 10: return w4 ? k_join_mfma_w4<D, 10, H> : k_join_mfma<D, 10, H>;
        case 20: return k_join_mfma<D, 20, H>;
        case 32: return k_join_mfma<D, 32, H>;
    }
    return nullptr;
}

// Instantiation groups, one per translation unit.
JoinFn join_mfma_pick_group0(int D, int kc);    // d 2..8, H = 0
JoinFn join_mfma_pick_group1(int D, int kc);    // d 9..16, H = 0
JoinFn join_mfma_pick_group2(int D, int kc);    // d 2..8, H = 1
JoinFn join_mfma_pick_group3(int D, int kc);    // d 9..16, H = 1

}  // namespace snaps
