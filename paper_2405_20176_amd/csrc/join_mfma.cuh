// Fused kNN + eps self-join with the expanded-form prefilter on the matrix
// cores.  Same work units, walk, pruning, per-query state and outputs as
// k_join with one wavefront per workgroup and one query per lane; what
// changes is how a (query tile, candidate tile) pair is screened.
//
// Prefilter.  A candidate j can matter to query i only if
//     q_i . p_j - L_i >= -h_j,
// with h_j = -pn_j (1 - c0) / 2 stored in the candidate's row and L_i the
// query's limit (f16_limit).  The left side is a dense contraction over a
// 64 x 64 tile pair, computed by v_mfma_f32_32x32x16_f16 in four 32 x 32
// blocks.  Each float32 coordinate x is split into two half-precision pieces
// x = xh + xl + e (xh = x rounded toward zero, xl = the exact float32
// remainder rounded toward zero, |e| <= 2^-20 |x| + 2^-24), and the product
// q_f p_f is taken as qh ph + qh pl + ql ph (three K slots; the dropped
// ql pl is below 2^-20 |q_f p_f|).  -L_i enters as two more slots (its two
// pieces times 1).  Half-precision products are exact in float32; the
// matrix core's accumulation may drop low-order bits of the smaller products
// (measured: products 2^-25 below the largest term vanish), which the limit
// bounds as at most 2^-22 of the summed magnitudes per product.  h_j is not
// a slot: the accumulator is compared with -h_j, per candidate column, in
// float32.  f16_limit widens the exact limit by the sum of these bounds, so
// every candidate that the direct form accepts passes; the rest of the
// derivation (norms, direct form) is the one of xf_limit.
//
// The pieces need |x| <= 32 (half-precision range, with the limit clamped
// to -30000, below every score such coordinates can produce).  A query tile
// or a candidate tile with a coordinate outside that range is not screened:
// every pair of it goes to the exact re-evaluation.
//
// Operand layout (32 x 32 x 16, one block; checked on the device): lane l
// holds A[l % 32][8 (l / 32) + e] and B[8 (l / 32) + e][l % 32], e = 0..7,
// as 4 registers of two halves each; accumulator register r of lane l is
// element (8 (r / 4) + 4 (l / 32) + r % 4, l % 32).  Rows are queries,
// columns candidates.  Lane half h carries coordinates [h M, h M + M) of its
// row or column (M = ceil(d / 2); for odd d the last one of half 1 is 0).
// Per pair of coordinates (a, b) three registers: A = (qh_a, qh_b), (qh_a,
// qh_b), (ql_a, ql_b) against B = (ph_a, ph_b), (pl_a, pl_b), (ph_a, ph_b);
// an odd M ends with A = (qh_c, qh_c), (ql_c, -L piece) against B = (ph_c,
// pl_c), (ph_c, 1), the piece being -Lh in half 0 and -Ll in half 1; an even
// M ends with A = (-Lh, -Ll) (half 0) or 0 (half 1) against B = (1, 1).
//
// Screening.  Most tile pairs have no passing pair, which a per-lane maximum
// over the accumulators and one ballot establish.  Otherwise the ballot of
// each accumulator register gives, in its low and high 32 bits, the passing
// candidates of two queries in one candidate block; those bits are written
// into the owning lanes' per-query candidate masks.  The tile's float32
// candidate rows go from the operand registers into LDS, and each lane walks
// its own mask in ascending candidate order: it re-evaluates the exact
// direct-form distance of each candidate and updates its query's kNN list
// and eps sums exactly as k_join does, in the same order, so the results
// are identical to both k_join flavours.
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
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

// Row (within the 64-query tile) of accumulator register r of block row rb
// in lane half h.
__device__ __forceinline__ constexpr int acc_row(int rb, int r, int h) {
    return 32 * rb + 8 * (r >> 2) + 4 * h + (r & 3);
}

// Register plan of one lane half: M coordinates, their pairs, an odd one
// left over, the registers that hold them and the K = 16 steps that take
// those registers four at a time.
template <int D>
struct Split {
    static constexpr int M = (D + 1) / 2;
    static constexpr int PAIRS = M / 2;
    static constexpr bool SINGLE = M % 2 == 1;
    static constexpr int WORDS = 3 * PAIRS + (SINGLE ? 2 : 1);
    static constexpr int NS = (WORDS + 3) / 4;
    static constexpr int NW = 4 * NS;
    // Limit widening: relative part c16 (qn + thr), absolute part cabs.
    static constexpr float c16 = (float)(139 * NS + 120 + D) * 5.9604644775390625e-8f;
    static constexpr float cabs = (float)(D + 8) * 5.9604644775390625e-8f;
};

// Largest coordinate magnitude the half-precision pieces take.
constexpr float kF16Range = 32.f;
constexpr unsigned kOnes16 = 0x3C003C00u;   // (1, 1) in half precision

// Two floats rounded toward zero to half precision, packed low | high.
__device__ __forceinline__ unsigned pk(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(a, b));
}
__device__ __forceinline__ float lo_f(unsigned w) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xFFFFu));
}
__device__ __forceinline__ float hi_f(unsigned w) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
}

// Lower limit L of q . p over the candidates that can still matter to a query
// (see the file comment): the exact limit (qn - thr) / 2 of xf_limit widened
// by c16 (qn + thr) + cabs, clamped to -30000 (every score of in-range
// coordinates is above it, so a lower limit would pass the same pairs).
template <int D>
__device__ __forceinline__ float f16_limit(float qn, float thr) {
    const float l = fmaf(-Split<D>::c16, qn + thr, 0.5f * (qn - thr)) - Split<D>::cabs;
    return fmaxf(l, -30000.f);
}

// Register j of an operand held as NS groups of four (one per K step).
template <int NS>
__device__ __forceinline__ unsigned& word(u4v (&w)[NS], int j) {
    return reinterpret_cast<unsigned*>(&w[j >> 2])[j & 3];
}

// Candidate-side registers from this lane half's M float32 coordinates.
template <int D>
__device__ __forceinline__ void b_words(const float (&v)[Split<D>::M], u4v (&wv)[Split<D>::NS]) {
    using S = Split<D>;
    unsigned w[S::NW];
#pragma unroll
    for (int j = 0; j < S::PAIRS; ++j) {
        const float a = v[2 * j], b = v[2 * j + 1];
        const unsigned h = pk(a, b);
        w[3 * j] = h;
        w[3 * j + 1] = pk(a - lo_f(h), b - hi_f(h));
        w[3 * j + 2] = h;
    }
    if constexpr (S::SINGLE) {
        const float c = v[S::M - 1];
        const unsigned h1 = pk(c, 1.f);
        w[3 * S::PAIRS] = pk(c, c - lo_f(h1));
        w[3 * S::PAIRS + 1] = h1;
    } else {
        w[3 * S::PAIRS] = kOnes16;
    }
#pragma unroll
    for (int j = S::WORDS; j < S::NW; ++j) w[j] = 0u;
#pragma unroll
    for (int i = 0; i < S::NS; ++i) wv[i] = u4v{w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]};
}

// Query-side registers (without the limit pieces, which limit_words sets);
// for an odd M, rq = the float32 remainder of the odd coordinate.
template <int D>
__device__ __forceinline__ void a_words(const float (&v)[Split<D>::M], u4v (&wv)[Split<D>::NS], float& rq) {
    using S = Split<D>;
    unsigned w[S::NW];
#pragma unroll
    for (int j = 0; j < S::PAIRS; ++j) {
        const float a = v[2 * j], b = v[2 * j + 1];
        const unsigned h = pk(a, b);
        w[3 * j] = h;
        w[3 * j + 1] = h;
        w[3 * j + 2] = pk(a - lo_f(h), b - hi_f(h));
    }
    rq = 0.f;
    if constexpr (S::SINGLE) {
        const float c = v[S::M - 1];
        const unsigned h1 = pk(c, c);
        w[3 * S::PAIRS] = h1;
        rq = c - lo_f(h1);
        w[3 * S::PAIRS + 1] = 0u;
    } else {
        w[3 * S::PAIRS] = 0u;
    }
#pragma unroll
    for (int j = S::WORDS; j < S::NW; ++j) w[j] = 0u;
#pragma unroll
    for (int i = 0; i < S::NS; ++i) wv[i] = u4v{w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]};
}

// The limit pieces of one block row's query (lim = L of that row): -Lh =
// -L rounded toward zero, -Ll = the float32 remainder rounded toward zero.
template <int D>
__device__ __forceinline__ void limit_words(float lim, int half, float rq, u4v (&w)[Split<D>::NS]) {
    using S = Split<D>;
    const float nl = -lim;
    const float nlh = lo_f(pk(nl, 0.f));
    const float r = nl - nlh;
    if constexpr (S::SINGLE)
        word(w, 3 * S::PAIRS + 1) = pk(rq, half ? r : nl);
    else
        word(w, 3 * S::PAIRS) = half ? 0u : pk(nl, r);
}

__device__ __forceinline__ h8v op(const u4v& w) {
    return __builtin_bit_cast(h8v, w);
}


}  // namespace mfma_detail

template <int D, int KC, int H>
__device__ __forceinline__ void join_mfma_body(JoinArgs A) {
    using namespace mfma_detail;
    constexpr int DP = row_stride(D);
    constexpr int KS = KC > 0 ? KC : 1;
    using S = Split<D>;
    constexpr int M = S::M;                  // coordinates per lane half
    constexpr int NS = S::NS;                // K = 16 steps per block
    constexpr int NW = S::NW;                // operand registers per lane
    __shared__ int s_unit, s_queue;
    // Candidate rows of two tiles (the one screened and the next), copied
    // from global memory straight into LDS.  Two separate arrays, each named
    // at compile time wherever it is used, so that the compiler can tell a
    // read of one from the copy in flight into the other.
    __shared__ __align__(16) float s_rows0[kTile * DP];
    __shared__ __align__(16) float s_rows1[kTile * DP];
    // Walk entries: tile index | the 32 x 32 blocks (query block row rb,
    // candidate half cb) that may hold a pair in reach, bit rb + 2 cb, << 26
    // (H = 0 sets both halves of a block row together).
    constexpr int kRowShift = 26;
    constexpr int kTileMask = (1 << kRowShift) - 1;

    const int lane = threadIdx.x;
    const int half = lane >> 5;
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
        u64 kk[KS];
#pragma unroll
        for (int j = 0; j < KS; ++j) kk[j] = j < KS - k ? 0ull : kEmptyKey;
        int cnt = 0;
        double sum = 0.0;
        float thr = KC > 0 ? fmaxf(key_dist(kk[KS - 1]), eps2) : eps2;
        if (qpos >= n) thr = -INFINITY;     // pad lane of the last tile: nothing is in its reach
        float qn = 0.f;
#pragma unroll
        for (int f = 0; f < D; ++f) qn = fmaf(q[f], q[f], qn);
        float lim = f16_limit<D>(qn, thr);
        const int nq = max(0, min(kTile, n - t0 * kTile));
        long long pairs = 0;
        int scanned = 0, skipped = 0;

        // A operands: query rows 32 rb + col of the tile, this lane half's
        // coordinates (pad rows beyond n hold NaN and never pass), then the
        // limit pieces of the same query.  A query tile with a coordinate out
        // of the pieces' range is not screened (every pair is re-evaluated).
        u4v aw[2][NS];
        float rq[2];
        bool unit_all;
        {
            float amax = 0.f;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const float* rowp = xs_g + (int64_t)(t0 * kTile + 32 * rb + col) * DP + half * M;
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
        auto refresh_limits = [&]() {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) limit_words<D>(__shfl(lim, 32 * rb + col, 64), half, rq[rb], aw[rb]);
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
                const u64 key = knn_key(dd, cid);
                if (key < kk[KS - 1]) key_insert<KS>(kk, key);
                const float nthr = fmaxf(key_dist(kk[KS - 1]), eps2);
                const bool moved = nthr != thr;
                thr = nthr;
                lim = f16_limit<D>(qn, thr);
                return moved;
            }
            return false;
        };

        // Next candidate tile of the walk whose box may hold a candidate (or
        // -1 at the end), in the order of walk_tile; bits 26-29 of the result
        // flag the 32 x 32 blocks with a query that may reach the candidates
        // (the other blocks' contractions are skipped).
        // (q - clamp(q, lo, hi) is the signed gap, the subtraction that the
        // direct form makes with the nearest box corner, so it rounds the
        // same way.)
        auto reach_of = [&](cptr<float> bx) -> unsigned long long {
            float lb = 0.f;
#pragma unroll
            for (int f = 0; f < D; ++f) {
                const float g = q[f] - __builtin_amdgcn_fmed3f(q[f], bx[f], bx[DP + f]);
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
        // H = 1: the next 64 super-tiles of a frontier are first tested at
        // once, one per lane, with the query tile's box against each
        // super-tile's box and the tile's largest threshold.  Per dimension
        // that gap is at most each query's own gap (the same subtractions
        // with the query replaced by its box's near corner, and float
        // rounding is monotone), so a super-tile this drops is out of every
        // query's reach; the ones it keeps get the per-query test.  Bit j of
        // wmr is super-tile wbr + j, bit j of wml is super-tile wbl - j.
        unsigned long long wmr = 0ull, wml = 0ull;
        int wbr = -128, wbl = Jp->nsuper + 128;
        auto super_window = [&](int s0, int dir) -> unsigned long long {
            const int sj = s0 + dir * lane;
            const float tmax = wave_max(thr);
            bool ok = false;
            if (sj >= 0 && sj < Jp->nsuper) {
                const float* sb = (const float*)Jp->sboxes + (int64_t)sj * 2 * DP;
                float lb = 0.f;
#pragma unroll
                for (int f = 0; f < D; ++f) {
                    const float g = fmaxf(fmaxf(sb[f] - boxes[(int64_t)t0 * 2 * DP + DP + f],
                                                boxes[(int64_t)t0 * 2 * DP + f] - sb[DP + f]), 0.f);
                    lb = fmaf(g, g, lb);
                }
                ok = lb <= tmax;
            }
            return __ballot(ok);
        };
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
                            if (sr >= wbr + 64) {
                                wbr = sr;
                                wmr = super_window(sr, 1);
                            }
                            const unsigned long long rest = wmr >> (sr - wbr);
                            if (!(rest & 1ull)) {
                                // this super-tile and the next ones up to the
                                // first the window keeps
                                const int jump = rest ? __builtin_ctzll(rest) : 64 - (sr - wbr);
                                const int e = min(nt, (sr + jump) * kSuper);
                                skipped += e - wr;
                                wr = e;
                                continue;
                            }
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
                            if (sl <= wbl - 64) {
                                wbl = sl;
                                wml = super_window(sl, -1);
                            }
                            const unsigned long long rest = wml >> (wbl - sl);
                            if (!(rest & 1ull)) {
                                const int jump = rest ? __builtin_ctzll(rest) : 64 - (wbl - sl);
                                const int e = max(-1, (sl - jump + 1) * kSuper - 1);
                                skipped += wl - e;
                                wl = e;
                                continue;
                            }
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
        // The 64 rows of tile t into LDS buffer `buf`: DP / 4 copies of 16
        // bytes per lane, global memory to LDS without registers.  The LDS
        // reads of the buffer's previous tile are complete first.
        typedef const __attribute__((address_space(1))) float* gfloat;
        const gfloat xg = (gfloat)xs_g;
        auto load_rows = [&](int tv, float* dst) {
            const int t = tv & kTileMask;
            const gfloat src = xg + (int64_t)t * kTile * DP + lane * 4;
            wait_lds();
#pragma unroll
            for (int i = 0; i < DP / 4; ++i)
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + i * 256),
                                                 (__attribute__((address_space(3))) void*)(dst + i * 256), 16, 0, 0);
        };

        // Software pipeline: the next tile is chosen (with the threshold as
        // it stands, which only ever shrinks, so the choice is conservative)
        // and its operands requested before the current tile is screened.
        // Two operand buffers, used alternately (no copies between them, so a
        // tile's loads are waited on only when that tile is screened).
        auto process = [&](int tv, const float* rows_l) {
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

            // One 32 x 32 block at a time (the candidate half's registers and
            // one block's accumulators live): its scores, a screen (most
            // blocks have no passing pair), then the ballots, whose low and
            // high halves go to the owning queries' lanes of the candidate
            // masks mk (one per candidate half).
            bool hit = false, all = unit_all;
            unsigned mk[2] = {0u, 0u};
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                // H = 1: a block row out of reach of this candidate half is
                // not contracted; its scores never pass.
                const int act = H ? ((blocks >> (2 * cb)) & 3) : rows;
                if (!act) continue;
                // This lane's candidate (row 32 cb + col): its half's
                // coordinates and h.
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
                const float nh = -rowc[D];        // pass threshold of this lane's candidate column
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    if (!((act >> rb) & 1)) continue;
                    f16v acc = f16v{};
#pragma unroll
                    for (int s2 = 0; s2 < NS; ++s2)
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(op(aw[rb][s2]), op(bw[s2]), acc, 0, 0, 0);
                    float mx = -INFINITY;     // NaN pads never pass
#pragma unroll
                    for (int r = 0; r < 16; ++r) mx = fmaxf(mx, acc[r]);
                    if (!__any(mx >= nh)) continue;
                    hit = true;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const unsigned long long bm = __ballot(acc[r] >= nh);
                        const int i0 = acc_row(rb, r, 0);
                        mk[cb] = (unsigned)lane_write((int)(unsigned)bm, i0, (int)mk[cb]);
                        mk[cb] = (unsigned)lane_write((int)(unsigned)(bm >> 32), i0 + 4, (int)mk[cb]);
                    }
                }
            }
            if (hit || all) {
                bool moved = false;
                // This lane's passing candidates in ascending order (block 0,
                // then block 1): the order in which the direct form meets them.
                // A tile that was not screened offers every candidate.
                unsigned long long mine = all ? ~0ull : (((unsigned long long)mk[1] << 32) | mk[0]);
                while (mine) {
                    const int j = __builtin_ctzll(mine);
                    mine &= mine - 1;
                    if (cbase + j == qpos) continue;
                    const float* row = rows_l + j * DP;
                    float dd = 0.f;
#pragma unroll
                    for (int f = 0; f < D; ++f) {
                        const float tq = q[f] - row[f];
                        dd = fmaf(tq, tq, dd);
                    }
                    if (dd <= thr) moved |= take(dd, reinterpret_cast<const int*>(row)[D + 1]);
                }
                if (__any(moved)) refresh_limits();
            }
        };
        // The rows of the next tile are requested before the current tile is
        // screened; the wait leaves those DP / 4 copies in flight.  The last
        // tile waits for everything, so no copy outlives the unit.
        int t = next_tile();
        if (t >= 0) load_rows(t, s_rows0);
        while (t >= 0) {
            int tn = next_tile();
            if (tn >= 0) {
                load_rows(tn, s_rows1);
                wait_vmem<DP / 4>();
            } else {
                wait_vmem<0>();
            }
            process(t, s_rows0);
            if (tn < 0) break;
            t = next_tile();
            if (t >= 0) {
                load_rows(t, s_rows0);
                wait_vmem<DP / 4>();
            } else {
                wait_vmem<0>();
            }
            process(tn, s_rows1);
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
                        const float dj = sqrtf(key_dist(kk[j]));
                        const int kid = (int)(unsigned)kk[j];
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
                if (kth) kth[id] = key_dist(kk[KS - 1]);
            }
        }
    }
}

template <int D, int KC, int H>
__global__ __launch_bounds__(64) void k_join_mfma(JoinArgs A) {
    join_mfma_body<D, KC, H>(A);
}

// The same kernel held to 96 VGPRs, five wavefronts per SIMD instead of
// four (at d = 5..10 it spills 4-10 registers and is still about 10 %
// faster; held to 80 for six, it spills 20-40 and is 25-55 % slower).
template <int D, int KC, int H>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_join_mfma_w5(JoinArgs A) {
    join_mfma_body<D, KC, H>(A);
}

template <int D, int H>
JoinFn join_mfma_pick_kc(int kc) {
    // Five waves per SIMD for the lean walk at d = 5..10 (measured per d over
    // all SNAPShot1-shaped subspaces of that d); the hierarchical walk would
    // spill 14-35 registers there and keeps four.
    constexpr bool w5 = H == 0 && D >= 5 && D <= 10;
    switch (kc) {
        case 0: return k_join_mfma<D, 0, H>;
        case 5: return w5 ? k_join_mfma_w5<D, 5, H> : k_join_mfma<D, 5, H>;
        case 10: return w5 ? k_join_mfma_w5<D, 10, H> : k_join_mfma<D, 10, H>;
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
