// Selection of k between under- and overfitting (paper Sec. 3.6.2): for a
// grid k_1 < ... < k_g (the paper: from k_min = 2 to k_max = 4096), the
// in-degree and the mean kNN distance of every object at every k, from the
// k_max nearest neighbours, which hold those of every smaller k.
//   k_kgrid_thresh: one workgroup per query, its distances to every object
//     held in registers (k_kgrid_thresh_stream, for populations above
//     kMaxKGridN objects: recomputed in every pass).  One radix selection
//     for all k_j at once gives, for every k_j, the (distance, id) bound of
//     the k_j nearest (ties in id order) and the sum of the k_j smallest
//     distances.
//   k_kgrid_indeg: one lane per object p scans every query q: p is among the
//     k_j nearest of q exactly when (distance, id of p) is at most q's k_j-th
//     (distance, id), so p's in-degree at every k needs no global atomics.
// The rankings, Eq. 2 similarities and the Eq. 3 choice are those of the
// radius grid (eps_grid.hip) with in-degree for the neighbour count and the
// mean kNN distance for the mean.
#include "snaps_internal.h"
#include "common.cuh"

namespace snaps {

namespace {

constexpr int kThreshThreads = 1024;
constexpr int kSlots = kMaxKGridN / kThreshThreads;   // distances per thread, in registers
constexpr int kLookupBatch = 8;

__device__ __forceinline__ int kjob_of(const int32_t* prefix, int n_jobs, int b) {
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// One radix digit of the selection of the r-th smallest (1-based) over the
// register-held values of the workgroup: the histogram of the digit [shift,
// shift + bits) of the values whose higher digits equal pre (every value in
// the first pass), then the bin that holds rank r.  Returns the prefix
// extended by that bin; r becomes the rank within it and *eq its size.
// Values of thread t, slot s belong to object t + s * kThreshThreads; only
// slots that start below n take part (the tail of the last one holds
// 0xFFFFFFFF, above every distance).
template <typename GetFn>
__device__ __forceinline__ unsigned select_digit(GetFn get, int n, int shift, int bits, bool first, unsigned pre,
                                                 unsigned& r, unsigned* eq, unsigned* hist, int* tmp,
                                                 unsigned* s_sel) {
    const int tid = threadIdx.x;
    const int nb = 1 << bits;
    for (int x = tid; x < nb; x += kThreshThreads) hist[x] = 0u;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        if (s * kThreshThreads < n) {
            bool on;
            const uint32_t v = get(s, on);
            if (on && (first || (v >> (shift + bits)) == pre)) atomicAdd(&hist[(v >> shift) & (unsigned)(nb - 1)], 1u);
        }
    }
    __syncthreads();
    const int per = (nb + kThreshThreads - 1) / kThreshThreads;
    const int b0 = tid * per;
    unsigned local = 0u;
    for (int b = 0; b < per; ++b)
        if (b0 + b < nb) local += hist[b0 + b];
    int total;
    const unsigned before = (unsigned)block_exclusive_scan((int)local, tmp, &total);
    if (before < r && before + local >= r) {
        unsigned cum = before;
        int b = b0;
        while (cum + hist[b] < r) cum += hist[b++];
        s_sel[0] = (pre << bits) | (unsigned)b;
        s_sel[1] = r - cum;
        s_sel[2] = hist[b];
    }
    __syncthreads();
    const unsigned out = s_sel[0];
    r = s_sel[1];
    *eq = s_sel[2];
    __syncthreads();
    return out;
}

// Bin of rank r (1-based) in the histogram h[0, 64 * per) (per a power of
// two, at most 64) by one whole wavefront, with the number of values in lower bins and in the bin itself:
// each lane sums per consecutive bins, a scan finds the lane whose bins
// reach rank r, and a second scan over that lane's bins finds the bin.
__device__ __forceinline__ void wave_rank_bin(const unsigned* h, int per, unsigned r, unsigned* bin,
                                              unsigned* below, unsigned* size) {
    const int lane = threadIdx.x & 63;
    unsigned local = 0u;
    for (int b = 0; b < per; ++b) local += h[lane * per + ((b + lane) & (per - 1))];   // rotated: fewer bank conflicts
    const unsigned incl = (unsigned)wave_scan_dpp((int)local);
    const unsigned excl = incl - local;
    const unsigned long long hit = __ballot(excl < r && incl >= r);
    const int L = hit ? __builtin_ctzll(hit) : 63;
    const unsigned base = (unsigned)__builtin_amdgcn_readlane((int)excl, L);
    const unsigned v = lane < per ? h[L * per + lane] : 0u;
    const unsigned incl2 = (unsigned)wave_scan_dpp((int)v) + base;
    const unsigned excl2 = incl2 - v;
    const unsigned long long hit2 = __ballot(lane < per && excl2 < r && incl2 >= r);
    const int B = hit2 ? __builtin_ctzll(hit2) : per - 1;
    *bin = (unsigned)(L * per + B);
    *below = (unsigned)__builtin_amdgcn_readlane((int)excl2, B);
    *size = (unsigned)__builtin_amdgcn_readlane((int)v, B);
}

// Targets t = 0..15 (the grid, padded with k_g) are ranks R_t = k_t of the
// query's distances.  All sixteen are selected together, radix digit by
// digit (12, 10, 10 bits of the float32 squared distance): the first
// histogram is shared; in the later passes targets whose higher digits
// agree share a histogram ("group"), and a value finds its group through
// tables indexed by its own higher digits.  Wavefront t then finds target
// t's bin.  Ties at a target's distance that do not all belong to its k_t
// nearest are split by id (rare: a separate selection over the ties' ids).
template <int D>
__global__ __launch_bounds__(kThreshThreads) void k_kgrid_thresh(const KGridJob* jobs, const int32_t* prefix,
                                                                  int n_jobs, int block0) {
    static_assert(kThreshThreads == 64 * kMaxGrid, "one wavefront per grid target");
    __shared__ unsigned hist[kMaxGrid * 1024];      // pass 0: one 4096-bin histogram; then [group][1024]
    __shared__ uint8_t tab1[4096];                  // 12-bit digit -> pass-1 group + 1 (0: none)
    __shared__ uint8_t tab2[kMaxGrid][1024];        // pass-1 group, 10-bit digit -> pass-2 group + 1
    __shared__ uint32_t list[kMaxKGridK];           // distances below the largest target's
    __shared__ unsigned s_pre[kMaxGrid], s_rank[kMaxGrid], s_eq[kMaxGrid], s_id[kMaxGrid];
    __shared__ unsigned s_g1[kMaxGrid], s_g2[kMaxGrid];
    __shared__ double s_part[kThreshThreads / 64][kMaxGrid];
    __shared__ int tmp[17];
    __shared__ unsigned s_sel[3];
    __shared__ unsigned s_fill, s_split;
    const int blk = block0 + (int)blockIdx.x;
    const int jb = kjob_of(prefix, n_jobs, blk);
    const KGridJob& J = jobs[jb];
    const int qid = blk - prefix[jb];
    const int n = J.n;
    const int g = J.g;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    {
        uint32_t* t1 = reinterpret_cast<uint32_t*>(tab1);
        uint32_t* t2 = reinterpret_cast<uint32_t*>(&tab2[0][0]);
        for (int x = tid; x < 4096 / 4; x += kThreshThreads) t1[x] = 0u;
        for (int x = tid; x < kMaxGrid * 1024 / 4; x += kThreshThreads) t2[x] = 0u;
        for (int x = tid; x < 4096; x += kThreshThreads) hist[x] = 0u;
        if (tid == 0) {
            s_fill = 0u;
            s_split = 0u;
        }
    }
    float q[D];
#pragma unroll
    for (int f = 0; f < D; ++f) q[f] = J.cols[(int64_t)J.feat[f] * J.ld + qid];
    uint32_t e[kSlots];                             // squared distance bits to object tid + s * kThreshThreads
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        const int i = tid + s * kThreshThreads;
        uint32_t v = 0xFFFFFFFFu;                   // past n: above every distance
        if (i < n) {
            float dd = 0.f;
#pragma unroll
            for (int f = 0; f < D; ++f) {
                const float tq = q[f] - J.cols[(int64_t)J.feat[f] * J.ld + i];   // query minus object
                dd = fmaf(tq, tq, dd);
            }
            v = i == qid ? 0x7F800000u : __float_as_uint(dd);                   // self: +inf, never chosen
        }
        e[s] = v;
    }
    __syncthreads();

    // Pass 0: bits [31:20], one histogram for every target.
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
        if (s * kThreshThreads < n) atomicAdd(&hist[e[s] >> 20], 1u);
    __syncthreads();
    const unsigned R = (unsigned)J.k[wave];
    {
        unsigned b, below, size;
        wave_rank_bin(hist, 4096 / 64, R, &b, &below, &size);
        if (lane == 0) {
            s_pre[wave] = b;
            s_rank[wave] = R - below;
        }
    }
    __syncthreads();
    // Pass 1: bits [19:10], a histogram per distinct 12-bit prefix.
    if (tid < kMaxGrid) {
        unsigned grp = 0u;
        for (int t = 1; t <= tid; ++t) grp += s_pre[t] != s_pre[t - 1] ? 1u : 0u;
        s_g1[tid] = grp;
        tab1[s_pre[tid]] = (uint8_t)(grp + 1u);
    }
    for (int x = tid; x < kMaxGrid * 1024; x += kThreshThreads) hist[x] = 0u;
    __syncthreads();
    // Table reads batched ahead of the increments (slots past n read the
    // empty entry of their 0xFFFFFFFF).
#pragma unroll
    for (int s0 = 0; s0 < kSlots; s0 += kLookupBatch) {
        unsigned g1[kLookupBatch];
#pragma unroll
        for (int u = 0; u < kLookupBatch; ++u) g1[u] = tab1[e[s0 + u] >> 20];
#pragma unroll
        for (int u = 0; u < kLookupBatch; ++u)
            if (g1[u]) atomicAdd(&hist[(g1[u] - 1u) * 1024u + ((e[s0 + u] >> 10) & 1023u)], 1u);
    }
    __syncthreads();
    {
        unsigned b, below, size;
        wave_rank_bin(hist + s_g1[wave] * 1024u, 1024 / 64, s_rank[wave], &b, &below, &size);
        if (lane == 0) {
            s_pre[wave] = (s_pre[wave] << 10) | b;
            s_rank[wave] -= below;
        }
    }
    __syncthreads();
    // Pass 2: bits [9:0], a histogram per distinct 22-bit prefix.
    if (tid < kMaxGrid) {
        unsigned grp = 0u;
        for (int t = 1; t <= tid; ++t) grp += s_pre[t] != s_pre[t - 1] ? 1u : 0u;
        s_g2[tid] = grp;
        tab2[s_g1[tid]][s_pre[tid] & 1023u] = (uint8_t)(grp + 1u);
    }
    for (int x = tid; x < kMaxGrid * 1024; x += kThreshThreads) hist[x] = 0u;
    __syncthreads();
#pragma unroll
    for (int s0 = 0; s0 < kSlots; s0 += kLookupBatch) {
        unsigned g1[kLookupBatch], g2[kLookupBatch];
#pragma unroll
        for (int u = 0; u < kLookupBatch; ++u) g1[u] = tab1[e[s0 + u] >> 20];
#pragma unroll
        for (int u = 0; u < kLookupBatch; ++u)
            g2[u] = tab2[g1[u] ? g1[u] - 1u : 0u][(e[s0 + u] >> 10) & 1023u];
#pragma unroll
        for (int u = 0; u < kLookupBatch; ++u)
            if (g1[u] && g2[u]) atomicAdd(&hist[(g2[u] - 1u) * 1024u + (e[s0 + u] & 1023u)], 1u);
    }
    __syncthreads();
    {
        unsigned b, below, size;
        wave_rank_bin(hist + s_g2[wave] * 1024u, 1024 / 64, s_rank[wave], &b, &below, &size);
        if (lane == 0) {
            s_pre[wave] = (s_pre[wave] << 10) | b;
            s_rank[wave] -= below;
            s_eq[wave] = size;
            s_id[wave] = 0xFFFFFFFFu;               // every tie at the distance belongs
            if (size > s_rank[wave]) atomicOr(&s_split, 1u << wave);
        }
    }
    __syncthreads();
    // Ties split by id (targets in s_split): the s_rank-th smallest id among
    // the ties.
    for (unsigned todo = s_split; todo; todo &= todo - 1u) {
        const int t = __builtin_ctz(todo);
        const unsigned vt = s_pre[t], rt = s_rank[t];
        if (t > 0 && vt == s_pre[t - 1] && rt == s_rank[t - 1]) {
            if (tid == 0) s_id[t] = s_id[t - 1];
            __syncthreads();
            continue;
        }
        auto id_of_tie = [&](int s, bool& on) {
            on = e[s] == vt;
            return (uint32_t)(tid + s * kThreshThreads);
        };
        unsigned r = rt, eq;
        unsigned id = select_digit(id_of_tie, n, 8, 8, false, 0u, r, &eq, hist, tmp, s_sel);
        id = select_digit(id_of_tie, n, 0, 8, false, id, r, &eq, hist, tmp, s_sel);
        if (tid == 0) s_id[t] = id;
        __syncthreads();
    }

    // Sums of the distances below each target's: the values below the
    // largest target's, binned by the number of targets at or below them.
    const uint32_t vtop = s_pre[kMaxGrid - 1];
    {
        unsigned cnt = 0u;
#pragma unroll
        for (int s = 0; s < kSlots; ++s)
            if (s * kThreshThreads < n) cnt += (unsigned)__popcll(__ballot(e[s] < vtop));
        unsigned base = 0u;
        if (lane == 0 && cnt) base = atomicAdd(&s_fill, cnt);
        base = __shfl(base, 0, 64);
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            if (s * kThreshThreads < n) {
                const bool in = e[s] < vtop;
                const unsigned long long bal = __ballot(in);
                const unsigned pos = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                if (in && pos < (unsigned)kMaxKGridK) list[pos] = e[s];
                base += (unsigned)__popcll(bal);
            }
        }
    }
    __syncthreads();
    const int m = (int)min(s_fill, (unsigned)kMaxKGridK);
    uint32_t vt[kMaxGrid];
#pragma unroll
    for (int t = 0; t < kMaxGrid; ++t) vt[t] = s_pre[t];
    double part[kMaxGrid];
#pragma unroll
    for (int t = 0; t < kMaxGrid; ++t) part[t] = 0.0;
    for (int x = tid; x < m; x += kThreshThreads) {
        const uint32_t v = list[x];
        int c = 0;                                  // targets whose distance is at most v
#pragma unroll
        for (int t = 0; t < kMaxGrid; ++t) c += v >= vt[t] ? 1 : 0;
        const double dv = (double)sqrtf(__uint_as_float(v));
#pragma unroll
        for (int t = 0; t < kMaxGrid; ++t) part[t] += c == t ? dv : 0.0;
    }
    {
        double run = 0.0;                           // lane 63: this wavefront's sums of bins 0..t
#pragma unroll
        for (int t = 0; t < kMaxGrid; ++t) {
            run += wave_scan_dpp(part[t]);
            if (lane == 63) s_part[wave][t] = run;
        }
    }
    __syncthreads();
    if (tid < kMaxGrid) {
        const int t = tid;
        double sum = 0.0;                           // distances below target t's
#pragma unroll
        for (int w = 0; w < kThreshThreads / 64; ++w) sum += s_part[w][t];
        sum += (double)s_rank[t] * (double)sqrtf(__uint_as_float(vt[t]));
        J.thr[(int64_t)qid * kMaxGrid + t] = ((uint64_t)vt[t] << 32) | (uint64_t)s_id[t];
        if (t < g) J.kmean[(int64_t)t * n + qid] = (float)(sum / (double)J.k[t]);
    }
}

// The same selection for populations above one workgroup's registers
// (n > kMaxKGridN): every pass recomputes the query's distances from the
// columns instead of holding them (the same operations, so the same float32
// values), and ties are split by id over 32 bits.
template <typename GetFn>
__device__ __forceinline__ unsigned select_digit_stream(GetFn get, int n, int shift, int bits, unsigned pre,
                                                        unsigned& r, unsigned* hist, int* tmp, unsigned* s_sel) {
    const int tid = threadIdx.x;
    const int nb = 1 << bits;
    for (int x = tid; x < nb; x += kThreshThreads) hist[x] = 0u;
    __syncthreads();
    for (int i = tid; i < n; i += kThreshThreads) {
        bool on;
        const uint32_t v = get(i, on);
        if (on && (shift + bits >= 32 || (v >> (shift + bits)) == pre))
            atomicAdd(&hist[(v >> shift) & (unsigned)(nb - 1)], 1u);
    }
    __syncthreads();
    const int per = (nb + kThreshThreads - 1) / kThreshThreads;
    const int b0 = tid * per;
    unsigned local = 0u;
    for (int b = 0; b < per; ++b)
        if (b0 + b < nb) local += hist[b0 + b];
    int total;
    const unsigned before = (unsigned)block_exclusive_scan((int)local, tmp, &total);
    if (before < r && before + local >= r) {
        unsigned cum = before;
        int b = b0;
        while (cum + hist[b] < r) cum += hist[b++];
        s_sel[0] = (pre << bits) | (unsigned)b;
        s_sel[1] = r - cum;
    }
    __syncthreads();
    const unsigned out = s_sel[0];
    r = s_sel[1];
    __syncthreads();
    return out;
}

template <int D>
__global__ __launch_bounds__(kThreshThreads) void k_kgrid_thresh_stream(const KGridJob* jobs, const int32_t* prefix,
                                                                         int n_jobs, int block0) {
    __shared__ unsigned hist[kMaxGrid * 1024];
    __shared__ uint8_t tab1[4096];
    __shared__ uint8_t tab2[kMaxGrid][1024];
    __shared__ uint32_t list[kMaxKGridK];
    __shared__ unsigned s_pre[kMaxGrid], s_rank[kMaxGrid], s_id[kMaxGrid];
    __shared__ unsigned s_g1[kMaxGrid], s_g2[kMaxGrid];
    __shared__ double s_part[kThreshThreads / 64][kMaxGrid];
    __shared__ int tmp[17];
    __shared__ unsigned s_sel[3];
    __shared__ unsigned s_fill, s_split;
    const int blk = block0 + (int)blockIdx.x;
    const int jb = kjob_of(prefix, n_jobs, blk);
    const KGridJob& J = jobs[jb];
    const int qid = blk - prefix[jb];
    const int n = J.n;
    const int g = J.g;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    {
        uint32_t* t1 = reinterpret_cast<uint32_t*>(tab1);
        uint32_t* t2 = reinterpret_cast<uint32_t*>(&tab2[0][0]);
        for (int x = tid; x < 4096 / 4; x += kThreshThreads) t1[x] = 0u;
        for (int x = tid; x < kMaxGrid * 1024 / 4; x += kThreshThreads) t2[x] = 0u;
        for (int x = tid; x < 4096; x += kThreshThreads) hist[x] = 0u;
        if (tid == 0) {
            s_fill = 0u;
            s_split = 0u;
        }
    }
    const float* col[D];
    float q[D];
#pragma unroll
    for (int f = 0; f < D; ++f) {
        col[f] = J.cols + (int64_t)J.feat[f] * J.ld;
        q[f] = col[f][qid];
    }
    auto dist_bits = [&](int i) -> uint32_t {
        float dd = 0.f;
#pragma unroll
        for (int f = 0; f < D; ++f) {
            const float tq = q[f] - col[f][i];                                  // query minus object
            dd = fmaf(tq, tq, dd);
        }
        return i == qid ? 0x7F800000u : __float_as_uint(dd);                    // self: +inf, never chosen
    };
    __syncthreads();

    // Pass 0: bits [31:20], one histogram for every target.
    for (int i = tid; i < n; i += kThreshThreads) atomicAdd(&hist[dist_bits(i) >> 20], 1u);
    __syncthreads();
    const unsigned R = (unsigned)J.k[wave];
    {
        unsigned b, below, size;
        wave_rank_bin(hist, 4096 / 64, R, &b, &below, &size);
        if (lane == 0) {
            s_pre[wave] = b;
            s_rank[wave] = R - below;
        }
    }
    __syncthreads();
    // Pass 1: bits [19:10], a histogram per distinct 12-bit prefix.
    if (tid < kMaxGrid) {
        unsigned grp = 0u;
        for (int t = 1; t <= tid; ++t) grp += s_pre[t] != s_pre[t - 1] ? 1u : 0u;
        s_g1[tid] = grp;
        tab1[s_pre[tid]] = (uint8_t)(grp + 1u);
    }
    for (int x = tid; x < kMaxGrid * 1024; x += kThreshThreads) hist[x] = 0u;
    __syncthreads();
    for (int i = tid; i < n; i += kThreshThreads) {
        const uint32_t v = dist_bits(i);
        const unsigned g1 = tab1[v >> 20];
        if (g1) atomicAdd(&hist[(g1 - 1u) * 1024u + ((v >> 10) & 1023u)], 1u);
    }
    __syncthreads();
    {
        unsigned b, below, size;
        wave_rank_bin(hist + s_g1[wave] * 1024u, 1024 / 64, s_rank[wave], &b, &below, &size);
        if (lane == 0) {
            s_pre[wave] = (s_pre[wave] << 10) | b;
            s_rank[wave] -= below;
        }
    }
    __syncthreads();
    // Pass 2: bits [9:0], a histogram per distinct 22-bit prefix.
    if (tid < kMaxGrid) {
        unsigned grp = 0u;
        for (int t = 1; t <= tid; ++t) grp += s_pre[t] != s_pre[t - 1] ? 1u : 0u;
        s_g2[tid] = grp;
        tab2[s_g1[tid]][s_pre[tid] & 1023u] = (uint8_t)(grp + 1u);
    }
    for (int x = tid; x < kMaxGrid * 1024; x += kThreshThreads) hist[x] = 0u;
    __syncthreads();
    for (int i = tid; i < n; i += kThreshThreads) {
        const uint32_t v = dist_bits(i);
        const unsigned g1 = tab1[v >> 20];
        if (!g1) continue;
        const unsigned g2 = tab2[g1 - 1u][(v >> 10) & 1023u];
        if (g2) atomicAdd(&hist[(g2 - 1u) * 1024u + (v & 1023u)], 1u);
    }
    __syncthreads();
    {
        unsigned b, below, size;
        wave_rank_bin(hist + s_g2[wave] * 1024u, 1024 / 64, s_rank[wave], &b, &below, &size);
        if (lane == 0) {
            s_pre[wave] = (s_pre[wave] << 10) | b;
            s_rank[wave] -= below;
            s_id[wave] = 0xFFFFFFFFu;               // every tie at the distance belongs
            if (size > s_rank[wave]) atomicOr(&s_split, 1u << wave);
        }
    }
    __syncthreads();
    // Ties split by id: the s_rank-th smallest id among the ties, 4 x 8 bits.
    for (unsigned todo = s_split; todo; todo &= todo - 1u) {
        const int t = __builtin_ctz(todo);
        const unsigned vt = s_pre[t], rt = s_rank[t];
        if (t > 0 && vt == s_pre[t - 1] && rt == s_rank[t - 1]) {
            if (tid == 0) s_id[t] = s_id[t - 1];
            __syncthreads();
            continue;
        }
        auto id_of_tie = [&](int i, bool& on) {
            on = dist_bits(i) == vt;
            return (uint32_t)i;
        };
        unsigned r = rt;
        unsigned id = select_digit_stream(id_of_tie, n, 24, 8, 0u, r, hist, tmp, s_sel);
        id = select_digit_stream(id_of_tie, n, 16, 8, id, r, hist, tmp, s_sel);
        id = select_digit_stream(id_of_tie, n, 8, 8, id, r, hist, tmp, s_sel);
        id = select_digit_stream(id_of_tie, n, 0, 8, id, r, hist, tmp, s_sel);
        if (tid == 0) s_id[t] = id;
        __syncthreads();
    }

    // Sums of the distances below each target's (as in k_kgrid_thresh).
    const uint32_t vtop = s_pre[kMaxGrid - 1];
    for (int i0 = 0; i0 < n; i0 += kThreshThreads) {
        const int i = i0 + tid;
        const uint32_t v = i < n ? dist_bits(i) : 0xFFFFFFFFu;
        const bool in = v < vtop;
        const unsigned long long bal = __ballot(in);
        unsigned base = 0u;
        if (lane == 0 && bal) base = atomicAdd(&s_fill, (unsigned)__popcll(bal));
        base = __shfl(base, 0, 64);
        const unsigned pos = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (in && pos < (unsigned)kMaxKGridK) list[pos] = v;
    }
    __syncthreads();
    const int m = (int)min(s_fill, (unsigned)kMaxKGridK);
    uint32_t vt[kMaxGrid];
#pragma unroll
    for (int t = 0; t < kMaxGrid; ++t) vt[t] = s_pre[t];
    double part[kMaxGrid];
#pragma unroll
    for (int t = 0; t < kMaxGrid; ++t) part[t] = 0.0;
    for (int x = tid; x < m; x += kThreshThreads) {
        const uint32_t v = list[x];
        int c = 0;
#pragma unroll
        for (int t = 0; t < kMaxGrid; ++t) c += v >= vt[t] ? 1 : 0;
        const double dv = (double)sqrtf(__uint_as_float(v));
#pragma unroll
        for (int t = 0; t < kMaxGrid; ++t) part[t] += c == t ? dv : 0.0;
    }
    {
        double run = 0.0;
#pragma unroll
        for (int t = 0; t < kMaxGrid; ++t) {
            run += wave_scan_dpp(part[t]);
            if (lane == 63) s_part[wave][t] = run;
        }
    }
    __syncthreads();
    if (tid < kMaxGrid) {
        const int t = tid;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < kThreshThreads / 64; ++w) sum += s_part[w][t];
        sum += (double)s_rank[t] * (double)sqrtf(__uint_as_float(vt[t]));
        J.thr[(int64_t)qid * kMaxGrid + t] = ((uint64_t)vt[t] << 32) | (uint64_t)s_id[t];
        if (t < g) J.kmean[(int64_t)t * n + qid] = (float)(sum / (double)J.k[t]);
    }
}

// Four 64-object tiles of one job per workgroup, lane = object p.  The
// queries come in chunks of 256, their coordinates and thresholds staged in
// LDS by the whole workgroup; p is among the k_j nearest of query q exactly
// when its (distance, id) key is at most q's j-th threshold, which each lane
// counts for all sixteen (padded) grid points in registers.
constexpr int kIndegWaves = 4;
constexpr int kIndegChunk = 256;

template <int D>
__global__ __launch_bounds__(64 * kIndegWaves) void k_kgrid_indeg(const KGridJob* jobs, const int32_t* group_prefix,
                                                                  int n_jobs) {
    __shared__ __align__(16) uint64_t s_thr[kIndegChunk][kMaxGrid];
    __shared__ float s_c[D][kIndegChunk];
    const int jb = kjob_of(group_prefix, n_jobs, blockIdx.x);
    const KGridJob& J = jobs[jb];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int n = J.n;
    const int g = J.g;
    const int p = ((blockIdx.x - group_prefix[jb]) * kIndegWaves + wave) * kTile + lane;
    const bool valid = p < n;
    const int pr = valid ? p : n - 1;
    float pc[D];
#pragma unroll
    for (int f = 0; f < D; ++f) pc[f] = J.cols[(int64_t)J.feat[f] * J.ld + pr];
    unsigned cnt[kMaxGrid];
#pragma unroll
    for (int t = 0; t < kMaxGrid; ++t) cnt[t] = 0u;
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    for (int c0 = 0; c0 < n; c0 += kIndegChunk) {
        const int m = min(kIndegChunk, n - c0);
        const u4* src = reinterpret_cast<const u4*>(J.thr + (int64_t)c0 * kMaxGrid);
        u4* dst = reinterpret_cast<u4*>(&s_thr[0][0]);
        for (int x = tid; x < m * (kMaxGrid / 2); x += blockDim.x) dst[x] = src[x];
#pragma unroll
        for (int f = 0; f < D; ++f)
            for (int x = tid; x < m; x += blockDim.x) s_c[f][x] = J.cols[(int64_t)J.feat[f] * J.ld + c0 + x];
        __syncthreads();
#pragma unroll 2
        for (int x = 0; x < m; ++x) {
            float dd = 0.f;
#pragma unroll
            for (int f = 0; f < D; ++f) {
                const float tq = s_c[f][x] - pc[f];                             // query minus object
                dd = fmaf(tq, tq, dd);
            }
            const uint64_t key = p == c0 + x ? ~0ull : (((uint64_t)__float_as_uint(dd) << 32) | (uint64_t)(uint32_t)p);
#pragma unroll
            for (int t = 0; t < kMaxGrid; ++t) cnt[t] += key <= s_thr[x][t] ? 1u : 0u;
        }
        __syncthreads();
    }
    if (!valid) return;
#pragma unroll
    for (int t = 0; t < kMaxGrid; ++t)
        if (t < g) J.indeg[(int64_t)t * n + p] = (int32_t)cnt[t];
}

using KThreshFn = void (*)(const KGridJob*, const int32_t*, int, int);
using KIndegFn = void (*)(const KGridJob*, const int32_t*, int);

template <int D>
void kgrid_fns(KThreshFn* a, KIndegFn* b, bool stream) {
    *a = stream ? k_kgrid_thresh_stream<D> : k_kgrid_thresh<D>;
    *b = k_kgrid_indeg<D>;
}

bool kgrid_pick(int d, KThreshFn* a, KIndegFn* b, bool stream) {
    switch (d) {
        case 2: kgrid_fns<2>(a, b, stream); return true;
        case 3: kgrid_fns<3>(a, b, stream); return true;
        case 4: kgrid_fns<4>(a, b, stream); return true;
        case 5: kgrid_fns<5>(a, b, stream); return true;
        case 6: kgrid_fns<6>(a, b, stream); return true;
        case 7: kgrid_fns<7>(a, b, stream); return true;
        case 8: kgrid_fns<8>(a, b, stream); return true;
        case 9: kgrid_fns<9>(a, b, stream); return true;
        case 10: kgrid_fns<10>(a, b, stream); return true;
        case 11: kgrid_fns<11>(a, b, stream); return true;
        case 12: kgrid_fns<12>(a, b, stream); return true;
        case 13: kgrid_fns<13>(a, b, stream); return true;
        case 14: kgrid_fns<14>(a, b, stream); return true;
        case 15: kgrid_fns<15>(a, b, stream); return true;
        case 16: kgrid_fns<16>(a, b, stream); return true;
    }
    return false;
}

}  // namespace

int kgrid_tiles_per_group() { return kIndegWaves; }

hipError_t launch_kgrid(const KGridJob* jobs, const int32_t* query_prefix, const int32_t* group_prefix, int n_jobs,
                        int total_queries, int total_groups, int d, bool stream, hipStream_t s) {
    KThreshFn thresh;
    KIndegFn indeg;
    if (!kgrid_pick(d, &thresh, &indeg, stream)) return hipErrorInvalidValue;
    if (n_jobs <= 0) return hipSuccess;
    // A dispatch counts its work-items in 32 bits: launches of at most 2^21
    // workgroups of 1024.
    constexpr int kMaxBlocks = 1 << 21;
    for (int b0 = 0; b0 < total_queries; b0 += kMaxBlocks) {
        const int nb = min(kMaxBlocks, total_queries - b0);
        hipLaunchKernelGGL(thresh, dim3(nb), dim3(kThreshThreads), 0, s, jobs, query_prefix, n_jobs, b0);
    }
    hipLaunchKernelGGL(indeg, dim3(total_groups), dim3(64 * kIndegWaves), 0, s, jobs, group_prefix, n_jobs);
    return hipGetLastError();
}

}  // namespace snaps
