// C ABI of libsnaps: argument validation, workspace layout, job tables and
// the launch sequence of the similarity self-join passes.
#include "snaps_internal.h"
#include "serve_internal.h"
#include "../../include/snaps.h"

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace snaps {
hipError_t launch_rank_single(const DevJob& j, hipStream_t s);
}

using namespace snaps;

namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SNAPS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr int64_t kMaxN = int64_t(1) << 30;   // objects per job (ids and tile counts stay in int32)
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Defaults of the walk when neither the call nor the job sets them: box
// pruning up to d = 14 on min(d, 4) indexed dimensions (what the autotuner
// picks for most classes of the SNAPShot1-shaped run; fewer dimensions cut
// each one finer), brute force above.  Serving states keep min(d, 6).
constexpr int kDefaultIndexDims = 4;
constexpr int kDefaultPruneMaxD = 14;

int popcount32(uint32_t m) { return __builtin_popcount(m); }

int ceil_log2(int64_t v) {
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

int check_population(const snaps_population* P, uint32_t mask) {
    if (!P) return fail(SNAPS_EINVAL, "population is NULL");
    if (!P->cols) return fail(SNAPS_EINVAL, "population columns are NULL");
    if (P->n < 2) return fail(SNAPS_EINVAL, "population needs n >= 2 objects (n = %lld)", (long long)P->n);
    if (P->ld < P->n) return fail(SNAPS_EINVAL, "leading dimension %lld < n %lld", (long long)P->ld, (long long)P->n);
    if (P->n_features < 2 || P->n_features > 32)
        return fail(SNAPS_EINVAL, "n_features must be in [2, 32] (got %d)", P->n_features);
    if (P->n_features < 32 && (mask >> P->n_features) != 0)
        return fail(SNAPS_EINVAL, "mask 0x%x names features beyond n_features = %d", mask, P->n_features);
    const int d = popcount32(mask);
    if (d < 2 || d > kMaxD) return fail(SNAPS_EINVAL, "subspace needs 2..%d features (mask 0x%x has %d)", kMaxD, mask, d);
    if (P->n > kMaxN)
        return fail(SNAPS_EUNSUPPORTED, "n = %lld objects exceeds this version's limit of %lld per job",
                    (long long)P->n, (long long)kMaxN);
    return SNAPS_OK;
}

int check_k(int64_t n, int32_t k) {
    if (k < 1 || k > n - 1) return fail(SNAPS_EINVAL, "k must be in [1, n-1] (k = %d, n = %lld)", k, (long long)n);
    return SNAPS_OK;
}

// Sorted kNN lists above kMaxK come from an LDS sort of up to kMaxListK keys.
int check_list_k(int32_t k) {
    if (k > kMaxListK)
        return fail(SNAPS_EUNSUPPORTED, "kNN lists are written for k <= %d (k = %d); the scores take any k", kMaxListK, k);
    return SNAPS_OK;
}

int check_eps(float eps) {
    if (!(eps > 0.f) || !std::isfinite(eps)) return fail(SNAPS_EINVAL, "eps must be positive and finite");
    return SNAPS_OK;
}

int check_tuning(const snaps_tuning* t) {
    if (!t) return SNAPS_OK;
    if (t->mode < 0 || t->mode > 2) return fail(SNAPS_EINVAL, "tuning.mode must be 0, 1 or 2");
    if (!(t->split == 0 || t->split == 1 || t->split == 2 || t->split == 4 || t->split == 8))
        return fail(SNAPS_EINVAL, "tuning.split must be 0, 1, 2, 4 or 8");
    if (t->index_dims < 0 || t->index_dims > kMaxIndexDims) return fail(SNAPS_EINVAL, "tuning.index_dims must be in [0, 6]");
    if (t->filter < 0 || t->filter > 3) return fail(SNAPS_EINVAL, "tuning.filter must be 0, 1, 2 or 3");
    if (t->passes < 0 || t->passes > 7) return fail(SNAPS_EINVAL, "tuning.passes must be a mask of SNAPS_PASS_*");
    if (!(t->mq == 0 || t->mq == 1 || t->mq == 2 || t->mq == 4 || t->mq == 8))
        return fail(SNAPS_EINVAL, "tuning.mq must be 0, 1, 2, 4 or 8");
    if (t->mq > 1 && t->split > 1) return fail(SNAPS_EINVAL, "tuning.mq and tuning.split cannot both exceed 1");
    if (t->index_sort < 0 || t->index_sort > 2) return fail(SNAPS_EINVAL, "tuning.index_sort must be 0, 1 or 2");
    if (t->tile_shape < 0 || t->tile_shape > 3) return fail(SNAPS_EINVAL, "tuning.tile_shape must be 0, 1, 2 or 3");
    return SNAPS_OK;
}

// Device properties, cached per device.
struct DeviceInfo {
    int cus = 0;
};

std::mutex g_dev_mu;
std::map<int, DeviceInfo> g_dev;

int device_info(DeviceInfo* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev.find(dev);
    if (it == g_dev.end()) {
        DeviceInfo di;
        e = hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        it = g_dev.emplace(dev, di).first;
    }
    *out = it->second;
    return SNAPS_OK;
}

// What one job needs, decided on the host.
struct JobPlan {
    int32_t n, d, k, kc, ntiles, nchunks;
    bool bigk;               // k above the fused join's lists: kNN metrics by the selection kernel
    bool large;              // index through the device-wide radix sort (full 32-bit cell keys)
    bool large_rank;         // ranks through the device-wide radix sort (n above one LDS)
    bool rank;               // rank scratch reserved
    int32_t nsuper;
    size_t xs_off, perm_off, box_off, sbox_off, hbox_off;
    size_t ihist_off, acc_off, sel_off;          // large index scratch
    size_t rkey_off, rpong_off, rhist_off, rnd_off;  // large rank scratch
    size_t bytes;
};

// Index sort of a job: kIndexAuto (the device-wide radix sort), kIndexPacked
// (object id packed under the cell key in 32 bits and sorted in one LDS;
// coarser cells, only for n within one LDS) or kIndexRadix.  force_large also
// ranks through the device-wide path (the serving state keeps its sorted keys).
constexpr int kIndexAuto = 0, kIndexPacked = 1, kIndexRadix = 2;

JobPlan plan_job(int64_t n, int d, int k, bool with_rank, int index_sort = kIndexAuto, bool force_large = false) {
    JobPlan p{};
    p.n = (int32_t)n;
    p.d = d;
    p.k = k;
    p.bigk = k > kMaxK;
    p.kc = p.bigk ? 0 : kc_class(k);        // the fused join then runs the eps side only
    p.ntiles = (int32_t)((n + kTile - 1) / kTile);
    p.nchunks = (int32_t)((n + kRadixChunk - 1) / kRadixChunk);
    p.large_rank = force_large || n > kLdsSortMax;
    p.large = p.large_rank || index_sort != kIndexPacked;
    p.rank = with_rank;
    const size_t rows = (size_t)p.ntiles * kTile;
    const int dp = row_stride(d);
    size_t off = 0;
    // xs also hosts the large-index sort keys (3 x rows words <= rows x dp
    // floats) before the reorder overwrites it with coordinates.
    p.xs_off = off;
    off += align_up(rows * dp * sizeof(float));
    p.perm_off = off;
    off += align_up(rows * sizeof(int32_t));
    p.box_off = off;
    off += align_up((size_t)p.ntiles * 2 * dp * sizeof(float));
    p.nsuper = (p.ntiles + kSuper - 1) / kSuper;
    p.sbox_off = off;
    off += align_up((size_t)p.nsuper * 2 * dp * sizeof(float));
    p.hbox_off = off;
    off += align_up((size_t)p.ntiles * 4 * dp * sizeof(float));
    if (p.large) {
        p.ihist_off = off;
        off += align_up((size_t)256 * p.nchunks * sizeof(int32_t));
        p.acc_off = off;
        off += align_up(2 * kMaxD * sizeof(double));
        p.sel_off = off;
        off += align_up(3 * kMaxIndexDims * sizeof(float));
        if (with_rank && p.large_rank) {
            p.rkey_off = off;
            off += align_up(4 * rows * sizeof(uint32_t));
            p.rpong_off = off;
            off += align_up(4 * rows * sizeof(uint32_t));
            p.rhist_off = off;
            off += align_up((size_t)4 * 256 * p.nchunks * sizeof(int32_t));
            p.rnd_off = off;
            off += align_up(4 * sizeof(int32_t));
        }
    }
    p.bytes = off;
    return p;
}

// Kernel classes of the join: (dimensionality, top-k capacity, walk).
constexpr int kNumClasses = (kMaxD + 1) * 5 * 2;
int class_id(int d, int kc, int hier) {
    const int ki = kc == 0 ? 0 : kc == 5 ? 1 : kc == 10 ? 2 : kc == 20 ? 3 : 4;
    return (d * 5 + ki) * 2 + (hier ? 1 : 0);
}
constexpr int kKcOfClass[5] = {0, 5, 10, 20, 32};
int class_d(int c) { return c / 10; }
int class_kc(int c) { return kKcOfClass[(c / 2) % 5]; }
int class_hier(int c) { return c % 2; }

// Tile shape of a job (snaps_tuning.tile_shape): 1 = the lean walk over
// 64-candidate tiles, 2 = super-tile culls and 32-candidate halves, 3 =
// super-tile culls over whole tiles.  Automatic: 3 for pruned jobs with at
// least kHierMinSupers super-tiles, else 1.
constexpr int kHierMinSupers = 16;
int resolve_shape(int shape, const JobPlan& p, int prune) {
    if (shape == 0) shape = (prune && p.nsuper >= kHierMinSupers) ? 3 : 1;
    return shape;
}
bool shape_hier(int shape, int prune) { return prune && (shape == 2 || shape == 3); }

struct MetaLayout {
    size_t table, order, unit_prefix, tile_prefix, super_prefix, counters;
    size_t li, iseg, ichunk, lr, rseg, rchunk, rsegchunk, bigk, bigk_prefix;
    size_t bytes;
};

// Selection-kernel classes: dimensionality 2..16, with or without lists.
constexpr int kBigKClasses = (kMaxD + 1) * 2;

MetaLayout meta_layout(int n_jobs, int n_large, int n_lrank, int n_bigk = 0) {
    MetaLayout m{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    m.table = take((size_t)n_jobs * sizeof(DevJob));
    m.order = take((size_t)n_jobs * sizeof(int32_t));
    m.unit_prefix = take((size_t)(n_jobs + kNumClasses * kQueues) * sizeof(int32_t));
    m.tile_prefix = take((size_t)(n_jobs + 1) * sizeof(int32_t));
    m.super_prefix = take((size_t)(n_jobs + 1) * sizeof(int32_t));
    m.counters = take((size_t)kNumClasses * kQueues * sizeof(int32_t));
    m.li = take((size_t)n_large * sizeof(LargeIndex));
    m.iseg = take((size_t)n_large * sizeof(SortSeg));
    m.ichunk = take((size_t)(n_large + 1) * sizeof(int32_t));
    m.lr = take((size_t)n_lrank * sizeof(LargeRank));
    m.rseg = take((size_t)4 * n_lrank * sizeof(SortSeg));
    m.rchunk = take((size_t)(n_lrank + 1) * sizeof(int32_t));
    m.rsegchunk = take((size_t)(4 * n_lrank + 1) * sizeof(int32_t));
    m.bigk = take((size_t)n_bigk * sizeof(BigKJob));
    m.bigk_prefix = take((size_t)(n_bigk > 0 ? n_bigk + kBigKClasses : 0) * sizeof(int64_t));
    m.bytes = off;
    return m;
}

struct Tune {
    int mode = 0, split = 0, index_dims = 0, filter = 0, passes = 7, mq = 0, tile_shape = 0;
    unsigned long long* stats = nullptr;
};

Tune resolve_tune(const snaps_tuning* t) {
    Tune r;
    if (t) {
        r.mode = t->mode;
        r.split = t->split;
        r.index_dims = t->index_dims;
        r.filter = t->filter;
        r.passes = t->passes ? t->passes : 7;
        r.mq = t->mq;
        r.tile_shape = t->tile_shape;
        r.stats = reinterpret_cast<unsigned long long*>(t->stats);
    }
    return r;
}

// Fill the device-side description of one job.
DevJob make_devjob(const snaps_population* P, uint32_t mask, const JobPlan& p, float eps, const Tune& tn,
                   char* ws_base) {
    DevJob j;
    std::memset(&j, 0, sizeof(j));
    j.cols = P->cols;
    j.ld = P->ld;
    j.n = p.n;
    j.d = p.d;
    j.k = p.k;
    j.ntiles = p.ntiles;
    j.eps2 = eps > 0.f ? (float)((double)eps * (double)eps) : -1.f;
    int c = tn.index_dims > 0 ? std::min(tn.index_dims, p.d) : std::min(p.d, kDefaultIndexDims);
    j.c = c;
    int f = 0;
    for (int b = 0; b < 32; ++b)
        if ((mask >> b) & 1u) j.feat[f++] = b;
    if (p.large) {
        // keys are sorted with the id as a separate payload: all 32 bits
        j.idbits = 0;
        j.bits = 32 / c;
    } else {
        j.idbits = std::max(1, ceil_log2(p.n));
        j.bits = std::max(1, (32 - j.idbits) / c);
    }
    j.flags = (p.large ? kJobRadixIndex : 0) | (p.large_rank ? kJobRadixRank : 0);
    if (tn.mode == 1) j.prune = 0;
    else if (tn.mode == 2) j.prune = 1;
    else j.prune = p.d <= kDefaultPruneMaxD ? 1 : 0;
    j.xs = reinterpret_cast<float*>(ws_base + p.xs_off);
    j.perm = reinterpret_cast<int32_t*>(ws_base + p.perm_off);
    j.boxes = reinterpret_cast<float*>(ws_base + p.box_off);
    j.sboxes = reinterpret_cast<float*>(ws_base + p.sbox_off);
    j.hboxes = reinterpret_cast<float*>(ws_base + p.hbox_off);
    j.nsuper = p.nsuper;
    const int shape = resolve_shape(tn.tile_shape, p, j.prune);
    j.halves = shape == 2 && j.prune ? 1 : 0;
    j.hier = shape_hier(shape, j.prune) ? 1 : 0;
    return j;
}

constexpr size_t kMaxJoinLds = 120 * 1024;

// Query tiles from which the matrix-core kernel (one wavefront per tile)
// beats the split vector-ALU kernel even with SIMDs left idle (measured on
// MI355X over single jobs of 500 to 31,693 objects, d = 2..15: about equal at
// 32 tiles, 7-12 % faster at 63, 25-45 % at 250 and more).
constexpr int64_t kMfmaMinUnits = 48;

int choose_split(const Tune& tn, int64_t total_units, int cus, int kc, bool mfma) {
    int s = 1;
    if (tn.split > 0) {
        s = tn.split;
    } else if (mfma && total_units >= kMfmaMinUnits) {
        s = 1;
    } else {
        // Aim for about eight wavefronts per SIMD (four SIMDs per CU).
        const int64_t target = (int64_t)cus * 4 * 8;
        while (s < 8 && total_units * s < target) s <<= 1;
    }
    while (s > 1 && join_lds_bytes(kc, s) > kMaxJoinLds) s >>= 1;
    return s;
}

// Waves per lockstep workgroup: off unless asked for (measured on MI355X: the
// per-tile barrier costs more than the shared scalar-cache lines save when
// tiles are pruned).
int choose_mq(const Tune& tn, int64_t units1, int cus) {
    (void)units1;
    (void)cus;
    if (tn.split > 1) return 1;
    return tn.mq > 0 ? tn.mq : 1;
}

// Per kernel class: its jobs dealt round-robin (most expensive first) over
// the per-XCD work queues.
struct ClassPlan {
    int count = 0;
    int units = 0;
    int q_order_off[kQueues] = {};
    int q_prefix_off[kQueues] = {};
    int q_jobs[kQueues] = {};
    int q_units[kQueues] = {};
};

// Launch the join kernels of every class present.
int launch_joins(const Meta& meta, const std::vector<ClassPlan>& plans, const Tune& tn, int mq, int cus,
                 hipStream_t s) {
    int64_t all_units = 0;
    for (const auto& p : plans) all_units += p.units;
    // auto: the matrix-core prefilter (the vector-ALU one where the work unit
    // spans several wavefronts)
    const int xf_pref = tn.filter == 1 ? 0 : tn.filter == 2 ? 1 : 2;
    hipError_t fe = launch_fill_i32(meta.counters, meta.n_counters, 0, s);
    if (fe != hipSuccess) return hip_fail(fe, "counter reset");
    for (int c = 0; c < kNumClasses; ++c) {
        const ClassPlan& p = plans[c];
        if (p.count == 0) continue;
        const int d = class_d(c);
        const int kc = class_kc(c);
        const int hier = class_hier(c);
        const int split = mq > 1 ? 1 : choose_split(tn, all_units, cus, kc, xf_pref == 2);
        // the matrix-core kernel runs one wavefront per query tile
        const int xf = (xf_pref == 2 && (split > 1 || mq > 1)) ? 1 : xf_pref;
        JoinArgs a{};
        a.table = meta.table;
        a.order = meta.order;
        a.unit_prefix = meta.unit_prefix;
        for (int q = 0; q < kQueues; ++q) {
            a.q_order_off[q] = p.q_order_off[q];
            a.q_prefix_off[q] = p.q_prefix_off[q];
            a.q_jobs[q] = p.q_jobs[q];
            a.q_units[q] = p.q_units[q];
        }
        a.counter = meta.counters + c * kQueues;
        a.split = split;
        a.mq = mq;
        a.stats = tn.stats;
        const int per_cu = join_blocks_per_cu(d, kc, xf, hier, split, mq);
        if (per_cu <= 0) return fail(SNAPS_EDEVICE, "no occupancy for join kernel d=%d kc=%d split=%d", d, kc, split);
        int grid = std::min<int64_t>((int64_t)per_cu * cus, p.units);
        hipError_t e = launch_join(d, kc, xf, hier, a, grid, s);
        if (e != hipSuccess) return hip_fail(e, "join kernel launch");
    }
    return SNAPS_OK;
}

// Shared driver of every entry point: jobs already validated and planned.
struct RunJob {
    const snaps_population* pop;
    uint32_t mask;
    float eps;              // <= 0: no range join
    JobPlan plan;
    int32_t* eps_count;
    float* eps_mean;
    int32_t* indeg;
    float* knn_mean;
    int32_t* rank;
    float* ensemble;
    int32_t* knn_ids;
    float* knn_dist;
    float* knn_kth;
    int64_t* pair_off;      // eps-only pair lists (snaps_eps_selfjoin)
    int32_t* pairs;
    int64_t pair_cap;
    int32_t mode;           // per-job overrides of the call's tuning (0: none)
    int32_t index_dims;
    int32_t tile_shape;
};

void count_large(const std::vector<RunJob>& jobs, int* n_large, int* n_lrank) {
    *n_large = 0;
    *n_lrank = 0;
    for (const auto& j : jobs) {
        if (j.plan.large) ++*n_large;
        if (j.plan.large_rank && j.rank) ++*n_lrank;
    }
}

int count_bigk(const std::vector<RunJob>& jobs) {
    int c = 0;
    for (const auto& j : jobs) c += j.plan.bigk ? 1 : 0;
    return c;
}

size_t run_workspace(const std::vector<RunJob>& jobs) {
    int nl = 0, nr = 0;
    count_large(jobs, &nl, &nr);
    size_t b = meta_layout((int)jobs.size(), nl, nr, count_bigk(jobs)).bytes;
    for (const auto& j : jobs) b += j.plan.bytes;
    return b;
}

std::vector<uint8_t>& staging() {
    thread_local std::vector<uint8_t> buf;
    return buf;
}

// How run() treats the metadata block of a multi-job or large-job call:
// upload it and launch (normal calls), upload only (before a graph capture),
// or launch only (inside a capture, after an upload of the same jobs).
enum class RunMode { Full, UploadOnly, LaunchOnly };

int run(const std::vector<RunJob>& jobs, const Tune& tn, void* ws, size_t ws_bytes, hipStream_t s,
        RunMode mode = RunMode::Full) {
    const int n_jobs = (int)jobs.size();
    const size_t need = run_workspace(jobs);
    if (!ws && need > 0) return fail(SNAPS_EINVAL, "workspace is NULL (%zu bytes needed)", need);
    if (ws_bytes < need) return fail(SNAPS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != SNAPS_OK) return rc;
    int n_large = 0, n_lrank = 0;
    count_large(jobs, &n_large, &n_lrank);
    const int n_bigk = count_bigk(jobs);

    char* base = static_cast<char*>(ws);
    const MetaLayout ml = meta_layout(n_jobs, n_large, n_lrank, n_bigk);
    Meta meta{};
    meta.table = reinterpret_cast<DevJob*>(base + ml.table);
    meta.order = reinterpret_cast<int32_t*>(base + ml.order);
    meta.unit_prefix = reinterpret_cast<int32_t*>(base + ml.unit_prefix);
    meta.tile_prefix = reinterpret_cast<int32_t*>(base + ml.tile_prefix);
    meta.super_prefix = reinterpret_cast<int32_t*>(base + ml.super_prefix);
    meta.counters = reinterpret_cast<int32_t*>(base + ml.counters);
    meta.n_counters = kNumClasses * kQueues;

    std::vector<DevJob> table(n_jobs);
    std::vector<char*> job_base(n_jobs);
    size_t off = ml.bytes;
    int64_t total_tiles = 0;
    std::vector<int32_t> tile_prefix(n_jobs + 1, 0);
    std::vector<int32_t> super_prefix(n_jobs + 1, 0);
    int64_t total_supers = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const RunJob& r = jobs[i];
        job_base[i] = base + off;
        Tune tj = tn;
        if (r.mode > 0) tj.mode = r.mode;
        if (r.index_dims > 0) tj.index_dims = r.index_dims;
        if (r.tile_shape > 0) tj.tile_shape = r.tile_shape;
        DevJob j = make_devjob(r.pop, r.mask, r.plan, r.eps, tj, base + off);
        j.eps_count = r.eps_count;
        j.eps_mean = r.eps_mean;
        j.indeg = r.indeg;
        j.knn_mean = r.knn_mean;
        j.rank = r.rank;
        j.ensemble = r.rank ? r.ensemble : nullptr;
        j.knn_ids = r.knn_ids;
        j.knn_dist = r.knn_dist;
        j.knn_kth = r.knn_kth;
        j.pair_off = r.pair_off;
        j.pairs = r.pairs;
        j.pair_cap = r.pair_cap;
        table[i] = j;
        off += r.plan.bytes;
        total_tiles += r.plan.ntiles;
        if (total_tiles > INT32_MAX / 2) return fail(SNAPS_EUNSUPPORTED, "too many tiles in one call");
        tile_prefix[i + 1] = (int32_t)total_tiles;
        total_supers += r.plan.nsuper;
        super_prefix[i + 1] = (int32_t)total_supers;
    }

    // Jobs with k above the fused join's lists: their kNN side runs in the
    // selection kernel, one launch per (dimensionality, lists) class.
    std::vector<std::vector<BigKJob>> bk_cls(kBigKClasses);
    for (int i = 0; i < n_jobs; ++i) {
        const RunJob& r = jobs[i];
        if (!r.plan.bigk) continue;
        BigKJob b{};
        b.cols = r.pop->cols;
        b.ld = r.pop->ld;
        b.n = r.plan.n;
        b.k = r.plan.k;
        for (int f = 0; f < kMaxD; ++f) b.feat[f] = table[i].feat[f];
        b.indeg = r.indeg;
        b.knn_mean = r.knn_mean;
        b.ids = r.knn_ids;
        b.dist = r.knn_dist;
        bk_cls[r.plan.d * 2 + (r.knn_ids ? 1 : 0)].push_back(b);
    }
    std::vector<BigKJob> bk_table;
    std::vector<int64_t> bk_prefix;
    std::vector<int> bk_off(kBigKClasses), bk_poff(kBigKClasses);
    std::vector<int64_t> bk_queries(kBigKClasses, 0);
    if (n_bigk > 0) {
        for (int c = 0; c < kBigKClasses; ++c) {
            bk_off[c] = (int)bk_table.size();
            bk_poff[c] = (int)bk_prefix.size();
            int64_t acc = 0;
            bk_prefix.push_back(0);
            for (const BigKJob& b : bk_cls[c]) {
                bk_table.push_back(b);
                acc += b.n;
                bk_prefix.push_back(acc);
            }
            bk_queries[c] = acc;
            if (acc > INT32_MAX) return fail(SNAPS_EUNSUPPORTED, "too many queries of large k in one call");
        }
    }

    // Group jobs into kernel classes (dimensionality, top-k capacity); within
    // a class, the most expensive jobs (largest n) first, dealt round-robin
    // over the per-XCD queues.
    std::vector<std::vector<int>> members(kNumClasses);
    std::vector<int> job_class(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        job_class[i] = class_id(jobs[i].plan.d, jobs[i].plan.kc, table[i].hier);
        members[job_class[i]].push_back(i);
    }
    int64_t units1 = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const int ql = join_ql(jobs[i].plan.kc);
        units1 += (jobs[i].plan.ntiles + ql - 1) / ql;
    }
    const int mq = choose_mq(tn, units1, di.cus);
    std::vector<ClassPlan> plans(kNumClasses);
    std::vector<int32_t> order;
    std::vector<int32_t> unit_prefix;
    order.reserve(n_jobs);
    unit_prefix.reserve(n_jobs + kNumClasses * kQueues);
    for (int c = 0; c < kNumClasses; ++c) {
        auto& m = members[c];
        std::stable_sort(m.begin(), m.end(), [&](int a, int b) { return jobs[a].plan.n > jobs[b].plan.n; });
        ClassPlan& p = plans[c];
        p.count = (int)m.size();
        if (p.count == 0) continue;
        const int per_unit = join_ql(class_kc(c)) * mq;      // query tiles per work unit
        for (int q = 0; q < kQueues; ++q) {
            p.q_order_off[q] = (int)order.size();
            p.q_prefix_off[q] = (int)unit_prefix.size();
            int64_t acc = 0;
            unit_prefix.push_back(0);
            for (size_t t = q; t < m.size(); t += kQueues) {
                const int i = m[t];
                order.push_back(i);
                acc += (jobs[i].plan.ntiles + per_unit - 1) / per_unit;
                unit_prefix.push_back((int32_t)acc);
            }
            p.q_jobs[q] = (int)((m.size() + kQueues - 1 - q) / kQueues);
            p.q_units[q] = (int)acc;
            p.units += (int)acc;
        }
    }

    // Device-wide sort descriptors of the large jobs.
    std::vector<LargeIndex> lidx;
    std::vector<SortSeg> iseg;
    std::vector<int32_t> ichunk(1, 0);
    std::vector<LargeRank> lrank;
    std::vector<SortSeg> rseg;
    std::vector<int32_t> rchunk(1, 0), rsegchunk(1, 0);
    int32_t* rank_nd_base = nullptr;
    (void)rank_nd_base;
    for (int i = 0; i < n_jobs; ++i) {
        const JobPlan& p = jobs[i].plan;
        if (!p.large) continue;
        char* jb = job_base[i];
        const size_t rows = (size_t)p.ntiles * kTile;
        uint32_t* xs_words = reinterpret_cast<uint32_t*>(jb + p.xs_off);
        LargeIndex L{};
        L.job = i;
        L.nchunks = p.nchunks;
        L.acc = reinterpret_cast<double*>(jb + p.acc_off);
        L.sel_col = reinterpret_cast<int32_t*>(jb + p.sel_off);
        L.sel_lo = reinterpret_cast<float*>(jb + p.sel_off) + kMaxIndexDims;
        L.sel_scale = reinterpret_cast<float*>(jb + p.sel_off) + 2 * kMaxIndexDims;
        L.keys = xs_words;
        L.vals = reinterpret_cast<uint32_t*>(table[i].perm);
        lidx.push_back(L);
        SortSeg g{};
        g.key[0] = xs_words;
        g.key[1] = xs_words + rows;
        g.val[0] = L.vals;
        g.val[1] = xs_words + 2 * rows;
        g.hist = reinterpret_cast<int32_t*>(jb + p.ihist_off);
        g.n = p.n;
        g.nchunks = p.nchunks;
        iseg.push_back(g);
        ichunk.push_back(ichunk.back() + p.nchunks);
        if (jobs[i].rank && p.large_rank) {
            LargeRank R{};
            R.job = i;
            R.nchunks = p.nchunks;
            R.n_distinct = reinterpret_cast<int32_t*>(jb + p.rnd_off);
            for (int m = 0; m < 4; ++m) {
                R.keys[m] = reinterpret_cast<uint32_t*>(jb + p.rkey_off) + m * rows;
                R.distinct[m] = reinterpret_cast<uint32_t*>(jb + p.rpong_off) + m * rows;
                SortSeg rg{};
                rg.key[0] = R.keys[m];
                rg.key[1] = R.distinct[m];
                rg.val[0] = rg.val[1] = nullptr;
                rg.hist = reinterpret_cast<int32_t*>(jb + p.rhist_off) + (size_t)m * 256 * p.nchunks;
                rg.n = p.n;
                rg.nchunks = p.nchunks;
                rseg.push_back(rg);
                rsegchunk.push_back(rsegchunk.back() + p.nchunks);
            }
            lrank.push_back(R);
            rchunk.push_back(rchunk.back() + p.nchunks);
        }
    }

    hipError_t e;
    const bool do_index = (tn.passes & SNAPS_PASS_INDEX) != 0;
    const bool do_join = (tn.passes & SNAPS_PASS_JOIN) != 0;
    const bool do_rank = (tn.passes & SNAPS_PASS_RANK) != 0;
    const bool seed_single = (n_jobs == 1 && n_large == 0 && n_bigk == 0);
    if (seed_single) {
        // The metadata of a single small job is written by its index kernel
        // from kernel arguments (no host-to-device copy); later passes of the
        // same job reuse it.
        // (the single job is the first entry of order and unit_prefix)
        if (do_index && mode != RunMode::UploadOnly) {
            IndexArgs ia{};
            ia.meta = meta;
            ia.n_jobs = 1;
            ia.seed = 1;
            const ClassPlan& p = plans[job_class[0]];
            ia.single_units = p.q_units[0];
            ia.single_tiles = table[0].ntiles;
            ia.single_supers = table[0].nsuper;
            ia.single = table[0];
            e = launch_index_sort(ia, 1, s);
            if (e != hipSuccess) return hip_fail(e, "index sort launch");
        }
    } else if (mode != RunMode::LaunchOnly) {
        // One host-to-device copy of the metadata block (synchronous for
        // pageable host memory, so the staging buffer can be reused).
        auto& st = staging();
        st.assign(ml.bytes, 0);
        auto put = [&](size_t at, const void* src, size_t bytes) {
            if (bytes) std::memcpy(st.data() + at, src, bytes);
        };
        put(ml.table, table.data(), table.size() * sizeof(DevJob));
        put(ml.order, order.data(), order.size() * sizeof(int32_t));
        put(ml.unit_prefix, unit_prefix.data(), unit_prefix.size() * sizeof(int32_t));
        put(ml.tile_prefix, tile_prefix.data(), tile_prefix.size() * sizeof(int32_t));
        put(ml.super_prefix, super_prefix.data(), super_prefix.size() * sizeof(int32_t));
        put(ml.li, lidx.data(), lidx.size() * sizeof(LargeIndex));
        put(ml.iseg, iseg.data(), iseg.size() * sizeof(SortSeg));
        put(ml.ichunk, ichunk.data(), ichunk.size() * sizeof(int32_t));
        put(ml.lr, lrank.data(), lrank.size() * sizeof(LargeRank));
        put(ml.rseg, rseg.data(), rseg.size() * sizeof(SortSeg));
        put(ml.rchunk, rchunk.data(), rchunk.size() * sizeof(int32_t));
        put(ml.rsegchunk, rsegchunk.data(), rsegchunk.size() * sizeof(int32_t));
        put(ml.bigk, bk_table.data(), bk_table.size() * sizeof(BigKJob));
        put(ml.bigk_prefix, bk_prefix.data(), bk_prefix.size() * sizeof(int64_t));
        e = hipMemcpyAsync(base, st.data(), ml.bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "job table upload");
    }
    if (mode == RunMode::UploadOnly) return SNAPS_OK;
    if (!seed_single) {
        if (do_index) {
            IndexArgs ia{};
            ia.meta = meta;
            ia.n_jobs = n_jobs;
            ia.seed = 0;
            e = launch_index_sort(ia, n_jobs, s);
            if (e != hipSuccess) return hip_fail(e, "index sort launch");
            e = launch_large_index(meta.table, reinterpret_cast<const LargeIndex*>(base + ml.li), n_large,
                                   reinterpret_cast<const int32_t*>(base + ml.ichunk), ichunk.back(),
                                   reinterpret_cast<const SortSeg*>(base + ml.iseg), s);
            if (e != hipSuccess) return hip_fail(e, "large index launch");
        }
    }
    if (do_index) {
        e = launch_reorder(meta, n_jobs, (int32_t)total_tiles, s);
        if (e != hipSuccess) return hip_fail(e, "reorder launch");
        e = launch_super_boxes(meta, n_jobs, (int32_t)total_supers, s);
        if (e != hipSuccess) return hip_fail(e, "super-tile boxes launch");
    }
    if (do_join) {
        e = launch_zero_indeg(meta, n_jobs, (int32_t)total_tiles, s);
        if (e != hipSuccess) return hip_fail(e, "in-degree reset launch");
        rc = launch_joins(meta, plans, tn, mq, di.cus, s);
        if (rc != SNAPS_OK) return rc;
        for (int c = 0; c < kBigKClasses; ++c) {
            if (bk_cls[c].empty()) continue;
            BigKArgs ba{};
            ba.table = reinterpret_cast<const BigKJob*>(base + ml.bigk) + bk_off[c];
            ba.prefix = reinterpret_cast<const int64_t*>(base + ml.bigk_prefix) + bk_poff[c];
            ba.n_jobs = (int32_t)bk_cls[c].size();
            e = launch_bigk(c / 2, (c % 2) != 0, ba, bk_queries[c], s);
            if (e != hipSuccess) return hip_fail(e, "large-k selection launch");
        }
    }
    bool any_rank = false;
    for (const auto& j : jobs) any_rank |= (j.rank != nullptr);
    if (do_rank && any_rank) {
        RankArgs ra{meta.table, n_jobs};
        e = launch_rank(ra, s);
        if (e != hipSuccess) return hip_fail(e, "rank launch");
        e = launch_large_rank(meta.table, reinterpret_cast<const LargeRank*>(base + ml.lr), n_lrank,
                              reinterpret_cast<const int32_t*>(base + ml.rchunk), rchunk.back(),
                              reinterpret_cast<const SortSeg*>(base + ml.rseg),
                              reinterpret_cast<const int32_t*>(base + ml.rsegchunk), rsegchunk.back(), s);
        if (e != hipSuccess) return hip_fail(e, "large rank launch");
        bool any_ens = false;
        for (const auto& j : jobs) any_ens |= (j.rank != nullptr && j.ensemble != nullptr);
        if (any_ens) {
            e = launch_ensemble(meta.table, n_jobs, meta.tile_prefix, (int32_t)total_tiles, s);
            if (e != hipSuccess) return hip_fail(e, "ensemble launch");
        }
    }
    return SNAPS_OK;
}

// Workspace of snaps_rank: none for n within one workgroup's LDS, else the
// metadata block plus key, ping-pong and histogram buffers of 4 segments.
size_t rank_workspace(int64_t n) {
    if (n <= kLdsSortMax) return 0;
    const int64_t nchunks = (n + kRadixChunk - 1) / kRadixChunk;
    const size_t rows = (size_t)((n + kTile - 1) / kTile) * kTile;
    return meta_layout(1, 0, 1).bytes + align_up(8 * rows * sizeof(uint32_t)) +
           align_up((size_t)4 * 256 * nchunks * sizeof(int32_t) + 4 * sizeof(int32_t));
}

}  // namespace

extern "C" {

const char* snaps_last_error(void) { return g_error.c_str(); }

const char* snaps_version(void) { return "snaps-mi355x 0.1 (gfx950)"; }

size_t snaps_workspace_bytes(int32_t op, int64_t n, int32_t d, int32_t k) {
    if (n < 2 || n > kMaxN) return 0;
    if (op == SNAPS_OP_RANK) return rank_workspace(n);
    if (d < 2 || d > kMaxD) return 0;
    if (op == SNAPS_OP_EPS) k = 0;
    else if (k < 1 || k > n - 1) return 0;
    if (op != SNAPS_OP_KNN && op != SNAPS_OP_EPS && op != SNAPS_OP_SCORES) return 0;
    if (op == SNAPS_OP_KNN && k > kMaxK) return k > kMaxListK ? 0 : kAlign;   // selection kernel: no workspace
    const JobPlan p = plan_job(n, d, k, op == SNAPS_OP_SCORES);
    const size_t run = meta_layout(1, p.large ? 1 : 0, (p.large_rank && op == SNAPS_OP_SCORES) ? 1 : 0,
                                   p.bigk ? 1 : 0).bytes + p.bytes;
    return op == SNAPS_OP_EPS ? align_up(run) + pair_scan_scratch(n) : run;
}

static int collect_jobs(const snaps_job* jobs, int32_t n_jobs, const snaps_tuning* tune, std::vector<RunJob>* out) {
    const int index_sort = tune ? tune->index_sort : kIndexAuto;
    if (n_jobs < 1) return fail(SNAPS_EINVAL, "n_jobs must be >= 1");
    if (!jobs) return fail(SNAPS_EINVAL, "jobs is NULL");
    out->clear();
    out->reserve(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        const snaps_job& j = jobs[i];
        int rc = check_population(j.pop, j.mask);
        if (rc != SNAPS_OK) return fail(rc, "job %d: %s", i, g_error.c_str());
        rc = check_k(j.pop->n, j.k);
        if (rc != SNAPS_OK) return fail(rc, "job %d: %s", i, g_error.c_str());
        rc = check_eps(j.eps);
        if (rc != SNAPS_OK) return fail(rc, "job %d: %s", i, g_error.c_str());
        if (!j.out.eps_count || !j.out.eps_mean || !j.out.indeg || !j.out.knn_mean)
            return fail(SNAPS_EINVAL, "job %d: every score output array is required", i);
        RunJob r{};
        r.pop = j.pop;
        r.mask = j.mask;
        r.eps = j.eps;
        r.plan = plan_job(j.pop->n, popcount32(j.mask), j.k, j.rank != nullptr, index_sort);
        r.eps_count = j.out.eps_count;
        r.eps_mean = j.out.eps_mean;
        r.indeg = j.out.indeg;
        r.knn_mean = j.out.knn_mean;
        r.rank = j.rank;
        if (j.ensemble && !j.rank) return fail(SNAPS_EINVAL, "job %d: the ensemble output needs the rank output", i);
        r.ensemble = j.ensemble;
        if (j.mode < 0 || j.mode > 2) return fail(SNAPS_EINVAL, "job %d: mode must be 0, 1 or 2", i);
        if (j.index_dims < 0 || j.index_dims > kMaxIndexDims)
            return fail(SNAPS_EINVAL, "job %d: index_dims must be in [0, %d]", i, kMaxIndexDims);
        if (j.tile_shape < 0 || j.tile_shape > 3) return fail(SNAPS_EINVAL, "job %d: tile_shape must be 0, 1, 2 or 3", i);
        if (j.reserved != 0) return fail(SNAPS_EINVAL, "job %d: reserved must be zero", i);
        r.mode = j.mode;
        r.index_dims = j.index_dims;
        r.tile_shape = j.tile_shape;
        if (j.knn_dist && !j.knn_ids) return fail(SNAPS_EINVAL, "job %d: knn_dist needs knn_ids", i);
        if (j.knn_ids && j.k > kMaxK) {
            rc = check_list_k(j.k);
            if (rc != SNAPS_OK) return fail(rc, "job %d: %s", i, g_error.c_str());
        }
        r.knn_ids = j.knn_ids;
        r.knn_dist = j.knn_dist;
        out->push_back(r);
    }
    return SNAPS_OK;
}

size_t snaps_outlier_scores_workspace(const snaps_job* jobs, int32_t n_jobs, const snaps_tuning* tune) {
    std::vector<RunJob> rj;
    if (check_tuning(tune) != SNAPS_OK) return 0;
    if (collect_jobs(jobs, n_jobs, tune, &rj) != SNAPS_OK) return 0;
    return run_workspace(rj);
}

int snaps_knn_selfjoin(const snaps_population* P, uint32_t mask, int32_t k, int32_t* ids, float* dist,
                       void* ws, size_t ws_bytes, void* stream) {
    int rc = check_population(P, mask);
    if (rc != SNAPS_OK) return rc;
    rc = check_k(P->n, k);
    if (rc != SNAPS_OK) return rc;
    if (!ids) return fail(SNAPS_EINVAL, "ids is NULL");
    if (k > kMaxK) {
        // selection kernel, straight from the population's columns
        rc = check_list_k(k);
        if (rc != SNAPS_OK) return rc;
        BigKArgs ba{};
        ba.use_single = 1;
        ba.single.cols = P->cols;
        ba.single.ld = P->ld;
        ba.single.n = (int32_t)P->n;
        ba.single.k = k;
        int f = 0;
        for (int b = 0; b < 32; ++b)
            if ((mask >> b) & 1u) ba.single.feat[f++] = b;
        ba.single.ids = ids;
        ba.single.dist = dist;
        hipError_t e = launch_bigk(popcount32(mask), true, ba, P->n, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "large-k selection launch");
        return SNAPS_OK;
    }
    RunJob r{};
    r.pop = P;
    r.mask = mask;
    r.eps = 0.f;
    r.plan = plan_job(P->n, popcount32(mask), k, false);
    r.knn_ids = ids;
    r.knn_dist = dist;
    return run({r}, Tune{0, 0, 0, 0}, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int snaps_eps_selfjoin(const snaps_population* P, uint32_t mask, float eps, int32_t* count, float* mean_dist,
                       int64_t* pair_off, int32_t* pairs, int64_t pair_cap, void* ws, size_t ws_bytes,
                       void* stream) {
    int rc = check_population(P, mask);
    if (rc != SNAPS_OK) return rc;
    rc = check_eps(eps);
    if (rc != SNAPS_OK) return rc;
    if (!count) return fail(SNAPS_EINVAL, "count is NULL");
    if (!mean_dist) return fail(SNAPS_EINVAL, "mean_dist is NULL");
    if (pair_cap < 0) return fail(SNAPS_EINVAL, "pair_cap must be >= 0");
    if ((pairs || pair_cap > 0) && !pair_off) return fail(SNAPS_EINVAL, "a pair list needs pair_off");
    if (pair_cap > 0 && !pairs) return fail(SNAPS_EINVAL, "pair_cap > 0 needs pairs");
    RunJob r{};
    r.pop = P;
    r.mask = mask;
    r.eps = eps;
    r.plan = plan_job(P->n, popcount32(mask), 0, false);
    r.eps_count = count;
    r.eps_mean = mean_dist;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!pair_off) return run({r}, Tune{0, 0, 0, 0}, ws, ws_bytes, s);
    // Pair lists: counts, their prefix sums, then the same join again (one
    // wavefront per query tile, so each query appends its own row), writing
    // each hit at its row start plus the hits before it.
    const size_t need_run = run_workspace({r});
    const size_t scan_at = align_up(need_run);
    const size_t need = scan_at + pair_scan_scratch(P->n);
    if (!ws) return fail(SNAPS_EINVAL, "workspace is NULL (%zu bytes needed)", need);
    if (ws_bytes < need) return fail(SNAPS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    Tune tn{};
    tn.split = 1;
    tn.mq = 1;
    int rc2 = run({r}, tn, ws, ws_bytes, s);
    if (rc2 != SNAPS_OK) return rc2;
    hipError_t e = launch_pair_offsets(count, P->n, pair_off, static_cast<char*>(ws) + scan_at, s);
    if (e != hipSuccess) return hip_fail(e, "pair offsets launch");
    if (pair_cap == 0) return SNAPS_OK;
    r.pair_off = pair_off;
    r.pairs = pairs;
    r.pair_cap = pair_cap;
    return run({r}, tn, ws, ws_bytes, s);
}

int snaps_outlier_scores(const snaps_job* jobs, int32_t n_jobs, const snaps_tuning* tune, void* ws,
                         size_t ws_bytes, void* stream) {
    int rc = check_tuning(tune);
    if (rc != SNAPS_OK) return rc;
    std::vector<RunJob> rj;
    rc = collect_jobs(jobs, n_jobs, tune, &rj);
    if (rc != SNAPS_OK) return rc;
    return run(rj, resolve_tune(tune), ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int snaps_rank(const int32_t* eps_count, const float* eps_mean, const int32_t* indeg, const float* knn_mean,
               int64_t n, int32_t* rank, void* ws, size_t ws_bytes, void* stream) {
    if (!eps_count || !eps_mean || !indeg || !knn_mean || !rank)
        return fail(SNAPS_EINVAL, "every metric array and the rank output are required");
    if (n < 1) return fail(SNAPS_EINVAL, "n must be >= 1");
    if (n > kMaxN) return fail(SNAPS_EUNSUPPORTED, "n = %lld exceeds this version's limit", (long long)n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevJob j;
    std::memset(&j, 0, sizeof(j));
    j.n = (int32_t)n;
    j.eps_count = const_cast<int32_t*>(eps_count);
    j.eps_mean = const_cast<float*>(eps_mean);
    j.indeg = const_cast<int32_t*>(indeg);
    j.knn_mean = const_cast<float*>(knn_mean);
    j.rank = rank;
    if (n <= kLdsSortMax) {
        hipError_t e = launch_rank_single(j, s);
        if (e != hipSuccess) return hip_fail(e, "rank launch");
        return SNAPS_OK;
    }
    const size_t need = rank_workspace(n);
    if (!ws) return fail(SNAPS_EINVAL, "workspace is NULL (%zu bytes needed)", need);
    if (ws_bytes < need) return fail(SNAPS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    char* base = static_cast<char*>(ws);
    const MetaLayout ml = meta_layout(1, 0, 1);
    const int nchunks = (int)((n + kRadixChunk - 1) / kRadixChunk);
    const size_t rows = (size_t)((n + kTile - 1) / kTile) * kTile;
    char* jb = base + ml.bytes;
    uint32_t* keys = reinterpret_cast<uint32_t*>(jb);
    uint32_t* pong = keys + 4 * rows;
    int32_t* hist = reinterpret_cast<int32_t*>(jb + align_up(8 * rows * sizeof(uint32_t)));
    int32_t* nd = hist + (size_t)4 * 256 * nchunks;
    LargeRank R{};
    R.job = 0;
    R.nchunks = nchunks;
    R.n_distinct = nd;
    std::vector<SortSeg> segs(4);
    std::vector<int32_t> segchunk(5, 0);
    for (int m = 0; m < 4; ++m) {
        R.keys[m] = keys + m * rows;
        R.distinct[m] = pong + m * rows;
        SortSeg& g = segs[m];
        g.key[0] = R.keys[m];
        g.key[1] = R.distinct[m];
        g.hist = hist + (size_t)m * 256 * nchunks;
        g.n = n;
        g.nchunks = nchunks;
        segchunk[m + 1] = segchunk[m] + nchunks;
    }
    const int32_t chunk[2] = {0, nchunks};
    auto& st = staging();
    st.assign(ml.bytes, 0);
    std::memcpy(st.data() + ml.table, &j, sizeof(DevJob));
    std::memcpy(st.data() + ml.lr, &R, sizeof(LargeRank));
    std::memcpy(st.data() + ml.rseg, segs.data(), 4 * sizeof(SortSeg));
    std::memcpy(st.data() + ml.rchunk, chunk, sizeof(chunk));
    std::memcpy(st.data() + ml.rsegchunk, segchunk.data(), 5 * sizeof(int32_t));
    hipError_t e = hipMemcpyAsync(base, st.data(), ml.bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "rank table upload");
    e = launch_large_rank(reinterpret_cast<const DevJob*>(base + ml.table), reinterpret_cast<const LargeRank*>(base + ml.lr),
                          1, reinterpret_cast<const int32_t*>(base + ml.rchunk), nchunks,
                          reinterpret_cast<const SortSeg*>(base + ml.rseg),
                          reinterpret_cast<const int32_t*>(base + ml.rsegchunk), 4 * nchunks, s);
    if (e != hipSuccess) return hip_fail(e, "large rank launch");
    return SNAPS_OK;
}

// -------------------------------------------------------------- graph plans

struct snaps_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int snaps_plan_create(const snaps_job* jobs, int32_t n_jobs, const snaps_tuning* tune, void* ws, size_t ws_bytes,
                      void* stream, snaps_plan** out) {
    if (!out) return fail(SNAPS_EINVAL, "plan output pointer is NULL");
    *out = nullptr;
    int rc = check_tuning(tune);
    if (rc != SNAPS_OK) return rc;
    std::vector<RunJob> rj;
    rc = collect_jobs(jobs, n_jobs, tune, &rj);
    if (rc != SNAPS_OK) return rc;
    const Tune tn = resolve_tune(tune);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // Upload the job table once, then capture the launches on a private
    // stream (the upload is not part of the graph).
    rc = run(rj, tn, ws, ws_bytes, s, RunMode::UploadOnly);
    if (rc != SNAPS_OK) return rc;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "plan upload");
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        hipStreamDestroy(cs);
        return hip_fail(e, "begin capture");
    }
    rc = run(rj, tn, ws, ws_bytes, cs, RunMode::LaunchOnly);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    hipStreamDestroy(cs);
    if (rc != SNAPS_OK) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return hip_fail(e, "graph instantiate");
    }
    snaps_plan* p = new snaps_plan;
    p->graph = g;
    p->exec = x;
    *out = p;
    return SNAPS_OK;
}

int snaps_plan_launch(const snaps_plan* plan, void* stream) {
    if (!plan || !plan->exec) return fail(SNAPS_EINVAL, "plan is NULL");
    hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return SNAPS_OK;
}

void snaps_plan_destroy(snaps_plan* plan) {
    if (!plan) return;
    if (plan->exec) hipGraphExecDestroy(plan->exec);
    if (plan->graph) hipGraphDestroy(plan->graph);
    delete plan;
}

}  // extern "C"

// ------------------------------------------- allocation-free batched form

// The workspace of snaps_outlier_scores_static: one fixed array per device,
// part of the library's code object, held until the process ends.  Host code
// never uses this name as an address (on the host it is only a stand-in):
// every use goes through the device address that hipGetSymbolAddress
// returns, looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[SNAPS_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

int static_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(SNAPS_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return SNAPS_OK;
}

}  // namespace

extern "C" {

int snaps_outlier_scores_static(const snaps_job* jobs, int32_t n_jobs, const snaps_tuning* tune, void* stream) {
    int rc = check_tuning(tune);
    if (rc != SNAPS_OK) return rc;
    std::vector<RunJob> rj;
    rc = collect_jobs(jobs, n_jobs, tune, &rj);
    if (rc != SNAPS_OK) return rc;
    const size_t need = run_workspace(rj);
    if (need > (size_t)SNAPS_STATIC_SCRATCH_BYTES)
        return fail(SNAPS_ENOMEM,
                    "these jobs need %zu bytes of workspace, more than the %zu of the static scratch: "
                    "use snaps_outlier_scores with a caller workspace",
                    need, (size_t)SNAPS_STATIC_SCRATCH_BYTES);
    void* ws = nullptr;
    rc = static_scratch(&ws);
    if (rc != SNAPS_OK) return rc;
    return run(rj, resolve_tune(tune), ws, SNAPS_STATIC_SCRATCH_BYTES, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ serving

namespace {

struct ServeLayout {
    JobPlan plan;
    size_t hdr, ws, ws_bytes, rk2, tmax, tkey, sbox, smax, cnt, mean, deg, kmean, kth, rank, bytes;
    int nsuper;
};

// Kernel of one alert job: 1 = one wavefront per alert (k_alerts), 2 = the
// matrix-core cross-join of 64-alert groups (k_alerts_mfma).  Automatic
// choice: the matrix cores from d = 6, and at d = 5 up to 512 alerts, where
// the per-alert walk meets most tiles (measured on 10^6-object states with
// 16..10^4 alerts per request: at d = 6 the matrix cores are 1.2-4.6x
// faster, at d = 10 7.6-21x, at d = 15 10-33x; at d = 5 1.6-1.9x faster up
// to 256 alerts and 0.8x from 1,024; at d <= 4 the per-alert index culling
// is the better tool).
int alert_method(int method, int d, int m) {
    if (method != 0) return method;
    return d >= 6 || (d == 5 && m <= 512) ? 2 : 1;
}

ServeLayout serve_layout(int64_t n, int d, int k) {
    ServeLayout L{};
    L.plan = plan_job(n, d, k, true, kIndexRadix, true);
    const size_t rows = (size_t)L.plan.ntiles * kTile;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align_up(b);
        return o;
    };
    L.hdr = take(sizeof(ServeState));
    L.ws_bytes = meta_layout(1, 1, 1).bytes + L.plan.bytes;
    L.ws = take(L.ws_bytes);
    L.rk2 = take(rows * sizeof(float));
    L.tmax = take((size_t)L.plan.ntiles * sizeof(float));
    L.tkey = take((size_t)L.plan.ntiles * sizeof(uint32_t));
    L.nsuper = (L.plan.ntiles + 63) / 64;
    L.sbox = take((size_t)L.nsuper * 2 * row_stride(d) * sizeof(float));
    L.smax = take((size_t)L.nsuper * sizeof(float));
    L.cnt = take((size_t)n * 4);
    L.mean = take((size_t)n * 4);
    L.deg = take((size_t)n * 4);
    L.kmean = take((size_t)n * 4);
    L.kth = take((size_t)n * 4);
    L.rank = take((size_t)4 * n * 4);
    L.bytes = off;
    return L;
}

}  // namespace

size_t snaps_serve_state_bytes(const snaps_population* P, uint32_t mask, int32_t k) {
    if (check_population(P, mask) != SNAPS_OK || check_k(P->n, k) != SNAPS_OK) return 0;
    return serve_layout(P->n, popcount32(mask), k).bytes;
}

int snaps_serve_state_build(const snaps_population* P, uint32_t mask, int32_t k, float eps, void* state,
                            size_t state_bytes, void* stream) {
    int rc = check_population(P, mask);
    if (rc != SNAPS_OK) return rc;
    rc = check_k(P->n, k);
    if (rc != SNAPS_OK) return rc;
    rc = check_eps(eps);
    if (rc != SNAPS_OK) return rc;
    const int d = popcount32(mask);
    const ServeLayout L = serve_layout(P->n, d, k);
    if (!state) return fail(SNAPS_EINVAL, "state memory is NULL (%zu bytes needed)", L.bytes);
    if (state_bytes < L.bytes) return fail(SNAPS_ENOMEM, "state of %zu bytes is smaller than the %zu needed", state_bytes, L.bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(state);
    RunJob r{};
    r.pop = P;
    r.mask = mask;
    r.eps = eps;
    r.plan = L.plan;
    r.eps_count = reinterpret_cast<int32_t*>(base + L.cnt);
    r.eps_mean = reinterpret_cast<float*>(base + L.mean);
    r.indeg = reinterpret_cast<int32_t*>(base + L.deg);
    r.knn_mean = reinterpret_cast<float*>(base + L.kmean);
    r.knn_kth = reinterpret_cast<float*>(base + L.kth);
    r.rank = reinterpret_cast<int32_t*>(base + L.rank);
    // A serving state indexes min(d, 6) dimensions: single alerts are culled
    // tile by tile, which the finer cut in more dimensions helps (measured:
    // the batched default of 4 made p50 and p99 latency worse).
    Tune ts{};
    ts.index_dims = kMaxIndexDims;
    rc = run({r}, ts, base + L.ws, L.ws_bytes, s);
    if (rc != SNAPS_OK) return rc;
    // Same addresses as run() chose for this single large job.
    char* wsb = base + L.ws;
    const MetaLayout ml = meta_layout(1, 1, 1);
    char* jb = wsb + ml.bytes;
    const JobPlan& p = L.plan;
    const size_t rows = (size_t)p.ntiles * kTile;
    DevJob j = make_devjob(P, mask, p, eps, ts, jb);
    LargeIndex li{};
    li.sel_col = reinterpret_cast<int32_t*>(jb + p.sel_off);
    li.sel_lo = reinterpret_cast<float*>(jb + p.sel_off) + kMaxIndexDims;
    li.sel_scale = reinterpret_cast<float*>(jb + p.sel_off) + 2 * kMaxIndexDims;
    hipError_t e = launch_serve_finish(j, li, reinterpret_cast<float*>(base + L.rk2), reinterpret_cast<float*>(base + L.tmax),
                                       reinterpret_cast<uint32_t*>(base + L.tkey), r.knn_kth, s);
    if (e != hipSuccess) return hip_fail(e, "serve state launch");
    e = launch_serve_super(p.ntiles, row_stride(d), j.boxes, reinterpret_cast<float*>(base + L.tmax),
                           reinterpret_cast<float*>(base + L.sbox), reinterpret_cast<float*>(base + L.smax), s);
    if (e != hipSuccess) return hip_fail(e, "serve state launch");
    ServeState st{};
    st.n = (int32_t)P->n;
    st.d = d;
    st.k = k;
    st.ntiles = p.ntiles;
    st.eps2 = j.eps2;
    st.c = j.c;
    st.bits = j.bits;
    st.cols = P->cols;
    st.ld = P->ld;
    for (int f = 0; f < kMaxD; ++f) st.feat[f] = j.feat[f];
    st.xs = j.xs;
    st.boxes = j.boxes;
    st.rk2 = reinterpret_cast<float*>(base + L.rk2);
    st.tmax = reinterpret_cast<float*>(base + L.tmax);
    st.tkey = reinterpret_cast<uint32_t*>(base + L.tkey);
    st.sbox = reinterpret_cast<float*>(base + L.sbox);
    st.smax = reinterpret_cast<float*>(base + L.smax);
    st.nsuper = L.nsuper;
    st.sel_col = li.sel_col;
    st.sel_lo = li.sel_lo;
    st.sel_scale = li.sel_scale;
    for (int m = 0; m < 4; ++m) st.distinct[m] = reinterpret_cast<uint32_t*>(jb + p.rpong_off) + m * rows;
    st.n_distinct = reinterpret_cast<int32_t*>(jb + p.rnd_off);
    auto& stg = staging();
    stg.assign(sizeof(ServeState), 0);
    std::memcpy(stg.data(), &st, sizeof(st));
    e = hipMemcpyAsync(base + L.hdr, stg.data(), sizeof(st), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "serve state header upload");
    return SNAPS_OK;
}

int snaps_serve_state_outputs(const void* state, int64_t n, int32_t d, int32_t k, const int32_t** eps_count,
                              const float** eps_mean, const int32_t** indeg, const float** knn_mean,
                              const int32_t** rank) {
    if (!state || n < 2 || d < 2 || d > kMaxD || k < 1) return fail(SNAPS_EINVAL, "invalid state description");
    const ServeLayout L = serve_layout(n, d, k);
    const char* base = static_cast<const char*>(state);
    if (eps_count) *eps_count = reinterpret_cast<const int32_t*>(base + L.cnt);
    if (eps_mean) *eps_mean = reinterpret_cast<const float*>(base + L.mean);
    if (indeg) *indeg = reinterpret_cast<const int32_t*>(base + L.deg);
    if (knn_mean) *knn_mean = reinterpret_cast<const float*>(base + L.kmean);
    if (rank) *rank = reinterpret_cast<const int32_t*>(base + L.rank);
    return SNAPS_OK;
}

namespace {

// Matrix-core alert jobs' workspace: the slices' partial results of every
// such job, then one k-th distance bound per alert slot (64 per group),
// shared by the workgroups of a group.
struct AlertWs {
    size_t part_bytes = 0, bound_count = 0;
    size_t bytes() const { return part_bytes + align_up(bound_count * sizeof(uint32_t)); }
};

AlertWs alert_ws(const snaps_alert_job* jobs, int32_t n_jobs, int32_t d, int kc) {
    AlertWs w;
    for (int i = 0; i < n_jobs; ++i) {
        const snaps_alert_job& a = jobs[i];
        if (a.m <= 0 || alert_method(a.method, d, a.m) != 2) continue;
        const int64_t groups = (a.m + kTile - 1) / kTile;
        w.part_bytes += align_up((size_t)(groups * alert_slices(a.m, d) * alert_part_floats(kc)) * sizeof(float));
        w.bound_count += (size_t)groups * kTile;
    }
    return w;
}

}  // namespace

size_t snaps_alerts_workspace_bytes(const snaps_alert_job* jobs, int32_t n_jobs, int32_t d, int32_t k) {
    if (n_jobs < 1 || !jobs || d < 2 || d > kMaxD || k < 1 || k > kMaxK) return 0;
    const AlertWs w = alert_ws(jobs, n_jobs, d, kc_class(k));
    return w.bound_count ? w.bytes() : 0;
}

int snaps_alerts_score(const snaps_alert_job* jobs, int32_t n_jobs, int32_t d, int32_t k, void* ws, size_t ws_bytes,
                       void* stream) {
    if (n_jobs < 1 || !jobs) return fail(SNAPS_EINVAL, "need at least one alert job");
    if (d < 2 || d > kMaxD) return fail(SNAPS_EINVAL, "d must be in [2, %d]", kMaxD);
    if (k < 1 || k > kMaxK) return fail(SNAPS_EINVAL, "k must be in [1, %d]", kMaxK);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < n_jobs; ++i) {
        const snaps_alert_job& a = jobs[i];
        if (!a.state || (a.m > 0 && (!a.alerts || !a.eps_count || !a.eps_mean || !a.indeg || !a.knn_mean)))
            return fail(SNAPS_EINVAL, "alert job %d: state, alerts and every score output are required", i);
        if (a.m < 0) return fail(SNAPS_EINVAL, "alert job %d: negative alert count", i);
        if (a.method < 0 || a.method > 2) return fail(SNAPS_EINVAL, "alert job %d: method must be 0, 1 or 2", i);
    }
    const size_t need = snaps_alerts_workspace_bytes(jobs, n_jobs, d, k);
    if (need > 0 && !ws) return fail(SNAPS_EINVAL, "workspace is NULL (%zu bytes needed)", need);
    if (ws_bytes < need) return fail(SNAPS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    const int kc = kc_class(k);
    const AlertWs aws = alert_ws(jobs, n_jobs, d, kc);
    uint32_t* bounds = aws.bound_count ? reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + aws.part_bytes) : nullptr;
    if (bounds) {
        if (aws.bound_count > (size_t)INT32_MAX) return fail(SNAPS_EINVAL, "too many alerts in one call");
        hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(bounds), (int32_t)aws.bound_count, 0x7F800000, s);
        if (e != hipSuccess) return hip_fail(e, "alert bound fill launch");
    }
    // Each job's kernel and slice count depend only on its own method, d and
    // size, so an alert's scores do not depend on the other jobs of the call.
    size_t part_at = 0;                          // floats into ws
    size_t bound_at = 0;                         // bound slots
    for (int mfma = 0; mfma < 2; ++mfma) {
        std::vector<int> sel;
        for (int i = 0; i < n_jobs; ++i)
            if (jobs[i].m > 0 && alert_method(jobs[i].method, d, jobs[i].m) == (mfma ? 2 : 1)) sel.push_back(i);
        for (size_t b = 0; b < sel.size(); b += kAlertJobs) {
            AlertArgs aa{};
            int64_t alerts = 0, blocks = 0, groups = 0;
            const int nb = (int)std::min<size_t>(kAlertJobs, sel.size() - b);
            aa.n_jobs = nb;
            aa.d = d;
            aa.part = static_cast<float*>(ws);
            aa.bounds = bounds;
            for (int i = 0; i < nb; ++i) {
                const snaps_alert_job& a = jobs[sel[b + i]];
                AlertJob& J = aa.jobs[i];
                J.st = static_cast<const ServeState*>(a.state);
                J.alerts = a.alerts;
                J.m = a.m;
                J.eps_count = a.eps_count;
                J.eps_mean = a.eps_mean;
                J.indeg = a.indeg;
                J.knn_mean = a.knn_mean;
                J.rank = a.rank;
                aa.alert_prefix[i] = (int32_t)alerts;
                aa.group_prefix[i] = (int32_t)blocks;
                aa.merge_prefix[i] = (int32_t)groups;
                alerts += a.m;
                if (alerts > INT32_MAX - kAlertWaves)
                    return fail(SNAPS_EINVAL, "more than 2^31 alerts in one call");
                if (mfma) {
                    const int64_t g = (a.m + kTile - 1) / kTile;
                    const int sl = alert_slices(a.m, d);
                    aa.slices[i] = sl;
                    aa.part_off[i] = (int64_t)part_at;
                    part_at += align_up((size_t)(g * sl * alert_part_floats(kc)) * sizeof(float)) / sizeof(float);
                    aa.bound_off[i] = (int64_t)bound_at;
                    bound_at += (size_t)g * kTile;
                    blocks += g * sl;
                    groups += g;
                    if (blocks > INT32_MAX) return fail(SNAPS_EINVAL, "too many alert groups in one call");
                }
            }
            aa.alert_prefix[nb] = (int32_t)alerts;
            aa.group_prefix[nb] = (int32_t)blocks;
            aa.merge_prefix[nb] = (int32_t)groups;
            hipError_t e = mfma ? launch_alerts_mfma(d, kc, aa, s) : launch_alerts(d, kc, aa, s);
            if (e != hipSuccess) return hip_fail(e, "alert scoring launch");
        }
    }
    return SNAPS_OK;
}

}  // extern "C"

// ------------------------------------------------------------ eps sampler

namespace {

struct EpsPlan {
    int n_jobs = 0;
    std::vector<int> d;                 // per job
    std::vector<std::array<uint32_t, kMaxEpsTargets>> rank;
    size_t table = 0, prefix = 0, hist = 0, state = 0, bytes = 0;
};

int plan_eps(const snaps_eps_job* jobs, int32_t n_jobs, EpsPlan* p) {
    if (n_jobs < 1 || !jobs) return fail(SNAPS_EINVAL, "need at least one eps job");
    p->n_jobs = n_jobs;
    p->d.resize(n_jobs);
    p->rank.resize(n_jobs);
    int64_t blocks = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const snaps_eps_job& j = jobs[i];
        int rc = check_population(j.pop, j.mask);
        if (rc != SNAPS_OK) return fail(rc, "eps job %d: %s", i, g_error.c_str());
        const int64_t n = j.pop->n;
        if (j.m < 1 || j.m > n) return fail(SNAPS_EINVAL, "eps job %d: sample size %d not in [1, n]", i, j.m);
        if (!j.sample || !j.eps) return fail(SNAPS_EINVAL, "eps job %d: sample and eps are required", i);
        if (j.n_targets < 1 || j.n_targets > kMaxEpsTargets)
            return fail(SNAPS_EINVAL, "eps job %d: n_targets must be in [1, %d]", i, kMaxEpsTargets);
        const int64_t pairs = (int64_t)j.m * (n - 1);
        if (pairs >= (int64_t)1 << 32)
            return fail(SNAPS_EUNSUPPORTED, "eps job %d: m (n - 1) = %lld sample distances exceed 2^32", i,
                        (long long)pairs);
        for (int t = 0; t < j.n_targets; ++t) {
            const double tt = j.target[t];
            if (!(tt > 0.0) || !std::isfinite(tt)) return fail(SNAPS_EINVAL, "eps job %d: target %d must be > 0", i, t);
            const double r = std::nearbyint(tt * (double)j.m);     // round half to even
            if (r < 1.0 || r > (double)(pairs - 1))
                return fail(SNAPS_EINVAL, "eps job %d: round(target m) = %.0f not in [1, m (n - 1) - 1]", i, r);
            p->rank[i][t] = (uint32_t)r;
        }
        p->d[i] = popcount32(j.mask);
        blocks += j.m;
    }
    if (blocks > INT32_MAX) return fail(SNAPS_EUNSUPPORTED, "more than 2^31 - 1 sample objects in one call");
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align_up(b);
        return o;
    };
    p->table = take((size_t)n_jobs * sizeof(EpsJob));
    p->prefix = take((size_t)(n_jobs + kMaxD + 2) * sizeof(int32_t));
    p->hist = take((size_t)n_jobs * kMaxEpsTargets * 256 * sizeof(uint32_t));
    p->state = take((size_t)n_jobs * kMaxEpsTargets * sizeof(EpsState));
    p->bytes = off;
    return SNAPS_OK;
}

}  // namespace

extern "C" {

size_t snaps_eps_sample_workspace(const snaps_eps_job* jobs, int32_t n_jobs) {
    EpsPlan p;
    if (plan_eps(jobs, n_jobs, &p) != SNAPS_OK) return 0;
    return p.bytes;
}

int snaps_eps_sample(const snaps_eps_job* jobs, int32_t n_jobs, void* ws, size_t ws_bytes, void* stream) {
    EpsPlan p;
    int rc = plan_eps(jobs, n_jobs, &p);
    if (rc != SNAPS_OK) return rc;
    if (!ws) return fail(SNAPS_EINVAL, "workspace is NULL (%zu bytes needed)", p.bytes);
    if (ws_bytes < p.bytes) return fail(SNAPS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, p.bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    // Jobs grouped by dimensionality (one instantiation per d), in order.
    std::vector<EpsJob> table;
    table.reserve(n_jobs);
    std::vector<int32_t> prefix;
    struct Group { int d, first, count, blocks, prefix_at; };
    std::vector<Group> groups;
    for (int d = 2; d <= kMaxD; ++d) {
        Group g{d, (int)table.size(), 0, 0, (int)prefix.size()};
        prefix.push_back(0);
        for (int i = 0; i < n_jobs; ++i) {
            if (p.d[i] != d) continue;
            const snaps_eps_job& j = jobs[i];
            EpsJob e{};
            e.cols = j.pop->cols;
            e.ld = j.pop->ld;
            e.n = (int32_t)j.pop->n;
            e.d = d;
            int f = 0;
            for (int b = 0; b < 32; ++b)
                if ((j.mask >> b) & 1u) e.feat[f++] = b;
            e.sample = j.sample;
            e.m = j.m;
            e.n_targets = j.n_targets;
            for (int t = 0; t < j.n_targets; ++t) e.rank[t] = p.rank[i][t];
            e.eps = j.eps;
            const size_t slot = table.size();
            e.hist = reinterpret_cast<uint32_t*>(base + p.hist) + slot * kMaxEpsTargets * 256;
            e.state = reinterpret_cast<EpsState*>(base + p.state) + slot * kMaxEpsTargets;
            table.push_back(e);
            g.count += 1;
            g.blocks += j.m;
            prefix.push_back(g.blocks);
        }
        if (g.count == 0) {
            prefix.pop_back();
            continue;
        }
        groups.push_back(g);
    }
    auto& stg = staging();
    const size_t tb = table.size() * sizeof(EpsJob), pb = prefix.size() * sizeof(int32_t);
    stg.resize(tb + pb);
    std::memcpy(stg.data(), table.data(), tb);
    std::memcpy(stg.data() + tb, prefix.data(), pb);
    hipError_t e = hipMemcpyAsync(base + p.table, stg.data(), tb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(base + p.prefix, stg.data() + tb, pb, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "eps table upload");
    const EpsJob* dt = reinterpret_cast<const EpsJob*>(base + p.table);
    const int32_t* dp = reinterpret_cast<const int32_t*>(base + p.prefix);
    for (const Group& g : groups) {
        e = launch_eps_sample(dt + g.first, dp + g.prefix_at, g.count, g.blocks, g.d, s);
        if (e != hipSuccess) return hip_fail(e, "eps sampler launch");
    }
    return SNAPS_OK;
}

}  // extern "C"

// ------------------------------------------------------------ eps grid

namespace {

struct GridPlan {
    std::vector<int> d, words;
    size_t table = 0, prefix = 0, scratch = 0, bytes = 0;
    std::vector<size_t> count_off, mean_off, member_off;
};

int plan_grid(const snaps_eps_grid_job* jobs, int32_t n_jobs, GridPlan* p) {
    if (n_jobs < 1 || !jobs) return fail(SNAPS_EINVAL, "need at least one eps-grid job");
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align_up(b);
        return o;
    };
    p->table = take((size_t)n_jobs * sizeof(GridJob));
    p->prefix = take((size_t)(n_jobs + kMaxD + 2) * sizeof(int32_t));
    int64_t tiles = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const snaps_eps_grid_job& j = jobs[i];
        int rc = check_population(j.pop, j.mask);
        if (rc != SNAPS_OK) return fail(rc, "eps-grid job %d: %s", i, g_error.c_str());
        const int64_t n = j.pop->n;
        if ((reinterpret_cast<uintptr_t>(j.pop->cols) & 15u) != 0 || (j.pop->ld & 3) != 0)
            return fail(SNAPS_EINVAL, "eps-grid job %d: columns must be 16-byte aligned with ld a multiple of 4", i);
        if (j.n_grid < 2 || j.n_grid > kMaxGrid)
            return fail(SNAPS_EINVAL, "eps-grid job %d: n_grid must be in [2, %d]", i, kMaxGrid);
        for (int g = 0; g < j.n_grid; ++g) {
            if (!(j.eps[g] > 0.f) || !std::isfinite(j.eps[g]) || (g > 0 && !(j.eps[g] > j.eps[g - 1])))
                return fail(SNAPS_EINVAL, "eps-grid job %d: radii must be positive, finite and strictly ascending", i);
        }
        if (j.top_n < 1 || j.top_n > n) return fail(SNAPS_EINVAL, "eps-grid job %d: top_n must be in [1, n]", i);
        if (!j.similarity || !j.select) return fail(SNAPS_EINVAL, "eps-grid job %d: similarity and select are required", i);
        p->d.push_back(popcount32(j.mask));
        const int words = (int)((n + 31) / 32);
        p->words.push_back(words);
        p->count_off.push_back(j.count ? 0 : take((size_t)j.n_grid * n * sizeof(int32_t)));
        p->mean_off.push_back(j.mean ? 0 : take((size_t)j.n_grid * n * sizeof(float)));
        p->member_off.push_back(take((size_t)2 * j.n_grid * words * sizeof(uint32_t)));
        tiles += (n + kTile - 1) / kTile;
    }
    if (tiles > INT32_MAX) return fail(SNAPS_EUNSUPPORTED, "too many query tiles in one call");
    p->bytes = off;
    return SNAPS_OK;
}

}  // namespace

extern "C" {

size_t snaps_eps_grid_workspace(const snaps_eps_grid_job* jobs, int32_t n_jobs) {
    GridPlan p;
    if (plan_grid(jobs, n_jobs, &p) != SNAPS_OK) return 0;
    return p.bytes;
}

int snaps_eps_grid(const snaps_eps_grid_job* jobs, int32_t n_jobs, void* ws, size_t ws_bytes, void* stream) {
    GridPlan p;
    int rc = plan_grid(jobs, n_jobs, &p);
    if (rc != SNAPS_OK) return rc;
    if (!ws) return fail(SNAPS_EINVAL, "workspace is NULL (%zu bytes needed)", p.bytes);
    if (ws_bytes < p.bytes) return fail(SNAPS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, p.bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    std::vector<GridJob> table;
    table.reserve(n_jobs);
    std::vector<int32_t> prefix;
    struct Group { int d, first, count, tiles, prefix_at; };
    std::vector<Group> groups;
    for (int d = 2; d <= kMaxD; ++d) {
        Group g{d, (int)table.size(), 0, 0, (int)prefix.size()};
        prefix.push_back(0);
        for (int i = 0; i < n_jobs; ++i) {
            if (p.d[i] != d) continue;
            const snaps_eps_grid_job& j = jobs[i];
            GridJob e{};
            e.cols = j.pop->cols;
            e.ld = j.pop->ld;
            e.n = (int32_t)j.pop->n;
            e.d = d;
            int f = 0;
            for (int b = 0; b < 32; ++b)
                if ((j.mask >> b) & 1u) e.feat[f++] = b;
            e.g = j.n_grid;
            e.top_n = j.top_n;
            for (int r = 0; r < kMaxGrid; ++r) {
                const float er = j.eps[r < j.n_grid ? r : j.n_grid - 1];
                e.e2[r] = (float)((double)er * (double)er);
            }
            e.count = j.count ? j.count : reinterpret_cast<int32_t*>(base + p.count_off[i]);
            e.mean = j.mean ? j.mean : reinterpret_cast<float*>(base + p.mean_off[i]);
            e.member = reinterpret_cast<uint32_t*>(base + p.member_off[i]);
            e.words = p.words[i];
            e.similarity = j.similarity;
            e.select = j.select;
            table.push_back(e);
            g.count += 1;
            g.tiles += (int)((j.pop->n + kTile - 1) / kTile);
            prefix.push_back(g.tiles);
        }
        if (g.count == 0) {
            prefix.pop_back();
            continue;
        }
        groups.push_back(g);
    }
    auto& stg = staging();
    const size_t tb = table.size() * sizeof(GridJob), pb = prefix.size() * sizeof(int32_t);
    stg.resize(tb + pb);
    std::memcpy(stg.data(), table.data(), tb);
    std::memcpy(stg.data() + tb, prefix.data(), pb);
    hipError_t e = hipMemcpyAsync(base + p.table, stg.data(), tb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(base + p.prefix, stg.data() + tb, pb, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "eps-grid table upload");
    const GridJob* dt = reinterpret_cast<const GridJob*>(base + p.table);
    const int32_t* dp = reinterpret_cast<const int32_t*>(base + p.prefix);
    for (const Group& g : groups) {
        e = launch_grid_join(dt + g.first, dp + g.prefix_at, g.count, g.tiles, g.d, s);
        if (e != hipSuccess) return hip_fail(e, "eps-grid join launch");
    }
    e = launch_grid_select(dt, n_jobs, s);
    if (e != hipSuccess) return hip_fail(e, "eps-grid selection launch");
    return SNAPS_OK;
}

}  // extern "C"

// ------------------------------------------------------------ k grid

namespace {

struct KGridPlan {
    std::vector<int> d, words;
    size_t table = 0, gtable = 0, prefix = 0, bytes = 0;
    std::vector<size_t> thr_off, indeg_off, kmean_off, member_off;
};

int plan_kgrid(const snaps_k_grid_job* jobs, int32_t n_jobs, KGridPlan* p) {
    if (n_jobs < 1 || !jobs) return fail(SNAPS_EINVAL, "need at least one k-grid job");
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align_up(b);
        return o;
    };
    p->table = take((size_t)n_jobs * sizeof(KGridJob));
    p->gtable = take((size_t)n_jobs * sizeof(GridJob));
    p->prefix = take((size_t)2 * (n_jobs + kMaxD + 2) * sizeof(int32_t));
    int64_t queries = 0, tiles = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const snaps_k_grid_job& j = jobs[i];
        int rc = check_population(j.pop, j.mask);
        if (rc != SNAPS_OK) return fail(rc, "k-grid job %d: %s", i, g_error.c_str());
        const int64_t n = j.pop->n;
        if ((reinterpret_cast<uintptr_t>(j.pop->cols) & 15u) != 0 || (j.pop->ld & 3) != 0)
            return fail(SNAPS_EINVAL, "k-grid job %d: columns must be 16-byte aligned with ld a multiple of 4", i);
        if (n < 2 || n > kMaxN)
            return fail(SNAPS_EUNSUPPORTED, "k-grid job %d: n = %lld outside [2, %lld]", i, (long long)n,
                        (long long)kMaxN);
        if (j.n_grid < 2 || j.n_grid > kMaxGrid)
            return fail(SNAPS_EINVAL, "k-grid job %d: n_grid must be in [2, %d]", i, kMaxGrid);
        for (int g = 0; g < j.n_grid; ++g) {
            if (j.k[g] < 1 || (g > 0 && j.k[g] <= j.k[g - 1]))
                return fail(SNAPS_EINVAL, "k-grid job %d: k must be >= 1 and strictly ascending", i);
        }
        const int kmax = j.k[j.n_grid - 1];
        if (kmax > kMaxKGridK || kmax > n - 1)
            return fail(SNAPS_EINVAL, "k-grid job %d: k_max = %d exceeds min(%d, n - 1)", i, kmax, kMaxKGridK);
        if (j.top_n < 1 || j.top_n > n) return fail(SNAPS_EINVAL, "k-grid job %d: top_n must be in [1, n]", i);
        if (!j.similarity || !j.select) return fail(SNAPS_EINVAL, "k-grid job %d: similarity and select are required", i);
        p->d.push_back(popcount32(j.mask));
        const int words = (int)((n + 31) / 32);
        p->words.push_back(words);
        p->thr_off.push_back(take((size_t)n * kMaxGrid * sizeof(uint64_t)));
        p->indeg_off.push_back(j.indeg ? 0 : take((size_t)j.n_grid * n * sizeof(int32_t)));
        p->kmean_off.push_back(j.knn_mean ? 0 : take((size_t)j.n_grid * n * sizeof(float)));
        p->member_off.push_back(take((size_t)2 * j.n_grid * words * sizeof(uint32_t)));
        queries += n;
        tiles += (n + kTile - 1) / kTile;
    }
    if (queries > INT32_MAX) return fail(SNAPS_EUNSUPPORTED, "too many objects in one call");
    p->bytes = off;
    return SNAPS_OK;
}

}  // namespace

extern "C" {

size_t snaps_k_grid_workspace(const snaps_k_grid_job* jobs, int32_t n_jobs) {
    KGridPlan p;
    if (plan_kgrid(jobs, n_jobs, &p) != SNAPS_OK) return 0;
    return p.bytes;
}

int snaps_k_grid(const snaps_k_grid_job* jobs, int32_t n_jobs, void* ws, size_t ws_bytes, void* stream) {
    KGridPlan p;
    int rc = plan_kgrid(jobs, n_jobs, &p);
    if (rc != SNAPS_OK) return rc;
    if (!ws) return fail(SNAPS_EINVAL, "workspace is NULL (%zu bytes needed)", p.bytes);
    if (ws_bytes < p.bytes) return fail(SNAPS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, p.bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    std::vector<KGridJob> table;
    std::vector<GridJob> gtable;
    table.reserve(n_jobs);
    gtable.reserve(n_jobs);
    std::vector<int32_t> qprefix, tprefix;
    // Launch groups: one dimensionality, and populations within one
    // workgroup's registers or above (the streaming threshold kernel).
    struct Group { int d, stream, first, count, queries, tiles, prefix_at; };
    std::vector<Group> groups;
    for (int gi = 0; gi < 2 * (kMaxD + 1); ++gi) {
        const int d = gi / 2, stream = gi % 2;
        if (d < 2) continue;
        Group g{d, stream, (int)table.size(), 0, 0, 0, (int)qprefix.size()};
        qprefix.push_back(0);
        tprefix.push_back(0);
        for (int i = 0; i < n_jobs; ++i) {
            if (p.d[i] != d || (jobs[i].pop->n > kMaxKGridN ? 1 : 0) != stream) continue;
            const snaps_k_grid_job& j = jobs[i];
            const int32_t n = (int32_t)j.pop->n;
            KGridJob e{};
            e.cols = j.pop->cols;
            e.ld = j.pop->ld;
            e.n = n;
            e.d = d;
            int f = 0;
            for (int b = 0; b < 32; ++b)
                if ((j.mask >> b) & 1u) e.feat[f++] = b;
            e.g = j.n_grid;
            for (int r = 0; r < kMaxGrid; ++r) e.k[r] = j.k[r < j.n_grid ? r : j.n_grid - 1];
            e.thr = reinterpret_cast<uint64_t*>(base + p.thr_off[i]);
            e.indeg = j.indeg ? j.indeg : reinterpret_cast<int32_t*>(base + p.indeg_off[i]);
            e.kmean = j.knn_mean ? j.knn_mean : reinterpret_cast<float*>(base + p.kmean_off[i]);
            table.push_back(e);
            GridJob s2{};
            s2.cols = e.cols;
            s2.ld = e.ld;
            s2.n = n;
            s2.d = d;
            s2.g = j.n_grid;
            s2.top_n = j.top_n;
            s2.count = e.indeg;
            s2.mean = e.kmean;
            s2.member = reinterpret_cast<uint32_t*>(base + p.member_off[i]);
            s2.words = p.words[i];
            s2.knn = 1;
            s2.similarity = j.similarity;
            s2.select = j.select;
            gtable.push_back(s2);
            g.count += 1;
            if ((int64_t)g.queries + n > INT32_MAX) return fail(SNAPS_EUNSUPPORTED, "too many k-grid queries in one call");
            g.queries += n;
            const int tg = kgrid_tiles_per_group();
            g.tiles += ((n + kTile - 1) / kTile + tg - 1) / tg;      // groups of tiles
            qprefix.push_back(g.queries);
            tprefix.push_back(g.tiles);
        }
        if (g.count == 0) {
            qprefix.pop_back();
            tprefix.pop_back();
            continue;
        }
        groups.push_back(g);
    }
    auto& stg = staging();
    const size_t tb = table.size() * sizeof(KGridJob), gb = gtable.size() * sizeof(GridJob);
    const size_t pb = qprefix.size() * sizeof(int32_t);
    stg.resize(tb + gb + 2 * pb);
    std::memcpy(stg.data(), table.data(), tb);
    std::memcpy(stg.data() + tb, gtable.data(), gb);
    std::memcpy(stg.data() + tb + gb, qprefix.data(), pb);
    std::memcpy(stg.data() + tb + gb + pb, tprefix.data(), pb);
    hipError_t e = hipMemcpyAsync(base + p.table, stg.data(), tb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(base + p.gtable, stg.data() + tb, gb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(base + p.prefix, stg.data() + tb + gb, 2 * pb, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "k-grid table upload");
    const KGridJob* dt = reinterpret_cast<const KGridJob*>(base + p.table);
    const GridJob* dg = reinterpret_cast<const GridJob*>(base + p.gtable);
    const int32_t* dq = reinterpret_cast<const int32_t*>(base + p.prefix);
    const int32_t* dtp = dq + qprefix.size();
    for (const Group& g : groups) {
        e = launch_kgrid(dt + g.first, dq + g.prefix_at, dtp + g.prefix_at, g.count, g.queries, g.tiles, g.d,
                         g.stream != 0, s);
        if (e != hipSuccess) return hip_fail(e, "k-grid launch");
    }
    e = launch_grid_select(dg, n_jobs, s);
    if (e != hipSuccess) return hip_fail(e, "k-grid selection launch");
    return SNAPS_OK;
}

}  // extern "C"
