/*
 * Brute-force float64 oracle of the per-object join results, in plain C.
 * TEST INFRASTRUCTURE: loaded only by the test suite and by the CPU
 * baseline leg of the benchmark; the product library never links it.
 *
 * It computes, for every object i of one feature space (paper Sec. 3.5,
 * 3.6, Fig. 1, Tab. 2):
 *   - D(i,j) = sqrt(sum_f (x_if - x_jf)^2) in float64, summed feature by
 *     feature in column order (the same order as the NumPy oracle, so the
 *     two agree bit for bit);
 *   - the k nearest other objects in ascending (D, id) order, plus the
 *     (k+1)-th distance (or +inf when it does not exist);
 *   - the number of other objects with D <= eps and the sum of their
 *     distances.
 * The loop over queries is split over OpenMP threads; each query is an
 * independent scan of all n objects.
 */
#include <math.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* (d, j) strictly before (bd, bj) in the (distance, id) order */
static int before(double d, int64_t j, double bd, int64_t bj) {
    return d < bd || (d == bd && j < bj);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * x        row-major float32 [n][d] (already projected to the space)
 * q        row-major float32 [m][d] queries; NULL means "the population
 *          itself" (self-join: object i never counts as its own neighbour)
 * ids      int32 [m][k]   nearest-neighbour ids, ascending order
 * dist     float64 [m][k] their distances
 * next     float64 [m]    (k+1)-th distance, +inf if none
 * cnt      int32 [m]      number of neighbours with D <= eps
 * sum      float64 [m]    sum of those distances
 * band     int32 [m]      number of other objects with band_lo <= D <= band_hi
 *                         (NULL to skip); tests use it to find objects that
 *                         have a neighbour within rounding distance of eps
 * qids     int64 [m]      with q == NULL: the self-join is evaluated only for
 *                         these object ids (row t of the outputs is object
 *                         qids[t]); NULL means every object
 * k may be 0 (no kNN), eps may be negative (no range join).
 */
int oracle_join(const float* x, int64_t n, int32_t d, const float* q, int64_t m,
                int32_t k, double eps, int32_t* ids, double* dist, double* next,
                int32_t* cnt, double* sum, int32_t* band, double band_lo, double band_hi,
                const int64_t* qids, int32_t nthreads) {
    if (n < 1 || d < 1 || k < 0 || k > 64) return -1;
    const int self = (q == 0);
    if (self) { q = x; if (!qids) m = n; }
    if (self && k > n - 1) return -1;
    if (!self && k > n) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t i = (self && qids) ? qids[t] : t;   /* object (self) or query row */
        double bd[65];
        int64_t bj[65];
        int kk = k + 1;              /* keep one extra to report the next distance */
        for (int t = 0; t < kk; ++t) { bd[t] = INFINITY; bj[t] = INT64_MAX; }
        int32_t c = 0, bc = 0;
        double s = 0.0;
        const float* qi = q + i * (int64_t)d;
        for (int64_t j = 0; j < n; ++j) {
            if (self && j == i) continue;
            const float* xj = x + j * (int64_t)d;
            double acc = 0.0;
            for (int f = 0; f < d; ++f) {
                double t = (double)qi[f] - (double)xj[f];
                acc += t * t;
            }
            double dj = sqrt(acc);
            if (dj <= eps) { c += 1; s += dj; }
            if (dj >= band_lo && dj <= band_hi) bc += 1;
            if (kk > 1 && before(dj, j, bd[kk - 1], bj[kk - 1])) {
                int p = kk - 1;
                while (p > 0 && before(dj, j, bd[p - 1], bj[p - 1])) {
                    bd[p] = bd[p - 1];
                    bj[p] = bj[p - 1];
                    --p;
                }
                bd[p] = dj;
                bj[p] = j;
            }
        }
        for (int u = 0; u < k; ++u) {
            ids[t * k + u] = (int32_t)bj[u];
            dist[t * k + u] = bd[u];
        }
        if (next) next[t] = (k > 0) ? bd[k] : INFINITY;
        if (cnt) cnt[t] = c;
        if (sum) sum[t] = s;
        if (band) band[t] = bc;
    }
    return 0;
}
