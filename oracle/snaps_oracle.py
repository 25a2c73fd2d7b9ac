"""Float64 brute-force oracle of the per-space outlier metrics.

TEST INFRASTRUCTURE: used only by tests, the smoke check and the CPU
baseline leg of the benchmark.  Nothing here is called by the product.

Definitions (paper Sec. 3.4-3.6; Fig. 1; Tab. 2):

* A feature space S is a subset of the normalised features; objects are
  compared by the Euclidean distance over the columns of S (Tab. 2's mean
  distances are means of Euclidean, not squared, distances).
* DSSJ (Sec. 3.5): the range self-join returns, for each object, the other
  objects within distance eps.  Its distance-oblivious metric is the number
  of such neighbours (fewest = most outlying); its distance-aware metric is
  their mean distance (largest = most outlying).  An object with no
  neighbour has mean 0 and is the most outlying on that metric (Sec. 3.7,
  Tab. 2 point 10).
* kNNSJ (Sec. 3.6): the k nearest other objects of each object (Fig. 1b:
  10 points, k = 3, 30 edges, so an object is not its own neighbour).  Its
  distance-oblivious metric is the in-degree of the kNN graph (fewest =
  most outlying); its distance-aware metric is the mean distance to the k
  neighbours (largest = most outlying).
* Ranks (Sec. 3.4): r_i = 0 is the most outlying object; equal metric
  values share a rank.  Tab. 2 shows the ranks are dense (in-degree values
  {0,1,2,3,5,6} have ranks 0..5).

Readings where the paper is silent: the eps ball is closed (D <= eps); at
the k-th distance, ties go to the lower object id; every arithmetic step is
float64 on the float32 inputs, accumulated feature by feature in the order
of the columns of S.
"""
from __future__ import annotations

import numpy as np

_BLOCK = 256


def project(x, mask=None) -> np.ndarray:
    """Columns of ``mask`` (ascending feature index) of the population
    ``x`` [n, F], as float64 [n, d].  ``mask=None`` keeps every column."""
    x = np.asarray(x)
    if mask is None:
        cols = list(range(x.shape[1]))
    else:
        cols = [f for f in range(x.shape[1]) if (int(mask) >> f) & 1]
    return np.ascontiguousarray(x[:, cols], dtype=np.float64)


def pair_distances(q: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Euclidean distances [len(q), len(p)] in float64, summing the squared
    per-feature differences in feature order, then taking the square root."""
    q = np.asarray(q, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    acc = np.zeros((q.shape[0], p.shape[0]), dtype=np.float64)
    for f in range(q.shape[1]):
        t = q[:, f][:, None] - p[:, f][None, :]
        acc += t * t
    return np.sqrt(acc)


def knn(X: np.ndarray, k: int, with_next: bool = False):
    """k nearest other objects of every object (Sec. 3.6, Fig. 1b).

    Neighbours are taken in ascending (distance, id) order, the object
    itself excluded.  Returns ``ids`` int64 [n, k] and ``dist`` float64
    [n, k]; with ``with_next`` also the (k+1)-th distance [n] (+inf when no
    (k+1)-th object exists), which measures how close the k-th choice is to
    a tie.
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if not (1 <= k <= n - 1):
        raise ValueError("need 1 <= k <= n-1")
    ids = np.empty((n, k), dtype=np.int64)
    dist = np.empty((n, k), dtype=np.float64)
    nxt = np.full(n, np.inf)
    for b0 in range(0, n, _BLOCK):
        b1 = min(n, b0 + _BLOCK)
        D = pair_distances(X[b0:b1], X)
        for r in range(b1 - b0):
            i = b0 + r
            row = np.delete(D[r], i)
            cand = np.delete(np.arange(n), i)
            order = np.argsort(row, kind="stable")   # equal distances keep id order
            ids[i] = cand[order[:k]]
            dist[i] = row[order[:k]]
            if k < n - 1:
                nxt[i] = row[order[k]]
    if with_next:
        return ids, dist, nxt
    return ids, dist


def eps_join(X: np.ndarray, eps: float):
    """Range self-join (Sec. 3.5): for every object, the number of other
    objects at distance <= eps and their mean distance (0 when there are
    none).  Returns ``count`` int64 [n], ``mean`` float64 [n]."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    eps = float(eps)
    count = np.zeros(n, dtype=np.int64)
    total = np.zeros(n, dtype=np.float64)
    for b0 in range(0, n, _BLOCK):
        b1 = min(n, b0 + _BLOCK)
        D = pair_distances(X[b0:b1], X)
        hit = D <= eps
        hit[np.arange(b1 - b0), np.arange(b0, b1)] = False
        count[b0:b1] = hit.sum(axis=1)
        total[b0:b1] = np.where(hit, D, 0.0).sum(axis=1)
    mean = np.where(count > 0, total / np.maximum(count, 1), 0.0)
    return count, mean


def eps_pairs(X: np.ndarray, eps: float) -> tuple[np.ndarray, np.ndarray]:
    """The range self-join's result set (Sec. 3.5, the set A of Sec. 3.5.3
    without the self-pairs) in CSR form: ``off`` int64 [n + 1] and ``ids``
    int64, row i = the objects at distance <= eps from object i in
    ascending id order."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    eps = float(eps)
    rows = []
    for b0 in range(0, n, _BLOCK):
        b1 = min(n, b0 + _BLOCK)
        D = pair_distances(X[b0:b1], X)
        for r in range(b1 - b0):
            hit = np.nonzero(D[r] <= eps)[0]
            rows.append(hit[hit != b0 + r])
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    ids = np.concatenate(rows).astype(np.int64) if rows else np.zeros(0, dtype=np.int64)
    return off, ids


def indegree(ids: np.ndarray, n: int) -> np.ndarray:
    """In-degree of the kNN graph (Sec. 3.6.1): how many objects list each
    object among their k neighbours."""
    return np.bincount(np.asarray(ids).ravel(), minlength=n).astype(np.int64)


def dense_rank(keys: np.ndarray) -> np.ndarray:
    """Dense 0-based rank: the number of distinct key values strictly
    smaller than each key (smaller key = more outlying)."""
    _, inv = np.unique(np.asarray(keys), return_inverse=True)
    return inv.astype(np.int64).ravel()


def rank_keys(eps_count, eps_mean, indeg, knn_mean):
    """Keys in which 'smaller' means 'more outlying', per metric (Sec. 3.5.1,
    3.6.1, Tab. 2): neighbour count ascending, mean eps-distance descending
    with objects that have no neighbour first, in-degree ascending, mean
    kNN distance descending."""
    eps_count = np.asarray(eps_count)
    k0 = eps_count.astype(np.float64)
    k1 = -np.where(eps_count > 0, np.asarray(eps_mean, dtype=np.float64), np.inf)
    k2 = np.asarray(indeg).astype(np.float64)
    k3 = -np.asarray(knn_mean, dtype=np.float64)
    return k0, k1, k2, k3


def rank_metrics(eps_count, eps_mean, indeg, knn_mean) -> np.ndarray:
    """The four dense rankings, int64 [4, n], in the order (eps_count,
    eps_mean, indeg, knn_mean)."""
    return np.stack([dense_rank(k) for k in rank_keys(eps_count, eps_mean, indeg, knn_mean)])


def ensemble(ranks: np.ndarray) -> np.ndarray:
    """Mean of an object's four dense ranks, the average over the four
    methods that Sec. 5 suggests for finding objects that are outlying in
    several of them (lower = more outlying)."""
    return np.asarray(ranks, dtype=np.float64).mean(axis=0)


def outlier_scores(X: np.ndarray, k: int, eps: float) -> dict:
    """All four metrics and their ranks for one (population, space) job."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    ids, dist, nxt = knn(X, k, with_next=True)
    count, mean = eps_join(X, eps)
    deg = indegree(ids, n)
    kmean = dist.sum(axis=1) / k
    ranks = rank_metrics(count, mean, deg, kmean)
    return dict(knn_ids=ids, knn_dist=dist, knn_next=nxt, eps_count=count,
                eps_mean=mean, indeg=deg, knn_mean=kmean, rank=ranks, ensemble=ensemble(ranks))


def alert_scores(P: np.ndarray, A: np.ndarray, k: int, eps: float, pop: dict | None = None) -> dict:
    """Score new objects ``A`` against a population ``P`` in one space.

    The paper has no serving path (its use is a batch over a catalogue), so
    this follows the reading adopted for alerts: an alert is scored as if it
    were one extra object that changes nothing in P and sees no other alert.
    Its kNN and eps metrics are taken over P; its in-degree is the number of
    population objects p with D(p, alert) strictly below p's own k-th
    neighbour distance in P; its rank on each metric is the number of
    distinct population key values strictly more outlying than its key.
    """
    P = np.asarray(P, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    n, m = P.shape[0], A.shape[0]
    if pop is None:
        pop = outlier_scores(P, k, eps)
    rk = pop["knn_dist"][:, k - 1]
    D = pair_distances(A, P)                     # [m, n]
    order = np.argsort(D, axis=1, kind="stable")[:, :k]
    ids = order
    dist = np.take_along_axis(D, order, axis=1)
    hit = D <= eps
    count = hit.sum(axis=1)
    mean = np.where(count > 0, np.where(hit, D, 0.0).sum(axis=1) / np.maximum(count, 1), 0.0)
    deg = (D < rk[None, :]).sum(axis=1)
    kmean = dist.sum(axis=1) / k
    pk = rank_keys(pop["eps_count"], pop["eps_mean"], pop["indeg"], pop["knn_mean"])
    ak = rank_keys(count, mean, deg, kmean)
    ranks = np.empty((4, m), dtype=np.int64)
    for t in range(4):
        u = np.unique(pk[t])
        ranks[t] = np.searchsorted(u, ak[t], side="left")
    return dict(knn_ids=ids, knn_dist=dist, eps_count=count, eps_mean=mean,
                indeg=deg, knn_mean=kmean, rank=ranks)


def selectivity(X: np.ndarray, eps: float) -> float:
    """Selectivity s = (|A| - |D|) / |D| of Sec. 3.5.3, where the result set
    A of the self-join includes every object paired with itself: the mean
    number of other objects within eps."""
    count, _ = eps_join(X, eps)
    n = np.asarray(X).shape[0]
    size_a = int(count.sum()) + n
    return (size_a - n) / n


def eps_exact_mean_count(X: np.ndarray, target: int) -> np.float32:
    """eps giving a mean neighbour count of exactly ``target`` (even total):
    the midpoint between the (target*n/2)-th and next smallest of the
    n(n-1)/2 pair distances, rounded to float32."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    D = pair_distances(X, X)
    iu = np.triu_indices(n, 1)
    d = np.sort(D[iu])
    m = target * n // 2
    return np.float32(0.5 * (d[m - 1] + d[m]))


def eps_from_sample(X: np.ndarray, sample: np.ndarray, target: float) -> np.float32:
    """Sampled-distance choice of eps (Sec. 3.5.3) for a given sample: the
    distances of the ``sample`` objects to every other object, and the radius
    at which the sample's mean neighbour count reaches ``target`` (the
    midpoint between the round(target * m)-th smallest of them and the next),
    as float32."""
    X = np.asarray(X, dtype=np.float64)
    sample = np.asarray(sample, dtype=np.int64)
    m = sample.size
    D = pair_distances(X[sample], X)
    D[np.arange(m), sample] = np.inf
    flat = D.ravel()
    r = int(round(target * m))
    r = max(1, min(r, flat.size - 1))
    part = np.partition(flat, (r - 1, r))
    return np.float32(0.5 * (part[r - 1] + part[r]))


def eps_sampled_mean_count(X: np.ndarray, target: float, m: int, seed: int) -> np.float32:
    """eps_from_sample with ``m`` seeded distinct objects (sorted ids)."""
    n = np.asarray(X).shape[0]
    m = min(m, n)
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(n, size=m, replace=False))
    return eps_from_sample(X, sample, target)


# ------------------------------------------------ eps-grid selection (F1) ---

def top_n(ranks: np.ndarray, n: int) -> np.ndarray:
    """The n most outlying objects of one ranking: the first n ids in
    (rank, id) order (Sec. 3.5.2 compares the top n = 1 % of |D| of two ranked
    lists; ties of rank are taken in ascending id)."""
    ranks = np.asarray(ranks)
    order = np.lexsort((np.arange(ranks.size), ranks))
    return order[:n]


def list_similarity(top_a: np.ndarray, top_b: np.ndarray, n: int) -> float:
    """Eq. 2: the fraction of the n objects that are in both top-n lists."""
    return len(set(np.asarray(top_a).tolist()) & set(np.asarray(top_b).tolist())) / n


def select_tradeoff(u_min: np.ndarray, u_max: np.ndarray) -> int:
    """Eq. 3: the grid index j minimising |U^min_j - U^max_j| (the first one
    if several tie)."""
    return int(np.argmin(np.abs(np.asarray(u_min, dtype=np.float64) - np.asarray(u_max, dtype=np.float64))))


def eps_grid(eps_min: float, eps_max: float, g: int) -> np.ndarray:
    """The evenly spaced grid G of Sec. 3.5.2 from eps_min to eps_max, as
    float32 (the values both sides use)."""
    j = np.arange(g, dtype=np.float64)
    return (eps_min + (eps_max - eps_min) * j / (g - 1)).astype(np.float32)


def eps_grid_metrics(X: np.ndarray, eps_list) -> tuple[np.ndarray, np.ndarray]:
    """Neighbour count and mean neighbour distance of every object at every
    radius of the grid ([g, n] each); the result sets of smaller radii are
    subsets of the largest one (Sec. 3.5.3, Fig. 4)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    g = len(eps_list)
    count = np.zeros((g, n), dtype=np.int64)
    mean = np.zeros((g, n), dtype=np.float64)
    for a in range(0, n, 512):
        D = pair_distances(X[a:a + 512], X)
        D[np.arange(D.shape[0]), np.arange(a, a + D.shape[0])] = np.inf
        for j, e in enumerate(eps_list):
            hit = D <= float(e)
            c = hit.sum(axis=1)
            s = np.where(hit, D, 0.0).sum(axis=1)
            count[j, a:a + D.shape[0]] = c
            mean[j, a:a + D.shape[0]] = np.where(c > 0, s / np.maximum(c, 1), 0.0)
    return count, mean


def _grid_select(keys_at, g: int, n_top: int) -> dict:
    """Sec. 3.5.2 / 3.6.2 given the ranking keys of both metrics at every
    grid point (keys_at(j) -> (key of metric 0, key of metric 1)): top n per
    ranking, Eq. 2 similarities to the first (U^min) and last (U^max) grid
    point, and Eq. 3 on the exact intersection counts."""
    u = np.zeros((2, 2, g))
    sel = np.zeros(2, dtype=np.int64)
    keys = [keys_at(j) for j in range(g)]
    for metric in range(2):
        tops = [top_n(dense_rank(keys[j][metric]), n_top) for j in range(g)]
        both = np.zeros((2, g), dtype=np.int64)
        for j in range(g):
            both[0, j] = len(set(tops[0].tolist()) & set(tops[j].tolist()))
            both[1, j] = len(set(tops[g - 1].tolist()) & set(tops[j].tolist()))
            u[metric, 0, j] = list_similarity(tops[0], tops[j], n_top)
            u[metric, 1, j] = list_similarity(tops[g - 1], tops[j], n_top)
        # the same n divides both, so the exact gaps compare as integers
        sel[metric] = select_tradeoff(both[0], both[1])
    return dict(similarity=u, select=sel)


def k_grid_metrics(X: np.ndarray, ks) -> tuple[np.ndarray, np.ndarray]:
    """In-degree and mean kNN distance of every object for every k of the
    grid ([g, n] each), from the k_max lists, which hold those of every
    smaller k (Sec. 3.6.2)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    kmax = int(max(ks))
    ids, dist = knn(X, kmax)
    deg = np.zeros((len(ks), n), dtype=np.int64)
    kmean = np.zeros((len(ks), n), dtype=np.float64)
    for j, k in enumerate(ks):
        deg[j] = indegree(ids[:, :k], n)
        kmean[j] = dist[:, :k].sum(axis=1) / k
    return deg, kmean


def k_grid_select(indeg: np.ndarray, kmean: np.ndarray, n_top: int) -> dict:
    """Sec. 3.6.2 on given per-k metrics: metric 0 is the in-degree
    (ascending), metric 1 the mean kNN distance (descending)."""
    g = indeg.shape[0]
    return _grid_select(lambda j: rank_keys(indeg[j], kmean[j], indeg[j], kmean[j])[2:], g, n_top)


def eps_grid_select(count: np.ndarray, mean: np.ndarray, n_top: int) -> dict:
    """Sec. 3.5.2 on given per-radius metrics: for both DSSJ metrics (number
    of neighbours, mean neighbour distance) the ranking at every radius, the
    similarity of its top n to those of the smallest and largest radius
    (U^min, U^max, Eq. 2) and the selected grid index (Eq. 3)."""
    g = count.shape[0]
    return _grid_select(lambda j: rank_keys(count[j], mean[j], count[j], mean[j])[:2], g, n_top)