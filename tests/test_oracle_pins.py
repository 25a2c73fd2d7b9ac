"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code: printed values of
the paper's worked examples, closed forms, textbook reductions, a second
library (scipy's k-d tree), pure-Python brute force on tiny inputs, and
invariants.  None of them needs a GPU.
"""
from __future__ import annotations

import bisect
import itertools
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle as O
from oracle import c_oracle as C
from tests.golden import exact_fp32_variant, load_fig3, load_tab2
import snaps_synth as S


# ------------------------------------------------ paper's worked examples ---

def _check_tab2(res, table, edges, mean_scale=1.0):
    np.testing.assert_array_equal(res["eps_count"], table[:, 0])
    np.testing.assert_array_equal(np.round(res["eps_mean"] * mean_scale, 4), table[:, 2])
    np.testing.assert_array_equal(res["indeg"], table[:, 4])
    np.testing.assert_array_equal(np.round(res["knn_mean"] * mean_scale, 4), table[:, 6])
    np.testing.assert_array_equal(res["rank"][0], table[:, 1])
    np.testing.assert_array_equal(res["rank"][1], table[:, 3])
    np.testing.assert_array_equal(res["rank"][2], table[:, 5])
    np.testing.assert_array_equal(res["rank"][3], table[:, 7])
    for i, nb in edges.items():
        assert set(res["knn_ids"][i].tolist()) == nb, f"point {i + 1}"


def test_tab2_fig1_float64():
    """All 40 values and 40 ranks of Tab. 2 and the 30 edges of Fig. 1b."""
    coords, eps, k, table, edges = load_tab2()
    _check_tab2(O.outlier_scores(coords, k, eps), table, edges)


def test_tab2_fig1_exact_fp32_variant():
    """Same example with coordinates rescaled to exact float32 dyadics;
    distances scale by 100/512, counts, in-degrees and ranks are unchanged,
    and point 1's exact tie (points 2 and 4 at the same distance) is won by
    the lower id, as in Fig. 1b."""
    coords, eps, k, table, edges = load_tab2()
    x = exact_fp32_variant(coords)
    e = np.float32(67.0 / 512.0)
    d12 = O.pair_distances(x[[0]], x[[1]])[0, 0]
    d14 = O.pair_distances(x[[0]], x[[3]])[0, 0]
    assert d12 == d14                                    # an exact tie
    _check_tab2(O.outlier_scores(x, k, e), table, edges, mean_scale=5.12)
    _check_tab2(C.outlier_scores(x, k, float(e)), table, edges, mean_scale=5.12)


def test_tab2_dense_not_competition_ranks():
    """Tab. 2's in-degree ranks {0,1,2,3,5,6} -> 0..5 are dense ranks."""
    coords, eps, k, table, _ = load_tab2()
    assert O.dense_rank(np.array([5, 6, 6, 3, 2, 3, 2, 2, 1, 0])).tolist() == table[:, 5].tolist()
    assert O.dense_rank(np.array([3, 1, 3, 2])).tolist() == [2, 0, 2, 1]


def test_ensemble_of_tab2():
    """Sec. 5's average over the four methods.  Tab. 2: only point 10 has
    rank 0 in all four methods, so it alone has ensemble score 0 and is the
    most outlying by it; every other point has some positive rank.  The
    score is the mean of the printed ranks whatever the method order, lies
    between the smallest and largest of them, and equals r when all four
    are r."""
    coords, eps, k, table, _ = load_tab2()
    out = O.outlier_scores(coords, k, eps)
    ens = out["ensemble"]
    printed = table[:, [1, 3, 5, 7]].T          # eps_count, eps_mean, indeg, knn_mean ranks
    assert np.nonzero(ens == 0)[0].tolist() == [9]
    assert (ens[:9] > 0).all()
    np.testing.assert_array_equal(ens, O.ensemble(printed[::-1]))
    assert ((ens >= printed.min(axis=0)) & (ens <= printed.max(axis=0))).all()
    same = np.full((4, 5), 3)
    assert (O.ensemble(same) == 3).all()


def test_fig3_nested_result_sets():
    coords, eps, k, _, _ = load_tab2()
    q, sets = load_fig3()
    D = O.pair_distances(q[None, :], coords)[0]
    prev = set()
    for r, expect in sets:
        got = set(np.nonzero(D <= r)[0].tolist())
        assert got == expect
        assert prev <= got                                # nested
        prev = got
        a = O.alert_scores(coords, q[None, :], k, r)
        assert a["eps_count"][0] == len(expect)
    assert 8 not in prev and 9 not in prev


# ------------------------------------------------------------ closed forms ---

@pytest.mark.parametrize("m,k", [(7, 3), (5, 1), (9, 8)])
def test_identical_points_closed_form(m, k):
    x = np.full((m, 3), 0.25, dtype=np.float32)
    r = O.outlier_scores(x, k, 0.01)
    for i in range(m):
        assert r["knn_ids"][i].tolist() == [j for j in range(m) if j != i][:k]
    expect = np.array([m - 1 if j < k else (k if j == k else 0) for j in range(m)])
    np.testing.assert_array_equal(r["indeg"], expect)
    np.testing.assert_array_equal(r["eps_count"], m - 1)
    np.testing.assert_array_equal(r["eps_mean"], 0.0)
    np.testing.assert_array_equal(r["knn_mean"], 0.0)
    assert O.selectivity(x, 0.01) == m - 1


def _lattice(w=12, h=2.0 ** -6, origin=0.25):
    ij = np.array([(r, c) for r in range(w) for c in range(w)])
    return (origin + h * ij).astype(np.float32), ij, w, h


def test_dyadic_lattice_counts_and_ties():
    x, ij, w, h = _lattice()
    interior = [(r * w + c) for r in range(1, w - 1) for c in range(1, w - 1)]
    cnt, mean = O.eps_join(x, h * (1 + 1e-6))
    assert (cnt[interior] == 4).all()
    np.testing.assert_allclose(mean[interior], h, rtol=0, atol=0)
    cnt, _ = O.eps_join(x, h * math.sqrt(2) * (1 + 1e-6))
    assert (cnt[interior] == 8).all()
    cnt, _ = O.eps_join(x, h)                         # closed ball: exactly h counts
    assert (cnt[interior] == 4).all()
    cnt, _ = O.eps_join(x, h * (1 - 1e-6))
    assert (cnt[interior] == 0).all()
    ids, dist = O.knn(x, 4)
    for i in interior:
        r, c = divmod(i, w)
        assert set(ids[i].tolist()) == {(r - 1) * w + c, r * w + c - 1, r * w + c + 1, (r + 1) * w + c}
        assert (dist[i] == h).all()
    ids, _ = O.knn(x, 2)                               # a four-way tie: lowest ids win
    for i in interior:
        r, c = divmod(i, w)
        assert ids[i].tolist() == [(r - 1) * w + c, r * w + c - 1]


def test_degenerate_eps_and_k():
    rng = np.random.default_rng(3)
    x = rng.random((23, 4)).astype(np.float32)
    n = x.shape[0]
    mean_all = [sum(math.dist(x[i].astype(float), x[j].astype(float)) for j in range(n) if j != i) / (n - 1)
                for i in range(n)]
    cnt, mean = O.eps_join(x, math.sqrt(4) + 1e-9)
    assert (cnt == n - 1).all()
    np.testing.assert_allclose(mean, mean_all, rtol=1e-13)
    r = O.outlier_scores(x, n - 1, 0.1)
    assert (r["indeg"] == n - 1).all()
    np.testing.assert_allclose(r["knn_mean"], mean_all, rtol=1e-13)
    assert (r["rank"][2] == 0).all()


# ---------------------------------------------------- textbook reductions ---

def test_one_dimensional_reduction():
    """A 2-D space whose second feature is constant is a 1-D problem:
    k nearest by a two-pointer walk outward from the sorted position, and
    the range count by bisection on the sorted values."""
    rng = np.random.default_rng(11)
    n, k, eps = 400, 6, 0.01
    v = rng.random(n)
    x = np.stack([v, np.full(n, 0.5)], axis=1).astype(np.float32)
    v32 = x[:, 0].astype(np.float64)
    order = np.argsort(v32, kind="stable")
    sv = v32[order]
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    r = O.outlier_scores(x, k, eps)
    for i in range(n):
        lo, hi, got = pos[i] - 1, pos[i] + 1, []
        while len(got) < k:
            dl = v32[i] - sv[lo] if lo >= 0 else math.inf
            dh = sv[hi] - v32[i] if hi < n else math.inf
            if dl <= dh:
                got.append(order[lo]); lo -= 1
            else:
                got.append(order[hi]); hi += 1
        assert set(got) == set(r["knn_ids"][i].tolist())
        c = bisect.bisect_right(sv, v32[i] + eps) - bisect.bisect_left(sv, v32[i] - eps) - 1
        assert c == r["eps_count"][i]


@pytest.mark.parametrize("d", [2, 3, 5])
def test_scipy_kdtree_crosscheck(d):
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(100 + d)
    x = rng.random((300, d)).astype(np.float32)
    k, eps = 7, 0.15 * d ** 0.5
    xd = x.astype(np.float64)
    tree = cKDTree(xd)
    dd, ii = tree.query(xd, k + 1)
    r = O.outlier_scores(x, k, eps)
    for i in range(x.shape[0]):
        assert set(ii[i, 1:].tolist()) == set(r["knn_ids"][i].tolist())
    np.testing.assert_allclose(r["knn_dist"], dd[:, 1:], rtol=1e-12)
    counts = np.array([len(b) - 1 for b in tree.query_ball_point(xd, eps)])
    np.testing.assert_array_equal(counts, r["eps_count"])


def _py_brute(x, k, eps):
    """Pure-Python O(n^2) reference: sorted() over (distance, id) pairs."""
    n = len(x)
    out = []
    for i in range(n):
        ds = []
        for j in range(n):
            if j == i:
                continue
            acc = 0.0
            for f in range(len(x[i])):
                t = float(x[i][f]) - float(x[j][f])
                acc += t * t
            ds.append((math.sqrt(acc), j))
        ds.sort()
        nn = ds[:k]
        within = [dj for dj, _ in ds if dj <= eps]
        out.append(([j for _, j in nn], [dj for dj, _ in nn], len(within),
                    (sum(within) / len(within)) if within else 0.0))
    return out


@settings(max_examples=60, deadline=None)
@given(st.integers(3, 11), st.integers(1, 4), st.integers(0, 10**6), st.integers(0, 3))
def test_pure_python_bruteforce_with_ties(n, d, seed, grid):
    """Tiny inputs on a coarse grid, so duplicates and exact ties abound."""
    rng = np.random.default_rng(seed)
    levels = [2, 3, 5, 1 << 20][grid]
    x = (rng.integers(0, levels, size=(n, d)) / float(levels)).astype(np.float32)
    k = int(rng.integers(1, n))
    eps = float(rng.choice([0.0, 0.2, 0.5, 1.0]))
    r = O.outlier_scores(x, k, eps)
    ref = _py_brute(x.tolist(), k, eps)
    deg = [0] * n
    for i, (ids, ds, c, m) in enumerate(ref):
        assert r["knn_ids"][i].tolist() == ids
        assert r["knn_dist"][i].tolist() == ds
        assert r["eps_count"][i] == c
        assert abs(r["eps_mean"][i] - m) <= 1e-12 * max(1.0, m)
        for j in ids:
            deg[j] += 1
    assert r["indeg"].tolist() == deg
    rc = C.outlier_scores(x, k, eps)
    np.testing.assert_array_equal(rc["knn_ids"], r["knn_ids"])
    np.testing.assert_array_equal(rc["eps_count"], r["eps_count"])
    np.testing.assert_array_equal(rc["rank"][[0, 2, 3]], r["rank"][[0, 2, 3]])


# -------------------------------------------------------------- invariants ---

def _blob(n=500, d=4, seed=5):
    rng = np.random.default_rng(seed)
    return rng.random((n, d)).astype(np.float32)


def test_invariants_symmetry_and_sums():
    x = _blob()
    n, k, eps = x.shape[0], 9, 0.2
    r = O.outlier_scores(x, k, eps)
    D = O.pair_distances(x, x)
    rel = (D <= eps) & ~np.eye(n, dtype=bool)
    assert (rel == rel.T).all()
    assert r["eps_count"].sum() % 2 == 0
    assert r["indeg"].sum() == n * k
    assert abs(O.selectivity(x, eps) - r["eps_count"].mean()) < 1e-12


def test_invariants_monotone_in_k_and_eps():
    x = _blob(300, 3)
    prev_kth, prev_mean = None, None
    for k in (1, 2, 5, 10, 20):
        _, dist = O.knn(x, k)
        kth, mean = dist[:, -1], dist.mean(axis=1)
        if prev_kth is not None:
            assert (kth >= prev_kth).all() and (mean >= prev_mean - 1e-15).all()
        prev_kth, prev_mean = kth, mean
    prev = None
    for eps in (0.01, 0.05, 0.1, 0.3, 2.0):
        c, _ = O.eps_join(x, eps)
        if prev is not None:
            assert (c >= prev).all()
        prev = c


def test_invariants_translation_permutation_relabel():
    x = _blob(200, 4, seed=9)
    k, eps = 5, 0.25
    r = O.outlier_scores(x, k, eps)
    shifted = (x.astype(np.float64) + 0.125).astype(np.float32)   # dyadic shift
    rs = O.outlier_scores(shifted, k, eps)
    np.testing.assert_array_equal(rs["knn_ids"], r["knn_ids"])
    np.testing.assert_allclose(rs["knn_mean"], r["knn_mean"], rtol=1e-6)
    rp = O.outlier_scores(x[:, [2, 0, 3, 1]], k, eps)
    np.testing.assert_array_equal(rp["knn_ids"], r["knn_ids"])
    np.testing.assert_array_equal(rp["eps_count"], r["eps_count"])
    np.testing.assert_allclose(rp["eps_mean"], r["eps_mean"], rtol=1e-13)
    perm = np.random.default_rng(1).permutation(x.shape[0])
    rr = O.outlier_scores(x[perm], k, eps)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    for key in ("eps_count", "indeg", "knn_mean", "eps_mean"):
        np.testing.assert_allclose(rr[key], r[key][perm], rtol=1e-13)
    np.testing.assert_array_equal(rr["rank"], r["rank"][:, perm])
    np.testing.assert_array_equal(np.sort(perm[rr["knn_ids"]], axis=1), np.sort(r["knn_ids"][perm], axis=1))


def test_isolated_points_rank_first():
    x, corners = S.gen_isolated_fixture()
    k, eps = 5, 0.1
    r = O.outlier_scores(x, k, eps)
    m = len(corners)
    assert (r["eps_count"][corners] == 0).all()
    assert (r["rank"][0][corners] == 0).all()
    assert (r["rank"][1][corners] == 0).all()
    assert (r["indeg"][corners] == 0).all() and (r["rank"][2][corners] == 0).all()
    assert sorted(r["rank"][3][corners].tolist()) == list(range(m))
    others = np.setdiff1d(np.arange(x.shape[0]), corners)
    assert (r["rank"][0][others] > 0).all() and (r["rank"][3][others] >= m).all()


# --------------------------------------------------------------- alerts ---

def test_alert_scores_against_brute_force():
    rng = np.random.default_rng(21)
    P = rng.random((60, 3)).astype(np.float32)
    A = rng.random((7, 3)).astype(np.float32)
    k, eps = 4, 0.3
    pop = O.outlier_scores(P, k, eps)
    a = O.alert_scores(P, A, k, eps, pop)
    Pl, Al = P.astype(float), A.astype(float)
    rk = [sorted(math.dist(Pl[p], Pl[j]) for j in range(60) if j != p)[k - 1] for p in range(60)]
    keys = O.rank_keys(pop["eps_count"], pop["eps_mean"], pop["indeg"], pop["knn_mean"])
    for i in range(7):
        ds = sorted((math.dist(Al[i], Pl[j]), j) for j in range(60))
        assert a["knn_ids"][i].tolist() == [j for _, j in ds[:k]]
        within = [dj for dj, _ in ds if dj <= eps]
        assert a["eps_count"][i] == len(within)
        assert a["indeg"][i] == sum(1 for p in range(60) if math.dist(Al[i], Pl[p]) < rk[p])
        akeys = O.rank_keys([a["eps_count"][i]], [a["eps_mean"][i]], [a["indeg"][i]], [a["knn_mean"][i]])
        for t in range(4):
            assert a["rank"][t][i] == len({v for v in keys[t] if v < akeys[t][0]})


# ------------------------------------------------- eps rules, ingest ---

def test_eps_rules_on_c0():
    x, k = S.gen_c0()
    e = O.eps_exact_mean_count(x, 10)
    c, _ = O.eps_join(x, e)
    assert c.sum() == 10 * x.shape[0]
    es = O.eps_sampled_mean_count(x, 10, 256, seed=1)
    rng = np.random.default_rng(1)
    sample = np.sort(rng.choice(x.shape[0], size=256, replace=False))
    D = O.pair_distances(x[sample], x)
    D[np.arange(256), sample] = np.inf
    assert abs((D <= es).sum() / 256 - 10) <= 1 / 256


def test_normalisation_definition():
    raw = np.array([[1.0, 5.0, 2.0], [3.0, 5.0, -2.0], [2.0, 5.0, 0.0]])
    x, lo, hi = S.normalize_minmax(raw)
    np.testing.assert_array_equal(x[:, 0], [0.0, 1.0, 0.5])
    np.testing.assert_array_equal(x[:, 1], 0.0)
    np.testing.assert_array_equal(x[:, 2], [1.0, 0.0, 0.5])
    c1, _, _ = S.gen_c1()
    assert c1.dtype == np.float32 and c1.min() == 0.0 and c1.max() == 1.0
    assert len(S.all_masks()) == 32752 == sum(math.comb(15, i) for i in range(2, 16))


def test_c_twin_matches_numpy_oracle():
    rng = np.random.default_rng(8)
    for n, d, k in [(257, 3, 5), (130, 7, 10), (64, 15, 20)]:
        x = (rng.integers(0, 50, size=(n, d)) / 50.0).astype(np.float32)   # many ties
        eps = 0.3
        a = O.outlier_scores(x, k, eps)
        b = C.outlier_scores(x, k, eps)
        np.testing.assert_array_equal(a["knn_ids"], b["knn_ids"])
        np.testing.assert_array_equal(a["knn_dist"], b["knn_dist"])
        np.testing.assert_array_equal(a["knn_next"], b["knn_next"])
        np.testing.assert_array_equal(a["eps_count"], b["eps_count"])
        np.testing.assert_allclose(a["eps_mean"], b["eps_mean"], rtol=1e-13)
        np.testing.assert_array_equal(a["rank"][[0, 2, 3]], b["rank"][[0, 2, 3]])


def test_c_twin_query_subset_mode():
    """The subset mode (used for sampled parity at large n) returns exactly
    the rows of the full self-join."""
    rng = np.random.default_rng(31)
    x = (rng.integers(0, 40, size=(700, 4)) / 40.0).astype(np.float32)
    full = C.join(x, 7, 0.2, band=(0.19, 0.21))
    q = np.array([0, 5, 123, 699, 350])
    sub = C.join(x, 7, 0.2, band=(0.19, 0.21), qids=q)
    for key in ("knn_ids", "knn_dist", "knn_next", "eps_count", "eps_sum", "band"):
        np.testing.assert_array_equal(sub[key], full[key][q])


# ------------------------------------------------ eps-grid selection ---

def test_eps_selection_worked_example():
    """Sec. 3.5.2's example: Eq. 2 on the three printed top-10 sets gives the
    printed U^min = {1.0, 0.4, 0.2} and U^max = {0.2, 0.5, 1.0}; Eq. 3 then
    selects the middle radius (|0.4 - 0.5| is the smallest gap); a list
    compared with itself matches fully."""
    from tests.golden import load_eps_select_example
    n, sets, umin, umax = load_eps_select_example()
    got_min = [O.list_similarity(sets[0], s, n) for s in sets]
    got_max = [O.list_similarity(sets[-1], s, n) for s in sets]
    assert got_min == umin and got_max == umax
    assert O.select_tradeoff(got_min, got_max) == 1
    assert O.select_tradeoff([1.0, 0.6, 0.5, 0.2], [0.2, 0.5, 0.6, 1.0]) == 1   # first of two equal gaps


def test_top_n_takes_ties_in_id_order():
    ranks = np.array([2, 0, 1, 0, 1, 3])
    assert O.top_n(ranks, 3).tolist() == [1, 3, 2]
    assert O.top_n(ranks, 6).tolist() == [1, 3, 2, 4, 0, 5]


def test_eps_grid_metrics_nested_and_equal_to_the_join():
    """The grid's result sets are nested (counts and sums grow with the
    radius, Sec. 3.5.3) and each equals the plain eps-join at that radius."""
    rng = np.random.default_rng(21)
    x = rng.random((300, 3))
    grid = O.eps_grid(0.05, 0.3, 6)
    count, mean = O.eps_grid_metrics(x, grid)
    assert (np.diff(count, axis=0) >= 0).all()
    sums = count * mean
    assert (np.diff(sums, axis=0) >= -1e-12).all()
    for j, e in enumerate(grid):
        c, m = O.eps_join(x, float(e))
        np.testing.assert_array_equal(count[j], c)
        np.testing.assert_allclose(mean[j], m, rtol=1e-12)
    np.testing.assert_allclose(grid, [0.05, 0.1, 0.15, 0.2, 0.25, 0.3], rtol=1e-7)
    sel = O.eps_grid_select(count, mean, 3)
    assert sel["similarity"].shape == (2, 2, 6)
    assert (sel["similarity"][:, 0, 0] == 1.0).all() and (sel["similarity"][:, 1, -1] == 1.0).all()


def test_k_grid_metrics_against_the_plain_knn():
    """Per-k metrics from the k_max lists equal the plain kNN self-join at
    every k (the lists of smaller k are prefixes, Sec. 3.6.2); in-degree
    sums to n k; mean kNN distance grows with k."""
    rng = np.random.default_rng(33)
    x = rng.random((200, 3))
    ks = [2, 5, 11, 40]
    deg, km = O.k_grid_metrics(x, ks)
    for j, k in enumerate(ks):
        ref = O.outlier_scores(x, k, 0.1)
        np.testing.assert_array_equal(deg[j], ref["indeg"])
        np.testing.assert_allclose(km[j], ref["knn_mean"], rtol=1e-12)
        assert deg[j].sum() == 200 * k
    assert (np.diff(km, axis=0) >= -1e-12).all()
    sel = O.k_grid_select(deg, km, 4)
    assert (sel["similarity"][:, 0, 0] == 1.0).all() and (sel["similarity"][:, 1, -1] == 1.0).all()


def test_k_grid_metrics_against_scipy_kdtree():
    """In-degree and mean kNN distance at every k of a grid against scipy's
    cKDTree (k + 1 nearest including self; continuous data, no ties)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(34)
    x = rng.random((250, 4))
    ks = [1, 3, 8, 30]
    deg, km = O.k_grid_metrics(x, ks)
    dist, ids = cKDTree(x).query(x, k=max(ks) + 1)
    for j, k in enumerate(ks):
        nb = ids[:, 1:k + 1]
        assert (nb != np.arange(250)[:, None]).all()
        np.testing.assert_array_equal(deg[j], np.bincount(nb.ravel(), minlength=250))
        np.testing.assert_allclose(km[j], dist[:, 1:k + 1].mean(axis=1), rtol=1e-12)


def test_grid_selection_by_hand():
    """Eq. 2-3 on per-grid-point metrics whose top-2 lists are known by
    hand.  In-degree (ascending) tops are {0,1}, {1,2}, {2,3}: U^min =
    (1, .5, 0), U^max = (0, .5, 1), so the middle point is selected.  The
    mean kNN distance ranks descending: tops {5,6}, {5,7}, {7,8} give U^min =
    (1, .5, 0), U^max = (0, .5, 1) again.  The radius grid ranks its mean
    the same way except that objects with no neighbour come first."""
    n = 10
    deg = np.full((3, n), 5)
    deg[0, [0, 1]] = [0, 1]
    deg[1, [1, 2]] = [0, 1]
    deg[2, [2, 3]] = [1, 0]
    km = np.ones((3, n))
    km[0, [5, 6]] = [3.0, 2.0]
    km[1, [5, 7]] = [2.0, 3.0]
    km[2, [7, 8]] = [3.0, 3.0]
    sel = O.k_grid_select(deg, km, 2)
    for metric in (0, 1):
        np.testing.assert_allclose(sel["similarity"][metric, 0], [1.0, 0.5, 0.0])
        np.testing.assert_allclose(sel["similarity"][metric, 1], [0.0, 0.5, 1.0])
    assert sel["select"].tolist() == [1, 1]
    # radius grid: object 9 has no neighbour at the first radius, so it leads
    # the mean ranking there although its mean is the smallest (0): tops
    # {9, 5}, {7, 5}, {8, 9} (without that rule the first would be {5, 6}
    # and U^min_3 would be 0)
    cnt = np.full((3, n), 4)
    cnt[0, 9] = 0
    mean = np.ones((3, n))
    mean[0, [5, 6, 9]] = [3.0, 2.0, 0.0]
    mean[1, [5, 7]] = [2.0, 3.0]
    mean[2, [8, 9]] = [3.0, 3.0]
    sel = O.eps_grid_select(cnt, mean, 2)
    np.testing.assert_allclose(sel["similarity"][1, 0], [1.0, 0.5, 0.5])
    np.testing.assert_allclose(sel["similarity"][1, 1], [0.5, 0.0, 1.0])
    assert int(sel["select"][1]) == 0


def test_eps_pairs_against_scipy_ball_query():
    """The pair list of the range join equals scipy's ball query (closed
    ball, self removed, ids ascending) row by row, and its row lengths are
    the join's counts."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(35)
    x = rng.random((300, 3))
    eps = 0.12
    off, ids = O.eps_pairs(x, eps)
    balls = cKDTree(x).query_ball_point(x, eps)
    for i in range(300):
        ref = sorted(j for j in balls[i] if j != i)
        assert ids[off[i]:off[i + 1]].tolist() == ref
    c, _ = O.eps_join(x, eps)
    np.testing.assert_array_equal(np.diff(off), c)
