"""kNN metrics and lists for k above the fused join's register lists (the
selection kernel): against the float64 oracle at k = 64, 256 and 4,096
(the paper's k_max, Sec. 3.6.2), exact ties at the k-th distance (the id
tie-break, closed form), mixed with small-k jobs in one batched call and in
a captured plan, and sampled at a population above one LDS."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from oracle import c_oracle as C
from tests.parity import TAU, check_knn, check_scores, knn_strict

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_20176_amd import snaps
    snaps.load_library()
    return snaps


def full_oracle(x, k, eps):
    """The NumPy oracle's scores and lists (any k), with the eps band counts
    of the C twin (k = 0: range side only)."""
    ora = O.outlier_scores(x, k, eps)
    ora["band"] = C.join(x, 0, eps, band=(eps * (1 - TAU), eps * (1 + TAU)))["band"]
    return ora


def out_of(job):
    keys = ("eps_count", "eps_mean", "indeg", "knn_mean", "rank", "knn_ids", "knn_dist")
    return {key: (None if getattr(job, key) is None else getattr(job, key).cpu().numpy()) for key in keys}


@pytest.mark.parametrize("k", [64, 256, 4096])
def test_large_k_scores_and_lists_against_oracle(S, k):
    rng = np.random.default_rng(k)
    n = 6000
    x = (rng.random((n, 6)) ** 1.5).astype(np.float32)
    mask = 0b101101
    xs = O.project(x, mask).astype(np.float32)
    eps = 0.12
    pop = S.Population.from_rows(x)
    job = S.Job.alloc(pop, mask, k, eps, with_lists=True)
    S.snaps_outlier_scores([job])
    torch.cuda.synchronize()
    g = out_of(job)
    rep = check_scores(g, full_oracle(xs, k, eps), k, eps, label=f"k={k}")
    print(f"k={k}: exempt {rep}")
    # snaps_knn_selfjoin gives the same lists
    ids = torch.empty((n, k), dtype=torch.int32, device="cuda")
    dist = torch.empty((n, k), dtype=torch.float32, device="cuda")
    S.snaps_knn_selfjoin(pop, mask, k, ids, dist)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ids.cpu().numpy(), g["knn_ids"])
    np.testing.assert_array_equal(dist.cpu().numpy(), g["knn_dist"])


def test_large_k_exact_ties_take_the_lower_ids(S):
    """m identical objects (ids 0..m-1) among others far away: with k < m
    each copy's neighbours are the first k other copies, in id order, at
    distance 0; in-degree is m - 1 for ids below k, k for id k, 0 above."""
    rng = np.random.default_rng(11)
    m, k, n = 400, 150, 2000
    x = np.empty((n, 3), dtype=np.float32)
    x[:m] = 0.25
    x[m:] = 0.5 + 0.5 * rng.random((n - m, 3)).astype(np.float32)
    pop = S.Population.from_rows(x)
    job = S.Job.alloc(pop, 0b111, k, 0.01, with_lists=True)
    S.snaps_outlier_scores([job])
    torch.cuda.synchronize()
    g = out_of(job)
    for i in (0, 1, k - 1, k, k + 1, m - 1):
        want = [j for j in range(m) if j != i][:k]
        assert g["knn_ids"][i].tolist() == want, i
        assert (g["knn_dist"][i] == 0).all()
    deg = g["indeg"][:m]
    assert (deg[:k] == m - 1).all() and deg[k] == k and (deg[k + 1:] == 0).all()
    assert (g["eps_count"][:m] == m - 1).all() and (g["eps_mean"][:m] == 0).all()
    check_scores(g, full_oracle(x, k, 0.01), k, 0.01, label="ties")


def test_large_k_mixed_with_small_k_batched_and_planned(S):
    """Jobs of k = 7 (fused join) and k = 100, 700 (selection kernel), with and
    without lists, in one call and in a captured plan replayed twice: equal,
    bit for bit, to each job run alone."""
    rng = np.random.default_rng(5)
    x = rng.random((3000, 8)).astype(np.float32)
    pop = S.Population.from_rows(x)
    specs = [(0b111, 7, 0.05, True), (0b1111, 100, 0.1, True), (0b11110000, 700, 0.2, False),
             (0b11, 100, 0.02, False)]

    def alloc():
        return [S.Job.alloc(pop, m, k, e, with_lists=lists) for m, k, e, lists in specs]

    alone = []
    for j in alloc():
        S.snaps_outlier_scores([j])
        alone.append(j)
    torch.cuda.synchronize()
    together = alloc()
    S.snaps_outlier_scores(together)
    planned = alloc()
    tune = [S.tuning(passes=p) for p in (S.PASS_INDEX, S.PASS_JOIN, S.PASS_RANK)]
    ws = torch.empty(S.snaps_outlier_scores_workspace(planned, tune[1]), dtype=torch.uint8, device="cuda")
    plans = [S.Plan(planned, t, ws=ws) for t in tune]
    for _ in range(2):
        for p in plans:
            p.launch()
    torch.cuda.synchronize()
    for a, b, c in zip(alone, together, planned):
        for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank", "knn_ids", "knn_dist"):
            if getattr(a, key) is None:
                continue
            assert torch.equal(getattr(a, key), getattr(b, key)), f"batched {key} k={a.k}"
            assert torch.equal(getattr(a, key), getattr(c, key)), f"planned {key} k={a.k}"
    for p in plans:
        p.close()
    j = alone[2]
    xs = O.project(x, j.mask).astype(np.float32)
    # without lists: kNN means to tau, the in-degree sum, and the in-degree
    # itself where no query is exempt
    ora = full_oracle(xs, j.k, j.eps)
    g = out_of(j)
    np.testing.assert_allclose(g["knn_mean"], ora["knn_mean"], rtol=TAU)
    strict = knn_strict(ora["knn_dist"][:, j.k - 1], ora["knn_next"])
    if strict.all():
        np.testing.assert_array_equal(g["indeg"], ora["indeg"])
    assert int(g["indeg"].astype(np.int64).sum()) == x.shape[0] * j.k


def test_large_k_above_one_lds_sampled(S):
    """n = 50,000 (device-wide index path for the eps side), k = 64: 64
    seeded queries against the oracle (C twin, subset mode)."""
    rng = np.random.default_rng(64)
    n, k = 50_000, 64
    x = rng.random((n, 5)).astype(np.float32)
    eps = 0.05
    pop = S.Population.from_rows(x)
    job = S.Job.alloc(pop, 0b11111, k, eps, with_lists=True)
    S.snaps_outlier_scores([job])
    torch.cuda.synchronize()
    g = out_of(job)
    assert int(g["indeg"].astype(np.int64).sum()) == n * k
    own = np.bincount(g["knn_ids"].astype(np.int64).ravel(), minlength=n)
    assert (own == g["indeg"]).all()
    qs = np.sort(rng.choice(n, size=64, replace=False))
    ora = C.join(x, k, eps, band=(eps * (1 - TAU), eps * (1 + TAU)), qids=qs)
    check_knn(g["knn_ids"][qs], g["knn_dist"][qs], ora, k, label="k=64 n=50000", row_ids=qs)
    exempt = ora["band"] > 0
    assert ((g["eps_count"][qs] == ora["eps_count"]) | exempt).all()
    o_km = ora["knn_dist"].sum(axis=1) / k
    assert (np.abs(g["knn_mean"][qs] - o_km) <= TAU * o_km).all()
