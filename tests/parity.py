"""Acceptance rule of GPU results against the float64 oracle.

tau = 1e-5 relative.  The GPU evaluates distances in float32, so where the
exact (float64) result is within float32 rounding of a decision boundary the
GPU may legitimately decide the other way; such objects are "exempt" and
checked for validity instead of equality:

* kNN: gap = (D_(k+1) - D_(k)) / D_(k+1).  If gap > tau (or both are 0, exact
  duplicates) the GPU's neighbour set must equal the oracle's; otherwise the
  query is exempt and the GPU set must still be a valid kNN set (every oracle
  neighbour strictly inside D_(k)(1 - tau) present, every returned distance
  <= D_(k)(1 + tau)).  Distances and the mean kNN distance hold to tau.
* eps: counts are exact for every object with no oracle distance in
  [eps(1 - tau), eps(1 + tau)]; such objects are exempt from the count and the
  mean.  Means of the others hold to tau.
* in-degree: (i) exactly the in-degree recomputed from the GPU's own kNN
  lists of the same call, after those lists pass the kNN rule above;
  (ii) exactly the oracle's for every object that no exempt query lists
  (in the oracle's lists or the GPU's), and everywhere when no query is
  exempt.  The sum is n*k.
* ranks: (i) exactly the dense ranks of the GPU's own metric values; (ii) for
  the integer metrics, equal to the oracle's ranks when the metric matched;
  (iii) for the float metrics, every pair whose oracle values differ by more
  than tau relative is ordered the same way.
"""
from __future__ import annotations

import numpy as np

TAU = 1e-5


def knn_strict(dk, dn) -> np.ndarray:
    """Queries whose kNN set the GPU must reproduce exactly: oracle gap
    (D_(k+1) - D_(k)) / D_(k+1) above tau, no (k+1)-th object, or exact
    duplicates at both ranks."""
    dk = np.asarray(dk, dtype=np.float64)
    dn = np.asarray(dn, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        gap = np.where(np.isinf(dn), np.inf, (dn - dk) / np.where(dn > 0, dn, 1.0))
    return (gap > TAU) | ((dk == 0) & (dn == 0))


def dense_rank_desc(values: np.ndarray) -> np.ndarray:
    """Dense rank, larger value first (rank 0)."""
    _, inv = np.unique(-np.asarray(values, dtype=np.float64), return_inverse=True)
    return inv.ravel()


def dense_rank_asc(values: np.ndarray) -> np.ndarray:
    _, inv = np.unique(np.asarray(values), return_inverse=True)
    return inv.ravel()


def self_ranks(eps_count, eps_mean, indeg, knn_mean) -> np.ndarray:
    """Dense ranks of given metric values, by the paper's ordering (used on
    the GPU's own float32 outputs)."""
    em = np.where(np.asarray(eps_count) > 0, np.asarray(eps_mean, dtype=np.float32).astype(np.float64), np.inf)
    return np.stack([dense_rank_asc(eps_count), dense_rank_desc(em), dense_rank_asc(indeg),
                     dense_rank_desc(np.asarray(knn_mean, dtype=np.float32).astype(np.float64))])


def _order_agrees(oracle_vals, gpu_rank, mask) -> int:
    """Count violations: pairs (a, b) with oracle a > b (1 + tau) (a more
    outlying) where the GPU does not rank a strictly before b."""
    idx = np.nonzero(mask)[0]
    if idx.size < 2:
        return 0
    v = np.asarray(oracle_vals, dtype=np.float64)[idx]
    r = np.asarray(gpu_rank)[idx]
    order = np.argsort(-v, kind="stable")
    v, r = v[order], r[order]
    # for each b, elements a with v_a > v_b (1 + tau) form a prefix of the
    # descending order; their max rank must stay below rank_b.
    thresh = np.where(np.isinf(v), np.inf, v * (1 + TAU) + (v == 0) * 1e-30)
    neg = -v
    cut = np.searchsorted(neg, -thresh, side="left")   # number of elements with v > thresh
    pmax = np.maximum.accumulate(r)
    has = cut > 0
    return int((pmax[cut[has] - 1] >= r[has]).sum())


def check_scores(gpu: dict, ora: dict, k: int, eps: float, check_ranks: bool = True, label: str = "") -> dict:
    """Compare a job's GPU outputs with the oracle's; raise AssertionError on
    any violation; return counts of exempt objects."""
    n = ora["eps_count"].shape[0]
    rep = {}
    # kNN exemptions from the oracle's k-th / (k+1)-th distances
    dk = ora["knn_dist"][:, k - 1]
    dn = ora["knn_next"]
    knn_exempt = ~knn_strict(dk, dn)
    rep["knn_exempt"] = int(knn_exempt.sum())

    # knn_mean within tau everywhere
    km_g = np.asarray(gpu["knn_mean"], dtype=np.float64)
    km_o = ora["knn_mean"]
    err = np.abs(km_g - km_o) / np.maximum(km_o, 1e-30)
    bad = (err > TAU) & (km_o > 0) | ((km_o == 0) & (km_g != 0))
    assert not bad.any(), f"{label} knn_mean off at {np.nonzero(bad)[0][:5]}: {km_g[bad][:5]} vs {km_o[bad][:5]}"

    # eps exemptions: an oracle distance within the band around eps
    if "band" in ora:
        eps_exempt = ora["band"] > 0
    else:
        eps_exempt = np.zeros(n, dtype=bool)
    rep["eps_exempt"] = int(eps_exempt.sum())
    ec_g = np.asarray(gpu["eps_count"])
    okc = (ec_g == ora["eps_count"]) | eps_exempt
    assert okc.all(), f"{label} eps_count off at {np.nonzero(~okc)[0][:5]}: {ec_g[~okc][:5]} vs {ora['eps_count'][~okc][:5]}"
    em_g = np.asarray(gpu["eps_mean"], dtype=np.float64)
    em_o = ora["eps_mean"]
    rel = np.abs(em_g - em_o) / np.maximum(em_o, 1e-30)
    okm = ((em_o == 0) & (em_g == 0)) | (rel <= TAU) | eps_exempt
    assert okm.all(), f"{label} eps_mean off at {np.nonzero(~okm)[0][:5]}: {em_g[~okm][:5]} vs {em_o[~okm][:5]}"

    # in-degree
    dg = np.asarray(gpu["indeg"]).astype(np.int64)
    assert dg.sum() == n * k, f"{label} in-degree sums to {dg.sum()}, not {n * k}"
    if gpu.get("knn_ids") is not None:
        ids_g = np.asarray(gpu["knn_ids"]).astype(np.int64)
        check_knn(ids_g, gpu["knn_dist"], ora, k, label=label)
        # (i) the GPU's in-degree is the in-degree of its own (validated) lists
        own = np.bincount(ids_g.ravel(), minlength=n)
        assert (dg == own).all(), f"{label} in-degree differs from its own kNN lists at {np.nonzero(dg != own)[0][:5]}"
        # (ii) objects no exempt query lists (either side) match the oracle
        touched = np.zeros(n, dtype=bool)
        touched[ora["knn_ids"][knn_exempt].ravel()] = True
        touched[ids_g[knn_exempt].ravel()] = True
        rep["indeg_exempt"] = int(touched.sum())
        ok = (dg == ora["indeg"]) | touched
        assert ok.all(), f"{label} in-degree off the oracle at {np.nonzero(~ok)[0][:5]}"
    elif rep["knn_exempt"] == 0:
        assert (dg == ora["indeg"]).all(), f"{label} in-degree off at {np.nonzero(dg != ora['indeg'])[0][:5]}"
    else:
        raise AssertionError(f"{label}: {rep['knn_exempt']} exempt queries and no GPU kNN lists to check "
                             "the in-degree against")

    if check_ranks and gpu.get("rank") is not None:
        rg = np.asarray(gpu["rank"]).astype(np.int64)
        sr = self_ranks(gpu["eps_count"], gpu["eps_mean"], gpu["indeg"], gpu["knn_mean"])
        for t in range(4):
            assert (rg[t] == sr[t]).all(), f"{label} rank row {t} not the dense rank of the GPU's own values"
        if (ec_g == ora["eps_count"]).all():
            assert (rg[0] == ora["rank"][0]).all(), f"{label} eps_count ranks differ"
        if (dg == ora["indeg"]).all():
            assert (rg[2] == ora["rank"][2]).all(), f"{label} indeg ranks differ"
        em_key = np.where(ora["eps_count"] > 0, em_o, np.inf)
        v1 = _order_agrees(em_key, rg[1], ~eps_exempt)
        v3 = _order_agrees(km_o, rg[3], np.ones(n, dtype=bool))
        assert v1 == 0, f"{label} eps_mean rank order disagrees on {v1} objects"
        assert v3 == 0, f"{label} knn_mean rank order disagrees on {v3} objects"
    return rep


def check_knn(ids_g, dist_g, ora: dict, k: int, label: str = "", row_ids=None) -> int:
    """Neighbour lists of snaps_knn_selfjoin against the oracle; ``row_ids``
    are the object ids of the rows (default: row i is object i)."""
    ids_g = np.asarray(ids_g).astype(np.int64)
    dist_g = np.asarray(dist_g, dtype=np.float64)
    dk = ora["knn_dist"][:, k - 1]
    dn = ora["knn_next"]
    strict = knn_strict(dk, dn)
    n = ids_g.shape[0]
    if row_ids is None:
        row_ids = np.arange(n)
    row_ids = np.asarray(row_ids).astype(np.int64)
    assert (np.diff(dist_g, axis=1) >= 0).all(), f"{label} GPU distances not ascending"
    # every row holds k distinct ids in [0, N), never its own
    srt = np.sort(ids_g, axis=1)
    assert (srt[:, 1:] != srt[:, :-1]).all() if k > 1 else True, f"{label} a kNN list repeats an id"
    assert (ids_g >= 0).all() and (ids_g != row_ids[:, None]).all(), f"{label} invalid id or own id in a list"
    # strict rows: the oracle's set exactly
    o_srt = np.sort(np.asarray(ora["knn_ids"]).astype(np.int64), axis=1)
    bad = np.nonzero(strict & (srt != o_srt).any(axis=1))[0]
    assert bad.size == 0, f"{label} kNN sets differ at {bad[:5]}"
    for i in np.nonzero(~strict)[0]:
        inner = ora["knn_ids"][i][ora["knn_dist"][i] < dk[i] * (1 - TAU)]
        assert set(inner.tolist()) <= set(ids_g[i].tolist()), f"{label} exempt {i} misses a strict neighbour"
        assert (dist_g[i] <= dk[i] * (1 + TAU) + 1e-30).all()
    od = ora["knn_dist"]
    rel = np.abs(np.sort(dist_g, axis=1) - od) / np.maximum(od, 1e-30)
    assert ((rel <= TAU) | ((od == 0) & (dist_g == 0))).all(), f"{label} kNN distances off"
    return int((~strict).sum())
