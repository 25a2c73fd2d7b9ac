"""GPU tests of the served form: alerts scored against resident states.

The oracle's reading (oracle.alert_scores): an alert is one extra object that
changes nothing in the population and sees no other alert.  Checked against
the paper's Fig. 3 nested result sets, against the oracle under the float32
tolerance rule, and for independence from the other alerts of a call.
"""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from oracle import c_oracle as C
import snaps_synth as G
from tests.golden import exact_fp32_variant, load_fig3, load_tab2
from tests.parity import TAU, dense_rank_asc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_20176_amd import snaps
    snaps.load_library()
    return snaps


def score(S, state, alerts_np):
    a = torch.from_numpy(np.ascontiguousarray(alerts_np, dtype=np.float32)).cuda()
    job = S.AlertJob.alloc(state, a)
    S.snaps_alerts_score([job])
    torch.cuda.synchronize()
    return {k: getattr(job, k).cpu().numpy() for k in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank")}


def test_fig3_nested_sets_served(S):
    """Fig. 3: a query at (1, 1) among the ten points of Fig. 1 finds 3, 6
    and 8 neighbours at the three drawn radii (exact float32 rescaling)."""
    coords, _, _, _, _ = load_tab2()
    q, sets = load_fig3()
    x = exact_fp32_variant(coords)
    qq = exact_fp32_variant(q[None, :])
    pop = S.Population.from_rows(x)
    for r, expect in sets:
        eps = float(np.float32(100.0 * r / 512.0))
        st = S.ServeState(pop, 0b11, 3, eps)
        out = score(S, st, qq)
        assert out["eps_count"][0] == len(expect)
        ref = O.alert_scores(x, qq, 3, eps)
        assert out["indeg"][0] == ref["indeg"][0]
        np.testing.assert_allclose(out["knn_mean"][0], ref["knn_mean"][0], rtol=TAU)
        np.testing.assert_array_equal(out["rank"][:, 0], ref["rank"][:, 0])


def _population_keys(po):
    cnt = po["eps_count"].cpu().numpy()
    mean = po["eps_mean"].cpu().numpy().astype(np.float64)
    km = po["knn_mean"].cpu().numpy().astype(np.float64)
    deg = po["indeg"].cpu().numpy()
    return [cnt.astype(np.float64), -np.where(cnt > 0, mean, np.inf), deg.astype(np.float64), -km]


@pytest.mark.parametrize("n,d,k", [(3000, 3, 10), (20000, 2, 5), (40000, 7, 10), (12000, 13, 20)])
def test_alerts_against_oracle(S, n, d, k):
    rng = np.random.default_rng(n + d)
    job = G.gen_c3_jobs(4)[2]
    x = G.gen_c3_population(job, n=n)
    mask = int(sum(1 << f for f in rng.choice(15, size=d, replace=False)))
    P = O.project(x, mask)
    eps = float(O.eps_sampled_mean_count(P, 10, 64, seed=d))
    # alerts in the population's frame: perturbed population rows (inside the
    # bulk) plus a few far away
    base_rows = x[rng.choice(n, size=400, replace=False)]
    alerts_full = np.clip(base_rows + rng.normal(0, 0.01, size=base_rows.shape), -0.1, 1.1).astype(np.float32)
    alerts_full[:8] = rng.uniform(-0.2, 1.2, size=(8, alerts_full.shape[1])).astype(np.float32)
    A = O.project(alerts_full, mask).astype(np.float32)
    pop = S.Population.from_rows(x)
    st = S.ServeState(pop, mask, k, eps)
    out = score(S, st, A)
    # the population's exact k-th neighbour distances from the oracle's C
    # twin (float64 brute force, identical to the NumPy oracle)
    P32 = P.astype(np.float32)
    popref = C.outlier_scores(P32, k, eps)
    ref = O.alert_scores(P32, A, k, eps, pop=popref)
    # exemptions: a population distance within tau of eps (eps count / mean),
    # or within tau of that object's own k-th distance (in-degree: each such
    # object may count either way, every other one exactly)
    D = O.pair_distances(A, P32)
    eps_ex = (np.abs(D - eps) <= TAU * eps).any(axis=1)
    np.testing.assert_allclose(out["knn_mean"], ref["knn_mean"], rtol=TAU)
    assert ((out["eps_count"] == ref["eps_count"]) | eps_ex).all()
    rel = np.abs(out["eps_mean"] - ref["eps_mean"]) / np.maximum(ref["eps_mean"], 1e-30)
    assert ((rel <= TAU) | eps_ex | ((ref["eps_mean"] == 0) & (out["eps_mean"] == 0))).all()
    rk = popref["knn_dist"][:, k - 1]
    deg_ex = (np.abs(D - rk[None, :]) <= TAU * rk[None, :]).sum(axis=1)
    assert (np.abs(out["indeg"] - ref["indeg"]) <= deg_ex).all(), "alert in-degree outside the band rule"
    assert (out["indeg"] == ref["indeg"])[deg_ex == 0].all()
    # rank positions against the GPU's own population values, exactly
    keys = _population_keys(st.population_outputs())
    em = out["eps_mean"].astype(np.float64)
    akeys = [out["eps_count"].astype(np.float64), -np.where(out["eps_count"] > 0, em, np.inf),
             out["indeg"].astype(np.float64), -out["knn_mean"].astype(np.float64)]
    for t in range(4):
        u = np.unique(keys[t])
        np.testing.assert_array_equal(out["rank"][t], np.searchsorted(u, akeys[t], side="left"))


def test_population_outputs_of_state_match_plain_join(S):
    rng = np.random.default_rng(3)
    x = rng.random((5000, 6)).astype(np.float32)
    pop = S.Population.from_rows(x)
    st = S.ServeState(pop, 0b101101, 10, 0.08)
    job = S.Job.alloc(pop, 0b101101, 10, 0.08)
    S.snaps_outlier_scores([job], S.tuning(split=1))
    torch.cuda.synchronize()
    po = st.population_outputs()
    for key in ("eps_count", "indeg", "knn_mean"):
        assert torch.equal(po[key], getattr(job, key)), key
    np.testing.assert_allclose(po["eps_mean"].cpu().numpy(), job.eps_mean.cpu().numpy(), rtol=1e-6)


def test_mix_vs_alone(S):
    """Every alert's scores are identical whether its request is scored alone
    or inside a call that mixes requests of different sizes, populations and
    subspaces."""
    rng = np.random.default_rng(11)
    pops = [S.Population.from_rows(rng.random((n, 15)).astype(np.float32)) for n in (6000, 9000)]
    states = [S.ServeState(pops[0], 0b111, 10, 0.05), S.ServeState(pops[0], 0b1100001, 10, 0.05),
              S.ServeState(pops[1], 0b11000000011, 10, 0.12), S.ServeState(pops[1], 0b101, 10, 0.03)]
    reqs = []
    for i in range(12):
        st = states[i % len(states)]
        m = int(rng.integers(1, 700))
        reqs.append((st, torch.from_numpy(rng.random((m, st.d)).astype(np.float32)).cuda()))
    alone = []
    for st, a in reqs:
        j = S.AlertJob.alloc(st, a)
        S.snaps_alerts_score([j])
        alone.append(j)
    mixed = [S.AlertJob.alloc(st, a) for st, a in reqs]
    S.snaps_alerts_score(mixed)
    torch.cuda.synchronize()
    for x, y in zip(alone, mixed):
        for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
            assert torch.equal(getattr(x, key), getattr(y, key)), key


def test_state_of_another_shape_is_flagged_not_read(S):
    """A job whose state has another dimensionality than the call's d is
    flagged on the device (-1 counts, NaN means) instead of being scored."""
    import ctypes
    rng = np.random.default_rng(5)
    pop = S.Population.from_rows(rng.random((3000, 6)).astype(np.float32))
    st = S.ServeState(pop, 0b111, 5, 0.1)
    alerts = torch.from_numpy(rng.random((70, 3)).astype(np.float32)).cuda()
    job = S.AlertJob.alloc(st, alerts)
    arr = (S.c_alert_job * 1)()
    arr[0].state = st.ptr()
    arr[0].alerts = alerts.data_ptr()
    arr[0].m = 70
    arr[0].eps_count = job.eps_count.data_ptr()
    arr[0].eps_mean = job.eps_mean.data_ptr()
    arr[0].indeg = job.indeg.data_ptr()
    arr[0].knn_mean = job.knn_mean.data_ptr()
    arr[0].rank = None
    lib = S.load_library()
    assert lib.snaps_alerts_score(arr, 1, 4, 5, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
    torch.cuda.synchronize()
    assert (job.eps_count.cpu().numpy() == -1).all() and (job.indeg.cpu().numpy() == -1).all()
    assert torch.isnan(job.knn_mean).all() and torch.isnan(job.eps_mean).all()
    # the same job with the right d is scored
    S.snaps_alerts_score([job])
    torch.cuda.synchronize()
    assert (job.eps_count.cpu().numpy() >= 0).all() and (job.indeg.cpu().numpy() >= 0).all()


def test_large_population_many_super_tiles(S):
    """A population of 300,000 objects (74 super-tiles): alerts inside the
    bulk, on its edge and far outside.  The alert-side metrics come from the
    oracle's pair distances; the population's k-th neighbour distances, which
    the in-degree needs, from scipy's exact k-d tree (checked against the
    oracle in the pins)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(17)
    n, d, k = 300_000, 4, 10
    x = (rng.random((n, d)) ** 2).astype(np.float32)            # denser near 0
    eps = 0.01
    alerts = np.concatenate([rng.random((40, d)) ** 2, rng.random((8, d)) * 0.05,
                             1.0 + rng.random((4, d))]).astype(np.float32)
    pop = S.Population.from_rows(x)
    st = S.ServeState(pop, (1 << d) - 1, k, eps)
    out = score(S, st, alerts)
    x64 = x.astype(np.float64)
    rk = cKDTree(x64).query(x64, k=k + 1)[0][:, k]              # self is the first hit
    D = O.pair_distances(alerts, x)
    knn_mean = np.sort(D, axis=1)[:, :k].mean(axis=1)
    hit = D <= eps
    cnt = hit.sum(axis=1)
    mean = np.where(cnt > 0, np.where(hit, D, 0).sum(axis=1) / np.maximum(cnt, 1), 0)
    deg = (D < rk[None, :]).sum(axis=1)
    eps_ex = (np.abs(D - eps) <= TAU * eps).any(axis=1)
    deg_ex = (np.abs(D - rk[None, :]) <= TAU * rk[None, :]).sum(axis=1)
    np.testing.assert_allclose(out["knn_mean"], knn_mean, rtol=TAU)
    assert ((out["eps_count"] == cnt) | eps_ex).all()
    rel = np.abs(out["eps_mean"] - mean) / np.maximum(mean, 1e-30)
    assert ((rel <= TAU) | eps_ex | ((mean == 0) & (out["eps_mean"] == 0))).all()
    assert (np.abs(out["indeg"] - deg) <= deg_ex).all()
    assert (deg[-4:] == 0).all() and (cnt[-4:] == 0).all()      # far alerts


def test_continuous_batching_mix_vs_alone(S):
    """Requests replayed through the continuous-batching server (Batcher +
    GpuExecutor: four streams, admission by a device-memory budget) arrive
    while earlier batches are still on the device, land in batches of mixed
    sizes, populations and subspaces, and overlap on the GPU; every request's
    results equal those of the same request scored alone, bit for bit."""
    from paper_2405_20176_amd.serve import Admission, Batcher, GpuExecutor, Request
    rng = np.random.default_rng(404)
    pops = [S.Population.from_rows(G.gen_c3_population(G.gen_c3_jobs(4)[i], n=n)) for i, n in ((0, 60_000),
                                                                                                 (1, 90_000))]
    specs = [(0, 0b111, 0.02), (0, 0b1100001010, 0.06), (1, 0b11, 0.004), (1, 0b110000000110111, 0.12)]
    states = {}
    for p, m, e in specs:
        states[(p, m)] = S.ServeState(pops[p], m, 10, e)
    torch.cuda.synchronize()
    keys = list(states)
    reqs, t = [], 0.0
    for rid in range(80):
        t += rng.exponential(1.0 / 1500.0)          # arrivals far faster than a batch finishes
        key = keys[int(rng.integers(len(keys)))]
        m = int(np.exp(rng.uniform(0.0, np.log(4000.0))))
        al = rng.random((m, bin(key[1]).count("1"))).astype(np.float32)
        reqs.append(Request(rid, t, key, al))
    ex = GpuExecutor(states, n_streams=4)
    b = Batcher(ex, Admission(64 << 20, 4), max_batch_alerts=6000)
    b.run_open_loop(reqs)
    done = {r.rid: r for r in b.finished}
    assert len(done) == len(reqs) and all(r.status == "done" for r in done.values())
    assert b.batches_launched > 4 and b.max_inflight > 1, (b.batches_launched, b.max_inflight)
    mixed_sizes = False
    for r in reqs:
        alone = S.AlertJob.alloc(states[r.key], torch.from_numpy(r.alerts).cuda())
        S.snaps_alerts_score([alone])
        torch.cuda.synchronize()
        got = done[r.rid].result
        for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
            np.testing.assert_array_equal(got[key], getattr(alone, key).cpu().numpy(),
                                          err_msg=f"request {r.rid} {key}")
        mixed_sizes |= r.m > 1000
    assert mixed_sizes
