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


def score(S, state, alerts_np, method=0):
    a = torch.from_numpy(np.ascontiguousarray(alerts_np, dtype=np.float32)).cuda()
    job = S.AlertJob.alloc(state, a, method=method)
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


@pytest.mark.parametrize("method", [1, 2])
@pytest.mark.parametrize("n,d,k", [(3000, 3, 10), (20000, 2, 5), (40000, 7, 10), (12000, 13, 20)])
def test_alerts_against_oracle(S, n, d, k, method):
    """Both kernels (1: one wavefront per alert, 2: matrix-core tiles of 64
    alerts) against the oracle."""
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
    out = score(S, st, A, method)
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
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for method in (1, 2):
        job.eps_count.zero_()
        job.indeg.zero_()
        job.knn_mean.zero_()
        job.eps_mean.zero_()
        arr[0].method = method
        need = lib.snaps_alerts_workspace_bytes(arr, 1, 4, 5)
        assert (need > 0) == (method == 2)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        if need:                                       # a workspace too small, or none, is refused
            assert lib.snaps_alerts_score(arr, 1, 4, 5, ctypes.c_void_p(ws.data_ptr()), need - 1, stream) != 0
            assert lib.snaps_alerts_score(arr, 1, 4, 5, None, 0, stream) != 0
        assert lib.snaps_alerts_score(arr, 1, 4, 5, ctypes.c_void_p(ws.data_ptr()), need, stream) == 0
        torch.cuda.synchronize()
        assert (job.eps_count.cpu().numpy() == -1).all() and (job.indeg.cpu().numpy() == -1).all(), method
        assert torch.isnan(job.knn_mean).all() and torch.isnan(job.eps_mean).all(), method
    arr[0].method = 3
    assert lib.snaps_alerts_score(arr, 1, 3, 5, None, 0, stream) != 0
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


def _both(S, st, a_np, with_rank=True):
    a = torch.from_numpy(np.ascontiguousarray(a_np, dtype=np.float32)).cuda()
    outs = []
    for method in (1, 2):
        j = S.AlertJob.alloc(st, a, with_rank=with_rank, method=method)
        S.snaps_alerts_score([j])
        outs.append(j)
    torch.cuda.synchronize()
    return [{k: getattr(j, k).cpu().numpy() for k in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank")
             if getattr(j, k) is not None} for j in outs]


def _assert_kernels_agree(w, t):
    """The matrix-core kernel against the per-alert kernel: in-degree, eps
    count and kNN mean (and their rank positions) identical; the eps mean,
    whose float64 sum runs in another order, within one float32 ulp, its
    rank position identical wherever the two means are."""
    for key in ("eps_count", "indeg", "knn_mean"):
        np.testing.assert_array_equal(t[key], w[key], err_msg=key)
    diff = np.abs(t["eps_mean"].astype(np.float64) - w["eps_mean"].astype(np.float64))
    assert (diff <= np.spacing(np.abs(w["eps_mean"])).astype(np.float64)).all()
    if "rank" in w:
        for r in (0, 2, 3):
            np.testing.assert_array_equal(t["rank"][r], w["rank"][r], err_msg=f"rank {r}")
        same = t["eps_mean"] == w["eps_mean"]
        np.testing.assert_array_equal(t["rank"][1][same], w["rank"][1][same])


@pytest.mark.parametrize("n,d,k,m", [(5000, 2, 5, 1), (20000, 6, 10, 63), (20000, 9, 20, 65), (70000, 12, 32, 700),
                                     (30000, 15, 10, 130), (8000, 16, 5, 64), (3000, 7, 10, 1000),
                                     (150000, 10, 10, 200), (20000, 15, 32, 100), (12000, 16, 20, 300),
                                     (40000, 11, 10, 5000)])
def test_matrix_core_alerts_match_wavefront(S, n, d, k, m):
    """Ragged alert counts (one alert, 63, 64, 65 ...), every k class, d from
    2 to 16 (four wavefronts per workgroup at d = 15-16, eight below), 13 to
    128 population slices, populations from one to 37 super-tiles: alerts
    inside the bulk, exact copies of population objects (distance 0), far
    outside, and on the edge of the bulk."""
    rng = np.random.default_rng(n + 31 * d + m)
    job = G.gen_c3_jobs(4)[3]
    x = G.gen_c3_population(job, n=n)
    mask = int(sum(1 << f for f in rng.choice(15, size=min(d, 15), replace=False))) if d <= 15 else None
    if mask is None:                                      # d = 16: one extra column
        x = np.concatenate([x, rng.random((n, 1)).astype(np.float32)], axis=1)
        mask = (1 << 16) - 1
    P = O.project(x, mask).astype(np.float32)
    eps = float(O.eps_sampled_mean_count(P.astype(np.float64), 10, 64, seed=d))
    rows = rng.choice(n, size=m, replace=m > n)
    a = P[rows] + rng.normal(0, 0.01, size=(m, d)).astype(np.float32)
    a[: m // 4] = P[rows[: m // 4]]                       # exact copies
    if m > 8:
        a[-3:] = rng.uniform(-0.5, 1.5, size=(3, d)).astype(np.float32)
        a[-1] = 5.0
    pop = S.Population.from_rows(x)
    st = S.ServeState(pop, mask, k, eps)
    w, t = _both(S, st, a)
    _assert_kernels_agree(w, t)
    assert (w["indeg"] >= 0).all() and np.isfinite(w["knn_mean"]).all()


@pytest.mark.parametrize("case", ["far_alerts", "large_population"])
def test_matrix_core_alerts_out_of_half_range(S, case):
    """Coordinates beyond the half-precision pieces' range (|x| > 32): a group
    holding such an alert, or a tile holding such an object, is not screened
    and every pair is re-evaluated; the scores stay those of the per-alert
    kernel, and the oracle's in-degree and kNN mean."""
    rng = np.random.default_rng(77)
    n, d, k = 6000, 8, 10
    x = rng.random((n, d)).astype(np.float32)
    a = x[rng.choice(n, size=150, replace=False)] + rng.normal(0, 0.02, size=(150, d)).astype(np.float32)
    if case == "far_alerts":
        a[5] = 40.0
        a[100, 3] = -1000.0
    else:
        x = x * 80.0 - 20.0                                # most objects beyond |x| = 32
        a = a * 80.0 - 20.0
    a = a.astype(np.float32)
    pop = S.Population.from_rows(x)
    eps = 0.3 if case == "far_alerts" else 20.0
    st = S.ServeState(pop, (1 << d) - 1, k, eps)
    w, t = _both(S, st, a)
    _assert_kernels_agree(w, t)
    popref = C.outlier_scores(x, k, eps)
    ref = O.alert_scores(x, a, k, eps, pop=popref)
    np.testing.assert_allclose(t["knn_mean"], ref["knn_mean"], rtol=TAU)
    D = O.pair_distances(a, x)
    rk = popref["knn_dist"][:, k - 1]
    deg_ex = (np.abs(D - rk[None, :]) <= TAU * rk[None, :]).sum(axis=1)
    assert (np.abs(t["indeg"] - ref["indeg"]) <= deg_ex).all()


def test_mixed_methods_in_one_call(S):
    """Jobs of both kernels and of states with different populations in one
    call: every job's scores equal those of the same job scored alone."""
    rng = np.random.default_rng(29)
    pops = [S.Population.from_rows(rng.random((n, 15)).astype(np.float32)) for n in (7000, 11000)]
    states = [S.ServeState(pops[0], 0b111111100, 10, 0.2), S.ServeState(pops[1], 0b1111111000000, 10, 0.25)]
    reqs = []
    for i in range(10):
        st = states[i % 2]
        m = int(rng.integers(1, 900))
        reqs.append((st, torch.from_numpy(rng.random((m, st.d)).astype(np.float32)).cuda(), 1 + (i // 2) % 2))
    alone = []
    for st, a, meth in reqs:
        j = S.AlertJob.alloc(st, a, method=meth)
        S.snaps_alerts_score([j])
        alone.append(j)
    mixed = [S.AlertJob.alloc(st, a, method=meth) for st, a, meth in reqs]
    S.snaps_alerts_score(mixed)
    torch.cuda.synchronize()
    for x, y in zip(alone, mixed):
        for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
            assert torch.equal(getattr(x, key), getattr(y, key)), key


def test_matrix_core_jobs_across_launch_chunks(S):
    """More matrix-core jobs than one launch holds (40 > 32): the second
    chunk's partial results and bounds sit after the first's in the call's
    workspace; every job equals the same job scored alone."""
    rng = np.random.default_rng(41)
    pop = S.Population.from_rows(rng.random((9000, 15)).astype(np.float32))
    st = S.ServeState(pop, 0b11111110000, 10, 0.25)
    reqs = [torch.from_numpy(rng.random((int(rng.integers(1, 300)), st.d)).astype(np.float32)).cuda()
            for _ in range(40)]
    alone = []
    for a in reqs:
        j = S.AlertJob.alloc(st, a, method=2)
        S.snaps_alerts_score([j])
        alone.append(j)
    together = [S.AlertJob.alloc(st, a, method=2) for a in reqs]
    S.snaps_alerts_score(together)
    torch.cuda.synchronize()
    for x, y in zip(alone, together):
        for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
            assert torch.equal(getattr(x, key), getattr(y, key)), key
