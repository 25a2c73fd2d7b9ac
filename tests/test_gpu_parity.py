"""GPU parity: libsnaps (through its C ABI) against the float64 oracle.

Every case runs the HIP path on seeded synthetic inputs and compares element
by element with the oracle under the acceptance rule of ``tests/parity.py``.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from oracle import c_oracle as C
import snaps_synth as G
from tests.golden import exact_fp32_variant, load_tab2
from tests.parity import TAU, check_knn, check_scores, knn_strict, self_ranks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_20176_amd import snaps
    snaps.load_library()
    return snaps


def job_out(job):
    """Host copies of a job's outputs (the kNN lists too when it has them)."""
    keys = ("eps_count", "eps_mean", "indeg", "knn_mean", "rank", "knn_ids", "knn_dist")
    return {key: (None if getattr(job, key) is None else getattr(job, key).cpu().numpy()) for key in keys}


def run_gpu(S, x, mask, k, eps, tune=None, with_rank=True):
    pop = S.Population.from_rows(x)
    job = S.Job.alloc(pop, mask, k, eps, with_rank, with_lists=True)
    S.snaps_outlier_scores([job], tune)
    torch.cuda.synchronize()
    return job_out(job)


def run_oracle(x, mask, k, eps):
    xs = O.project(x, mask).astype(np.float32)
    return C.outlier_scores(xs, k, float(eps), band=(float(eps) * (1 - TAU), float(eps) * (1 + TAU)))


def full_mask(f):
    return (1 << f) - 1


def test_tab2_worked_example_exact(S):
    coords, _, k, table, _ = load_tab2()
    x = exact_fp32_variant(coords)
    eps = np.float32(67.0 / 512.0)
    g = run_gpu(S, x, 0b11, k, float(eps))
    np.testing.assert_array_equal(g["eps_count"], table[:, 0])
    np.testing.assert_array_equal(np.round(g["eps_mean"].astype(np.float64) * 5.12, 4), table[:, 2])
    np.testing.assert_array_equal(g["indeg"], table[:, 4])
    np.testing.assert_array_equal(np.round(g["knn_mean"].astype(np.float64) * 5.12, 4), table[:, 6])
    for t, col in enumerate((1, 3, 5, 7)):
        np.testing.assert_array_equal(g["rank"][t], table[:, col])
    ids = torch.empty((10, k), dtype=torch.int32, device="cuda")
    dist = torch.empty((10, k), dtype=torch.float32, device="cuda")
    pop = S.Population.from_rows(x)
    S.snaps_knn_selfjoin(pop, 0b11, k, ids, dist)
    torch.cuda.synchronize()
    _, _, _, _, edges = load_tab2()
    for i, nb in edges.items():
        assert set(ids[i].cpu().tolist()) == nb


@pytest.fixture(scope="module")
def c0():
    x, k = G.gen_c0()
    return x, k, O.eps_exact_mean_count(x, 10)


@pytest.mark.parametrize("split", [1, 2, 4, 8])
@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("filt", [1, 2, 3])
def test_c0_parity(S, c0, split, mode, filt):
    x, k, eps = c0
    g = run_gpu(S, x, 0b111, k, float(eps), S.tuning(mode=mode, split=split, filter=filt))
    ora = run_oracle(x, 0b111, k, eps)
    rep = check_scores(g, ora, k, float(eps), label=f"C0 split={split} mode={mode}")
    # eps is the midpoint of two pair distances closer than tau: those two
    # pairs (four objects) sit inside the boundary band
    assert rep["knn_exempt"] <= 0.01 * x.shape[0] and rep["eps_exempt"] <= 0.01 * x.shape[0]


def test_pruning_and_split_invariance_bitwise(S, c0):
    """Skipping provably out-of-reach tiles never changes a result; the split
    of candidates over wavefronts changes only the eps-mean summation order."""
    x, k, eps = c0
    for split in (1, 4):
        a = run_gpu(S, x, 0b111, k, float(eps), S.tuning(mode=1, split=split))
        b = run_gpu(S, x, 0b111, k, float(eps), S.tuning(mode=2, split=split))
        for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
            np.testing.assert_array_equal(a[key], b[key], err_msg=f"{key} split={split}")
    a = run_gpu(S, x, 0b111, k, float(eps), S.tuning(split=1))
    b = run_gpu(S, x, 0b111, k, float(eps), S.tuning(split=8))
    for key in ("eps_count", "indeg", "knn_mean"):
        np.testing.assert_array_equal(a[key], b[key])


def _prefilter_cases():
    rng = np.random.default_rng(77)
    cases = [(G.gen_c0()[0], 0b111, 5, None)]
    for d in (2, 3, 5, 8, 12, 15, 16):
        x = rng.random((900, 16)).astype(np.float32)
        mask = int(sum(1 << f for f in rng.choice(16, size=d, replace=False)))
        cases.append((x, mask, 10, 0.1 * math.sqrt(d)))
    dup = (rng.integers(0, 3, size=(300, 6)) / 3.0).astype(np.float32)
    cases.append((dup, 0b111111, 20, 0.34))
    off = (rng.random((500, 4)) * 0.001 + 0.9).astype(np.float32)   # large norms, tiny distances
    cases.append((off, 0b1111, 7, 2e-4))
    return cases


@pytest.mark.parametrize("case", range(10))
def test_prefilter_is_bitwise_identical_to_direct_form(S, case):
    """The expanded-form prefilter only skips candidates that provably cannot
    matter; every surviving candidate is re-evaluated in the direct form, so
    all outputs equal those of the direct-form scan bit for bit."""
    x, mask, k, eps = _prefilter_cases()[case]
    if eps is None:
        eps = float(O.eps_exact_mean_count(x, 10))
    for split in (1, 4):
        a = run_gpu(S, x, mask, k, eps, S.tuning(split=split, filter=1))
        b = run_gpu(S, x, mask, k, eps, S.tuning(split=split, filter=2))
        for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
            np.testing.assert_array_equal(a[key], b[key], err_msg=f"{key} case={case} split={split}")
        if split == 1:
            m = run_gpu(S, x, mask, k, eps, S.tuning(split=1, filter=3))
            for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
                np.testing.assert_array_equal(a[key], m[key], err_msg=f"{key} case={case} matrix cores")
    check_scores(b, run_oracle(x, mask, k, eps), k, eps, label=f"prefilter case {case}")


@pytest.mark.parametrize("d", list(range(2, 17)))
def test_matrix_core_prefilter_every_d_and_k(S, d):
    """The matrix-core prefilter (every dimensionality and top-k capacity,
    ragged last tiles, several jobs per call) gives the direct form's results
    bit for bit, and meets the oracle."""
    rng = np.random.default_rng(300 + d)
    x = rng.random((777, 16)).astype(np.float32)
    mask = int(sum(1 << f for f in rng.choice(16, size=d, replace=False)))
    pop = S.Population.from_rows(x)
    eps = 0.1 * math.sqrt(d)
    ks = (1, 5, 10, 20, 32)
    outs = {}
    for filt in (1, 3):
        jobs = [S.Job.alloc(pop, mask, k, eps, with_lists=True) for k in ks]
        S.snaps_outlier_scores(jobs, S.tuning(split=1, filter=filt))
        torch.cuda.synchronize()
        outs[filt] = [job_out(j) for j in jobs]
    for k, a, b in zip(ks, outs[1], outs[3]):
        for key in a:
            np.testing.assert_array_equal(a[key], b[key], err_msg=f"{key} d={d} k={k}")
    for k, b in zip((1, 10, 32), [outs[3][0], outs[3][2], outs[3][4]]):
        check_scores(b, run_oracle(x, mask, k, eps), k, eps, label=f"matrix cores d={d} k={k}")


@pytest.mark.parametrize("case", ["beyond_range", "some_beyond_range", "tiny_scale", "offset_negative", "edge_of_range"])
@pytest.mark.parametrize("d", [3, 8, 15])
def test_matrix_core_half_precision_range(S, case, d):
    """The matrix cores screen with half-precision pieces of coordinates up to
    32 in magnitude: populations beyond that (all of them, or a few objects
    in some tiles) take the exact re-evaluation for the affected tiles,
    coordinates near the half-precision subnormal range and populations far
    from the origin keep a valid limit.  Outputs equal the direct form's bit
    for bit and meet the oracle."""
    rng = np.random.default_rng(["beyond_range", "some_beyond_range", "tiny_scale", "offset_negative",
                                 "edge_of_range"].index(case) * 31 + d)
    n = 3000
    x = rng.random((n, 16)).astype(np.float32)
    if case == "beyond_range":
        x = (x * 200.0 - 50.0).astype(np.float32)
    elif case == "some_beyond_range":
        x[rng.choice(n, 5, replace=False)] *= np.float32(100.0)
    elif case == "tiny_scale":
        x = (x * 3e-6).astype(np.float32)
    elif case == "edge_of_range":
        # exactly +-32 is in range, the next float above 32 is not
        x = ((x - 0.5) * 64.0).astype(np.float32)
        x[rng.choice(n, 20, replace=False), rng.integers(0, 16, 20)] = np.float32(32.0)
        x[rng.choice(n, 20, replace=False), rng.integers(0, 16, 20)] = np.float32(-32.0)
        x[rng.choice(n, 3, replace=False), 0] = np.nextafter(np.float32(32.0), np.float32(64.0))
    else:
        x = (x * 0.5 - 31.0).astype(np.float32)
    mask = (1 << d) - 1
    xs = O.project(x, mask).astype(np.float32)
    eps = float(O.eps_exact_mean_count(xs, 10))
    k = 10
    a = run_gpu(S, x, mask, k, eps, S.tuning(split=1, filter=1))
    m = run_gpu(S, x, mask, k, eps, S.tuning(split=1, filter=3))
    for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
        np.testing.assert_array_equal(a[key], m[key], err_msg=f"{key} {case} d={d}")
    check_scores(m, run_oracle(x, mask, k, eps), k, eps, label=f"half-precision range {case} d={d}")


@pytest.mark.parametrize("d", [2, 5, 8, 12])
def test_index_sorts_agree(S, d):
    """The packed-key LDS index and the full-key device-wide index order the
    objects differently; every result that does not depend on the summation
    order is identical, eps means agree to float32 rounding, and both meet
    the oracle."""
    rng = np.random.default_rng(900 + d)
    x = rng.random((4000, 16)).astype(np.float32)
    mask = int(sum(1 << f for f in rng.choice(16, size=d, replace=False)))
    eps = 0.09 * math.sqrt(d)
    a = run_gpu(S, x, mask, 10, eps, S.tuning(index_sort=1))
    b = run_gpu(S, x, mask, 10, eps, S.tuning(index_sort=2))
    for key in ("eps_count", "indeg", "knn_mean"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)
    np.testing.assert_allclose(a["eps_mean"], b["eps_mean"], rtol=1e-6)
    for r in (0, 2, 3):
        np.testing.assert_array_equal(a["rank"][r], b["rank"][r])
    ora = run_oracle(x, mask, 10, eps)
    check_scores(a, ora, 10, eps, label=f"packed index d={d}")
    check_scores(b, ora, 10, eps, label=f"radix index d={d}")


@pytest.mark.parametrize("n", [1000, 40000])
def test_ensemble_output(S, n):
    """The ensemble output is the mean of the GPU's own four ranks (exactly),
    equals the oracle's wherever the four ranks match it, and is written for
    jobs ranked by either rank path (LDS, or device-wide above 32,768)."""
    rng = np.random.default_rng(n)
    x = rng.random((n, 4)).astype(np.float32)
    pop = S.Population.from_rows(x)
    jobs = [S.Job.alloc(pop, 0b111, 7, 0.07, with_ensemble=True), S.Job.alloc(pop, 0b1011, 5, 0.09)]
    S.snaps_outlier_scores(jobs)
    torch.cuda.synchronize()
    r = jobs[0].rank.cpu().numpy().astype(np.int64)
    ens = jobs[0].ensemble.cpu().numpy()
    np.testing.assert_array_equal(ens, (r.sum(axis=0) / 4.0).astype(np.float32))
    assert jobs[1].ensemble is None
    if n <= 1000:
        ora = run_oracle(x, 0b111, 7, 0.07)
        same = (r == ora["rank"]).all(axis=0)
        assert same.mean() > 0.99
        np.testing.assert_array_equal(ens[same], ora["ensemble"][same].astype(np.float32))


def test_determinism(S, c0):
    x, k, eps = c0
    a = run_gpu(S, x, 0b111, k, float(eps))
    b = run_gpu(S, x, 0b111, k, float(eps))
    for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
        np.testing.assert_array_equal(a[key], b[key])


@pytest.mark.parametrize("n", [2, 3, 17, 63, 64, 65, 129, 1000])
def test_ragged_and_tiny_sizes(S, n):
    rng = np.random.default_rng(n)
    x = rng.random((n, 4)).astype(np.float32)
    for k in sorted({1, min(5, n - 1), min(n - 1, 32)}):
        eps = 0.3
        g = run_gpu(S, x, 0b1011, k, eps)
        check_scores(g, run_oracle(x, 0b1011, k, eps), k, eps, label=f"n={n} k={k}")


@pytest.mark.parametrize("d", list(range(2, 17)))
def test_every_dimensionality(S, d):
    rng = np.random.default_rng(100 + d)
    x = rng.random((700, 16)).astype(np.float32)
    mask = int(sum(1 << f for f in rng.choice(16, size=d, replace=False)))
    for k in (1, 5, 10, 20, 32):
        eps = 0.12 * math.sqrt(d)
        g = run_gpu(S, x, mask, k, eps, S.tuning(split=2))
        check_scores(g, run_oracle(x, mask, k, eps), k, eps, label=f"d={d} k={k}")


def test_duplicates_and_ties(S):
    rng = np.random.default_rng(7)
    base = (rng.integers(0, 4, size=(40, 3)) / 4.0).astype(np.float32)   # many exact duplicates
    x = np.concatenate([base, base, np.full((30, 3), 0.5, np.float32)])
    for k in (1, 3, 10, 32):
        ora = run_oracle(x, 0b111, k, 0.25)
        for filt in (0, 3):
            g = run_gpu(S, x, 0b111, k, 0.25, S.tuning(split=1, filter=filt))
            check_scores(g, ora, k, 0.25, label=f"dups k={k} filter={filt}")
    m = 9
    same = np.full((m, 2), 0.25, np.float32)
    g = run_gpu(S, same, 0b11, 3, 0.01)
    np.testing.assert_array_equal(g["indeg"], [m - 1, m - 1, m - 1, 3, 0, 0, 0, 0, 0])
    np.testing.assert_array_equal(g["eps_count"], m - 1)
    np.testing.assert_array_equal(g["eps_mean"], 0.0)


def test_degenerate_eps_and_k(S):
    rng = np.random.default_rng(3)
    n = 33
    x = rng.random((n, 3)).astype(np.float32)
    g = run_gpu(S, x, 0b111, n - 1, 2.0)
    assert (g["eps_count"] == n - 1).all()
    assert (g["indeg"] == n - 1).all()
    np.testing.assert_allclose(g["eps_mean"], g["knn_mean"], rtol=2e-6)
    g = run_gpu(S, x, 0b111, 2, 1e-6)
    assert (g["eps_count"] == 0).all() and (g["eps_mean"] == 0).all() and (g["rank"][0] == 0).all()


def test_isolated_points_rank_first(S):
    x, corners = G.gen_isolated_fixture()
    g = run_gpu(S, x, 0b111, 5, 0.1)
    assert (g["eps_count"][corners] == 0).all() and (g["rank"][0][corners] == 0).all()
    assert (g["rank"][1][corners] == 0).all() and (g["rank"][2][corners] == 0).all()
    assert sorted(g["rank"][3][corners].tolist()) == list(range(len(corners)))


def test_batched_equals_single(S):
    rng = np.random.default_rng(12)
    x = rng.random((3000, 15)).astype(np.float32)
    pop = S.Population.from_rows(x)
    specs = []
    for i in range(24):
        d = int(rng.integers(2, 16))
        mask = int(sum(1 << f for f in rng.choice(15, size=d, replace=False)))
        k = int(rng.choice([5, 10, 20]))
        specs.append((mask, k, 0.05 * math.sqrt(d)))
    tune = S.tuning(split=1)
    jobs = [S.Job.alloc(pop, m, k, e, with_lists=True) for m, k, e in specs]
    S.snaps_outlier_scores(jobs, tune)
    torch.cuda.synchronize()
    for (m, k, e), job in zip(specs, jobs):
        single = S.Job.alloc(pop, m, k, e)
        S.snaps_outlier_scores([single], tune)
        torch.cuda.synchronize()
        for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
            assert torch.equal(getattr(job, key), getattr(single, key)), f"{key} mask={m:x}"
    for (m, k, e), job in list(zip(specs, jobs))[:4]:
        check_scores(job_out(job), run_oracle(x, m, k, e), k, e, label=f"batched mask={m:x}")


def test_knn_and_eps_entry_points(S):
    rng = np.random.default_rng(5)
    x = rng.random((1500, 6)).astype(np.float32)
    pop = S.Population.from_rows(x)
    k, mask, eps = 10, 0b110101, 0.2
    ids = torch.empty((1500, k), dtype=torch.int32, device="cuda")
    dist = torch.empty((1500, k), dtype=torch.float32, device="cuda")
    S.snaps_knn_selfjoin(pop, mask, k, ids, dist)
    cnt = torch.empty(1500, dtype=torch.int32, device="cuda")
    mean = torch.empty(1500, dtype=torch.float32, device="cuda")
    S.snaps_eps_selfjoin(pop, mask, eps, cnt, mean)
    torch.cuda.synchronize()
    ora = run_oracle(x, mask, k, eps)
    check_knn(ids.cpu().numpy(), dist.cpu().numpy(), ora, k)
    exempt = ora["band"] > 0
    assert ((cnt.cpu().numpy() == ora["eps_count"]) | exempt).all()
    rel = np.abs(mean.cpu().numpy() - ora["eps_mean"]) / np.maximum(ora["eps_mean"], 1e-30)
    assert ((rel <= TAU) | exempt | (ora["eps_mean"] == 0)).all()


def test_rank_entry_point(S):
    rng = np.random.default_rng(9)
    for n in (1, 2, 100, 4097, 32768):
        cnt = rng.integers(0, 7, size=n).astype(np.int32)
        mean = np.where(cnt > 0, rng.integers(0, 50, size=n) / 7.0, 0.0).astype(np.float32)
        deg = rng.integers(0, 9, size=n).astype(np.int32)
        km = (rng.integers(0, 1000, size=n) / 13.0).astype(np.float32)
        rank = torch.empty((4, n), dtype=torch.int32, device="cuda")
        t = [torch.from_numpy(a).cuda() for a in (cnt, mean, deg, km)]
        S.snaps_rank(*t, rank)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(rank.cpu().numpy(), self_ranks(cnt, mean, deg, km))


@pytest.fixture(scope="module")
def c1():
    x, masks, k = G.gen_c1()
    try:
        eps = G.load_c1_eps()
    except (OSError, ValueError):
        eps = None
    return x, masks, k, eps


@pytest.mark.parametrize("which", [0, 104, 105, 560, 5000, 20000, 32751])
def test_c1_full_size_spaces(S, c1, which):
    """Spaces of the SNAPShot1-shaped population at its full size, with the
    stored per-space eps (oracle-computed)."""
    x, masks, k, eps_tab = c1
    mask = int(masks[which])
    if eps_tab is not None:
        eps = float(eps_tab[which])
    else:
        eps = float(O.eps_sampled_mean_count(O.project(x, mask), 10, 128, seed=mask))
    g = run_gpu(S, x, mask, k, eps)
    rep = check_scores(g, run_oracle(x, mask, k, eps), k, eps, label=f"C1 space {which}")
    assert rep["knn_exempt"] < 0.01 * x.shape[0]


# ------------------------------------------------------------------ large n ---

def sampled_check(S, x, mask, k, eps, jobs_out, n_samples=384, seed=0, label=""):
    """Parity at sizes the full oracle cannot finish: exact float64 answers
    for seeded sample objects (C twin, subset mode), GPU kNN lists for the
    same objects, and properties that hold at any size (sum of in-degrees,
    in-degree recomputed from the GPU's own kNN lists, rank self-consistency)."""
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    q = np.sort(rng.choice(n, size=min(n_samples, n), replace=False))
    xs = O.project(x, mask).astype(np.float32)
    ora = C.join(xs, k, float(eps), band=(float(eps) * (1 - TAU), float(eps) * (1 + TAU)), qids=q)
    cnt = jobs_out["eps_count"]
    mean = jobs_out["eps_mean"].astype(np.float64)
    km = jobs_out["knn_mean"].astype(np.float64)
    dk = ora["knn_dist"][:, k - 1]
    o_km = ora["knn_dist"].sum(axis=1) / k
    np.testing.assert_allclose(km[q], o_km, rtol=TAU, err_msg=f"{label} knn_mean")
    exempt = ora["band"] > 0
    assert ((cnt[q] == ora["eps_count"]) | exempt).all(), f"{label} eps_count"
    o_mean = np.where(ora["eps_count"] > 0, ora["eps_sum"] / np.maximum(ora["eps_count"], 1), 0.0)
    rel = np.abs(mean[q] - o_mean) / np.maximum(o_mean, 1e-30)
    assert ((rel <= TAU) | exempt | ((o_mean == 0) & (mean[q] == 0))).all(), f"{label} eps_mean"
    deg = jobs_out["indeg"].astype(np.int64)
    assert deg.sum() == n * k
    rg = jobs_out["rank"]
    sr = self_ranks(cnt, jobs_out["eps_mean"], jobs_out["indeg"], jobs_out["knn_mean"])
    for t in range(4):
        assert (rg[t] == sr[t]).all(), f"{label} rank row {t}"
    # kNN lists of the sample and in-degree recomputed from the GPU's own lists
    pop = S.Population.from_rows(x)
    ids = torch.empty((n, k), dtype=torch.int32, device="cuda")
    dist = torch.empty((n, k), dtype=torch.float32, device="cuda")
    S.snaps_knn_selfjoin(pop, mask, k, ids, dist)
    torch.cuda.synchronize()
    ids_h = ids.cpu().numpy()
    sub = {"knn_ids": ora["knn_ids"], "knn_dist": ora["knn_dist"], "knn_next": ora["knn_next"]}
    check_knn(ids_h[q], dist.cpu().numpy()[q], sub, k, label=label, row_ids=q)
    np.testing.assert_array_equal(np.bincount(ids_h.ravel(), minlength=n), deg, err_msg=f"{label} indeg vs lists")
    return int(exempt.sum())


_out = job_out


@pytest.mark.parametrize("n,d", [(32769, 3), (100_000, 2), (100_000, 6), (150_000, 12)])
def test_large_n_device_wide_sort_path(S, n, d):
    """n above one workgroup's LDS: index and ranks go through the device-wide
    radix sort."""
    rng = np.random.default_rng(n + d)
    job = G.gen_c3_jobs(8)[0]
    x = G.gen_c3_population(job, n=n)
    mask = int(sum(1 << f for f in rng.choice(15, size=d, replace=False)))
    eps = float(O.eps_sampled_mean_count(O.project(x, mask), 10, 64, seed=d))
    pop = S.Population.from_rows(x)
    j = S.Job.alloc(pop, mask, 10, eps)
    S.snaps_outlier_scores([j])
    torch.cuda.synchronize()
    sampled_check(S, x, mask, 10, eps, _out(j), label=f"n={n} d={d}")


def test_large_rank_entry_point(S):
    rng = np.random.default_rng(19)
    for n in (32769, 250_000):
        cnt = rng.integers(0, 40, size=n).astype(np.int32)
        mean = np.where(cnt > 0, rng.integers(0, 5000, size=n) / 77.0, 0.0).astype(np.float32)
        deg = rng.integers(0, 30, size=n).astype(np.int32)
        km = (rng.integers(0, 100000, size=n) / 13.0).astype(np.float32)
        rank = torch.empty((4, n), dtype=torch.int32, device="cuda")
        t = [torch.from_numpy(a).cuda() for a in (cnt, mean, deg, km)]
        S.snaps_rank(*t, rank)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(rank.cpu().numpy(), self_ranks(cnt, mean, deg, km))


def test_mixed_small_and_large_batch(S):
    """One call mixing LDS-path and device-wide-path jobs gives the same
    results as separate calls."""
    rng = np.random.default_rng(4)
    x = G.gen_c3_population(G.gen_c3_jobs(8)[1], n=60_000)
    small = x[:20_000]
    pl, ps = S.Population.from_rows(x), S.Population.from_rows(small)
    specs = [(pl, 0b111, 5, 0.02), (ps, 0b1100000011, 10, 0.05), (pl, 0b11110000, 20, 0.08),
             (ps, 0b11, 10, 0.004)]
    tune = S.tuning(split=1)
    jobs = [S.Job.alloc(p, m, k, e) for p, m, k, e in specs]
    S.snaps_outlier_scores(jobs, tune)
    torch.cuda.synchronize()
    for (p, m, k, e), job in zip(specs, jobs):
        one = S.Job.alloc(p, m, k, e)
        S.snaps_outlier_scores([one], tune)
        torch.cuda.synchronize()
        for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
            assert torch.equal(getattr(job, key), getattr(one, key)), f"{key} mask={m:x}"


@pytest.fixture(scope="module")
def c2():
    x, masks, k, target = G.gen_c2()
    return x, masks, k, target


@pytest.mark.parametrize("which", [0, 1, 57])
def test_c2_lsst_scale_spaces(S, c2, which):
    """LSST-scale population (5,000,000 objects): the full 15-feature space and
    two of the 105 two-feature spaces, eps for a mean of 20 neighbours;
    sampled exact checks plus whole-array properties."""
    x, masks, k, target = c2
    mask = int(masks[which])
    xs = O.project(x, mask)
    eps = float(O.eps_sampled_mean_count(xs, target, 24, seed=mask))
    del xs
    pop = S.Population.from_rows(x)
    j = S.Job.alloc(pop, mask, k, eps)
    S.snaps_outlier_scores([j])
    torch.cuda.synchronize()
    out = _out(j)
    del j
    ex = sampled_check(S, x, mask, k, eps, out, n_samples=128, seed=which, label=f"C2 space {which}")
    assert ex <= 5


@pytest.mark.parametrize("mq", [2, 4, 8])
def test_lockstep_workgroups(S, mq):
    """Workgroups of mq wavefronts with their own query tiles walking the same
    candidate tiles: same neighbours, counts and kNN means as one wavefront
    per workgroup (only the eps-sum order may differ), and oracle parity."""
    rng = np.random.default_rng(60 + mq)
    x = rng.random((5000, 15)).astype(np.float32)
    pop = S.Population.from_rows(x)
    specs = [(0b111, 5, 0.05), (0b1111100000, 10, 0.3), (0x7FFF, 20, 0.6), (0b11, 10, 0.01)]
    for mask, k, eps in specs:
        a = S.Job.alloc(pop, mask, k, eps)
        b = S.Job.alloc(pop, mask, k, eps, with_lists=True)
        S.snaps_outlier_scores([a], S.tuning(split=1, mq=1))
        S.snaps_outlier_scores([b], S.tuning(split=1, mq=mq))
        torch.cuda.synchronize()
        for key in ("eps_count", "indeg", "knn_mean"):
            assert torch.equal(getattr(a, key), getattr(b, key)), f"{key} mask={mask:x} mq={mq}"
        np.testing.assert_allclose(b.eps_mean.cpu().numpy(), a.eps_mean.cpu().numpy(), rtol=1e-6)
        check_scores(_out(b), run_oracle(x, mask, k, eps), k, eps, label=f"mq={mq} mask={mask:x}")


def test_graph_plans_replay(S):
    """The batched form captured as HIP graphs (one per pass) replays to the
    same results as direct calls, several times, with other work between
    replays."""
    rng = np.random.default_rng(23)
    x = rng.random((4000, 15)).astype(np.float32)
    pop = S.Population.from_rows(x)
    specs = [(0b111, 10, 0.05), (0b1111100000, 10, 0.3), (0x7FFF, 20, 0.6), (0b11, 5, 0.01), (0b101010101, 10, 0.2)]
    tune = S.tuning(split=1)
    ref = [S.Job.alloc(pop, m, k, e) for m, k, e in specs]
    S.snaps_outlier_scores(ref, tune)
    jobs = [S.Job.alloc(pop, m, k, e) for m, k, e in specs]
    ws = torch.empty(S.snaps_outlier_scores_workspace(jobs, tune), dtype=torch.uint8, device="cuda")
    plans = [S.Plan(jobs, S.tuning(split=1, passes=p), ws=ws) for p in (S.PASS_INDEX, S.PASS_JOIN, S.PASS_RANK)]
    for rep in range(3):
        for j in jobs:
            for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
                getattr(j, key).fill_(-7)
        for p in plans:
            p.launch()
        junk = torch.randn(1 << 20, device="cuda").sum()          # eager work between replays
        torch.cuda.synchronize()
        for a, b in zip(ref, jobs):
            for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank"):
                assert torch.equal(getattr(a, key), getattr(b, key)), f"replay {rep} {key}"
        del junk
    # the join pass alone, replayed again and again, recomputes the same
    # in-degrees (it clears them itself before adding)
    for rep in range(3):
        plans[1].launch()
        torch.cuda.synchronize()
        for a, b in zip(ref, jobs):
            assert torch.equal(a.indeg, b.indeg), f"join-only replay {rep}"
    single = [S.Job.alloc(pop, *specs[0])]
    whole = S.Plan(single, S.tuning())
    whole.launch()
    torch.cuda.synchronize()
    for key in ("eps_count", "indeg", "knn_mean"):
        assert torch.equal(getattr(single[0], key), getattr(ref[0], key)), key


# ---------------------------------------------------- sampled eps (Sec. 3.5.3)

def _eps_case(S, x, mask, m, targets, seed):
    rng = np.random.default_rng(seed)
    n = x.shape[0]
    sample = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)
    pop = S.Population.from_rows(x)
    got = S.snaps_eps_sample([(pop, mask, torch.from_numpy(sample).cuda(), targets)])[0].cpu().numpy()
    P = O.project(x, mask).astype(np.float32)
    ref = np.array([O.eps_from_sample(P, sample, t) for t in targets], dtype=np.float64)
    return got, ref


@pytest.mark.parametrize("d", [2, 5, 9, 16])
def test_eps_sampler_against_oracle(S, d):
    """The GPU radius equals the oracle's for the same sample to float32
    rounding of the distances, at small, middle and extreme targets
    (r = 1 and r = m (n - 1) - 1)."""
    rng = np.random.default_rng(40 + d)
    n, m = 3000, 64
    x = rng.random((n, 16)).astype(np.float32)
    mask = int(sum(1 << f for f in rng.choice(16, size=d, replace=False)))
    targets = [1.0 / m, 0.5, 10.0, 300.0, 0.0015 * n, 0.15 * n, (m * (n - 1) - 1) / m]
    got, ref = _eps_case(S, x, mask, m, targets, seed=d)
    np.testing.assert_allclose(got, ref, rtol=TAU)


def test_eps_sampler_ties_and_duplicates(S):
    """Many exactly equal distances (a coarse lattice with duplicates): the
    selection handles ties of the r-th and (r+1)-th smallest exactly."""
    rng = np.random.default_rng(5)
    x = (rng.integers(0, 4, size=(500, 3)) / 4.0).astype(np.float32)
    got, ref = _eps_case(S, x, 0b111, 50, [0.02, 1.0, 7.0, 33.3, 120.0, 400.0], seed=1)
    np.testing.assert_allclose(got, ref, rtol=TAU)


def test_eps_sampler_reproduces_the_stored_c1_radii(S, c1):
    """The stored C1 radii were written by the oracle (m = 128 seeded by the
    subspace mask, target 10); the GPU sampler with the same samples
    reproduces them."""
    x, masks, k, eps_tab = c1
    pop = S.Population.from_rows(x)
    n = x.shape[0]
    specs, want = [], []
    for i in (0, 104, 560, 5000, 20000, 32751):
        rng = np.random.default_rng(int(masks[i]))
        sample = np.sort(rng.choice(n, size=128, replace=False)).astype(np.int32)
        specs.append((pop, int(masks[i]), torch.from_numpy(sample).cuda(), [10.0]))
        want.append(eps_tab[i])
    got = [o.cpu().numpy()[0] for o in S.snaps_eps_sample(specs)]
    np.testing.assert_allclose(got, want, rtol=TAU)


def test_eps_sampler_batched_equals_single(S):
    rng = np.random.default_rng(8)
    pops = [S.Population.from_rows(rng.random((n, 15)).astype(np.float32)) for n in (800, 2500)]
    specs = []
    for i in range(10):
        pop = pops[i % 2]
        d = int(rng.integers(2, 16))
        mask = int(sum(1 << f for f in rng.choice(15, size=d, replace=False)))
        sample = torch.from_numpy(np.sort(rng.choice(pop.n, size=40, replace=False)).astype(np.int32)).cuda()
        specs.append((pop, mask, sample, [0.001 * pop.n, 0.15 * pop.n]))
    batched = S.snaps_eps_sample(specs)
    for spec, b in zip(specs, batched):
        single = S.snaps_eps_sample([spec])[0]
        assert torch.equal(single, b)
    # ids outside [0, n) are ignored: too few distances leave the radius NaN
    bad = torch.full((40,), -1, dtype=torch.int32, device="cuda")
    out = S.snaps_eps_sample([(pops[0], 0b111, bad, [1.0])])[0]
    assert torch.isnan(out).all()


# ------------------------------------------- eps-grid selection (Sec. 3.5.2)

def _grid_exempt(P, radii):
    """Per radius, objects with a float64 distance within tau of it."""
    D = O.pair_distances(P, P)
    np.fill_diagonal(D, np.inf)
    return np.stack([(np.abs(D - float(r)) <= TAU * float(r)).any(axis=1) for r in radii])


@pytest.mark.parametrize("d", [2, 5, 9])
def test_eps_grid_against_oracle(S, d):
    """Per-object counts and means at every radius meet the oracle; the
    similarity curves and the selected radii are exactly the oracle's
    selection applied to the GPU's own per-radius metrics, and equal the
    oracle's outright when no object sits on a radius."""
    rng = np.random.default_rng(60 + d)
    n = 1500
    x = rng.random((n, 16)).astype(np.float32)
    mask = int(sum(1 << f for f in rng.choice(16, size=d, replace=False)))
    P = O.project(x, mask).astype(np.float32)
    sample = np.sort(rng.choice(n, size=64, replace=False))
    lo, hi = O.eps_from_sample(P, sample, 2.0), O.eps_from_sample(P, sample, 0.15 * n)
    radii = O.eps_grid(float(lo), float(hi), 8)
    top = 15
    pop = S.Population.from_rows(x)
    out = S.snaps_eps_grid([(pop, mask, radii, top)], with_metrics=True)[0]
    cnt = out["count"].cpu().numpy()
    mean = out["mean"].cpu().numpy()
    rc, rm = O.eps_grid_metrics(P, radii)
    ex = _grid_exempt(P, radii)
    assert ((cnt == rc) | ex).all()
    rel = np.abs(mean - rm) / np.maximum(rm, 1e-30)
    assert ((rel <= TAU) | ex | ((rm == 0) & (mean == 0))).all()
    mine = O.eps_grid_select(cnt, mean.astype(np.float64), top)
    np.testing.assert_array_equal(out["similarity"].cpu().numpy(), mine["similarity"].astype(np.float32))
    np.testing.assert_array_equal(out["select"].cpu().numpy(), mine["select"])
    if not ex.any():
        ref = O.eps_grid_select(rc, rm, top)
        np.testing.assert_array_equal(out["select"].cpu().numpy()[0], ref["select"][0])


def test_eps_grid_batched_equals_single_and_degenerate_top(S):
    rng = np.random.default_rng(9)
    pops = [S.Population.from_rows(rng.random((n, 15)).astype(np.float32)) for n in (700, 1300)]
    specs = []
    for i in range(8):
        pop = pops[i % 2]
        d = int(rng.integers(2, 16))
        mask = int(sum(1 << f for f in rng.choice(15, size=d, replace=False)))
        r0 = 0.05 * math.sqrt(d)
        specs.append((pop, mask, [r0 * (1 + 0.5 * j) for j in range(6)], max(1, pop.n // 100)))
    batched = S.snaps_eps_grid(specs)
    for spec, b in zip(specs, batched):
        single = S.snaps_eps_grid([spec])[0]
        for key in ("similarity", "select"):
            assert torch.equal(single[key], b[key]), key
    # top n = every object: every list is the whole population, all gaps are 0
    allt = S.snaps_eps_grid([(pops[0], 0b111, [0.05, 0.1, 0.2], pops[0].n)])[0]
    assert (allt["similarity"] == 1).all() and (allt["select"] == 0).all()


def _knn_gap_exempt(P, ks):
    """Per k of the grid, queries whose k-th and (k+1)-th float64 distances
    lie within tau (relative) of each other and are not exact duplicates."""
    D = O.pair_distances(P, P)
    np.fill_diagonal(D, np.inf)
    Ds = np.sort(D, axis=1)
    out = []
    for k in ks:
        dk = Ds[:, k - 1]
        dn = Ds[:, k] if k < P.shape[0] - 1 else np.full(P.shape[0], np.inf)
        gap = np.where(np.isinf(dn), np.inf, (dn - dk) / np.where(dn > 0, dn, 1.0))
        out.append(~((gap > TAU) | ((dk == 0) & (dn == 0))))
    return np.stack(out)


@pytest.mark.parametrize("d", [2, 5, 9])
def test_k_grid_against_oracle(S, d):
    """In-degrees and mean kNN distances at every k meet the oracle (exact
    in-degrees where no query sits on a near-tie at that k); the similarity
    curves and selected k are exactly the oracle's selection applied to the
    GPU's own per-k metrics, and the in-degree choice equals the oracle's
    outright when the in-degrees agree."""
    rng = np.random.default_rng(80 + d)
    n = 1500
    x = rng.random((n, 16)).astype(np.float32)
    mask = int(sum(1 << f for f in rng.choice(16, size=d, replace=False)))
    P = O.project(x, mask).astype(np.float32)
    ks = [2, 3, 4, 6, 8, 12, 16, 24, 32, 64, 128, 256]
    top = 15
    pop = S.Population.from_rows(x)
    out = S.snaps_k_grid([(pop, mask, ks, top)], with_metrics=True)[0]
    deg = out["indeg"].cpu().numpy().astype(np.int64)
    km = out["knn_mean"].cpu().numpy()
    rd, rk = O.k_grid_metrics(P, ks)
    ex = _knn_gap_exempt(P, ks)
    for j, k in enumerate(ks):
        assert deg[j].sum() == n * k, k
        if not ex[j].any():
            assert (deg[j] == rd[j]).all(), k
        else:
            assert np.abs(deg[j] - rd[j]).sum() <= 2 * int(ex[j].sum()) * k, k
        rel = np.abs(km[j] - rk[j]) / np.maximum(rk[j], 1e-30)
        assert (rel <= TAU).all(), (k, float(rel.max()))
    assert (np.diff(km, axis=0) >= 0).all()            # more neighbours, farther on average
    mine = O.k_grid_select(deg, km.astype(np.float64), top)
    np.testing.assert_array_equal(out["similarity"].cpu().numpy(), mine["similarity"].astype(np.float32))
    np.testing.assert_array_equal(out["select"].cpu().numpy(), mine["select"])
    if (deg == rd).all():
        ref = O.k_grid_select(rd, rk, top)
        assert int(out["select"].cpu().numpy()[0]) == int(ref["select"][0])


def test_k_grid_ties_duplicates_and_every_neighbour(S):
    """Coordinates on a 1/8 grid: every squared distance is exact in float32
    and float64, so ties (and duplicates at distance 0) are resolved by id on
    both sides and the in-degrees must agree exactly at every k, up to
    k = n - 1 (every other object)."""
    rng = np.random.default_rng(5)
    n = 300
    x = (rng.integers(0, 6, size=(n, 4)) / 8.0).astype(np.float32)
    mask = 0b1111
    P = O.project(x, mask).astype(np.float32)
    ks = [1, 2, 5, 17, 100, n - 1]
    out = S.snaps_k_grid([(S.Population.from_rows(x), mask, ks, 10)], with_metrics=True)[0]
    deg = out["indeg"].cpu().numpy().astype(np.int64)
    km = out["knn_mean"].cpu().numpy()
    rd, rk = O.k_grid_metrics(P, ks)
    np.testing.assert_array_equal(deg, rd)
    assert (deg[-1] == n - 1).all()
    rel = np.abs(km - rk) / np.maximum(rk, 1e-30)
    assert ((rel <= TAU) | ((rk == 0) & (km == 0))).all()
    mine = O.k_grid_select(deg, km.astype(np.float64), 10)
    np.testing.assert_array_equal(out["select"].cpu().numpy(), mine["select"])


def test_k_grid_batched_equals_single_and_degenerate_top(S):
    rng = np.random.default_rng(19)
    pops = [S.Population.from_rows(rng.random((n, 15)).astype(np.float32)) for n in (700, 1301)]
    specs = []
    for i in range(8):
        pop = pops[i % 2]
        d = int(rng.integers(2, 16))
        mask = int(sum(1 << f for f in rng.choice(15, size=d, replace=False)))
        ks = sorted(set(int(v) for v in rng.integers(1, 400, size=int(rng.integers(2, 17)))))
        if len(ks) < 2:
            ks = [1, 400]
        specs.append((pop, mask, ks, max(1, pop.n // 100)))
    batched = S.snaps_k_grid(specs, with_metrics=True)
    for spec, b in zip(specs, batched):
        single = S.snaps_k_grid([spec], with_metrics=True)[0]
        for key in ("similarity", "select", "indeg", "knn_mean"):
            assert torch.equal(single[key], b[key]), key
    # top n = every object: every list is the whole population, all gaps are 0
    allt = S.snaps_k_grid([(pops[0], 0b111, [2, 10, 50], pops[0].n)])[0]
    assert (allt["similarity"] == 1).all() and (allt["select"] == 0).all()


def test_k_grid_beyond_one_dispatch(S):
    """More queries of one dimensionality in one call than one dispatch of
    1024-wide workgroups can count (2^32 work-items): the last job still
    equals its own call."""
    rng = np.random.default_rng(13)
    n = 32768
    pop = S.Population.from_rows(rng.random((n, 15)).astype(np.float32))
    masks = [int(sum(1 << f for f in c)) for c in itertools.islice(itertools.combinations(range(15), 3), 130)]
    ks = [2, 16, 128]
    specs = [(pop, m, ks, 100) for m in masks]
    assert len(specs) * n > (1 << 22)
    out = S.snaps_k_grid(specs, with_metrics=True)
    for i in (0, len(specs) - 1):
        single = S.snaps_k_grid([specs[i]], with_metrics=True)[0]
        for key in ("similarity", "select", "indeg", "knn_mean"):
            assert torch.equal(single[key], out[i][key]), (i, key)


def test_eps_sampler_beyond_one_dispatch(S):
    """More sample objects in one call than one dispatch of 256-wide
    workgroups can count: the first and last jobs equal their own calls."""
    rng = np.random.default_rng(12)
    n = 1024
    pop = S.Population.from_rows(rng.random((n, 15)).astype(np.float32))
    sample = torch.arange(n, dtype=torch.int32, device="cuda")
    jobs = (1 << 22) // n + 2
    specs = [(pop, 0b111 << (i % 12), sample, [0.01 * n, 0.15 * n]) for i in range(jobs)]
    out = S.snaps_eps_sample(specs)
    for i in (0, jobs - 1):
        assert torch.equal(S.snaps_eps_sample([specs[i]])[0], out[i]), i


# ------------------------------------------------ eps pair lists (Sec. 3.5)

def _check_pair_rows(P, eps, off, pairs, rows):
    """Rows of the GPU pair list against the float64 oracle: equal as sets
    unless an oracle distance of the row sits in the eps band; then every
    neighbour strictly inside the band is listed and nothing outside it."""
    D = O.pair_distances(P[rows], P)
    for r, i in enumerate(rows):
        got = np.sort(pairs[off[i]:off[i + 1]])
        assert np.unique(got).size == got.size and i not in got, i
        di = D[r].copy()
        di[i] = np.inf
        if (np.abs(di - eps) <= TAU * eps).any():
            inner = np.nonzero(di < eps * (1 - TAU))[0]
            outer = np.nonzero(di <= eps * (1 + TAU))[0]
            assert set(inner.tolist()) <= set(got.tolist()) <= set(outer.tolist()), i
        else:
            np.testing.assert_array_equal(got, np.nonzero(di <= eps)[0])


@pytest.mark.parametrize("n,d", [(1000, 3), (3000, 7), (40000, 4)])
def test_eps_pair_list(S, n, d):
    """The CSR pair list of snaps_eps_selfjoin: row starts are the prefix
    sums of the counts, rows match the oracle's result set (band rule), the
    counts and means equal the call without a list, and a capacity below the
    total writes exactly the first entries of the full list and nothing past
    the capacity.  n = 40,000 runs through the device-wide index."""
    rng = np.random.default_rng(70 + d)
    x = rng.random((n, 8)).astype(np.float32)
    mask = (1 << d) - 1
    P = O.project(x, mask).astype(np.float32)
    sample = np.sort(rng.choice(n, size=64, replace=False))
    eps = float(O.eps_from_sample(P, sample, 8.0))
    pop = S.Population.from_rows(x)
    count, mean, off, pairs = S.snaps_eps_pairs(pop, mask, eps)
    count, mean = count.cpu().numpy(), mean.cpu().numpy()
    off, pl = off.cpu().numpy(), pairs.cpu().numpy()
    assert off[0] == 0 and (np.diff(off) == count).all() and off[-1] == pl.size
    c0 = torch.empty(n, dtype=torch.int32, device="cuda")
    m0 = torch.empty(n, dtype=torch.float32, device="cuda")
    S.snaps_eps_selfjoin(pop, mask, eps, c0, m0)
    np.testing.assert_array_equal(c0.cpu().numpy(), count)
    np.testing.assert_array_equal(m0.cpu().numpy(), mean)
    rows = np.arange(n) if n <= 3000 else np.sort(rng.choice(n, size=300, replace=False))
    _check_pair_rows(P, eps, off, pl, rows)
    if n <= 3000:                                   # the relation is symmetric outside the band
        ro, rid = O.eps_pairs(P, eps)
        assert abs(int(ro[-1]) - pl.size) <= 2 * int((np.abs(O.pair_distances(P, P) - eps) <= TAU * eps).sum())
    # capacity below the total
    cap = pl.size // 2
    buf = torch.full((cap + 100,), -7, dtype=torch.int32, device="cuda")
    off2 = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    S.snaps_eps_selfjoin(pop, mask, eps, c0, m0, pair_off=off2, pairs=buf[:cap])
    b = buf.cpu().numpy()
    np.testing.assert_array_equal(off2.cpu().numpy(), off)
    np.testing.assert_array_equal(b[:cap], pl[:cap])
    assert (b[cap:] == -7).all()


# ------------------------------------- per-job walk settings and the autotuner

def test_per_job_walk_settings_and_autotuner(S):
    """Per-job mode / index_dims (brute force, or box pruning on 2..6
    indexed dimensions) change only the time: counts, in-degrees and kNN
    means are identical, eps means agree to the summation order.  The
    autotuner times every candidate setting of each class and its choices,
    applied, keep the results."""
    from paper_2405_20176_amd import autotune as AT
    rng = np.random.default_rng(91)
    x = rng.random((5000, 15)).astype(np.float32)
    pop = S.Population.from_rows(x)
    masks = [0b111, 0b1111111, 0b111111111111]
    epss = [0.08 * math.sqrt(bin(m).count("1")) for m in masks]

    def run(settings, jobs=None):
        jobs = jobs or [S.Job.alloc(pop, m, 10, e, with_lists=True) for m, e in zip(masks, epss)]
        for j, st in zip(jobs, settings):
            j.mode, j.index_dims = st[0], st[1]
            j.tile_shape = st[2] if len(st) > 2 else 0
        S.snaps_outlier_scores(jobs, S.tuning(split=1))
        torch.cuda.synchronize()
        return [job_out(j) for j in jobs]

    def same(a, b, label):
        for ra, rb in zip(a, b):
            for key in ("eps_count", "indeg", "knn_mean"):
                np.testing.assert_array_equal(ra[key], rb[key], err_msg=f"{key} {label}")
            np.testing.assert_allclose(ra["eps_mean"], rb["eps_mean"], rtol=TAU, err_msg=label)
            for t in (0, 2, 3):
                np.testing.assert_array_equal(ra["rank"][t], rb["rank"][t], err_msg=f"rank {t} {label}")

    ref = run([(0, 0)] * 3)
    check_scores(ref[1], run_oracle(x, masks[1], 10, epss[1]), 10, epss[1], label="defaults d=7")
    for setting in [(1, 0), (2, 2), (2, 3), (2, 6), (2, 2, 2), (2, 4, 3), (1, 0, 2)]:
        same(ref, run([setting] * 3), f"setting {setting}")
    # super-tile culls and candidate halves only skip work no query can
    # reach, in the same walk order: bit for bit the same
    for c in (2, 4):
        a = run([(2, c, 1)] * 3)
        for shape in (2, 3):
            b = run([(2, c, shape)] * 3)
            for ra, rb in zip(a, b):
                for key in ra:
                    np.testing.assert_array_equal(ra[key], rb[key], err_msg=f"shape {shape} {key} c={c}")
    jobs = [S.Job.alloc(pop, m, 10, e) for m, e in zip(masks, epss)]
    table = AT.tune(jobs, sample=2, reps=1)
    assert set(table) == {AT.class_key(AT.job_class(j)) for j in jobs}
    for key, v in table.items():
        d = int(key[1:key.index("_")])
        assert (v["mode"], v["index_dims"]) in AT.candidates(d)
        assert v["tile_shape"] in (AT.TILE_FULL, AT.TILE_HALVES, AT.TILE_SUPER)
        plain_keys = {f"{m},{c}" for m, c in AT.candidates(d)}
        assert plain_keys <= set(v["ms"])
        extra = set(v["ms"]) - plain_keys
        assert extra == ({f"{v['mode']},{v['index_dims']},{t}" for t in "hs"} if v["mode"] == AT.MODE_PRUNE
                         else set())
    assert AT.apply(jobs, table) == 3
    same(ref, run([(j.mode, j.index_dims, j.tile_shape) for j in jobs], jobs), "autotuned")


# ----------------------------------------------- super-tile walk at large n

@pytest.mark.parametrize("d", [2, 5])
def test_super_tile_walk_and_candidate_halves_large_n(S, d):
    """A population of 200,000 objects (49 super-tiles of 64 tiles): the
    matrix-core join culls super-tiles, then tiles (or 32-candidate halves)
    by their boxes, or walks tile by tile; the vector-ALU direct form walks
    the same tile order tile by tile.  All give identical results, bit for
    bit, and 64 seeded queries match the oracle."""
    rng = np.random.default_rng(200 + d)
    n, k = 200_000, 10
    x = (rng.random((n, d)) ** 2).astype(np.float32)
    eps = 0.004 if d == 2 else 0.05
    mask = (1 << d) - 1
    pop = S.Population.from_rows(x)
    outs = {}
    for name, tune in (("mfma", S.tuning(split=1, filter=3, tile_shape=3)),
                       ("mfma_halves", S.tuning(split=1, filter=3, tile_shape=2)),
                       ("mfma_lean", S.tuning(split=1, filter=3, tile_shape=1)),
                       ("valu_direct", S.tuning(split=1, filter=1))):
        job = S.Job.alloc(pop, mask, k, eps, with_lists=True)
        st = torch.zeros(4, dtype=torch.int64, device="cuda")
        tune.stats = st.data_ptr()
        S.snaps_outlier_scores([job], tune)
        torch.cuda.synchronize()
        outs[name] = job_out(job)
        outs[name]["stats"] = st.cpu().numpy()
    for name in ("mfma_halves", "mfma_lean", "valu_direct"):
        for key in ("eps_count", "eps_mean", "indeg", "knn_mean", "rank", "knn_ids", "knn_dist"):
            np.testing.assert_array_equal(outs["mfma"][key], outs[name][key], err_msg=f"{name} {key} d={d}")
    # the super-tile level skips most tiles; halves evaluate no more pairs
    if d == 2:
        assert outs["mfma"]["stats"][2] > 10 * outs["mfma"]["stats"][1]
    assert outs["mfma_halves"]["stats"][0] <= outs["mfma"]["stats"][0]
    qs = np.sort(rng.choice(n, size=64, replace=False))
    ora = C.join(x, k, eps, band=(eps * (1 - TAU), eps * (1 + TAU)), qids=qs)
    g = outs["mfma"]
    exempt = ora["band"] > 0
    assert ((g["eps_count"][qs] == ora["eps_count"]) | exempt).all()
    check_knn(g["knn_ids"][qs], g["knn_dist"][qs], ora, k, label=f"super-tile walk d={d}", row_ids=qs)
    assert int(g["indeg"].astype(np.int64).sum()) == n * k


# --------------------------------------- k grid above one workgroup's registers

@pytest.mark.parametrize("case", ["random", "coarse_grid_ties"])
def test_k_grid_streaming_selection_above_32768(S, case):
    """Populations above 32,768 objects take the k-grid threshold kernel that
    recomputes each query's distances in every selection pass.  At every
    k <= 64 the in-degree of every object equals the one counted from the
    oracle's kNN lists (C twin, all 40,000 queries) exactly, except where an
    exempt query could list it; on a coarse grid (squared distances exact in
    float32, many ties and duplicates split by id on both sides) exactly
    everywhere.  Mean kNN distances hold to tau at every k for sampled
    queries, and the in-degrees sum to n k."""
    rng = np.random.default_rng(4096)
    n, d = 40_000, 3
    if case == "random":
        x = rng.random((n, d)).astype(np.float32)
    else:
        x = (rng.integers(0, 20, size=(n, d)) / 16.0).astype(np.float32)
    ks = [2, 5, 16, 64, 256]
    out = S.snaps_k_grid([(S.Population.from_rows(x), (1 << d) - 1, ks, 400)], with_metrics=True)[0]
    deg = out["indeg"].cpu().numpy().astype(np.int64)
    km = out["knn_mean"].cpu().numpy().astype(np.float64)
    for j, k in enumerate(ks):
        assert deg[j].sum() == n * k, k
    ora = C.join(x, 64, -1.0)
    for j, k in enumerate(ks):
        if k > 64:
            continue
        want = O.indegree(ora["knn_ids"][:, :k], n)
        if case == "random":
            dk = ora["knn_dist"][:, k - 1]
            dn = ora["knn_dist"][:, k] if k < 64 else ora["knn_next"]
            ex = ~knn_strict(dk, dn)
            # an exempt query lists every object closer than its k-th
            # distance (1 - tau) on both sides; they differ only in objects
            # within tau of that distance
            touched = np.zeros(n, dtype=bool)
            exq = np.nonzero(ex)[0]
            if exq.size:
                Dq = O.pair_distances(x[exq], x)
                Dq[np.arange(exq.size), exq] = np.inf
                band = (Dq >= dk[exq, None] * (1 - TAU)) & (Dq <= dk[exq, None] * (1 + TAU))
                touched[np.nonzero(band)[1]] = True
            assert ((deg[j] == want) | touched).all(), k
            assert touched.sum() < n // 100, (k, int(touched.sum()))
        else:
            np.testing.assert_array_equal(deg[j], want, err_msg=f"k={k}")
    qs = np.sort(rng.choice(n, size=48, replace=False))
    D = O.pair_distances(x[qs], x)
    D[np.arange(qs.size), qs] = np.inf
    Ds = np.sort(D, axis=1)
    for j, k in enumerate(ks):
        want = Ds[:, :k].mean(axis=1)
        got = km[j][qs]
        ok = (np.abs(got - want) <= TAU * want) | ((want == 0) & (got == 0))
        assert ok.all(), (k, got[~ok][:3], want[~ok][:3])
