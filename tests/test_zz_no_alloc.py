"""snaps_outlier_scores_static (the library's fixed per-device scratch, no
workspace argument, no device allocation) against snaps_outlier_scores with
a caller workspace: the same kernels on the same jobs, so every output must
be identical bit for bit.  Two calls in a row, the second with smaller
jobs, so that it runs on the scratch contents the first call left behind;
then a request above the scratch size is refused with nothing launched."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

KEYS = ("eps_count", "eps_mean", "indeg", "knn_mean", "rank", "ensemble", "knn_ids", "knn_dist")


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_20176_amd import snaps
    snaps.load_library()
    return snaps


def _jobs(S, specs):
    out = []
    for x, mask, k, eps in specs:
        pop = S.Population.from_rows(x)
        out.append(S.Job.alloc(pop, mask, k, eps, with_ensemble=True, with_lists=True))
    return out


def _same(a, b, label):
    for key in KEYS:
        ta, tb = getattr(a, key), getattr(b, key)
        va, vb = ta.cpu().numpy(), tb.cpu().numpy()
        assert va.dtype == vb.dtype and va.shape == vb.shape, (label, key)
        assert np.array_equal(va.view(np.uint8), vb.view(np.uint8)), f"{label}: {key} differs"


def _poison(jobs):
    for j in jobs:
        for key in KEYS:
            t = getattr(j, key)
            t.view(torch.uint8).fill_(0xA5)


@pytest.mark.parametrize("tune_kind", ["default", "packed_index"])
def test_static_scratch_equals_workspace_call_twice(S, tune_kind):
    rng = np.random.default_rng(77)
    big = [(rng.random((20000, 7)).astype(np.float32), 0b1011011, 10, 0.06),
           (rng.random((3000, 5)).astype(np.float32), 0b00111, 5, 0.08),
           (rng.random((40000, 4)).astype(np.float32), 0b1111, 20, 0.02)]   # above one LDS: device-wide sort
    small = [(rng.random((1500, 6)).astype(np.float32), 0b110101, 7, 0.12)]
    tune = S.tuning(index_sort=1) if tune_kind == "packed_index" else None
    if tune_kind == "packed_index":
        big = big[:2]
    for call, specs in enumerate((big, small)):
        ref = _jobs(S, specs)
        got = [S.Job(j.pop, j.mask, j.k, j.eps, *(torch.empty_like(getattr(j, key)) for key in
                                                    ("eps_count", "eps_mean", "indeg", "knn_mean", "rank",
                                                     "ensemble")),
                     knn_ids=torch.empty_like(j.knn_ids), knn_dist=torch.empty_like(j.knn_dist)) for j in ref]
        _poison(ref)
        _poison(got)
        S.snaps_outlier_scores(ref, tune=tune)
        S.snaps_outlier_scores_static(got, tune=tune)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(ref, got)):
            _same(a, b, f"call {call} job {i} ({tune_kind})")
        # plain sanity of the outputs themselves
        for j in got:
            assert int(j.indeg.sum()) == j.pop.n * j.k


def test_static_scratch_refuses_oversized_jobs(S):
    n = 1_200_000                     # 1.2e6 objects at d = 15: about 96 MB of index scratch
    cols = torch.zeros((15, n), dtype=torch.float32, device="cuda")
    pop = S.Population(cols, n)
    job = S.Job.alloc(pop, (1 << 15) - 1, 10, 0.1, with_rank=False)   # full-size outputs all the same
    need = S.snaps_outlier_scores_workspace([job])
    assert need > S.STATIC_SCRATCH_BYTES
    with pytest.raises(S.SnapsError) as ei:
        S.snaps_outlier_scores_static([job])
    assert ei.value.code == S.SNAPS_ENOMEM
    torch.cuda.synchronize()
