"""Host-side pieces of the autotuner: candidate settings, class keys, the
table's application to jobs and its per-device cache file."""
from __future__ import annotations

from types import SimpleNamespace

import pytest

pytest.importorskip("torch")
from paper_2405_20176_amd import autotune as AT  # noqa: E402


def _job(mask, n):
    return SimpleNamespace(pop=SimpleNamespace(n=n), mask=mask, k=10, eps=0.1, mode=0, index_dims=0)


def test_candidates_cover_brute_force_and_every_index_width():
    assert AT.candidates(2) == [(1, 0), (2, 2)]
    assert AT.candidates(8) == [(1, 0)] + [(2, c) for c in range(2, 7)]
    assert all(c <= 6 for _, c in AT.candidates(15))


def test_class_keys_and_apply():
    jobs = [_job(0b111, 31693), _job(0b1111, 31693), _job(0b111, 1000)]
    assert AT.job_class(jobs[0]) == (3, 14) and AT.job_class(jobs[2]) == (3, 9)
    table = {AT.class_key((3, 14)): {"mode": 2, "index_dims": 3}, AT.class_key((4, 14)): {"mode": 1, "index_dims": 0}}
    assert AT.apply(jobs, table) == 2
    assert (jobs[0].mode, jobs[0].index_dims) == (2, 3)
    assert (jobs[1].mode, jobs[1].index_dims) == (1, 0)
    assert (jobs[2].mode, jobs[2].index_dims) == (0, 0)          # class not in the table: unchanged


def test_cache_round_trip_per_device(tmp_path):
    path = str(tmp_path / "tune.json")
    assert AT.load(path, "dev A") is None
    AT.save(path, "dev A", {"d3_n2^14": {"mode": 2, "index_dims": 3}})
    AT.save(path, "dev B", {"d3_n2^14": {"mode": 1, "index_dims": 0}})
    assert AT.load(path, "dev A")["d3_n2^14"]["mode"] == 2
    assert AT.load(path, "dev B")["d3_n2^14"]["mode"] == 1
    assert AT.load(path, "dev C") is None
