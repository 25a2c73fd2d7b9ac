"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the public header declares, sizes workspaces, and rejects
invalid arguments before touching a device."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "snaps.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(snaps_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2405_20176_amd import snaps
    return snaps.load_library()


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for f in ("snaps_knn_selfjoin", "snaps_eps_selfjoin", "snaps_outlier_scores", "snaps_rank"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_empty_error(lib):
    assert b"gfx950" in lib.snaps_version()


def test_workspace_sizes(lib):
    from paper_2405_20176_amd.snaps import OP_EPS, OP_KNN, OP_RANK, OP_SCORES
    a = lib.snaps_workspace_bytes(OP_SCORES, 31693, 15, 10)
    b = lib.snaps_workspace_bytes(OP_SCORES, 31693, 2, 10)
    assert a > b > 31693 * 4
    assert lib.snaps_workspace_bytes(OP_SCORES, 1, 3, 1) == 0          # n < 2
    assert lib.snaps_workspace_bytes(OP_KNN, 100, 3, 100) == 0         # k > n-1
    assert lib.snaps_workspace_bytes(OP_KNN, 100, 17, 5) == 0          # d > 16
    assert lib.snaps_workspace_bytes(OP_KNN, 100, 3, 40) > 0           # k above the fused join: selection kernel
    assert lib.snaps_workspace_bytes(OP_KNN, 6000, 3, 5000) == 0       # lists above k = 4096 are not written
    assert lib.snaps_workspace_bytes(OP_SCORES, 6000, 3, 5000) > 0     # the scores take any k
    assert lib.snaps_workspace_bytes(OP_EPS, 100, 3, 0) > 0
    assert lib.snaps_workspace_bytes(OP_RANK, 100, 0, 0) == 0          # LDS-resident rank needs none
    assert lib.snaps_workspace_bytes(OP_RANK, 40000, 0, 0) > 8 * 40000 * 4
    big = lib.snaps_workspace_bytes(OP_SCORES, 40000, 3, 5)            # device-wide sort path
    assert big > lib.snaps_workspace_bytes(OP_KNN, 40000, 3, 5) > 0
    assert lib.snaps_workspace_bytes(OP_SCORES, (1 << 30) + 1, 3, 5) == 0   # beyond the n limit


def _pop(n=100, f=15):
    from paper_2405_20176_amd.snaps import c_population
    return c_population(0x1000, 128, n, f)   # never dereferenced: validation fails first


@pytest.mark.parametrize("mask,k,expect", [
    (0b1, 5, -1),            # one feature
    (1 << 15, 5, -1),        # beyond n_features
    (0b111, 0, -1),          # k < 1
    (0b111, 100, -1),        # k > n - 1
])
def test_knn_validation(lib, mask, k, expect):
    p = _pop()
    ids = ctypes.c_void_p(0x2000)
    rc = lib.snaps_knn_selfjoin(ctypes.byref(p), mask, k, ids, None, None, 0, None)
    assert rc == expect, lib.snaps_last_error()
    assert lib.snaps_last_error()


def test_large_k_list_limit(lib):
    """Sorted kNN lists are written up to k = 4096; above, the call is
    refused before any device work (the scores alone take any k <= n - 1)."""
    from paper_2405_20176_amd.snaps import c_job, c_population, c_scores
    p = c_population(0x1000, 6016, 6000, 15)
    ids = ctypes.c_void_p(0x2000)
    assert lib.snaps_knn_selfjoin(ctypes.byref(p), 0b111, 4097, ids, None, None, 0, None) == -4
    assert lib.snaps_knn_selfjoin(ctypes.byref(p), 0b111, 6000, ids, None, None, 0, None) == -1   # k > n - 1
    job = c_job()
    job.pop = ctypes.pointer(p)
    job.mask, job.k, job.eps = 0b111, 5000, 0.1
    job.out = c_scores(0x10, 0x20, 0x30, 0x40)
    assert lib.snaps_outlier_scores_workspace(ctypes.byref(job), 1, None) > 0
    job.knn_ids = 0x50
    assert lib.snaps_outlier_scores(ctypes.byref(job), 1, None, None, 0, None) == -4


def test_eps_validation(lib):
    p = _pop()
    c = ctypes.c_void_p(0x2000)
    for eps in (0.0, -1.0, float("inf"), float("nan")):
        assert lib.snaps_eps_selfjoin(ctypes.byref(p), 0b11, eps, c, c, None, None, 0, None, 0, None) == -1
    # pair list arguments: a capacity needs the list and its row starts;
    # a negative capacity is rejected; a workspace is required (checked
    # before any device work)
    assert lib.snaps_eps_selfjoin(ctypes.byref(p), 0b11, 0.1, c, c, None, c, 10, None, 0, None) == -1
    assert lib.snaps_eps_selfjoin(ctypes.byref(p), 0b11, 0.1, c, c, c, None, 10, None, 0, None) == -1
    assert lib.snaps_eps_selfjoin(ctypes.byref(p), 0b11, 0.1, c, c, c, c, -1, None, 0, None) == -1
    assert lib.snaps_eps_selfjoin(ctypes.byref(p), 0b11, 0.1, c, c, c, c, 10, None, 0, None) == -1
    need = lib.snaps_workspace_bytes(1, 100, 2, 0)          # SNAPS_OP_EPS
    assert lib.snaps_eps_selfjoin(ctypes.byref(p), 0b11, 0.1, c, c, c, c, 10, c, need - 1, None) == -2


def test_population_validation(lib):
    from paper_2405_20176_amd.snaps import c_population
    c = ctypes.c_void_p(0x2000)
    bad = [c_population(0, 128, 100, 15), c_population(0x1000, 50, 100, 15), c_population(0x1000, 128, 1, 15),
           c_population(0x1000, 128, 100, 1), c_population(0x1000, 128, 100, 33)]
    for p in bad:
        assert lib.snaps_knn_selfjoin(ctypes.byref(p), 0b11, 1, c, None, None, 0, None) == -1
    big = c_population(0x1000, 1 << 31, 1 << 31, 15)
    assert lib.snaps_knn_selfjoin(ctypes.byref(big), 0b11, 1, c, None, None, 0, None) == -4


def test_outlier_scores_validation(lib):
    from paper_2405_20176_amd.snaps import c_job, c_scores, c_tuning
    p = _pop()
    job = c_job()
    job.pop = ctypes.pointer(p)
    job.mask, job.k, job.eps = 0b111, 5, 0.1
    job.out = c_scores(0x10, 0x20, 0x30, 0x40)
    assert lib.snaps_outlier_scores(ctypes.byref(job), 0, None, None, 0, None) == -1      # n_jobs = 0
    bad = c_job.from_buffer_copy(job)
    bad.out = c_scores(0, 0x20, 0x30, 0x40)
    assert lib.snaps_outlier_scores(ctypes.byref(bad), 1, None, None, 0, None) == -1      # missing output
    t = c_tuning()
    t.split = 3
    assert lib.snaps_outlier_scores(ctypes.byref(job), 1, ctypes.byref(t), None, 0, None) == -1
    for field, value in (("index_sort", 3), ("tile_shape", 4), ("tile_shape", -1), ("filter", 4), ("mq", 3)):
        t = c_tuning()
        setattr(t, field, value)
        assert lib.snaps_outlier_scores(ctypes.byref(job), 1, ctypes.byref(t), None, 0, None) == -1, field
    # per-job overrides of the walk: mode 0..2, index_dims 0..6
    for field, value in (("mode", 3), ("mode", -1), ("index_dims", 7), ("index_dims", -1), ("tile_shape", 4),
                         ("tile_shape", -1), ("reserved", 1)):
        bj = c_job.from_buffer_copy(job)
        setattr(bj, field, value)
        assert lib.snaps_outlier_scores(ctypes.byref(bj), 1, None, None, 0, None) == -1, (field, value)
        assert lib.snaps_outlier_scores_workspace(ctypes.byref(bj), 1, None) == 0, (field, value)
    okj = c_job.from_buffer_copy(job)
    okj.mode, okj.index_dims = 2, 3
    assert lib.snaps_outlier_scores_workspace(ctypes.byref(okj), 1, None) > 0
    # an ensemble output needs the rank output
    ej = c_job.from_buffer_copy(job)
    ej.ensemble = 0x50
    assert lib.snaps_outlier_scores(ctypes.byref(ej), 1, None, None, 0, None) == -1
    # the packed LDS index needs no device-wide sort scratch
    tp, tr = c_tuning(), c_tuning()
    tp.index_sort, tr.index_sort = 1, 2
    assert (lib.snaps_outlier_scores_workspace(ctypes.byref(job), 1, ctypes.byref(tp))
            < lib.snaps_outlier_scores_workspace(ctypes.byref(job), 1, ctypes.byref(tr)))
    t = c_tuning()
    need = lib.snaps_outlier_scores_workspace(ctypes.byref(job), 1, ctypes.byref(t))
    assert need > 0
    # a workspace that is too small is reported before any device work
    rc = lib.snaps_outlier_scores(ctypes.byref(job), 1, ctypes.byref(t), ctypes.c_void_p(0x1000), need - 1, None)
    assert rc == -2, lib.snaps_last_error()


def test_rank_validation(lib):
    c = ctypes.c_void_p(0x2000)
    assert lib.snaps_rank(None, c, c, c, 10, c, None, 0, None) == -1
    assert lib.snaps_rank(c, c, c, c, 0, c, None, 0, None) == -1
    assert lib.snaps_rank(c, c, c, c, 1 << 20, c, None, 0, None) == -1      # needs a workspace
    assert lib.snaps_rank(c, c, c, c, 1 << 20, c, c, 10, None) == -2        # too small
    assert lib.snaps_rank(c, c, c, c, 1 << 31, c, None, 0, None) == -4


def test_eps_sampler_validation(lib):
    from paper_2405_20176_amd.snaps import c_eps_job
    p = _pop(n=100)
    j = c_eps_job()
    j.pop = ctypes.pointer(p)
    j.mask, j.m, j.sample, j.n_targets, j.eps = 0b111, 10, 0x3000, 2, 0x4000
    j.target[0], j.target[1] = 1.0, 50.0
    assert lib.snaps_eps_sample_workspace(ctypes.byref(j), 1) > 0
    assert lib.snaps_eps_sample(ctypes.byref(j), 0, None, 0, None) == -1             # no jobs
    assert lib.snaps_eps_sample(ctypes.byref(j), 1, None, 0, None) == -1             # no workspace
    need = lib.snaps_eps_sample_workspace(ctypes.byref(j), 1)
    assert lib.snaps_eps_sample(ctypes.byref(j), 1, ctypes.c_void_p(0x1000), need - 1, None) == -2
    for field, value in (("m", 0), ("m", 101), ("n_targets", 0), ("n_targets", 9), ("sample", None), ("eps", None)):
        bad = c_eps_job.from_buffer_copy(j)
        setattr(bad, field, value)
        assert lib.snaps_eps_sample_workspace(ctypes.byref(bad), 1) == 0, field
        assert lib.snaps_eps_sample(ctypes.byref(bad), 1, ctypes.c_void_p(0x1000), need, None) == -1, field
    for t in (0.0, -1.0, float("nan"), 0.04, 99.0):     # r = round(t m) must be in [1, m (n - 1) - 1]
        bad = c_eps_job.from_buffer_copy(j)
        bad.target[1] = t
        assert lib.snaps_eps_sample_workspace(ctypes.byref(bad), 1) == 0, t
    ok = c_eps_job.from_buffer_copy(j)
    ok.target[1] = 98.9                                 # r = 989 = m (n - 1) - 1
    assert lib.snaps_eps_sample_workspace(ctypes.byref(ok), 1) > 0


def test_eps_grid_validation(lib):
    from paper_2405_20176_amd.snaps import c_eps_grid_job, c_population
    p = _pop(n=100)
    j = c_eps_grid_job()
    j.pop = ctypes.pointer(p)
    j.mask, j.n_grid, j.top_n, j.similarity, j.select = 0b111, 3, 5, 0x5000, 0x6000
    j.eps[0], j.eps[1], j.eps[2] = 0.1, 0.2, 0.3
    assert lib.snaps_eps_grid_workspace(ctypes.byref(j), 1) > 0
    need = lib.snaps_eps_grid_workspace(ctypes.byref(j), 1)
    assert lib.snaps_eps_grid(ctypes.byref(j), 1, None, 0, None) == -1
    assert lib.snaps_eps_grid(ctypes.byref(j), 1, ctypes.c_void_p(0x1000), need - 1, None) == -2
    cases = [("n_grid", 1), ("n_grid", 17), ("top_n", 0), ("top_n", 101), ("similarity", None), ("select", None)]
    for field, value in cases:
        bad = c_eps_grid_job.from_buffer_copy(j)
        setattr(bad, field, value)
        assert lib.snaps_eps_grid_workspace(ctypes.byref(bad), 1) == 0, field
    for radii in ((0.1, 0.1, 0.3), (0.3, 0.2, 0.1), (0.0, 0.2, 0.3), (0.1, 0.2, float("inf"))):
        bad = c_eps_grid_job.from_buffer_copy(j)
        for r, v in enumerate(radii):
            bad.eps[r] = v
        assert lib.snaps_eps_grid_workspace(ctypes.byref(bad), 1) == 0, radii
    for cols, ld in ((0x1004, 128), (0x1000, 102)):    # misaligned columns, ld not a multiple of 4
        q = c_population(cols, ld, 100, 15)
        bad = c_eps_grid_job.from_buffer_copy(j)
        bad.pop = ctypes.pointer(q)
        assert lib.snaps_eps_grid_workspace(ctypes.byref(bad), 1) == 0, (cols, ld)


def test_k_grid_validation(lib):
    from paper_2405_20176_amd.snaps import c_k_grid_job, c_population
    p = _pop(n=100)
    j = c_k_grid_job()
    j.pop = ctypes.pointer(p)
    j.mask, j.n_grid, j.top_n, j.similarity, j.select = 0b111, 3, 5, 0x5000, 0x6000
    j.k[0], j.k[1], j.k[2] = 2, 8, 99
    need = lib.snaps_k_grid_workspace(ctypes.byref(j), 1)
    assert need > 100 * 16 * 8                     # per-object thresholds of every grid point
    assert lib.snaps_k_grid(ctypes.byref(j), 1, None, 0, None) == -1
    assert lib.snaps_k_grid(ctypes.byref(j), 1, ctypes.c_void_p(0x1000), need - 1, None) == -2
    cases = [("n_grid", 1), ("n_grid", 17), ("top_n", 0), ("top_n", 101), ("similarity", None), ("select", None)]
    for field, value in cases:
        bad = c_k_grid_job.from_buffer_copy(j)
        setattr(bad, field, value)
        assert lib.snaps_k_grid_workspace(ctypes.byref(bad), 1) == 0, field
    # k >= 1, strictly ascending, k_max <= n - 1
    for ks in ((0, 8, 20), (2, 2, 20), (8, 2, 20), (2, 8, 100)):
        bad = c_k_grid_job.from_buffer_copy(j)
        for r, v in enumerate(ks):
            bad.k[r] = v
        assert lib.snaps_k_grid_workspace(ctypes.byref(bad), 1) == 0, ks
    for cols, ld, n in ((0x1004, 128, 100), (0x1000, 102, 100)):
        q = c_population(cols, ld, n, 15)           # misaligned, ld not a multiple of 4
        bad = c_k_grid_job.from_buffer_copy(j)
        bad.pop = ctypes.pointer(q)
        assert lib.snaps_k_grid_workspace(ctypes.byref(bad), 1) == 0, (cols, ld, n)
    q = c_population(0x1000, 32768, 32768, 15)      # the largest population, k_max beyond 4096
    big = c_k_grid_job.from_buffer_copy(j)
    big.pop = ctypes.pointer(q)
    big.k[2] = 4096
    assert lib.snaps_k_grid_workspace(ctypes.byref(big), 1) > 0
    big.k[2] = 4097
    assert lib.snaps_k_grid_workspace(ctypes.byref(big), 1) == 0
    q2 = c_population(0x1000, 5_000_000, 5_000_000, 15)   # above one workgroup's registers: streaming selection
    lsst = c_k_grid_job.from_buffer_copy(j)
    lsst.pop = ctypes.pointer(q2)
    assert lib.snaps_k_grid_workspace(ctypes.byref(lsst), 1) > 5_000_000 * 16 * 8


def test_static_scratch_entry_validation(lib):
    """The allocation-free form validates like snaps_outlier_scores and
    refuses, before any device work, jobs whose workspace exceeds its fixed
    scratch."""
    from paper_2405_20176_amd.snaps import STATIC_SCRATCH_BYTES, c_job, c_population, c_scores
    p = _pop()
    job = c_job()
    job.pop = ctypes.pointer(p)
    job.mask, job.k, job.eps = 0b111, 5, 0.1
    job.out = c_scores(0x10, 0x20, 0x30, 0x40)
    assert lib.snaps_outlier_scores_static(ctypes.byref(job), 0, None, None) == -1
    bad = c_job.from_buffer_copy(job)
    bad.k = 0
    assert lib.snaps_outlier_scores_static(ctypes.byref(bad), 1, None, None) == -1
    big = c_population(0x1000, 1_200_000, 1_200_000, 15)
    bj = c_job.from_buffer_copy(job)
    bj.pop = ctypes.pointer(big)
    bj.mask = (1 << 15) - 1
    assert lib.snaps_outlier_scores_workspace(ctypes.byref(bj), 1, None) > STATIC_SCRATCH_BYTES
    rc = lib.snaps_outlier_scores_static(ctypes.byref(bj), 1, None, None)
    assert rc == -2, lib.snaps_last_error()
    assert b"static scratch" in lib.snaps_last_error()


def _alert_jobs(ms, methods):
    from paper_2405_20176_amd.snaps import c_alert_job
    arr = (c_alert_job * len(ms))()
    for i, (m, meth) in enumerate(zip(ms, methods)):
        arr[i].state = 0x1000                 # never dereferenced on the host
        arr[i].alerts = 0x2000
        arr[i].m = m
        arr[i].method = meth
        arr[i].eps_count, arr[i].eps_mean, arr[i].indeg, arr[i].knn_mean = 0x3000, 0x4000, 0x5000, 0x6000
    return arr


def _alert_ws_expected(ms, d, kc):
    """The documented layout: per matrix-core job, groups x slices partial
    results of (kc + 4) x 64 floats, then one 4-byte bound per alert slot,
    each part rounded up to 256 bytes."""
    align = lambda b: (b + 255) // 256 * 256
    w = 4 if (d + 5) // 4 * 4 > 16 else 8     # wavefronts per workgroup
    part, slots = 0, 0
    for m in ms:
        g = -(-m // 64)
        sl = min(max(-(-(8192 // w) // g), 1), 512 // w)
        part += align(g * sl * (kc + 4) * 64 * 4)
        slots += g * 64
    return part + align(slots * 4) if slots else 0


def test_alert_workspace_and_kernel_choice(lib):
    """Workspace of the matrix-core alert kernel, and which jobs run it:
    method 2 always, method 1 never, method 0 from d = 6 and at d = 5 up to
    512 alerts."""
    ws = lambda ms, meths, d, k: lib.snaps_alerts_workspace_bytes(_alert_jobs(ms, meths), len(ms), d, k)
    assert ws([1000], [0], 4, 10) == 0
    assert ws([1000], [1], 10, 10) == 0
    assert ws([1000], [2], 4, 10) == _alert_ws_expected([1000], 4, 10)
    assert ws([1, 64, 65, 10000], [0] * 4, 6, 10) == _alert_ws_expected([1, 64, 65, 10000], 6, 10)
    assert ws([100, 1000], [0, 0], 5, 10) == _alert_ws_expected([100], 5, 10)
    assert ws([300], [0], 15, 20) == _alert_ws_expected([300], 15, 20)      # four wavefronts at d = 15
    assert ws([300], [0], 15, 20) != _alert_ws_expected([300], 14, 20)
    assert ws([0, 500], [2, 1], 12, 32) == 0                                # no alerts / per-alert kernel
    assert ws([500], [0], 1, 10) == 0 and ws([500], [0], 8, 0) == 0       # invalid d, k


def test_alert_score_validation(lib):
    """snaps_alerts_score refuses, before any device work, an unknown method,
    a missing workspace and one that is too small."""
    jobs = _alert_jobs([200], [3])
    assert lib.snaps_alerts_score(jobs, 1, 8, 10, None, 0, None) == -1
    jobs = _alert_jobs([200], [2])
    need = lib.snaps_alerts_workspace_bytes(jobs, 1, 8, 10)
    assert need > 0
    assert lib.snaps_alerts_score(jobs, 1, 8, 10, None, 0, None) == -1
    assert lib.snaps_alerts_score(jobs, 1, 8, 10, ctypes.c_void_p(0x10000), need - 1, None) == -2
    assert b"workspace" in lib.snaps_last_error()
    bad = _alert_jobs([-1], [1])
    assert lib.snaps_alerts_score(bad, 1, 8, 10, None, 0, None) == -1
