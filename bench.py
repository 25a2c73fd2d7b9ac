"""Benchmark: SNAPS outlier scores over every subspace of a SNAPShot1-shaped
population on one MI355X.

Workload (one step): N = 31,693 objects x 15 float32 features (seeded
synthetic stand-in for the SNAPShot1 catalogue), all 32,752 subspaces of 2..15
features, k = 10, eps per subspace from the stored table (mean neighbour count
10).  A step runs the whole hot path for every subspace: index build, fused
kNN + eps join with the four metrics, dense ranks.  Outputs of all subspaces
stay resident in HBM (35 GiB: four metrics, four ranks and their mean).  The timed steps use the batched form: every
subspace in one job table, its three passes captured as HIP graphs and
replayed.  A plain pass (one library call per subspace) is timed once
afterwards for comparison, and the served form (alerts scored against
resident populations under continuous batching) reports p50/p99 latency.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "object·subspace outlier scores/sec (batched vs plain, 1 GPU) + p50/p99 latency"
UNIT = "object·subspace scores/s"
# MI355X published fp32 peak, flop/s (vector and dense matrix alike: 256 CUs
# x 2.4 GHz x 256 flop per clock and CU).  The join's algorithmic work is the
# direct form's 3d fp32 flops per evaluated pair; its contraction runs on the
# matrix cores in half-precision pieces and what bounds it is the vector ALU
# (screening, walk, exact re-evaluation), so it is priced against this peak.
PEAK_FP32 = 157.3e12
PEAK_HBM = 8.0e12                # MI355X HBM3E, byte/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_join_c1_all_subspaces_hbm_traffic.md")
JOIN_SOURCES = ["join_kernel.cuh", "join_mfma.cuh", "join.hip", "join_inst0.hip", "join_inst1.hip",
                "join_inst2.hip", "join_inst3.hip", "join_mfma0.hip", "join_mfma1.hip", "join_mfma2.hip",
                "join_mfma3.hip", "common.cuh", "snaps_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(x, masks, eps_tab, k):
    """Time the CPU oracle (C twin with OpenMP, float64 brute force, ranks in
    NumPy) on one subspace of each dimensionality at full size and
    extrapolate to all subspaces by the number of subspaces of each d."""
    import oracle as O
    from oracle import c_oracle
    n = x.shape[0]
    dims = np.array([bin(int(m)).count("1") for m in masks])
    t_by_d = {}
    t0 = time.time()
    per_d = 3
    for d in range(2, 16):
        idx = np.nonzero(dims == d)[0]
        pick = idx[np.linspace(0, idx.size - 1, min(per_d, idx.size)).astype(int)]
        t = time.perf_counter()
        for i in pick:
            xs = O.project(x, int(masks[i])).astype(np.float32)
            c_oracle.outlier_scores(xs, k, float(eps_tab[i]))
        t_by_d[d] = (time.perf_counter() - t) / len(pick)
    total = sum(math.comb(15, d) * t_by_d[d] for d in t_by_d)
    log(f"cpu baseline: sample of {per_d * 14 - 1} spaces took {time.time() - t0:.1f} s, "
        f"extrapolated {total / 3600:.2f} h")
    return {"value": n * len(masks) / total, "unit": UNIT, "cores": c_oracle.num_threads(), "kind": "oracle",
            "sample": "three full-size subspaces per dimensionality d=2..15 (41 of 32,752; d=15 has one), timed "
                      "with the C/OpenMP float64 oracle and extrapolated by the number of subspaces of each d",
            "extrapolated_s": total, "cpu_model": _cpu_model()}


def alert_ab_bench(S, G, dev, sizes=(16, 256, 1024, 4096, 10000)):
    """Per-request time of the two alert kernels (method 1: one wavefront per
    alert; method 2: matrix-core cross-join of 64-alert groups) on one
    10^6-object serving population, one catalogue subspace per d, alerts from
    the serving generator (the largest request of that subspace, repeated
    with a 10^-3 shift when short).  HIP events over 3 calls after a warm-up;
    eps counts, in-degrees and kNN means compared between the kernels."""
    import torch
    w = G.gen_c4()
    masks_tab, eps_tab = G.load_c4_eps()
    x, lo, hi = w.population(0)
    pop = S.Population.from_rows(x, device=dev)
    del x
    best = {}
    for r in w.requests(60.0):
        if r.pop != 0:
            continue
        d = bin(int(masks_tab[0, r.space])).count("1")
        if d not in best or r.n_alerts > best[d].n_alerts:
            best[d] = r
    out = {}
    for d, r in sorted(best.items()):
        m_ = int(masks_tab[0, r.space])
        st = S.ServeState(pop, m_, w.k, float(eps_tab[0, r.space]))
        al = np.ascontiguousarray(w.alerts(r, lo, hi)[:, G.mask_features(m_)], dtype=np.float32)
        while al.shape[0] < max(sizes):
            al = np.concatenate([al, al + np.float32(1e-3)]).astype(np.float32)
        row = {}
        for m in sizes:
            a = torch.tensor(al[:m], device=dev)
            times, jobs = {}, {}
            for meth in (1, 2):
                job = S.AlertJob.alloc(st, a, method=meth)
                S.snaps_alerts_score([job])
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(3):
                    S.snaps_alerts_score([job])
                e1.record()
                torch.cuda.synchronize()
                times[meth] = e0.elapsed_time(e1) / 3
                jobs[meth] = job
            same = all(torch.equal(getattr(jobs[1], key), getattr(jobs[2], key))
                       for key in ("eps_count", "indeg", "knn_mean"))
            row[str(m)] = {"per_alert_kernel_ms": times[1], "matrix_core_ms": times[2],
                           "speedup": times[1] / times[2], "identical_counts_and_knn_mean": same}
        out[str(d)] = row
        log(f"alert A/B d={d}: " + ", ".join(f"m={m} {v['per_alert_kernel_ms']:.2f}/{v['matrix_core_ms']:.2f} ms"
                                              for m, v in row.items()))
        del st
        torch.cuda.empty_cache()
    return {"per_d": out, "population_n": pop.n, "k": w.k,
            "what": "ms per request, one wavefront per alert / matrix cores, same state and alerts"}


def serve_bench(S, G, dev, seconds: float, warmup_s: float = 10.0, n_streams: int = 4, plain_s: float = 20.0,
                capacity_s: float = 10.0):
    """Served form: 4 resident populations of 1,000,000 objects (the serving
    generator), every subspace of each population's seeded catalogue (64 per
    population, 256 states) built at start-up (cold builds, timed one by one),
    and an open-loop Poisson stream (200 requests/s, 1..10,000 alerts per
    request, log-uniform) replayed in real time through the
    continuous-batching server: ``warmup_s`` seconds of arrivals whose
    requests are served but not counted, then ``seconds`` measured.
    Compared with the plain form (one request at a time, each alone, no
    overlap) on the same states: both serve the same backlog of requests as
    fast as they can (capacity, results compared bit for bit), and the plain
    form replays ``plain_s`` seconds of the same arrivals."""
    import torch
    from paper_2405_20176_amd.serve import Admission, Batcher, GpuExecutor, Request, serve_serial
    w = G.gen_c4()
    masks_tab, eps_tab = G.load_c4_eps()
    t0 = time.perf_counter()
    bounds, states = [], {}
    build_s = []
    pops = []
    for p in range(w.n_pop):
        x, lo, hi = w.population(p)
        pop = S.Population.from_rows(x, device=dev)
        del x
        pops.append(pop)
        bounds.append((lo, hi))
        assert np.array_equal(masks_tab[p], w.spaces[p]), "eps table does not match the serving catalogue"
        for si, m in enumerate(int(v) for v in masks_tab[p]):
            tb = time.perf_counter()
            states[(p, m)] = S.ServeState(pop, m, w.k, float(eps_tab[p, si]))
            torch.cuda.synchronize()
            build_s.append(time.perf_counter() - tb)
    state_bytes = sum(st.nbytes for st in states.values())
    log(f"serving: {len(states)} states ({state_bytes / 2**30:.1f} GiB) built in {time.perf_counter() - t0:.1f} s "
        f"(cold build per state {np.median(build_s):.3f} s median)")
    tg = time.perf_counter()
    reqs = []
    for r in w.requests(warmup_s + seconds):
        p = r.pop
        m = int(masks_tab[p, r.space])
        cols = G.mask_features(m)
        lo, hi = bounds[p]
        al = np.ascontiguousarray(w.alerts(r, lo, hi)[:, cols], dtype=np.float32)
        reqs.append(Request(r.rid, r.arrival_s, (p, m), al))
    log(f"serving: {len(reqs)} requests over {warmup_s + seconds:.0f} s of arrivals generated in "
        f"{time.perf_counter() - tg:.1f} s")
    ex = GpuExecutor(states, n_streams=n_streams, device=dev)
    warm = Batcher(ex, Admission(8 << 30, n_streams))
    for i, key in enumerate(states):
        warm.submit(Request(-1 - i, 0.0, key, np.zeros((64, bin(key[1]).count("1")), np.float32)))
    warm.drain()
    fresh = lambda rs: [Request(r.rid, r.arrival, r.key, r.alerts) for r in rs]

    # continuous batching, open loop
    b = Batcher(ex, Admission(8 << 30, n_streams), max_batch_alerts=1 << 16)
    t_start = time.perf_counter()
    b.run_open_loop(fresh(reqs), t0=t_start)
    wall = time.perf_counter() - t_start
    meas = [r for r in b.finished if r.status == "done" and r.arrival - t_start >= warmup_s]
    lat = np.array([r.done - r.arrival for r in meas])
    span = max(r.done for r in meas) - min(r.arrival for r in meas)
    res = {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3), "requests": len(meas),
           "rejected": sum(1 for r in b.finished if r.status != "done"),
           "alerts": int(sum(r.m for r in meas)), "alert_scores_per_s": float(sum(r.m for r in meas) / span),
           "requests_per_s": len(meas) / span, "measured_s": seconds, "warmup_s": warmup_s, "wall_s": wall,
           "arrival_rate_hz": w.rate_hz, "populations": w.n_pop, "population_n": w.pop_n,
           "resident_states": len(states), "resident_state_gib": state_bytes / 2**30,
           "cold_builds": {"count": len(build_s), "median_s": float(np.median(build_s)),
                           "max_s": float(np.max(build_s)), "total_s": float(np.sum(build_s)),
                           "when": "at start-up, before the first request (every catalogue state resident; no "
                                   "request meets a missing state)"},
           "cold_misses": 0, "k": w.k, "batches": b.batches_launched, "max_batches_in_flight": b.max_inflight,
           "form": f"continuous batching over {n_streams} streams, admission by an 8 GiB in-flight budget, "
                   "latency = completion (results in host memory) - arrival"}
    log(f"serving: p50 {res['p50_ms']:.1f} ms, p99 {res['p99_ms']:.1f} ms over {len(meas)} requests, "
        f"{res['alert_scores_per_s']:.3e} alert scores/s")

    # capacity: the same backlog served as fast as possible, batched vs plain
    back = [r for r in reqs if warmup_s <= r.arrival < warmup_s + capacity_s]
    bq = fresh(back)
    for r in bq:
        r.arrival = 0.0
    bb = Batcher(ex, Admission(8 << 30, n_streams), max_batch_alerts=1 << 16)
    tc = time.perf_counter()
    bb.run_open_loop(bq, t0=tc)
    cap_batched_s = time.perf_counter() - tc
    pq = fresh(back)
    tc = time.perf_counter()
    pdone = serve_serial(ex, pq, open_loop=False)
    cap_plain_s = time.perf_counter() - tc
    got = {r.rid: r.result for r in bb.finished}
    same = all(np.array_equal(got[r.rid][key], r.result[key]) for r in pdone for key in r.result)
    n_al = int(sum(r.m for r in back))
    cap = {"requests": len(back), "alerts": n_al, "batched_s": cap_batched_s, "plain_s": cap_plain_s,
           "batched_alerts_per_s": n_al / cap_batched_s, "plain_alerts_per_s": n_al / cap_plain_s,
           "results_identical": bool(same),
           "what": f"the requests arriving in [{warmup_s:.0f}, {warmup_s + capacity_s:.0f}) s, all queued at once"}
    res["capacity"] = cap
    res["served_over_plain"] = cap["batched_alerts_per_s"] / cap["plain_alerts_per_s"]
    log(f"serving capacity: batched {cap['batched_alerts_per_s']:.3e} vs plain {cap['plain_alerts_per_s']:.3e} "
        f"alerts/s (identical results: {same})")

    # the plain form under the same arrivals (a shorter slice)
    if plain_s > 0:
        sl = fresh([r for r in reqs if r.arrival < warmup_s + plain_s])
        tp = time.perf_counter()
        pd = serve_serial(ex, sl, open_loop=True)
        pm = [r for r in pd if r.arrival - tp >= warmup_s]
        pl = np.array([r.done - r.arrival for r in pm])
        res["plain_open_loop"] = {"p50_ms": float(np.percentile(pl, 50) * 1e3),
                                  "p99_ms": float(np.percentile(pl, 99) * 1e3), "requests": len(pm),
                                  "measured_s": plain_s, "warmup_s": warmup_s,
                                  "form": "one request at a time, each alone, same states and kernels"}
        log(f"serving plain open loop: p50 {res['plain_open_loop']['p50_ms']:.1f} ms, "
            f"p99 {res['plain_open_loop']['p99_ms']:.1f} ms")
    del states, pops
    return res


def _c3_gen(job):
    """One C3 population as feature-major float32 columns [d, ld] (ld a
    multiple of 64), built in the worker process."""
    import snaps_synth as G
    x = G.gen_c3_projected(job)
    n, d = x.shape
    cols = np.zeros((d, (n + 63) // 64 * 64), dtype=np.float32)
    cols[:, :n] = x.T
    return job.index, n, cols


def c3_bench(S, G, lib, dev, stream, steps: int, warmup: int, autotune_sample: int, plain: bool):
    """Batched uneven workload: 4,096 (population, subspace) jobs, each with
    its own population (N log-uniform in [1e4, 5e5], the SNAPShot1-shaped
    generator), d uniform in 2..15, k in {5, 10, 20}, eps from the stored
    table (sampler target k).  Populations are held as their d subspace
    columns.  The walk of each (d, log2 n) class comes from the autotuner
    (measured on a few jobs per class before timing); the three passes of
    the whole table are HIP graphs.  Compared with the plain form (one
    library call per job, one stream)."""
    import multiprocessing as mp
    import torch
    from paper_2405_20176_amd import autotune as AT
    t0 = time.perf_counter()
    jobs = G.gen_c3_jobs()
    eps = G.load_c3_eps()
    pops = [None] * len(jobs)
    workers = max(1, min(16, os.cpu_count() or 4))
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        for idx, n, cols in pool.imap_unordered(_c3_gen, jobs, chunksize=4):
            pops[idx] = S.Population(torch.from_numpy(cols).to(dev), n)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    ns = np.array([j.n for j in jobs], dtype=np.int64)
    ds = np.array([bin(j.mask).count("1") for j in jobs])
    ks = np.array([j.k for j in jobs])
    log(f"C3: {len(jobs)} populations ({ns.sum():.3e} objects, {sum(p.cols.numel() for p in pops) * 4 / 2**30:.1f} "
        f"GiB of subspace columns) generated and uploaded in {t_gen:.1f} s")
    specs = [(pops[i], (1 << int(ds[i])) - 1, int(ks[i]), float(eps[i])) for i in range(len(jobs))]
    tab = S.JobTable(specs, with_rank=True)
    tuned = None
    if autotune_sample > 0:
        ta = time.perf_counter()
        recs = tab.walk_specs()
        table = AT.tune(recs, sample=autotune_sample, reps=1)
        AT.apply(recs, table)
        tab.apply_walk(recs)
        tuned = {"seconds": time.perf_counter() - ta, "sample_per_class": autotune_sample, "classes": len(table),
                 "choice": {key: [v["mode"], v["index_dims"], v.get("tile_shape", 1)] for key, v in table.items()}}
        log(f"C3: autotuned {len(table)} classes in {tuned['seconds']:.1f} s")
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    tp = time.perf_counter()
    ws, plans = tab.plans(stats=stats)
    log(f"C3: plans built in {time.perf_counter() - tp:.1f} s, workspace {ws.numel() / 2**30:.1f} GiB")

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    for _ in range(warmup):
        for p in plans:
            p.launch(stream)
    torch.cuda.synchronize()
    stats.zero_()
    marks = []
    tt = time.perf_counter()
    for _ in range(steps):
        m = [ev()]
        for p in plans:
            p.launch(stream)
            m.append(ev())
        marks.append(m)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - tt) / steps
    total_n = float(ns.sum())
    value = total_n / sec
    join_ms = sum(m[1].elapsed_time(m[2]) for m in marks) / steps
    pairs, scanned, skipped, pd = (stats.cpu().numpy().astype(np.float64) / steps)
    launches = len(set(zip(ds.tolist(), ks.tolist())))
    achieved = 3.0 * pd / (join_ms / 1000.0)
    # every job's in-degrees sum to n k (each object lists k neighbours)
    off = torch.tensor(tab.off, dtype=torch.int64, device=dev)
    seg = torch.repeat_interleave(torch.arange(len(jobs), device=dev), off[1:] - off[:-1])
    sums = torch.zeros(len(jobs), dtype=torch.int64, device=dev).index_add_(0, seg, tab.indeg.to(torch.int64))
    indeg_ok = bool((sums.cpu().numpy() == ns * ks).all())
    results = float((ns * ks).sum()) + float(tab.eps_count.sum(dtype=torch.int64).item())
    res = {"value": value, "unit": UNIT, "ms_per_step": sec * 1000.0, "steps": steps, "warmup": warmup,
           "jobs": len(jobs), "objects": total_n, "scores_per_step": total_n,
           "passes_ms_per_step": {name: sum(m[i].elapsed_time(m[i + 1]) for m in marks) / steps
                                  for i, name in enumerate(("index", "join", "rank"))},
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_FP32, "avg_launch_ms": join_ms / launches,
                        "launches_per_step": launches, "flops_per_pair": "3d"},
           "join": {"pairs_evaluated": pairs, "brute_force_pairs": float((ns.astype(np.float64) ** 2).sum()),
                    "candidates_per_result": pairs / results, "tiles_scanned": scanned, "tiles_skipped": skipped},
           "indeg_sums_equal_nk": indeg_ok, "generate_upload_s": t_gen, "autotune": tuned,
           "form": "one job table, index/join/rank passes replayed as HIP graphs"}
    log(f"C3: {sec:.2f} s per step, {value:.3e} scores/s, join {join_ms:.0f} ms, frac {achieved / PEAK_FP32:.3f}")
    for p in plans:
        p.close()
    del plans, ws
    torch.cuda.empty_cache()
    if plain:
        need = max(tab.workspace_bytes(None, i, i + 1) for i in range(len(jobs)))
        pws = torch.empty(need, dtype=torch.uint8, device=dev)
        tab.run(None, ws=pws, stream=stream, start=0, stop=1)
        torch.cuda.synchronize()
        tq = time.perf_counter()
        for i in range(len(jobs)):
            tab.run(None, ws=pws, stream=stream, start=i, stop=i + 1)
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - tq
        res["plain"] = {"value": total_n / plain_s, "unit": UNIT, "ms_per_pass": plain_s * 1000.0,
                        "form": "one library call per job, one stream, the same per-job walk settings"}
        res["batched_over_plain"] = value / res["plain"]["value"]
        log(f"C3 plain: {plain_s:.2f} s per pass")
    del tab, pops
    torch.cuda.empty_cache()
    return res


def c2_bench(S, G, dev, stream, steps: int, lsst_k_grid: bool = False):
    """LSST-scale population: N = 5,000,000 objects (the SNAPShot1-shaped
    generator), the full 15-feature space plus all 105 two-feature spaces,
    k = 10, eps from the stored table (target mean count 20), in one job
    table with ranks, passes replayed as HIP graphs, walk settings from the
    library defaults (box pruning with super-tile culls at d = 2, brute force
    at d = 15)."""
    import torch
    t0 = time.perf_counter()
    x, masks, k, _ = G.gen_c2()
    eps = G.load_c2_eps()
    n = x.shape[0]
    pop = S.Population.from_rows(x, device=dev)
    del x
    log(f"C2: population {n} x 15 generated and uploaded in {time.perf_counter() - t0:.1f} s")
    tab = S.JobTable([(pop, int(m), k, float(e)) for m, e in zip(masks, eps)], with_rank=True)
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    ws, plans = tab.plans(stats=stats)
    dims = np.array([bin(int(m)).count("1") for m in masks])

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    for p in plans:                       # warm-up
        p.launch(stream)
    torch.cuda.synchronize()
    res = {"objects": n, "spaces": len(masks), "k": k, "eps_target_mean_count": 20,
           "scores_per_step": float(n) * len(masks), "steps": steps}
    # the full space and the 105 two-feature spaces are timed as one table;
    # the join's per-d split comes from one more pass per part with events
    stats.zero_()
    marks = []
    tt = time.perf_counter()
    for _ in range(steps):
        m = [ev()]
        for p in plans:
            p.launch(stream)
            m.append(ev())
        marks.append(m)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - tt) / steps
    join_ms = sum(m[1].elapsed_time(m[2]) for m in marks) / steps
    pairs, scanned, skipped, pd = stats.cpu().numpy().astype(np.float64) / steps
    res.update({"value": float(n) * len(masks) / sec, "unit": UNIT, "ms_per_step": sec * 1000.0,
                "passes_ms_per_step": {name: sum(m[i].elapsed_time(m[i + 1]) for m in marks) / steps
                                       for i, name in enumerate(("index", "join", "rank"))},
                "roofline": {"bound": "alu", "achieved": 3.0 * pd / (join_ms / 1000.0) / 1e12,
                             "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                             "frac": 3.0 * pd / (join_ms / 1000.0) / PEAK_FP32,
                             "launches_per_step": len(set(dims.tolist())), "flops_per_pair": "3d"},
                "join": {"pairs_evaluated": pairs, "brute_force_pairs": float(n) * n * len(masks),
                         "tiles_scanned": scanned, "tiles_skipped": skipped}})
    for p in plans:
        p.close()
    del plans
    # per part: the full space alone and the 105 two-feature spaces alone
    parts = {}
    for name, sl in (("d15", slice(0, 1)), ("d2_x105", slice(1, len(masks)))):
        st = torch.zeros(4, dtype=torch.int64, device=dev)
        s0, s1 = sl.start, sl.stop
        tab.run(S.tuning(passes=S.PASS_INDEX), ws=ws, stream=stream, start=s0, stop=s1)
        e0 = ev()
        tab.run(S.tuning(passes=S.PASS_JOIN, stats=st), ws=ws, stream=stream, start=s0, stop=s1)
        e1 = ev()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        pr, sc, sk, pdd = st.cpu().numpy().astype(np.float64)
        cnt = float(tab.eps_count[tab.off[s0]:tab.off[s1]].sum(dtype=torch.int64).item())
        parts[name] = {"join_ms": ms, "pairs": pr, "pairs_over_brute_force": pr / (float(n) * n * (s1 - s0)),
                       "candidates_per_result": pr / (float(n) * k * (s1 - s0) + cnt),
                       "tflops": 3.0 * pdd / (ms / 1000.0) / 1e12,
                       "frac": 3.0 * pdd / (ms / 1000.0) / PEAK_FP32,
                       "tiles_scanned": sc, "tiles_skipped": sk}
    res["parts"] = parts
    off = torch.tensor(tab.off, dtype=torch.int64, device=dev)
    sums = torch.stack([tab.indeg[tab.off[i]:tab.off[i + 1]].sum(dtype=torch.int64) for i in range(len(masks))])
    res["indeg_sums_equal_nk"] = bool((sums.cpu().numpy() == n * k).all())
    del off
    # the paper's k selection at this scale (k up to 256 as in the LSST
    # runs, Sec. 4.5): one two-feature space, on request (brute force over
    # n^2 pairs: minutes)
    tk = time.perf_counter()
    if not lsst_k_grid:
        tk = None
    if tk is not None:
        ks = [2, 4, 8, 16, 32, 64, 128, 256]
        kg = S.snaps_k_grid([(pop, int(masks[1]), ks, max(1, int(round(0.01 * n))))], with_metrics=False)[0]
        torch.cuda.synchronize()
        res["k_grid_selection_one_space"] = {
            "seconds": time.perf_counter() - tk, "mask": int(masks[1]), "grid": ks, "objects": n,
            "selected_k": [int(ks[i]) for i in kg["select"].cpu().numpy()],
            "clock": "host wall clock around one k-grid call (thresholds by the streaming selection, "
                     "in-degrees by comparing every object with every query's bounds)"}
        log(f"C2: k-grid selection of one two-feature space in {res['k_grid_selection_one_space']['seconds']:.1f} s")
    log(f"C2: {sec:.2f} s per step, {res['value']:.3e} scores/s, join {join_ms:.0f} ms "
        f"(d15 {parts['d15']['join_ms']:.0f} ms frac {parts['d15']['frac']:.2f}, "
        f"105 x d2 {parts['d2_x105']['join_ms']:.0f} ms, {parts['d2_x105']['candidates_per_result']:.1f} cand/result)")
    del tab, ws, pop
    torch.cuda.empty_cache()
    return res


def join_source_hash() -> str:
    """sha256 over the join kernel's sources, to tie stored counter readings
    to the kernel they were taken on."""
    h = hashlib.sha256()
    for f in JOIN_SOURCES:
        with open(os.path.join(ROOT, "paper_2405_20176_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic():
    """HBM bytes per join launch from the stored rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a plain-copy calibration), or None if
    there is none or the join sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line[2:].split(": ", 1) for line in fh if line.startswith("- ") and ": " in line)
    except OSError:
        return None
    if kv.get("join_source_sha256", "").strip("` \n") != join_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"].strip("` \n"))
    except (KeyError, ValueError):
        return None


def copy_calibration(mib: int):
    """A plain device-to-device copy of known size, run under rocprofv3 --pmc
    to scale FETCH_SIZE / WRITE_SIZE readings into bytes."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 3}), flush=True)


def eps_sampler_bench(S, pop, masks, n, dev, m: int = 128):
    """The paper's eps_min / eps_max radii (selectivity 0.1 % and 15 % of the
    population, Sec. 3.5.3) of every subspace in one sampled-distance call:
    m seeded sample objects per subspace."""
    import torch
    rng = np.random.default_rng(2405)
    specs = []
    targets = [0.001 * n, 0.15 * n]
    for mk in masks:
        sample = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)
        specs.append((pop, int(mk), torch.from_numpy(sample).to(dev), targets))
    S.snaps_eps_sample(specs)                       # warm-up (and workspace)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    outs = S.snaps_eps_sample(specs)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    radii = torch.stack(outs).cpu().numpy()
    pairs = float(len(masks)) * m * (n - 1)
    log(f"eps sampler: {len(masks)} subspaces in {ms:.1f} ms")
    return {"ms": ms, "subspaces": len(masks), "sample_size": m, "targets": "0.001 n and 0.15 n neighbours",
            "sample_pairs_per_pass": pairs, "passes": 5, "pair_evals_per_s": 5 * pairs / (ms / 1000.0),
            "eps_min_median": float(np.median(radii[:, 0])), "eps_max_median": float(np.median(radii[:, 1])),
            "note": "includes the host-to-device upload of the job table"}


def eps_grid_bench(S, pop, masks, n, dev, spaces: int = 1024, g: int = 16, m: int = 128):
    """The paper's eps selection (Sec. 3.5.2-3.5.3) on an evenly spaced slice
    of the subspaces: eps_min / eps_max from the sampler (selectivity 0.1 %
    and 15 %), a grid of g evenly spaced radii, the per-radius rankings and
    the Eq. 3 choice for both DSSJ metrics, top n = 1 % of the population."""
    import torch
    idx = np.linspace(0, len(masks) - 1, min(spaces, len(masks))).astype(int)
    rng = np.random.default_rng(3576)
    specs = []
    for i in idx:
        sample = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)
        specs.append((pop, int(masks[i]), torch.from_numpy(sample).to(dev), [0.001 * n, 0.15 * n]))
    top = max(1, int(round(0.01 * n)))

    def run():
        radii = torch.stack(S.snaps_eps_sample(specs)).cpu().numpy()
        grid = [(pop, int(masks[i]), np.linspace(lo, hi, g).astype(np.float32), top)
                for i, (lo, hi) in zip(idx, radii)]
        return S.snaps_eps_grid(grid), radii

    run()                                           # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs, radii = run()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    sel = torch.stack([o["select"] for o in outs]).cpu().numpy()
    # the slice is evenly spaced over subspaces ordered by (d, mask), so its
    # mix of dimensionalities follows the full list
    full = sec * len(masks) / len(idx)
    log(f"eps-grid selection: {len(idx)} subspaces in {sec:.2f} s")
    return {"seconds": sec, "subspaces": len(idx), "grid": g, "top_n": top, "sample_size": m,
            "seconds_per_subspace": sec / len(idx), "extrapolated_all_subspaces_s": full,
            "pairs_per_subspace": float(n) * (n - 1),
            "selected_index_median": [float(np.median(sel[:, 0])), float(np.median(sel[:, 1]))],
            "clock": "host wall clock around sampler + grid calls (includes table uploads and the radii copy)"}


# The paper's k grid runs from k_min = 2 to k_max = 4096 and is sampled
# finely at small k, where the choice falls (Sec. 3.6.2).
K_GRID = [2, 3, 4, 6, 8, 11, 16, 23, 32, 45, 64, 128, 256, 512, 1024, 4096]


def k_grid_bench(S, pop, masks, n, dev, spaces: int = 1024):
    """The paper's k selection (Sec. 3.6.2) on an evenly spaced slice of the
    subspaces: in-degree and mean kNN distance at every k of K_GRID, the
    per-k rankings and the Eq. 3 choice for both KNNSJ metrics, top n = 1 %
    of the population."""
    import torch
    idx = np.linspace(0, len(masks) - 1, min(spaces, len(masks))).astype(int)
    top = max(1, int(round(0.01 * n)))
    ks = [k for k in K_GRID if k <= n - 1]
    specs = [(pop, int(masks[i]), ks, top) for i in idx]
    S.snaps_k_grid(specs[:1])                       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = S.snaps_k_grid(specs)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    sel = torch.stack([o["select"] for o in outs]).cpu().numpy()
    full = sec * len(masks) / len(idx)
    log(f"k-grid selection: {len(idx)} subspaces in {sec:.2f} s")
    return {"seconds": sec, "subspaces": len(idx), "grid": ks, "top_n": top,
            "seconds_per_subspace": sec / len(idx), "extrapolated_all_subspaces_s": full,
            "pairs_per_subspace": float(n) * (n - 1),
            "selected_k_median": [float(np.median(np.asarray(ks)[sel[:, 0]])),
                                  float(np.median(np.asarray(ks)[sel[:, 1]]))],
            "clock": "host wall clock around one k-grid call (includes the table upload)"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def per_d_breakdown(lib, S, jobs, dims, n, k, dev, stream, out_cnt, filt=0):
    """One eager index + join pass per dimensionality with its own counters
    and HIP events (after the timed steps): join time, pairs evaluated,
    candidates per result and the fraction of the fp32 peak, per d.  filt
    selects the per-pair test (0 default, 2 prefilter on the vector ALU,
    3 on the matrix cores)."""
    import torch
    sptr = ctypes.c_void_p(stream.cuda_stream)
    out = {}
    for d in sorted(set(int(v) for v in dims)):
        idx = np.nonzero(dims == d)[0]
        s0, cnt = int(idx[0]), int(idx.size)
        assert idx[-1] - s0 + 1 == cnt
        ptr = ctypes.cast(ctypes.byref(jobs, s0 * ctypes.sizeof(S.c_job)), ctypes.POINTER(S.c_job))
        st = torch.zeros(4, dtype=torch.int64, device=dev)
        t_idx, t_join = S.tuning(passes=S.PASS_INDEX), S.tuning(passes=S.PASS_JOIN, stats=st, filter=filt)
        need = lib.snaps_outlier_scores_workspace(ptr, cnt, ctypes.byref(t_join))
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        wsp = ctypes.c_void_p(ws.data_ptr())
        for t in (t_idx, t_join):      # a warm-up of both passes
            if lib.snaps_outlier_scores(ptr, cnt, ctypes.byref(t), wsp, need, sptr) != 0:
                raise RuntimeError(S.last_error())
        st.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if lib.snaps_outlier_scores(ptr, cnt, ctypes.byref(t_join), wsp, need, sptr) != 0:
            raise RuntimeError(S.last_error())
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        pairs, scanned, skipped, pd = st.cpu().numpy().astype(np.float64)
        results = float(cnt) * n * k + float(out_cnt[s0:s0 + cnt].sum(dtype=torch.int64).item())
        out[str(d)] = {"subspaces": cnt, "join_ms": ms, "pairs": pairs, "pairs_over_brute_force": pairs / (cnt * n * n),
                       "candidates_per_result": pairs / results,
                       "tiles_scanned": scanned, "tiles_skipped": skipped,
                       "tflops": 3.0 * pd / (ms / 1000.0) / 1e12, "frac": 3.0 * pd / (ms / 1000.0) / PEAK_FP32}
        del ws
    return out


class _Eager:
    """One batched pass launched by a direct snaps_outlier_scores call (same
    interface as a captured plan)."""

    def __init__(self, lib, S, c_jobs, n_jobs, tune, ws):
        self.lib, self.S, self.c_jobs, self.n_jobs, self.tune, self.ws = lib, S, c_jobs, n_jobs, tune, ws

    def launch(self, stream):
        rc = self.lib.snaps_outlier_scores(self.c_jobs, self.n_jobs, ctypes.byref(self.tune),
                                           ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                           ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"batched call failed ({rc}): {self.S.last_error()}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chunk", type=int, default=0, help="subspaces per batched plan (0: all in one)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="measured serving run length after a 10 s warm-up (0: skip serving)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-subspace pass")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--spaces", type=int, default=0, help="debug: use only the first N subspaces")
    ap.add_argument("--eager", action="store_true", help="launch the batched passes directly, without HIP graphs")
    ap.add_argument("--no-eps-sampler", dest="eps_sampler", action="store_false",
                    help="skip timing the sampled eps_min / eps_max radii of every subspace")
    ap.add_argument("--no-eps-grid", dest="eps_grid", action="store_false",
                    help="skip timing the eps-grid selection on a slice of the subspaces")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="use the library's fixed per-d defaults instead of the measured per-class walk")
    ap.add_argument("--autotune-sample", type=int, default=64, help="jobs timed per class by the autotuner")
    ap.add_argument("--autotune-cache", default="", metavar="FILE",
                    help="take the autotuner's table for this device from FILE if it holds one, else measure "
                         "and store it there (profiling runs use it to keep the tuning launches out)")
    ap.add_argument("--no-k-grid", dest="k_grid", action="store_false",
                    help="skip timing the k-grid selection on a slice of the subspaces")
    ap.add_argument("--grid-spaces", type=int, default=1024,
                    help="subspaces in the eps-grid and k-grid slices")
    ap.add_argument("--no-per-d", dest="per_d", action="store_false",
                    help="skip the per-dimensionality join breakdown (one eager pass per d after the timed steps)")
    ap.add_argument("--filter-ab", action="store_true",
                    help="after the per-d breakdown, time each d's join with the prefilter on the vector ALU and on the matrix cores")
    ap.add_argument("--alert-ab", action="store_true",
                    help="time both alert kernels per d and request size on one serving population (alert_ab)")
    ap.add_argument("--no-c2", dest="c2", action="store_false",
                    help="skip the LSST-scale population (5,000,000 objects, the full space + 105 two-feature spaces)")
    ap.add_argument("--c2-steps", type=int, default=1, help="timed steps of the LSST-scale population")
    ap.add_argument("--lsst-k-grid", action="store_true",
                    help="also time the k-grid selection (k = 2..256) of one two-feature space at 5,000,000 objects")
    ap.add_argument("--no-c3", dest="c3", action="store_false",
                    help="skip the batched-uneven workload (4,096 jobs of their own populations)")
    ap.add_argument("--c3-steps", type=int, default=2, help="timed steps of the batched-uneven workload")
    ap.add_argument("--c3-autotune-sample", type=int, default=2,
                    help="jobs timed per (d, log2 n) class by the autotuner on the batched-uneven workload (0: off)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain MIB-MiB device copy (counter calibration) and exit")
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: the path is measured on one GPU only (no multi-GPU form is built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return

    import torch
    from paper_2405_20176_amd import snaps as S
    import snaps_synth as G

    lib = S.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    sptr = ctypes.c_void_p(stream.cuda_stream)

    x, masks, k = G.gen_c1()
    eps_tab = G.load_c1_eps()
    if a.spaces:
        masks, eps_tab = masks[:a.spaces], eps_tab[:a.spaces]
    n = x.shape[0]
    n_sp = len(masks)
    dims = np.array([bin(int(m)).count("1") for m in masks])
    pop = S.Population.from_rows(x, device=dev)
    log(f"population {n} x 15, {n_sp} subspaces, k={k}")

    # Resident outputs of every subspace.
    out_cnt = torch.empty((n_sp, n), dtype=torch.int32, device=dev)
    out_mean = torch.empty((n_sp, n), dtype=torch.float32, device=dev)
    out_deg = torch.empty((n_sp, n), dtype=torch.int32, device=dev)
    out_kmean = torch.empty((n_sp, n), dtype=torch.float32, device=dev)
    out_rank = torch.empty((n_sp, 4, n), dtype=torch.int32, device=dev)
    out_ens = torch.empty((n_sp, n), dtype=torch.float32, device=dev)

    jobs = (S.c_job * n_sp)()
    pp = ctypes.pointer(pop.c)
    for i in range(n_sp):
        j = jobs[i]
        j.pop = pp
        j.mask = int(masks[i])
        j.k = k
        j.eps = float(eps_tab[i])
        j.out = S.c_scores(out_cnt[i].data_ptr(), out_mean[i].data_ptr(), out_deg[i].data_ptr(),
                           out_kmean[i].data_ptr())
        j.rank = out_rank[i].data_ptr()
        j.ensemble = out_ens[i].data_ptr()
    # Per-class choice of the candidate walk (box pruning and its indexed
    # dimensions, or brute force), measured on a sample of each class's jobs
    # before anything is timed.
    tuned = None
    if a.autotune:
        from types import SimpleNamespace
        from paper_2405_20176_amd import autotune as AT
        t_at = time.perf_counter()
        specs = [SimpleNamespace(pop=pop, mask=int(masks[i]), k=k, eps=float(eps_tab[i]), mode=0, index_dims=0,
                                 tile_shape=0)
                 for i in range(n_sp)]
        devname = AT.device_key(dev)
        table = AT.load(a.autotune_cache, devname) if a.autotune_cache else None
        source = "cache" if table else "measured"
        if not table:
            table = AT.tune(specs, sample=a.autotune_sample)
            if a.autotune_cache:
                AT.save(a.autotune_cache, devname, table)
        AT.apply(specs, table)
        for i in range(n_sp):
            jobs[i].mode, jobs[i].index_dims = specs[i].mode, specs[i].index_dims
            jobs[i].tile_shape = getattr(specs[i], "tile_shape", 0)
        tuned = {"seconds": time.perf_counter() - t_at, "source": source, "sample_per_class": a.autotune_sample,
                 "choice": {key: [v["mode"], v["index_dims"], v.get("tile_shape", 1)] for key, v in table.items()},
                 "note": "[mode, index_dims, tile_shape]: mode 1 = every candidate tile, 2 = box pruning on "
                         "index_dims indexed dimensions; tile_shape 1 = 64-candidate tiles, 2 = 32-candidate "
                         "halves culled by their own boxes; "
                         "measured per (d, log2 n) class on sampled jobs, outside the timed region"}
        log(f"autotune: {len(table)} classes in {tuned['seconds']:.1f} s: "
            + ", ".join(f"{key}={v['mode']}/{v['index_dims']}/{v.get('tile_shape', 1)}" for key, v in table.items()))
    chunk = a.chunk if a.chunk > 0 else n_sp
    chunks = [(s, min(n_sp, s + chunk)) for s in range(0, n_sp, chunk)]
    job_ptr = lambda s: ctypes.cast(ctypes.byref(jobs, s * ctypes.sizeof(S.c_job)), ctypes.POINTER(S.c_job))
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    tunes = {p: S.tuning(passes=p, stats=stats if p == S.PASS_JOIN else None)
             for p in (S.PASS_INDEX, S.PASS_JOIN, S.PASS_RANK)}
    t_plan = time.perf_counter()
    plans = []
    for s0, e0 in chunks:
        need = lib.snaps_outlier_scores_workspace(job_ptr(s0), e0 - s0, ctypes.byref(tunes[S.PASS_JOIN]))
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        if a.eager:
            trio = [_Eager(lib, S, job_ptr(s0), e0 - s0, tunes[p], ws) for p in (S.PASS_INDEX, S.PASS_JOIN, S.PASS_RANK)]
        else:
            trio = [S.Plan(None, tunes[p], ws=ws, c_jobs=job_ptr(s0), n_jobs=e0 - s0)
                    for p in (S.PASS_INDEX, S.PASS_JOIN, S.PASS_RANK)]
        plans.append((ws, trio))
    ws_total = sum(w.numel() for w, _ in plans)
    log(f"{len(chunks)} plan(s) of 3 {'eager passes' if a.eager else 'graphs'} built in {time.perf_counter() - t_plan:.1f} s, workspace "
        f"{ws_total / 2**30:.2f} GiB, outputs {n_sp * n * 36 / 2**30:.1f} GiB")

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def step(marks=None):
        """One step; with marks, events around each pass of each plan
        (start, after index, after join, after rank)."""
        for _, (p_index, p_join, p_rank) in plans:
            m = [ev()] if marks is not None else None
            p_index.launch(stream)
            if m is not None:
                m.append(ev())
            p_join.launch(stream)
            if m is not None:
                m.append(ev())
            p_rank.launch(stream)
            if m is not None:
                m.append(ev())
                marks.append(m)

    for w in range(a.warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup {w}: {time.perf_counter() - t:.2f} s")

    stats.zero_()
    marks = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(marks)
        log(f"step {i} enqueued")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1000.0 / a.steps
    value = n * n_sp / (ms_per_step / 1000.0)
    per_plan = len(plans)
    step_ms = [sum(marks[i * per_plan + j][0].elapsed_time(marks[i * per_plan + j][3]) for j in range(per_plan))
               for i in range(a.steps)]
    index_ms = sum(m[0].elapsed_time(m[1]) for m in marks)
    join_ms = sum(m[1].elapsed_time(m[2]) for m in marks)
    rank_ms = sum(m[2].elapsed_time(m[3]) for m in marks)
    results_per_step = float(n_sp) * n * k + float(out_cnt.sum(dtype=torch.int64).item())
    st = stats.cpu().numpy().astype(np.float64)
    pairs, scanned, skipped, pair_dims = st
    brute_pairs = a.steps * float(n) * n * n_sp
    join_launches = a.steps * sum(len(set(dims[s:e])) for s, e in chunks)
    avg_launch_s = join_ms / 1000.0 / join_launches
    flops_per_launch = 3.0 * pair_dims / join_launches
    achieved = flops_per_launch / avg_launch_s
    log(f"timed: {ms_per_step:.1f} ms/step, join {join_ms / a.steps:.1f} ms/step, "
        f"{value:.3e} obj-space/s, join {achieved / 1e12:.1f} TFLOP/s")

    result = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded SNAPShot1-shaped generator; the catalogue itself is not available)",
        "config": {"workload": "SNAPShot1-shaped full run: N=31,693 objects x 15 features, all 32,752 subspaces "
                               "(d=2..15), k=10, per-subspace eps for mean neighbour count 10, batched form "
                               "(one job table, " + ("passes launched directly)" if a.eager else
                                                     "passes replayed as HIP graphs)"),
                   "n_objects": n, "n_subspaces": n_sp, "k": k, "subspaces_per_plan": chunk},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": stored_traffic(),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "k_join_mfma (fused kNN + eps join, prefilter on fp16 MFMA over split fp32 coordinates), all instantiations",
                     "flops_per_pair": "3d", "avg_launch_ms": avg_launch_s * 1000.0, "launches": join_launches},
        "step_ms": {"median": float(np.median(step_ms)), "min": float(min(step_ms)), "max": float(max(step_ms)),
                    "each": step_ms, "clock": "HIP events on the library stream around each whole step"},
        "passes_ms_per_step": {"index": index_ms / a.steps, "join": join_ms / a.steps, "rank": rank_ms / a.steps},
        "join": {"ms_per_step": join_ms / a.steps, "pairs_evaluated_per_step": pairs / a.steps,
                 "brute_force_pairs_per_step": brute_pairs / a.steps,
                 "results_per_step": results_per_step,
                 "candidates_per_result": pairs / a.steps / results_per_step,
                 "tiles_scanned": scanned / a.steps, "tiles_skipped": skipped / a.steps,
                 "evals_per_s": pairs / (join_ms / 1000.0)},
        "autotune": tuned,
    }

    if a.per_d:
        del plans
        torch.cuda.empty_cache()
        plans = None
        result["join_per_d"] = per_d_breakdown(lib, S, jobs, dims, n, k, dev, stream, out_cnt)
        log("per d: " + ", ".join(f"d={d} {v['join_ms']:.0f} ms frac {v['frac']:.2f} pairs/bf {v['pairs_over_brute_force']:.2f}"
                                  for d, v in result["join_per_d"].items()))
        if a.filter_ab:
            # the same passes with the prefilter on the vector ALU, then on the
            # matrix cores (identical results; the kernels differ)
            ab = {f: per_d_breakdown(lib, S, jobs, dims, n, k, dev, stream, out_cnt, filt=f) for f in (2, 3)}
            result["filter_ab_per_d"] = {
                d: {"valu_prefilter_ms": ab[2][d]["join_ms"], "mfma_ms": ab[3][d]["join_ms"],
                    "mfma_speedup": ab[2][d]["join_ms"] / ab[3][d]["join_ms"]} for d in ab[3]}
            log("filter A/B (vector-ALU prefilter / matrix cores): " + ", ".join(
                f"d={d} {v['valu_prefilter_ms']:.0f}/{v['mfma_ms']:.0f} ms" for d, v in result["filter_ab_per_d"].items()))

    if not a.no_plain:
        tune = S.tuning()
        per_ws = max(lib.snaps_outlier_scores_workspace(job_ptr(i), 1, ctypes.byref(tune)) for i in (0, n_sp - 1))
        pws = torch.empty(per_ws, dtype=torch.uint8, device=dev)
        lat = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n_sp):
            rc = lib.snaps_outlier_scores(job_ptr(i), 1, ctypes.byref(tune), ctypes.c_void_p(pws.data_ptr()),
                                          per_ws, sptr)
            if rc != 0:
                raise RuntimeError(f"plain call failed ({rc}): {S.last_error()}")
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - t0
        result["plain"] = {"value": n * n_sp / plain_s, "unit": UNIT, "ms_per_pass": plain_s * 1000.0,
                           "form": "one library call per subspace, one stream", "passes": 1}
        result["batched_over_plain"] = value / result["plain"]["value"]
        log(f"plain: {plain_s:.2f} s per pass")

    if a.eps_sampler:
        result["eps_sampler"] = eps_sampler_bench(S, pop, masks, n, dev)
    if a.eps_grid:
        result["eps_grid_selection"] = eps_grid_bench(S, pop, masks, n, dev, spaces=a.grid_spaces)
    if a.k_grid:
        result["k_grid_selection"] = k_grid_bench(S, pop, masks, n, dev, spaces=a.grid_spaces)

    if a.c3 or a.c2 or a.serve_seconds > 0 or a.alert_ab:
        del plans, out_cnt, out_mean, out_deg, out_kmean, out_rank, out_ens
        torch.cuda.empty_cache()
    if a.c3:
        result["c3"] = c3_bench(S, G, lib, dev, stream, a.c3_steps, 1, a.c3_autotune_sample, not a.no_plain)
    if a.c2:
        result["c2"] = c2_bench(S, G, dev, stream, a.c2_steps, a.lsst_k_grid)
    if a.serve_seconds > 0:
        result["serving"] = serve_bench(S, G, dev, a.serve_seconds)
    if a.alert_ab:
        result["alert_ab"] = alert_ab_bench(S, G, dev)

    if not a.no_cpu:
        cb = cpu_baseline(x, masks if not a.spaces else G.all_masks(), G.load_c1_eps(), k)
        result["cpu_baseline"] = cb

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
