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
PEAK_FP32_MFMA = 157.3e12        # MI355X published dense FP32 matrix peak, flop/s
PEAK_HBM = 8.0e12                # MI355X HBM3E, byte/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_join_c1_all_subspaces_hbm_traffic.md")
JOIN_SOURCES = ["join_kernel.cuh", "join_mfma.cuh", "join.hip", "join_inst0.hip", "join_inst1.hip",
                "join_inst2.hip", "join_inst3.hip", "join_mfma0.hip", "join_mfma1.hip", "common.cuh",
                "snaps_internal.h"]


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


def serve_bench(S, G, dev, seconds: float, spaces_per_pop: int = 4, n_streams: int = 4):
    """Served form: 4 resident populations of 1,000,000 objects (the serving
    generator), the first `spaces_per_pop` subspaces of each population's
    seeded catalogue resident as scoring states, and an open-loop Poisson
    stream (200 requests/s, 1..10,000 alerts per request, log-uniform) replayed
    in real time through the continuous-batching server.  Requests naming a
    non-resident catalogue entry are mapped onto the resident ones."""
    import torch
    from paper_2405_20176_amd.serve import Admission, Batcher, GpuExecutor, Request
    w = G.gen_c4()
    masks_tab, eps_tab = G.load_c4_eps()
    t0 = time.perf_counter()
    pops, bounds, states = [], [], {}
    build_s = []
    for p in range(w.n_pop):
        x, lo, hi = w.population(p)
        pop = S.Population.from_rows(x, device=dev)
        del x
        pops.append(pop)
        bounds.append((lo, hi))
        for si in range(spaces_per_pop):
            m = int(masks_tab[p, si])
            assert m == int(w.spaces[p][si])
            tb = time.perf_counter()
            states[(p, m)] = S.ServeState(pop, m, w.k, float(eps_tab[p, si]))
            torch.cuda.synchronize()
            build_s.append(time.perf_counter() - tb)
    log(f"serving: {len(states)} states built in {time.perf_counter() - t0:.1f} s "
        f"(cold build per state {np.median(build_s):.2f} s median)")
    reqs = []
    for r in w.requests(seconds):
        p = r.pop
        m = int(masks_tab[p, r.space % spaces_per_pop])
        cols = G.mask_features(m)
        lo, hi = bounds[p]
        al = np.ascontiguousarray(w.alerts(r, lo, hi)[:, cols], dtype=np.float32)
        reqs.append(Request(r.rid, r.arrival_s, (p, m), al))
    n_alerts = sum(q.m for q in reqs)
    log(f"serving: {len(reqs)} requests, {n_alerts} alerts over {seconds:.0f} s of arrivals")
    ex = GpuExecutor(states, n_streams=n_streams, device=dev)
    # warm-up: one request per state, not timed
    warm = Batcher(ex, Admission(8 << 30, n_streams))
    for i, key in enumerate(states):
        warm.submit(Request(-1 - i, 0.0, key, np.zeros((64, bin(key[1]).count("1")), np.float32)))
    warm.drain()
    b = Batcher(ex, Admission(8 << 30, n_streams), max_batch_alerts=1 << 16)
    t_start = time.perf_counter()
    b.run_open_loop(reqs)
    t_end = time.perf_counter()
    lat = b.latencies()
    done = [r for r in b.finished if r.status == "done"]
    span = max(r.done for r in done) - min(r.arrival for r in done)
    res = {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "mean_ms": float(lat.mean() * 1e3), "requests": len(done), "rejected": len(b.finished) - len(done),
           "alerts": int(sum(r.m for r in done)), "alert_scores_per_s": float(sum(r.m for r in done) / span),
           "wall_s": t_end - t_start, "arrival_rate_hz": w.rate_hz, "populations": w.n_pop, "population_n": w.pop_n,
           "resident_states": len(states), "state_build_s_median": float(np.median(build_s)), "k": w.k,
           "form": "continuous batching over 4 streams, admission by an 8 GiB in-flight budget"}
    log(f"serving: p50 {res['p50_ms']:.1f} ms, p99 {res['p99_ms']:.1f} ms, "
        f"{res['alert_scores_per_s']:.3e} alert scores/s")
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
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="serving run length (0: skip)")
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
        specs = [SimpleNamespace(pop=pop, mask=int(masks[i]), k=k, eps=float(eps_tab[i]), mode=0, index_dims=0)
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
        tuned = {"seconds": time.perf_counter() - t_at, "source": source, "sample_per_class": a.autotune_sample,
                 "choice": {key: [v["mode"], v["index_dims"]] for key, v in table.items()},
                 "note": "mode 1 = every candidate tile, 2 = box pruning on index_dims indexed dimensions; "
                         "measured per (d, log2 n) class on sampled jobs, outside the timed region"}
        log(f"autotune: {len(table)} classes in {tuned['seconds']:.1f} s: "
            + ", ".join(f"{key}={v['mode']}/{v['index_dims']}" for key, v in table.items()))
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
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA, "traffic": stored_traffic(),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "k_join_mfma (fused kNN + eps join, prefilter on fp32 MFMA), all instantiations",
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

    if a.serve_seconds > 0:
        del plans
        torch.cuda.empty_cache()
        result["serving"] = serve_bench(S, G, dev, a.serve_seconds)

    if not a.no_cpu:
        cb = cpu_baseline(x, masks if not a.spaces else G.all_masks(), G.load_c1_eps(), k)
        result["cpu_baseline"] = cb

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
