"""Benchmark: SNAPS outlier scores over every subspace of a SNAPShot1-shaped
population on one MI355X.

Workload (one step): N = 31,693 objects x 15 float32 features (seeded
synthetic stand-in for the SNAPShot1 catalogue), all 32,752 subspaces of 2..15
features, k = 10, eps per subspace from the stored table (mean neighbour count
10).  A step runs the whole hot path for every subspace: index build, fused
kNN + eps join with the four metrics, dense ranks.  Outputs of all subspaces
stay resident in HBM (33 GB).  The timed steps use the batched form (thousands
of subspaces per library call); a plain pass (one library call per subspace)
is timed once afterwards for comparison.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import ctypes
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
PEAK_FP32_VECTOR = 157.3e12      # MI355X published FP32 vector peak, flop/s
PEAK_HBM = 8.0e12                # MI355X HBM3E, byte/s


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


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chunk", type=int, default=4096, help="subspaces per library call in the batched form")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-subspace pass")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--spaces", type=int, default=0, help="debug: use only the first N subspaces")
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only (each GPU box has one); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

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
    chunks = [(s, min(n_sp, s + a.chunk)) for s in range(0, n_sp, a.chunk)]
    job_ptr = lambda s: ctypes.cast(ctypes.byref(jobs, s * ctypes.sizeof(S.c_job)), ctypes.POINTER(S.c_job))
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    tunes = {p: S.tuning(passes=p, stats=stats if p == S.PASS_JOIN else None)
             for p in (S.PASS_INDEX, S.PASS_JOIN, S.PASS_RANK)}
    ws_bytes = max(lib.snaps_outlier_scores_workspace(job_ptr(s), e - s, ctypes.byref(tunes[S.PASS_JOIN]))
                   for s, e in chunks)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    log(f"{len(chunks)} chunks, workspace {ws_bytes / 2**30:.2f} GiB, outputs {n_sp * n * 32 / 2**30:.1f} GiB")

    def call(s, e, tune):
        rc = lib.snaps_outlier_scores(job_ptr(s), e - s, ctypes.byref(tune), ctypes.c_void_p(ws.data_ptr()),
                                      ws_bytes, sptr)
        if rc != 0:
            raise RuntimeError(f"snaps_outlier_scores failed ({rc}): {S.last_error()}")

    def step(events=None):
        for s, e in chunks:
            call(s, e, tunes[S.PASS_INDEX])
            if events is not None:
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record(stream)
            call(s, e, tunes[S.PASS_JOIN])
            if events is not None:
                ev1.record(stream)
                events.append((ev0, ev1))
            call(s, e, tunes[S.PASS_RANK])

    for w in range(a.warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup {w}: {time.perf_counter() - t:.2f} s")

    stats.zero_()
    events = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(events)
        log(f"step {i} enqueued")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1000.0 / a.steps
    value = n * n_sp / (ms_per_step / 1000.0)
    join_ms = sum(e0.elapsed_time(e1) for e0, e1 in events)
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
                               "(d=2..15), k=10, per-subspace eps for mean neighbour count 10, batched form",
                   "n_objects": n, "n_subspaces": n_sp, "k": k, "subspaces_per_call": a.chunk},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": None,
                     "kernel": "k_join (fused kNN + eps join), all instantiations",
                     "flops_per_pair": "3d", "avg_launch_ms": avg_launch_s * 1000.0, "launches": join_launches},
        "join": {"ms_per_step": join_ms / a.steps, "pairs_evaluated_per_step": pairs / a.steps,
                 "brute_force_pairs_per_step": brute_pairs / a.steps,
                 "tiles_scanned": scanned / a.steps, "tiles_skipped": skipped / a.steps,
                 "evals_per_s": pairs / (join_ms / 1000.0)},
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

    if not a.no_cpu:
        cb = cpu_baseline(x, masks if not a.spaces else G.all_masks(), G.load_c1_eps(), k)
        result["cpu_baseline"] = cb

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
