"""Write the stored per-space epsilon tables of the synthetic workloads.

Each epsilon is chosen by the CPU oracle's sampled-distance rule
(``oracle.eps_sampled_mean_count``: m seeded sample objects, their float64
distances to every other object, the radius at which the sample's mean
neighbour count reaches the target), rounded to float32, and stored so that
the oracle and the GPU library receive the identical value.  This script
calls only the oracle and the generators.

    python -m snaps_synth.make_eps_tables c1      # 32,752 spaces, target 10
    python -m snaps_synth.make_eps_tables c2      # LSST-scale: full space + 105 two-feature spaces, target 20
    python -m snaps_synth.make_eps_tables c3      # 4,096 batched uneven jobs, target k
    python -m snaps_synth.make_eps_tables c4      # served spaces of the serving workload
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O                      # noqa: E402
from snaps_synth import generators as G  # noqa: E402

C1_SAMPLES = 128
C1_TARGET = 10

_X = None


def _init(x):
    global _X
    _X = x


def _c1_one(args):
    idx, mask = args
    xs = O.project(_X, int(mask))
    return idx, O.eps_sampled_mean_count(xs, C1_TARGET, C1_SAMPLES, seed=int(mask))


def c1(workers: int) -> str:
    x, masks, _ = G.gen_c1()
    eps = np.zeros(len(masks), dtype=np.float32)
    t0 = time.time()
    with Pool(workers, initializer=_init, initargs=(x,)) as pool:
        for i, (idx, e) in enumerate(pool.imap_unordered(_c1_one, list(enumerate(masks)), chunksize=64)):
            eps[idx] = e
            if i % 2048 == 0:
                print(f"{i}/{len(masks)} spaces, {time.time() - t0:.0f} s", flush=True)
    os.makedirs(G.TABLE_DIR, exist_ok=True)
    out = os.path.join(G.TABLE_DIR, "c1_eps.npz")
    np.savez(out, masks=masks, eps=eps, samples=np.int64(C1_SAMPLES), target=np.int64(C1_TARGET))
    return out


C4_SAMPLES = 32
C4_TARGET = 10
C4_SPACES = 64         # served subspaces of each population (its whole catalogue)


C2_SAMPLES = 64
C2_TARGET = 20


def _c2_one(mask):
    return int(mask), O.eps_sampled_mean_count(O.project(_X, int(mask)), C2_TARGET, C2_SAMPLES, seed=int(mask))


def c2(workers: int) -> str:
    x, masks, _, target = G.gen_c2()
    assert target == C2_TARGET
    t0 = time.time()
    with Pool(workers, initializer=_init, initargs=(x,)) as pool:
        got = dict(pool.map(_c2_one, [int(m) for m in masks]))
    eps = np.array([got[int(m)] for m in masks], dtype=np.float32)
    print(f"{len(masks)} spaces in {time.time() - t0:.0f} s, eps median {np.median(eps):.6g}", flush=True)
    out = os.path.join(G.TABLE_DIR, "c2_eps.npz")
    np.savez(out, masks=masks, eps=eps, samples=np.int64(C2_SAMPLES), target=np.int64(C2_TARGET))
    return out


C3_SAMPLES = 32


def _c3_one(j):
    x = G.gen_c3_projected(j)
    return j.index, O.eps_sampled_mean_count(x, j.k, C3_SAMPLES, seed=j.index)


def c3(workers: int) -> str:
    jobs = G.gen_c3_jobs()
    eps = np.zeros(len(jobs), dtype=np.float32)
    t0 = time.time()
    with Pool(workers) as pool:
        for i, (idx, e) in enumerate(pool.imap_unordered(_c3_one, jobs, chunksize=8)):
            eps[idx] = e
            if i % 512 == 0:
                print(f"{i}/{len(jobs)} jobs, {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(G.TABLE_DIR, "c3_eps.npz")
    np.savez(out, masks=np.array([j.mask for j in jobs], dtype=np.uint32), n=np.array([j.n for j in jobs]),
             k=np.array([j.k for j in jobs]), eps=eps, samples=np.int64(C3_SAMPLES))
    return out


def _c4_one(mask):
    return int(mask), O.eps_sampled_mean_count(O.project(_X, int(mask)), C4_TARGET, C4_SAMPLES, seed=int(mask))


def c4(workers: int) -> str:
    w = G.gen_c4()
    eps = np.zeros((w.n_pop, C4_SPACES), dtype=np.float32)
    masks = np.zeros((w.n_pop, C4_SPACES), dtype=np.uint32)
    t0 = time.time()
    for p in range(w.n_pop):
        x, _, _ = w.population(p)
        masks[p] = w.spaces[p][:C4_SPACES]
        with Pool(workers, initializer=_init, initargs=(x,)) as pool:
            got = dict(pool.map(_c4_one, [int(m) for m in masks[p]]))
        eps[p] = [got[int(m)] for m in masks[p]]
        print(f"population {p}: {C4_SPACES} spaces, eps median {np.median(eps[p]):.6g} ({time.time() - t0:.0f} s)",
              flush=True)
        del x
    out = os.path.join(G.TABLE_DIR, "c4_eps.npz")
    np.savez(out, masks=masks, eps=eps, samples=np.int64(C4_SAMPLES), target=np.int64(C4_TARGET))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 4)
    a = ap.parse_args()
    print({"c1": c1, "c2": c2, "c3": c3, "c4": c4}[a.which](a.workers))


if __name__ == "__main__":
    main()
