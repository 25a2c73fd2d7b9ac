"""Measured choice of the join's candidate walk and tile shape per class of jobs.

For a job the library can either walk the candidate tiles of its grid index
and skip those whose bounding box is provably out of reach (the grid search
of Sec. 3.8.1, over c indexed dimensions, the paper's c = min(d, 6)), or
scan every tile (brute force, which the paper notes wins once the index stops
pruning at high d).  Which is faster, and with which c, depends on d, on the
population size and on the data, so it is measured: for each class of jobs
(d, floor(log2 n)) in a job list, a sample of its jobs runs the index and join
passes under every candidate setting, and the fastest setting is kept.  With
pruning, the tile shape is measured too: the lean walk over 64-query x
64-candidate tile pairs culled by the candidate tile's box (shape 1), the
walk that first culls runs of 64 tiles by their box (shape 3, for large
populations), or that walk with each candidate tile taken as two 32-object
halves culled by boxes of their own (shape 2: twice the box tests, fewer
pairs; the finer cut pays where the boxes are small against the reach).  The
choices go into the jobs' per-job ``mode`` / ``index_dims`` / ``tile_shape``
and can be cached per device (architecture and compute units) in a JSON file.
Every setting gives the same results (the pruning is exact); only the time
differs.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import torch

from . import snaps as S

MODE_BRUTE, MODE_PRUNE = 1, 2
TILE_FULL, TILE_HALVES, TILE_SUPER = 1, 2, 3
MAX_INDEX_DIMS = 6


def job_class(job: S.Job) -> Tuple[int, int]:
    """(d, floor(log2 n)) of a job."""
    return bin(int(job.mask)).count("1"), int(math.log2(max(2, job.pop.n)))


def class_key(cls: Tuple[int, int]) -> str:
    return f"d{cls[0]}_n2^{cls[1]}"


def candidates(d: int) -> List[Tuple[int, int]]:
    """(mode, index_dims) settings tried for dimensionality d."""
    return [(MODE_BRUTE, 0)] + [(MODE_PRUNE, c) for c in range(2, min(d, MAX_INDEX_DIMS) + 1)]


def _time_setting(jobs: Sequence[S.Job], mode: int, c: int, tune, reps: int, shape: int = TILE_FULL) -> float:
    for j in jobs:
        j.mode, j.index_dims, j.tile_shape = mode, c, shape
    ws = torch.empty(S.snaps_outlier_scores_workspace(jobs, tune), dtype=torch.uint8, device=jobs[0].pop.cols.device)
    S.snaps_outlier_scores(jobs, tune, ws=ws)                  # warm-up
    best = math.inf
    stream = torch.cuda.current_stream()
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        S.snaps_outlier_scores(jobs, tune, ws=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(jobs: Sequence[S.Job], sample: int = 64, reps: int = 3, base=None) -> Dict[str, dict]:
    """Measure every candidate setting on up to ``sample`` jobs of each class
    of ``jobs`` (evenly spread over the class, fresh outputs so the jobs'
    own are untouched).  ``base`` is the call-level tuning of the timed calls
    (default: one wavefront per query tile, as in a large batched call).
    Returns {class key: {"mode", "index_dims", "tile_shape", "ms": {setting: ms}}};
    a setting is "mode,index_dims" with the lean walk (shape 1), and the
    best pruning setting is also timed with shapes 2 ("mode,index_dims,h")
    and 3 ("mode,index_dims,s")."""
    if base is None:
        base = S.tuning(split=1, passes=S.PASS_INDEX | S.PASS_JOIN)
    by_class: Dict[Tuple[int, int], List[S.Job]] = {}
    for j in jobs:
        by_class.setdefault(job_class(j), []).append(j)
    table: Dict[str, dict] = {}
    for cls, members in sorted(by_class.items()):
        step = max(1, len(members) // sample)
        pick = members[::step][:sample]
        probe = [S.Job.alloc(j.pop, j.mask, j.k, j.eps, with_rank=False) for j in pick]
        ms = {f"{m},{c}": _time_setting(probe, m, c, base, reps) for m, c in candidates(cls[0])}
        best = min(ms, key=ms.get)
        m, c = (int(v) for v in best.split(","))
        shape = TILE_FULL
        if m == MODE_PRUNE:
            for sh, tag in ((TILE_HALVES, "h"), (TILE_SUPER, "s")):
                ms[f"{m},{c},{tag}"] = _time_setting(probe, m, c, base, reps, sh)
                if ms[f"{m},{c},{tag}"] < ms[best]:
                    best, shape = f"{m},{c},{tag}", sh
        table[class_key(cls)] = {"mode": m, "index_dims": c, "tile_shape": shape, "ms": ms,
                                 "jobs_timed": len(probe)}
    return table


def apply(jobs: Iterable[S.Job], table: Dict[str, dict]) -> int:
    """Set each job's mode / index_dims from the table (jobs of classes
    missing from it keep theirs); returns the number of jobs set."""
    done = 0
    for j in jobs:
        entry = table.get(class_key(job_class(j)))
        if entry is None:
            continue
        j.mode, j.index_dims = int(entry["mode"]), int(entry["index_dims"])
        j.tile_shape = int(entry.get("tile_shape", 0))
        done += 1
    return done


def device_key(device=None) -> str:
    """Cache key of a device: its architecture and compute-unit count (the
    marketing name is not always available)."""
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "") or props.name
    return f"{arch} {props.multi_processor_count}cu"


def load(path: str, device: str) -> Optional[Dict[str, dict]]:
    """The cached table of a device, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh).get(device)


def save(path: str, device: str, table: Dict[str, dict]) -> None:
    """Store a device's table (other devices' entries are kept)."""
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data[device] = table
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
