"""ctypes front of the C twin of the oracle (``oracle/c/snaps_oracle.c``).

TEST INFRASTRUCTURE: used by tests and by the benchmark's CPU baseline only.
The C twin computes the same float64 join results as
:mod:`oracle.snaps_oracle` with OpenMP over queries; metrics and ranks are
then derived with the NumPy oracle's own functions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import snaps_oracle as O

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "c", "snaps_oracle.c")
_LIB = os.path.join(_HERE, "c", "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C twin with gcc (-O2, OpenMP, no FMA contraction so the
    float64 sums match the NumPy oracle exactly)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_join.restype = ctypes.c_int
        lib.oracle_join.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
            ctypes.c_void_p, ctypes.c_int32]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def join(X, k: int, eps: float, queries=None, nthreads: int = 0, band=None, qids=None):
    """Raw join results for a projected population ``X`` [n, d] (float32
    values).  Returns dict(knn_ids, knn_dist, knn_next, eps_count, eps_sum)
    and, when ``band=(lo, hi)`` is given, ``band``: the number of other
    objects at a distance in [lo, hi].  ``qids`` restricts the self-join to
    those object ids (rows of the result follow ``qids``)."""
    lib = _load()
    x = np.ascontiguousarray(X, dtype=np.float32)
    n, d = x.shape
    qid_arr = None
    if queries is None:
        qp, m = None, n
        q = None
        if qids is not None:
            qid_arr = np.ascontiguousarray(qids, dtype=np.int64)
            m = qid_arr.size
    else:
        q = np.ascontiguousarray(queries, dtype=np.float32)
        m = q.shape[0]
        qp = q.ctypes.data
    kk = max(k, 1)
    ids = np.zeros((m, kk), dtype=np.int32)
    dist = np.zeros((m, kk), dtype=np.float64)
    nxt = np.zeros(m, dtype=np.float64)
    cnt = np.zeros(m, dtype=np.int32)
    ssum = np.zeros(m, dtype=np.float64)
    bnd = np.zeros(m, dtype=np.int32)
    blo, bhi = (band if band is not None else (1.0, -1.0))
    rc = lib.oracle_join(x.ctypes.data, n, d, qp, m, k, float(eps), ids.ctypes.data,
                         dist.ctypes.data, nxt.ctypes.data, cnt.ctypes.data, ssum.ctypes.data,
                         bnd.ctypes.data if band is not None else None, float(blo), float(bhi),
                         qid_arr.ctypes.data if qid_arr is not None else None, int(nthreads))
    if rc != 0:
        raise ValueError("oracle_join rejected its arguments")
    out = dict(knn_ids=ids[:, :k].astype(np.int64), knn_dist=dist[:, :k], knn_next=nxt,
               eps_count=cnt.astype(np.int64), eps_sum=ssum)
    if band is not None:
        out["band"] = bnd.astype(np.int64)
    return out


def outlier_scores(X, k: int, eps: float, nthreads: int = 0, band=None) -> dict:
    """Same result as :func:`oracle.snaps_oracle.outlier_scores`, with the
    O(n^2) scan done by the C twin (plus ``band`` counts when asked)."""
    r = join(X, k, eps, nthreads=nthreads, band=band)
    n = r["eps_count"].shape[0]
    cnt = r["eps_count"]
    mean = np.where(cnt > 0, r["eps_sum"] / np.maximum(cnt, 1), 0.0)
    deg = O.indegree(r["knn_ids"], n)
    kmean = r["knn_dist"].sum(axis=1) / k
    ranks = O.rank_metrics(cnt, mean, deg, kmean)
    out = dict(knn_ids=r["knn_ids"], knn_dist=r["knn_dist"], knn_next=r["knn_next"],
               eps_count=cnt, eps_mean=mean, indeg=deg, knn_mean=kmean, rank=ranks, ensemble=O.ensemble(ranks))
    if band is not None:
        out["band"] = r["band"]
    return out
