"""Python binding of libsnaps (ctypes), with the C ABI's names.

Only argument marshalling happens here: device memory and streams come from
PyTorch tensors, every computation runs in the library's HIP kernels.  The
binding raises if the shared library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnaps.so")

SNAPS_OK = 0
SNAPS_EINVAL = -1
SNAPS_ENOMEM = -2
SNAPS_EDEVICE = -3
SNAPS_EUNSUPPORTED = -4
OP_KNN, OP_EPS, OP_SCORES, OP_RANK = 0, 1, 2, 3
MAX_N = 1 << 30
LDS_N = 32768          # jobs up to this size are indexed and ranked inside LDS
MAX_K = 32             # largest k of the fused join (larger k: the selection kernel)
MAX_LIST_K = 4096      # largest k whose sorted kNN lists are written


class SnapsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"snaps error {code}: {msg}")
        self.code = code


class c_population(ctypes.Structure):
    _fields_ = [("cols", ctypes.c_void_p), ("ld", ctypes.c_int64), ("n", ctypes.c_int64),
                ("n_features", ctypes.c_int32)]


class c_scores(ctypes.Structure):
    _fields_ = [("eps_count", ctypes.c_void_p), ("eps_mean", ctypes.c_void_p),
                ("indeg", ctypes.c_void_p), ("knn_mean", ctypes.c_void_p)]


class c_job(ctypes.Structure):
    _fields_ = [("pop", ctypes.POINTER(c_population)), ("mask", ctypes.c_uint32), ("k", ctypes.c_int32),
                ("eps", ctypes.c_float), ("out", c_scores), ("rank", ctypes.c_void_p),
                ("ensemble", ctypes.c_void_p), ("mode", ctypes.c_int32), ("index_dims", ctypes.c_int32),
                ("knn_ids", ctypes.c_void_p), ("knn_dist", ctypes.c_void_p), ("tile_shape", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class c_tuning(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("split", ctypes.c_int32), ("index_dims", ctypes.c_int32),
                ("filter", ctypes.c_int32), ("passes", ctypes.c_int32), ("mq", ctypes.c_int32),
                ("index_sort", ctypes.c_int32), ("tile_shape", ctypes.c_int32), ("stats", ctypes.c_void_p)]


PASS_INDEX, PASS_JOIN, PASS_RANK = 1, 2, 4


class c_alert_job(ctypes.Structure):
    _fields_ = [("state", ctypes.c_void_p), ("alerts", ctypes.c_void_p), ("m", ctypes.c_int32),
                ("method", ctypes.c_int32), ("eps_count", ctypes.c_void_p), ("eps_mean", ctypes.c_void_p),
                ("indeg", ctypes.c_void_p), ("knn_mean", ctypes.c_void_p), ("rank", ctypes.c_void_p)]


MAX_EPS_TARGETS = 8


class c_eps_job(ctypes.Structure):
    _fields_ = [("pop", ctypes.POINTER(c_population)), ("mask", ctypes.c_uint32), ("m", ctypes.c_int32),
                ("sample", ctypes.c_void_p), ("n_targets", ctypes.c_int32),
                ("target", ctypes.c_float * MAX_EPS_TARGETS), ("eps", ctypes.c_void_p)]


MAX_GRID = 16


class c_eps_grid_job(ctypes.Structure):
    _fields_ = [("pop", ctypes.POINTER(c_population)), ("mask", ctypes.c_uint32), ("n_grid", ctypes.c_int32),
                ("eps", ctypes.c_float * MAX_GRID), ("top_n", ctypes.c_int32), ("count", ctypes.c_void_p),
                ("mean", ctypes.c_void_p), ("similarity", ctypes.c_void_p), ("select", ctypes.c_void_p)]


class c_k_grid_job(ctypes.Structure):
    _fields_ = [("pop", ctypes.POINTER(c_population)), ("mask", ctypes.c_uint32), ("n_grid", ctypes.c_int32),
                ("k", ctypes.c_int32 * MAX_GRID), ("top_n", ctypes.c_int32), ("indeg", ctypes.c_void_p),
                ("knn_mean", ctypes.c_void_p), ("similarity", ctypes.c_void_p), ("select", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsnaps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2405_20176_amd.build (no fallback exists)")
    lib = ctypes.CDLL(path)
    vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    lib.snaps_last_error.restype = ctypes.c_char_p
    lib.snaps_version.restype = ctypes.c_char_p
    lib.snaps_workspace_bytes.restype = sz
    lib.snaps_workspace_bytes.argtypes = [i32, i64, i32, i32]
    lib.snaps_outlier_scores_workspace.restype = sz
    lib.snaps_outlier_scores_workspace.argtypes = [P(c_job), i32, P(c_tuning)]
    lib.snaps_knn_selfjoin.restype = ctypes.c_int
    lib.snaps_knn_selfjoin.argtypes = [P(c_population), ctypes.c_uint32, i32, vp, vp, vp, sz, vp]
    lib.snaps_eps_selfjoin.restype = ctypes.c_int
    lib.snaps_eps_selfjoin.argtypes = [P(c_population), ctypes.c_uint32, ctypes.c_float, vp, vp, vp, vp, i64,
                                       vp, sz, vp]
    lib.snaps_outlier_scores.restype = ctypes.c_int
    lib.snaps_outlier_scores.argtypes = [P(c_job), i32, P(c_tuning), vp, sz, vp]
    lib.snaps_rank.restype = ctypes.c_int
    lib.snaps_rank.argtypes = [vp, vp, vp, vp, i64, vp, vp, sz, vp]
    lib.snaps_outlier_scores_static.restype = ctypes.c_int
    lib.snaps_outlier_scores_static.argtypes = [P(c_job), i32, P(c_tuning), vp]
    lib.snaps_plan_create.restype = ctypes.c_int
    lib.snaps_plan_create.argtypes = [P(c_job), i32, P(c_tuning), vp, sz, vp, P(vp)]
    lib.snaps_plan_launch.restype = ctypes.c_int
    lib.snaps_plan_launch.argtypes = [vp, vp]
    lib.snaps_plan_destroy.restype = None
    lib.snaps_plan_destroy.argtypes = [vp]
    lib.snaps_serve_state_bytes.restype = sz
    lib.snaps_serve_state_bytes.argtypes = [P(c_population), ctypes.c_uint32, i32]
    lib.snaps_serve_state_build.restype = ctypes.c_int
    lib.snaps_serve_state_build.argtypes = [P(c_population), ctypes.c_uint32, i32, ctypes.c_float, vp, sz, vp]
    lib.snaps_serve_state_outputs.restype = ctypes.c_int
    lib.snaps_serve_state_outputs.argtypes = [vp, i64, i32, i32, P(vp), P(vp), P(vp), P(vp), P(vp)]
    lib.snaps_alerts_score.restype = ctypes.c_int
    lib.snaps_alerts_score.argtypes = [P(c_alert_job), i32, i32, i32, vp, sz, vp]
    lib.snaps_alerts_workspace_bytes.restype = sz
    lib.snaps_alerts_workspace_bytes.argtypes = [P(c_alert_job), i32, i32, i32]
    lib.snaps_eps_sample_workspace.restype = sz
    lib.snaps_eps_sample_workspace.argtypes = [P(c_eps_job), i32]
    lib.snaps_eps_sample.restype = ctypes.c_int
    lib.snaps_eps_sample.argtypes = [P(c_eps_job), i32, vp, sz, vp]
    lib.snaps_eps_grid_workspace.restype = sz
    lib.snaps_eps_grid_workspace.argtypes = [P(c_eps_grid_job), i32]
    lib.snaps_eps_grid.restype = ctypes.c_int
    lib.snaps_eps_grid.argtypes = [P(c_eps_grid_job), i32, vp, sz, vp]
    lib.snaps_k_grid_workspace.argtypes = [P(c_k_grid_job), i32]
    lib.snaps_k_grid_workspace.restype = sz
    lib.snaps_k_grid.argtypes = [P(c_k_grid_job), i32, vp, sz, vp]
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().snaps_last_error().decode()


def _check(rc: int):
    if rc != SNAPS_OK:
        raise SnapsError(rc, last_error())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Population:
    """A resident population: feature-major float32 columns [F, ld] on the
    GPU, n objects (values normalised to [0, 1])."""

    def __init__(self, cols: torch.Tensor, n: int):
        if cols.dtype != torch.float32 or cols.dim() != 2 or not cols.is_cuda or not cols.is_contiguous():
            raise ValueError("cols must be a contiguous float32 CUDA tensor [n_features, ld]")
        self.cols = cols
        self.n = int(n)
        self.c = c_population(cols.data_ptr(), cols.shape[1], self.n, cols.shape[0])

    @classmethod
    def from_rows(cls, x, device="cuda") -> "Population":
        """Upload a row-major [n, F] float32 array as feature-major columns
        (leading dimension rounded up to 64)."""
        x = torch.as_tensor(x, dtype=torch.float32)
        n, f = x.shape
        ld = (n + 63) // 64 * 64
        cols = torch.zeros((f, ld), dtype=torch.float32)
        cols[:, :n] = x.T
        return cls(cols.to(device).contiguous(), n)


def tuning(mode=0, split=0, index_dims=0, filter=0, passes=0, stats: Optional[torch.Tensor] = None,
           mq=0, index_sort=0, tile_shape=0) -> c_tuning:
    """Tuning record; ``stats`` is an optional int64 CUDA tensor of 4
    accumulated join counters (pairs evaluated, tiles scanned, tiles
    skipped, pairs x dimensionality)."""
    t = c_tuning()
    t.mode, t.split, t.index_dims, t.filter, t.passes, t.mq = mode, split, index_dims, filter, passes, mq
    t.index_sort = index_sort
    t.tile_shape = tile_shape
    t.stats = None if stats is None else stats.data_ptr()
    return t


def snaps_workspace_bytes(op: int, n: int, d: int, k: int) -> int:
    return int(load_library().snaps_workspace_bytes(op, n, d, k))


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def snaps_knn_selfjoin(pop: Population, mask: int, k: int, ids: torch.Tensor, dist: Optional[torch.Tensor] = None,
                       ws: Optional[torch.Tensor] = None, stream=None):
    lib = load_library()
    d = bin(int(mask)).count("1")
    need = lib.snaps_workspace_bytes(OP_KNN, pop.n, d, k)
    if ws is None:
        ws = _workspace(need, pop.cols.device)
    _check(lib.snaps_knn_selfjoin(ctypes.byref(pop.c), int(mask), int(k), _ptr(ids), _ptr(dist), _ptr(ws),
                                  ws.numel(), _stream(stream)))


def snaps_eps_selfjoin(pop: Population, mask: int, eps: float, count: torch.Tensor, mean_dist: torch.Tensor,
                       ws: Optional[torch.Tensor] = None, stream=None, pair_off: Optional[torch.Tensor] = None,
                       pairs: Optional[torch.Tensor] = None):
    """Range self-join; with ``pair_off`` ([n + 1] int64) also the CSR pair
    list into ``pairs`` (int32, its length is the capacity)."""
    lib = load_library()
    d = bin(int(mask)).count("1")
    need = lib.snaps_workspace_bytes(OP_EPS, pop.n, d, 0)
    if ws is None:
        ws = _workspace(need, pop.cols.device)
    cap = int(pairs.numel()) if pairs is not None else 0
    _check(lib.snaps_eps_selfjoin(ctypes.byref(pop.c), int(mask), float(eps), _ptr(count), _ptr(mean_dist),
                                  _ptr(pair_off), _ptr(pairs), cap, _ptr(ws), ws.numel(), _stream(stream)))


def snaps_eps_pairs(pop: Population, mask: int, eps: float, stream=None):
    """Counts, mean distances and the complete pair list of one subspace:
    a first call sizes the list, a second fills it.  Returns (count,
    mean_dist, pair_off, pairs) as CUDA tensors."""
    dev = pop.cols.device
    count = torch.empty(pop.n, dtype=torch.int32, device=dev)
    mean = torch.empty(pop.n, dtype=torch.float32, device=dev)
    off = torch.empty(pop.n + 1, dtype=torch.int64, device=dev)
    snaps_eps_selfjoin(pop, mask, eps, count, mean, stream=stream, pair_off=off)
    total = int(off[-1].item())
    pairs = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
    snaps_eps_selfjoin(pop, mask, eps, count, mean, stream=stream, pair_off=off, pairs=pairs)
    return count, mean, off, pairs[:total]


@dataclass
class Job:
    """One (population, subspace) job and its output tensors (length n)."""
    pop: Population
    mask: int
    k: int
    eps: float
    eps_count: torch.Tensor
    eps_mean: torch.Tensor
    indeg: torch.Tensor
    knn_mean: torch.Tensor
    rank: Optional[torch.Tensor] = None      # [4, n] int32
    ensemble: Optional[torch.Tensor] = None  # [n] float32, mean of the four ranks
    mode: int = 0                            # per-job overrides of the call's tuning (0: none)
    index_dims: int = 0
    knn_ids: Optional[torch.Tensor] = None   # [n, k] int32, the kNN lists the in-degree was counted from
    knn_dist: Optional[torch.Tensor] = None  # [n, k] float32
    tile_shape: int = 0                      # per-job override of the call's tile shape (0: none)

    @classmethod
    def alloc(cls, pop: Population, mask: int, k: int, eps: float, with_rank: bool = True,
              with_ensemble: bool = False, with_lists: bool = False) -> "Job":
        dev = pop.cols.device
        n = pop.n
        return cls(pop, int(mask), int(k), float(eps),
                   torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.float32, device=dev),
                   torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.float32, device=dev),
                   torch.empty((4, n), dtype=torch.int32, device=dev) if with_rank else None,
                   torch.empty(n, dtype=torch.float32, device=dev) if (with_rank and with_ensemble) else None,
                   knn_ids=torch.empty((n, k), dtype=torch.int32, device=dev) if with_lists else None,
                   knn_dist=torch.empty((n, k), dtype=torch.float32, device=dev) if with_lists else None)


def _c_jobs(jobs: Sequence[Job]):
    arr = (c_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i].pop = ctypes.pointer(j.pop.c)
        arr[i].mask = j.mask
        arr[i].k = j.k
        arr[i].eps = j.eps
        arr[i].out = c_scores(j.eps_count.data_ptr(), j.eps_mean.data_ptr(), j.indeg.data_ptr(),
                              j.knn_mean.data_ptr())
        arr[i].rank = None if j.rank is None else j.rank.data_ptr()
        arr[i].ensemble = None if j.ensemble is None else j.ensemble.data_ptr()
        arr[i].mode = j.mode
        arr[i].index_dims = j.index_dims
        arr[i].knn_ids = None if j.knn_ids is None else j.knn_ids.data_ptr()
        arr[i].knn_dist = None if j.knn_dist is None else j.knn_dist.data_ptr()
        arr[i].tile_shape = j.tile_shape
    return arr


def snaps_outlier_scores_workspace(jobs: Sequence[Job], tune: Optional[c_tuning] = None) -> int:
    lib = load_library()
    arr = _c_jobs(jobs)
    return int(lib.snaps_outlier_scores_workspace(arr, len(jobs), None if tune is None else ctypes.byref(tune)))


def snaps_outlier_scores(jobs: Sequence[Job], tune: Optional[c_tuning] = None, ws: Optional[torch.Tensor] = None,
                         stream=None):
    lib = load_library()
    arr = _c_jobs(jobs)
    tp = None if tune is None else ctypes.byref(tune)
    need = lib.snaps_outlier_scores_workspace(arr, len(jobs), tp)
    if need == 0:
        # let the library report why
        _check(lib.snaps_outlier_scores(arr, len(jobs), tp, None, 0, _stream(stream)))
    if ws is None:
        ws = _workspace(need, jobs[0].pop.cols.device)
    _check(lib.snaps_outlier_scores(arr, len(jobs), tp, _ptr(ws), ws.numel(), _stream(stream)))


STATIC_SCRATCH_BYTES = 64 << 20


def snaps_outlier_scores_static(jobs: Sequence[Job], tune: Optional[c_tuning] = None, stream=None):
    """snaps_outlier_scores with the library's static per-device scratch
    (no workspace argument, no device allocation)."""
    lib = load_library()
    arr = _c_jobs(jobs)
    tp = None if tune is None else ctypes.byref(tune)
    _check(lib.snaps_outlier_scores_static(arr, len(jobs), tp, _stream(stream)))


class Plan:
    """A captured batched launch (snaps_plan_*) over a list of jobs."""

    def __init__(self, jobs: Sequence[Job], tune: Optional[c_tuning] = None, ws: Optional[torch.Tensor] = None,
                 stream=None, c_jobs=None, n_jobs: Optional[int] = None):
        lib = load_library()
        arr = c_jobs if c_jobs is not None else _c_jobs(jobs)
        n = n_jobs if n_jobs is not None else len(jobs)
        tp = None if tune is None else ctypes.byref(tune)
        need = lib.snaps_outlier_scores_workspace(arr, n, tp)
        if ws is None:
            ws = _workspace(need, jobs[0].pop.cols.device)
        self.ws, self.jobs, self.arr, self.tune = ws, jobs, arr, tune
        h = ctypes.c_void_p()
        _check(lib.snaps_plan_create(arr, n, tp, _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        _check(load_library().snaps_plan_launch(self.h, _stream(stream)))

    def close(self):
        if self.h:
            load_library().snaps_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class JobTable:
    """Many jobs in one job table over resident outputs: the outputs of every
    job live in flat device buffers (job i at offset off[i], [4][n] ranks at
    4 off[i], lists at off_k[i]), so thousands of jobs cost one allocation
    per output.  ``specs``: sequence of (Population, mask, k, eps).  Per-job
    walk settings (``mode``, ``index_dims``) can be set before plans are
    built; ``plans`` captures the three passes of the whole table as graphs
    over one workspace."""

    def __init__(self, specs, with_rank: bool = True, with_ensemble: bool = False, with_lists: bool = False,
                 device=None):
        self.specs = [(p, int(m), int(k), float(e)) for p, m, k, e in specs]
        nj = len(self.specs)
        if nj == 0:
            raise ValueError("no jobs")
        dev = device or self.specs[0][0].cols.device
        ns = [p.n for p, _, _, _ in self.specs]
        self.off = [0]
        self.off_k = [0]
        for (p, _, k, _), n in zip(self.specs, ns):
            self.off.append(self.off[-1] + n)
            self.off_k.append(self.off_k[-1] + n * k)
        total, total_k = self.off[-1], self.off_k[-1]
        self.eps_count = torch.empty(total, dtype=torch.int32, device=dev)
        self.eps_mean = torch.empty(total, dtype=torch.float32, device=dev)
        self.indeg = torch.empty(total, dtype=torch.int32, device=dev)
        self.knn_mean = torch.empty(total, dtype=torch.float32, device=dev)
        self.rank = torch.empty(4 * total, dtype=torch.int32, device=dev) if with_rank else None
        self.ensemble = torch.empty(total, dtype=torch.float32, device=dev) if (with_rank and with_ensemble) else None
        self.knn_ids = torch.empty(total_k, dtype=torch.int32, device=dev) if with_lists else None
        self.knn_dist = torch.empty(total_k, dtype=torch.float32, device=dev) if with_lists else None
        self.mode = [0] * nj
        self.index_dims = [0] * nj
        self.tile_shape = [0] * nj
        self.arr = (c_job * nj)()
        self._pops = {}
        for i, (pop, mask, k, eps) in enumerate(self.specs):
            key = id(pop)
            if key not in self._pops:
                self._pops[key] = (pop, ctypes.pointer(pop.c))
            j = self.arr[i]
            j.pop = self._pops[key][1]
            j.mask, j.k, j.eps = mask, k, eps
            o = self.off[i]
            j.out = c_scores(self._at(self.eps_count, o), self._at(self.eps_mean, o), self._at(self.indeg, o),
                             self._at(self.knn_mean, o))
            j.rank = self._at(self.rank, 4 * o)
            j.ensemble = self._at(self.ensemble, o)
            j.knn_ids = self._at(self.knn_ids, self.off_k[i])
            j.knn_dist = self._at(self.knn_dist, self.off_k[i])

    @staticmethod
    def _at(t: Optional[torch.Tensor], off: int):
        return None if t is None else t.data_ptr() + off * t.element_size()

    def __len__(self):
        return len(self.specs)

    def set_walk(self, i: int, mode: int, index_dims: int, tile_shape: int = 0):
        self.mode[i], self.index_dims[i], self.tile_shape[i] = int(mode), int(index_dims), int(tile_shape)
        self.arr[i].mode, self.arr[i].index_dims = int(mode), int(index_dims)
        self.arr[i].tile_shape = int(tile_shape)

    def walk_specs(self):
        """Lightweight per-job records (pop, mask, k, eps, mode, index_dims,
        tile_shape) for the autotuner; ``apply_walk`` copies their settings
        back."""
        from types import SimpleNamespace
        return [SimpleNamespace(pop=p, mask=m, k=k, eps=e, mode=self.mode[i], index_dims=self.index_dims[i],
                                tile_shape=self.tile_shape[i])
                for i, (p, m, k, e) in enumerate(self.specs)]

    def apply_walk(self, recs):
        for i, r in enumerate(recs):
            self.set_walk(i, r.mode, r.index_dims, getattr(r, "tile_shape", 0))

    def c_ptr(self, start: int = 0):
        return ctypes.cast(ctypes.byref(self.arr, start * ctypes.sizeof(c_job)), ctypes.POINTER(c_job))

    def workspace_bytes(self, tune: Optional[c_tuning] = None, start: int = 0, stop: Optional[int] = None) -> int:
        stop = len(self) if stop is None else stop
        return int(load_library().snaps_outlier_scores_workspace(self.c_ptr(start), stop - start,
                                                                 None if tune is None else ctypes.byref(tune)))

    def run(self, tune: Optional[c_tuning] = None, ws: Optional[torch.Tensor] = None, stream=None,
            start: int = 0, stop: Optional[int] = None):
        """One direct call over jobs [start, stop)."""
        lib = load_library()
        stop = len(self) if stop is None else stop
        tp = None if tune is None else ctypes.byref(tune)
        if ws is None:
            ws = _workspace(self.workspace_bytes(tune, start, stop), self.eps_count.device)
        _check(lib.snaps_outlier_scores(self.c_ptr(start), stop - start, tp, _ptr(ws), ws.numel(), _stream(stream)))

    def plans(self, stats: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None):
        """(workspace, [index, join, rank] plans) over every job; ``stats``
        accumulates the join pass's counters."""
        tunes = [tuning(passes=p, stats=stats if p == PASS_JOIN else None) for p in (PASS_INDEX, PASS_JOIN, PASS_RANK)]
        if ws is None:
            ws = _workspace(self.workspace_bytes(tunes[1]), self.eps_count.device)
        self._tunes = tunes
        return ws, [Plan(None, t, ws=ws, stream=stream, c_jobs=self.c_ptr(), n_jobs=len(self)) for t in tunes]

    def out(self, i: int) -> dict:
        """Device views of job i's outputs."""
        _, _, k, _ = self.specs[i]
        a, b = self.off[i], self.off[i + 1]
        n = b - a
        o = {"eps_count": self.eps_count[a:b], "eps_mean": self.eps_mean[a:b], "indeg": self.indeg[a:b],
             "knn_mean": self.knn_mean[a:b]}
        o["rank"] = None if self.rank is None else self.rank[4 * a:4 * b].view(4, n)
        o["ensemble"] = None if self.ensemble is None else self.ensemble[a:b]
        ka, kb = self.off_k[i], self.off_k[i + 1]
        o["knn_ids"] = None if self.knn_ids is None else self.knn_ids[ka:kb].view(n, k)
        o["knn_dist"] = None if self.knn_dist is None else self.knn_dist[ka:kb].view(n, k)
        return o


def snaps_rank(eps_count: torch.Tensor, eps_mean: torch.Tensor, indeg: torch.Tensor, knn_mean: torch.Tensor,
               rank: torch.Tensor, ws: Optional[torch.Tensor] = None, stream=None):
    lib = load_library()
    n = eps_count.numel()
    need = lib.snaps_workspace_bytes(OP_RANK, n, 0, 0)
    if ws is None and need > 0:
        ws = _workspace(need, eps_count.device)
    _check(lib.snaps_rank(_ptr(eps_count), _ptr(eps_mean), _ptr(indeg), _ptr(knn_mean), n, _ptr(rank), _ptr(ws),
                          0 if ws is None else ws.numel(), _stream(stream)))


def score_space(pop: Population, mask: int, k: int, eps: float, tune: Optional[c_tuning] = None,
                with_rank: bool = True) -> Job:
    """Convenience: allocate the outputs and run one job."""
    job = Job.alloc(pop, mask, k, eps, with_rank)
    snaps_outlier_scores([job], tune)
    return job


class ServeState:
    """Resident scoring state of one (population, subspace) in device memory
    (owned by this object as a torch tensor)."""

    def __init__(self, pop: Population, mask: int, k: int, eps: float, stream=None):
        lib = load_library()
        self.pop, self.mask, self.k, self.eps = pop, int(mask), int(k), float(eps)
        self.d = bin(self.mask).count("1")
        nbytes = lib.snaps_serve_state_bytes(ctypes.byref(pop.c), self.mask, self.k)
        if nbytes == 0:
            raise SnapsError(SNAPS_EINVAL, "invalid serve state request")
        self.nbytes = int(nbytes)
        self.mem = torch.empty(self.nbytes, dtype=torch.uint8, device=pop.cols.device)
        _check(lib.snaps_serve_state_build(ctypes.byref(pop.c), self.mask, self.k, self.eps,
                                           ctypes.c_void_p(self.mem.data_ptr()), self.nbytes, _stream(stream)))

    def ptr(self) -> int:
        return self.mem.data_ptr()

    def population_outputs(self) -> dict:
        """The population's own metrics and ranks (views into the state)."""
        lib = load_library()
        ptrs = [ctypes.c_void_p() for _ in range(5)]
        _check(lib.snaps_serve_state_outputs(ctypes.c_void_p(self.mem.data_ptr()), self.pop.n, self.d, self.k,
                                             *[ctypes.byref(p) for p in ptrs]))
        base = self.mem.data_ptr()
        n = self.pop.n

        def view(p, dtype, shape):
            off = p.value - base
            count = 1
            for v in shape:
                count *= v
            return self.mem[off:off + count * 4].view(dtype).view(*shape)

        return {"eps_count": view(ptrs[0], torch.int32, (n,)), "eps_mean": view(ptrs[1], torch.float32, (n,)),
                "indeg": view(ptrs[2], torch.int32, (n,)), "knn_mean": view(ptrs[3], torch.float32, (n,)),
                "rank": view(ptrs[4], torch.int32, (4, n))}


@dataclass
class AlertJob:
    """A batch of alerts [m, d] (float32, subspace columns in ascending feature
    order, population-normalised) for one ServeState, with its outputs."""
    state: ServeState
    alerts: torch.Tensor
    eps_count: torch.Tensor
    eps_mean: torch.Tensor
    indeg: torch.Tensor
    knn_mean: torch.Tensor
    rank: Optional[torch.Tensor] = None
    method: int = 0          # 0 automatic, 1 one wavefront per alert, 2 matrix-core tiles of 64 alerts

    @classmethod
    def alloc(cls, state: ServeState, alerts: torch.Tensor, with_rank: bool = True, method: int = 0) -> "AlertJob":
        m = alerts.shape[0]
        dev = alerts.device
        return cls(state, alerts, torch.empty(m, dtype=torch.int32, device=dev),
                   torch.empty(m, dtype=torch.float32, device=dev), torch.empty(m, dtype=torch.int32, device=dev),
                   torch.empty(m, dtype=torch.float32, device=dev),
                   torch.empty((4, m), dtype=torch.int32, device=dev) if with_rank else None, method)


def snaps_alerts_score(jobs: Sequence[AlertJob], stream=None):
    """Score alert batches; jobs are grouped by (d, k) into library calls,
    each with the workspace it needs (allocated on the calling stream)."""
    lib = load_library()
    groups = {}
    for j in jobs:
        if j.alerts.dtype != torch.float32 or not j.alerts.is_contiguous() or j.alerts.shape[1] != j.state.d:
            raise ValueError("alerts must be contiguous float32 [m, d] for the state's subspace")
        groups.setdefault((j.state.d, j.state.k), []).append(j)
    for (d, k), js in groups.items():
        arr = (c_alert_job * len(js))()
        for i, j in enumerate(js):
            arr[i].state = j.state.ptr()
            arr[i].alerts = j.alerts.data_ptr()
            arr[i].m = j.alerts.shape[0]
            arr[i].eps_count = j.eps_count.data_ptr()
            arr[i].eps_mean = j.eps_mean.data_ptr()
            arr[i].indeg = j.indeg.data_ptr()
            arr[i].knn_mean = j.knn_mean.data_ptr()
            arr[i].rank = None if j.rank is None else j.rank.data_ptr()
            arr[i].method = int(j.method)
        need = lib.snaps_alerts_workspace_bytes(arr, len(js), d, k)
        ws = _workspace(need, js[0].alerts.device) if need else None
        _check(lib.snaps_alerts_score(arr, len(js), d, k, _ptr(ws), need, _stream(stream)))


def snaps_eps_sample(specs, stream=None):
    """Sampled-distance radii (Sec. 3.5.3) for several subspaces in one call.
    ``specs``: sequence of (Population, mask, sample int32 CUDA tensor of
    object ids, targets); returns one float32 CUDA tensor of radii per spec."""
    lib = load_library()
    arr = (c_eps_job * len(specs))()
    outs = []
    for i, (pop, mask, sample, targets) in enumerate(specs):
        if sample.dtype != torch.int32 or not sample.is_contiguous():
            raise ValueError("sample must be a contiguous int32 tensor of object ids")
        targets = list(targets)
        out = torch.empty(len(targets), dtype=torch.float32, device=sample.device)
        arr[i].pop = ctypes.pointer(pop.c)
        arr[i].mask = int(mask)
        arr[i].m = sample.numel()
        arr[i].sample = sample.data_ptr()
        arr[i].n_targets = len(targets)
        for t, v in enumerate(targets):
            arr[i].target[t] = float(v)
        arr[i].eps = out.data_ptr()
        outs.append(out)
    need = lib.snaps_eps_sample_workspace(arr, len(specs))
    if need == 0:
        _check(lib.snaps_eps_sample(arr, len(specs), None, 0, _stream(stream)))
        return outs
    ws = _workspace(need, outs[0].device)
    _check(lib.snaps_eps_sample(arr, len(specs), _ptr(ws), ws.numel(), _stream(stream)))
    return outs


def snaps_eps_grid(specs, with_metrics: bool = False, stream=None):
    """Radius selection on grids of radii (Sec. 3.5.2).  ``specs``: sequence
    of (Population, mask, radii, top_n).  Returns per spec a dict with
    ``similarity`` [2, 2, g] (metric: count, mean; U^min, U^max), ``select``
    [2] and, with ``with_metrics``, ``count`` / ``mean`` [g, n] (CUDA
    tensors)."""
    lib = load_library()
    arr = (c_eps_grid_job * len(specs))()
    outs = []
    for i, (pop, mask, radii, top_n) in enumerate(specs):
        radii = [float(r) for r in radii]
        g = len(radii)
        dev = pop.cols.device
        o = {"similarity": torch.empty((2, 2, g), dtype=torch.float32, device=dev),
             "select": torch.empty(2, dtype=torch.int32, device=dev)}
        if with_metrics:
            o["count"] = torch.empty((g, pop.n), dtype=torch.int32, device=dev)
            o["mean"] = torch.empty((g, pop.n), dtype=torch.float32, device=dev)
        arr[i].pop = ctypes.pointer(pop.c)
        arr[i].mask = int(mask)
        arr[i].n_grid = g
        for r, v in enumerate(radii):
            arr[i].eps[r] = v
        arr[i].top_n = int(top_n)
        arr[i].count = o["count"].data_ptr() if with_metrics else None
        arr[i].mean = o["mean"].data_ptr() if with_metrics else None
        arr[i].similarity = o["similarity"].data_ptr()
        arr[i].select = o["select"].data_ptr()
        outs.append(o)
    need = lib.snaps_eps_grid_workspace(arr, len(specs))
    if need == 0:
        _check(lib.snaps_eps_grid(arr, len(specs), None, 0, _stream(stream)))
    ws = _workspace(need, outs[0]["select"].device)
    _check(lib.snaps_eps_grid(arr, len(specs), _ptr(ws), ws.numel(), _stream(stream)))
    return outs


def snaps_k_grid(specs, with_metrics: bool = False, stream=None):
    """k selection on grids of k (Sec. 3.6.2).  ``specs``: sequence of
    (Population, mask, ks, top_n).  Returns per spec a dict with
    ``similarity`` [2, 2, g] (metric: in-degree, mean kNN distance; U^min,
    U^max), ``select`` [2] and, with ``with_metrics``, ``indeg`` /
    ``knn_mean`` [g, n] (CUDA tensors)."""
    lib = load_library()
    arr = (c_k_grid_job * len(specs))()
    outs = []
    for i, (pop, mask, ks, top_n) in enumerate(specs):
        ks = [int(k) for k in ks]
        g = len(ks)
        dev = pop.cols.device
        o = {"similarity": torch.empty((2, 2, g), dtype=torch.float32, device=dev),
             "select": torch.empty(2, dtype=torch.int32, device=dev)}
        if with_metrics:
            o["indeg"] = torch.empty((g, pop.n), dtype=torch.int32, device=dev)
            o["knn_mean"] = torch.empty((g, pop.n), dtype=torch.float32, device=dev)
        arr[i].pop = ctypes.pointer(pop.c)
        arr[i].mask = int(mask)
        arr[i].n_grid = g
        for r, v in enumerate(ks[:MAX_GRID]):
            arr[i].k[r] = v
        arr[i].top_n = int(top_n)
        arr[i].indeg = o["indeg"].data_ptr() if with_metrics else None
        arr[i].knn_mean = o["knn_mean"].data_ptr() if with_metrics else None
        arr[i].similarity = o["similarity"].data_ptr()
        arr[i].select = o["select"].data_ptr()
        outs.append(o)
    need = lib.snaps_k_grid_workspace(arr, len(specs))
    if need == 0:
        _check(lib.snaps_k_grid(arr, len(specs), None, 0, _stream(stream)))
    ws = _workspace(need, outs[0]["select"].device)
    _check(lib.snaps_k_grid(arr, len(specs), _ptr(ws), ws.numel(), _stream(stream)))
    return outs
