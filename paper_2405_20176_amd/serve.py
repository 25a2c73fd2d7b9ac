"""Continuous-batching server for scoring alerts against resident states.

Requests (a population, one of its served subspaces, and a batch of alert
objects) arrive over time.  The server
  * admits a request when the device memory it needs (alerts plus outputs)
    fits in the remaining budget next to the resident states, and a batch slot
    is free; requests larger than the whole budget are rejected;
  * packs every admitted, waiting request into one batch (different sizes,
    populations and subspaces) and launches it on its own stream, so batches
    overlap on the device while later requests keep arriving;
  * completes a request when its batch's event has fired and its results
    have been copied back, and records its latency (completion - arrival).
Scoring itself runs in libsnaps (snaps_alerts_score); results of an alert do
not depend on the batch it lands in.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds on the server clock
    key: Tuple[int, int]           # (population id, subspace mask)
    alerts: np.ndarray             # float32 [m, d], subspace columns, population-normalised
    # filled by the server
    admitted: Optional[float] = None
    done: Optional[float] = None
    status: str = "pending"        # pending | running | done | rejected
    result: Optional[Dict[str, np.ndarray]] = None

    @property
    def m(self) -> int:
        return int(self.alerts.shape[0])

    def device_bytes(self) -> int:
        """Device memory of the request while in flight: alerts, four metric
        arrays and the [4, m] ranks."""
        return self.m * (4 * self.alerts.shape[1] + 16 + 16)


class Admission:
    """Device-memory budget for in-flight requests and a cap on batches in
    flight.  Pure host logic."""

    def __init__(self, budget_bytes: int, max_batches: int):
        self.budget = int(budget_bytes)
        self.max_batches = int(max_batches)
        self.used = 0
        self.batches = 0

    def fits(self, nbytes: int) -> bool:
        return self.used + nbytes <= self.budget

    def never_fits(self, nbytes: int) -> bool:
        return nbytes > self.budget

    def take(self, nbytes: int):
        assert self.fits(nbytes)
        self.used += nbytes

    def release(self, nbytes: int):
        self.used -= nbytes
        assert self.used >= 0

    def slot_free(self) -> bool:
        return self.batches < self.max_batches


class Batcher:
    """Continuous batching over an executor.  The executor launches a list of
    requests asynchronously and later reports completion:
        handle = executor.launch(requests)
        executor.poll(handle) -> bool            (non-blocking)
        executor.finish(handle) -> [result dict per request]
    """

    def __init__(self, executor, admission: Admission, max_batch_alerts: int = 1 << 16,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.adm = admission
        self.max_batch_alerts = int(max_batch_alerts)
        self.clock = clock
        self.waiting: Deque[Request] = collections.deque()
        self.inflight: List[Tuple[object, List[Request], int]] = []
        self.finished: List[Request] = []
        self.max_inflight = 0          # most batches on the device at once
        self.batches_launched = 0

    def submit(self, r: Request):
        if self.adm.never_fits(r.device_bytes()):
            r.status = "rejected"
            r.done = self.clock()
            self.finished.append(r)
            return
        self.waiting.append(r)

    def _launch(self) -> bool:
        if not self.waiting or not self.adm.slot_free():
            return False
        batch, nbytes, alerts = [], 0, 0
        while self.waiting:
            r = self.waiting[0]
            b = r.device_bytes()
            if not self.adm.fits(nbytes + b) or (batch and alerts + r.m > self.max_batch_alerts):
                break
            self.waiting.popleft()
            batch.append(r)
            nbytes += b
            alerts += r.m
        if not batch:
            return False
        self.adm.take(nbytes)
        self.adm.batches += 1
        now = self.clock()
        for r in batch:
            r.admitted = now
            r.status = "running"
        self.inflight.append((self.ex.launch(batch), batch, nbytes))
        self.batches_launched += 1
        self.max_inflight = max(self.max_inflight, len(self.inflight))
        return True

    def _reap(self) -> bool:
        progressed = False
        still = []
        for h, batch, nbytes in self.inflight:
            if self.ex.poll(h):
                results = self.ex.finish(h)
                now = self.clock()
                for r, res in zip(batch, results):
                    r.result = res
                    r.done = now
                    r.status = "done"
                    self.finished.append(r)
                self.adm.release(nbytes)
                self.adm.batches -= 1
                progressed = True
            else:
                still.append((h, batch, nbytes))
        self.inflight = still
        return progressed

    def step(self) -> bool:
        """One scheduling round; returns True if anything happened."""
        a = self._reap()
        b = self._launch()
        return a or b

    def drain(self):
        while self.waiting or self.inflight:
            if not self.step():
                time.sleep(0)

    def run_open_loop(self, requests: Sequence[Request], t0: Optional[float] = None):
        """Replay requests at their arrival times (seconds after t0), then
        drain.  Arrivals are released into the queue as the clock passes them,
        while earlier batches are still running."""
        t0 = self.clock() if t0 is None else t0
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        while pending or self.waiting or self.inflight:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                r.arrival += t0            # to the server clock
                self.submit(r)
            if not self.step():
                if self.inflight:
                    # a batch on the device: poll again at once (a sleep
                    # here would add up to its length to every completion)
                    time.sleep(0)
                elif pending:
                    wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0.0005:
                        time.sleep(min(wait, 0.001))

    def latencies(self) -> np.ndarray:
        return np.array([r.done - r.arrival for r in self.finished if r.status == "done"])


def serve_serial(executor, requests: Sequence[Request], open_loop: bool = True,
                 clock: Callable[[], float] = time.perf_counter) -> List[Request]:
    """The plain form of serving, for comparison: one request at a time, in
    arrival order, each launched alone and waited for before the next one
    starts (no batching, no overlap).  With ``open_loop`` a request is not
    started before its arrival time (seconds after the start); otherwise all
    are taken as arrived at the start.  Returns the finished requests."""
    t0 = clock()
    out = []
    for r in sorted(requests, key=lambda q: q.arrival):
        if open_loop:
            while clock() - t0 < r.arrival:
                time.sleep(min(0.001, max(0.0, r.arrival - (clock() - t0))))
            r.arrival += t0
        else:
            r.arrival = t0
        r.admitted = clock()
        h = executor.launch([r])
        r.result = executor.finish(h)[0]
        r.done = clock()
        r.status = "done"
        out.append(r)
    return out


class GpuExecutor:
    """Executor over libsnaps: one stream per in-flight batch slot.  Each
    slot owns pinned host staging buffers, reused from batch to batch (grown
    when a batch needs more): a batch's alerts are packed into one of them
    and go up in one copy, all its outputs come back in one copy into the
    other, and are copied out into ordinary host arrays once the batch has
    finished, so no pinned memory stays with a request."""

    def __init__(self, states: Dict[Tuple[int, int], object], n_streams: int = 4, device="cuda"):
        import torch
        from . import snaps as S
        self.torch, self.S = torch, S
        self.states = states
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.free = list(range(n_streams))
        self.h_in = [torch.empty(0, dtype=torch.float32).pin_memory() for _ in range(n_streams)]
        self.h_out = [torch.empty(0, dtype=torch.int32).pin_memory() for _ in range(n_streams)]

    def _host(self, bufs, si, n, dtype):
        torch = self.torch
        if bufs[si].numel() < n:
            bufs[si] = torch.empty(max(n, 2 * bufs[si].numel()), dtype=dtype).pin_memory()
        return bufs[si]

    def launch(self, batch: List[Request]):
        torch, S = self.torch, self.S
        si = self.free.pop()
        stream = self.streams[si]
        sizes = [r.alerts.size for r in batch]
        ms = [r.m for r in batch]
        n_in, n_al = sum(sizes), sum(ms)
        hin = self._host(self.h_in, si, n_in, torch.float32)
        hout = self._host(self.h_out, si, 8 * n_al, torch.int32)
        hv = hin.numpy()
        at = 0
        for r, sz in zip(batch, sizes):
            hv[at:at + sz] = r.alerts.ravel()
            at += sz
        with torch.cuda.stream(stream):
            dev_in = hin[:n_in].to(self.device, non_blocking=True)
            dev_out = torch.empty(8 * n_al, dtype=torch.int32, device=self.device)
            # per alert of the batch: eps_count, eps_mean, indeg, knn_mean, then the 4 ranks
            cnt, mean = dev_out[:n_al], dev_out[n_al:2 * n_al].view(torch.float32)
            deg, kmean = dev_out[2 * n_al:3 * n_al], dev_out[3 * n_al:4 * n_al].view(torch.float32)
            rank = dev_out[4 * n_al:]
            jobs, at, ai = [], 0, 0
            for r, sz, m in zip(batch, sizes, ms):
                st = self.states[r.key]
                a = dev_in[at:at + sz].view(m, r.alerts.shape[1])
                jobs.append(S.AlertJob(st, a, cnt[ai:ai + m], mean[ai:ai + m], deg[ai:ai + m], kmean[ai:ai + m],
                                       rank[4 * ai:4 * (ai + m)].view(4, m)))
                at += sz
                ai += m
            S.snaps_alerts_score(jobs, stream=stream)
            hout[:8 * n_al].copy_(dev_out, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return (si, ev, ms, dev_in, dev_out)

    def poll(self, h) -> bool:
        return h[1].query()

    def finish(self, h):
        si, ev, ms, _, _ = h
        ev.synchronize()
        n_al = sum(ms)
        v = self.h_out[si][:8 * n_al].numpy()
        out, ai = [], 0
        for m in ms:
            out.append({"eps_count": v[ai:ai + m].copy(),
                        "eps_mean": v[n_al + ai:n_al + ai + m].view(np.float32).copy(),
                        "indeg": v[2 * n_al + ai:2 * n_al + ai + m].copy(),
                        "knn_mean": v[3 * n_al + ai:3 * n_al + ai + m].view(np.float32).copy(),
                        "rank": v[4 * n_al + 4 * ai:4 * n_al + 4 * (ai + m)].reshape(4, m).copy()})
            ai += m
        self.free.append(si)
        return out
