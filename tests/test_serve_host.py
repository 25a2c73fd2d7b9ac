"""Host-side logic of the continuous-batching server, with a fake executor
(no GPU): admission by device-memory budget, rejection of requests that can
never fit, the cap on batches in flight, arrivals joining later batches while
earlier ones run, and first-come order."""
from __future__ import annotations

import numpy as np

from paper_2405_20176_amd.serve import Admission, Batcher, Request


class FakeExecutor:
    """Completes a batch after a fixed number of polls; records what ran."""

    def __init__(self, polls: int, budget_probe=None):
        self.polls = polls
        self.launched = []
        self.probe = budget_probe

    def launch(self, batch):
        if self.probe:
            self.probe()
        h = {"batch": list(batch), "left": self.polls}
        self.launched.append(h)
        return h

    def poll(self, h):
        h["left"] -= 1
        return h["left"] <= 0

    def finish(self, h):
        return [{"m": r.m} for r in h["batch"]]


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.001
        return self.t


def _req(i, m, d=3, t=0.0):
    return Request(i, t, (0, 0b111), np.zeros((m, d), np.float32))


def test_budget_is_never_exceeded_and_everything_completes():
    adm = Admission(budget_bytes=_req(0, 1000).device_bytes() * 3, max_batches=2)
    peak = []
    ex = FakeExecutor(polls=3, budget_probe=lambda: peak.append(adm.used))
    b = Batcher(ex, adm, max_batch_alerts=2500, clock=Clock())
    rng = np.random.default_rng(0)
    reqs = [_req(i, int(rng.integers(1, 1200))) for i in range(40)]
    for r in reqs:
        b.submit(r)
    b.drain()
    assert all(r.status == "done" for r in reqs)
    assert max(peak) <= adm.budget
    assert adm.used == 0 and adm.batches == 0
    assert all(len(h["batch"]) >= 1 for h in ex.launched)
    assert all(sum(r.m for r in h["batch"]) <= 2500 or len(h["batch"]) == 1 for h in ex.launched)
    # first come, first admitted
    order = [r.rid for h in ex.launched for r in h["batch"]]
    assert order == sorted(order)


def test_requests_larger_than_the_budget_are_rejected():
    adm = Admission(budget_bytes=_req(0, 100).device_bytes(), max_batches=1)
    b = Batcher(FakeExecutor(polls=1), adm, clock=Clock())
    big, small = _req(0, 101), _req(1, 100)
    b.submit(big)
    b.submit(small)
    b.drain()
    assert big.status == "rejected" and small.status == "done"


def test_batches_in_flight_are_capped_and_later_arrivals_join_later_batches():
    adm = Admission(budget_bytes=1 << 30, max_batches=2)
    ex = FakeExecutor(polls=5)
    b = Batcher(ex, adm, clock=Clock())
    for i in range(4):
        b.submit(_req(i, 10))
    b.step()                                   # batch 1 takes all four waiting
    assert len(ex.launched) == 1 and len(ex.launched[0]["batch"]) == 4
    for i in range(4, 6):
        b.submit(_req(i, 10))
    b.step()                                   # batch 2 while batch 1 is still running
    assert len(ex.launched) == 2 and adm.batches == 2
    b.submit(_req(6, 10))
    b.step()                                   # both slots busy: request 6 waits
    assert len(ex.launched) == 2 and len(b.waiting) == 1
    b.drain()
    assert len(ex.launched) == 3 and [r.rid for r in ex.launched[2]["batch"]] == [6]
    assert all(r.done >= r.arrival for r in b.finished)
