"""Scheduler of the request loop, driven by a fake executor on the CPU:
admission by memory and view slots, arrival order, overlap of batches on
several workers, failure isolation and latency bookkeeping."""
import math
import threading
import time

import numpy as np
import pytest

from paper_1606_04427_amd import serve, synth


class FakeExecutor:
    """Sleeps a fixed time per batch plus a time per view and records what
    was in flight when each batch started."""

    def __init__(self, log, lock, per_batch=0.004, per_view=0.001, fail_on=None):
        self.log, self.lock = log, lock
        self.per_batch, self.per_view = per_batch, per_view
        self.fail_on = fail_on

    def run(self, reqs):
        with self.lock:
            self.log.append(("start", time.perf_counter(), [r.rid for r in reqs]))
        if self.fail_on is not None and any(r.rid == self.fail_on for r in reqs):
            raise RuntimeError("injected")
        time.sleep(self.per_batch + self.per_view * len(reqs))
        with self.lock:
            self.log.append(("end", time.perf_counter(), [r.rid for r in reqs]))
        return [f"img{r.rid}" for r in reqs], [{"rid": r.rid} for r in reqs]


def _reqs(n, sizes=(64, 128, 256)):
    poses = [synth.Pose((0, 0, 2), (0, 0, 0), (0, 1, 0), 50.0, 0.01, s, s)
             for s in sizes]
    return [serve.Request(k, poses[k % len(poses)], 1) for k in range(n)]


def _server(log, lock, **kw):
    ex_kw = {k: kw.pop(k) for k in ("per_batch", "per_view", "fail_on") if k in kw}
    return serve.Server(lambda w: FakeExecutor(log, lock, **ex_kw), **kw)


def test_every_request_completes_with_its_own_result():
    log, lock = [], threading.Lock()
    srv = _server(log, lock, n_workers=2, max_views=4).start()
    reqs = _reqs(40)
    serve.drive(srv, reqs, np.linspace(0, 0.05, len(reqs)))
    srv.stop()
    assert all(r.image == f"img{r.rid}" and r.stats["rid"] == r.rid for r in reqs)
    assert all(r.arrival <= r.admitted <= r.done for r in reqs)
    assert sorted(r.rid for r in srv.completed) == list(range(40))


def test_memory_budget_is_never_exceeded():
    log, lock = [], threading.Lock()
    cost = lambda r: 12 * r.pose.width * r.pose.height
    budget = cost(_reqs(3)[2]) + cost(_reqs(3)[1])  # one 256^2 and one 128^2 at a time
    srv = _server(log, lock, n_workers=3, max_views=8, budget_bytes=budget, cost=cost).start()
    reqs = _reqs(30)
    serve.drive(srv, reqs, np.zeros(len(reqs)))
    srv.stop()
    assert srv.peak_reserved <= budget
    assert srv.reserved == 0 and srv.in_flight == 0
    # replay the log: bytes of batches running at once never exceed the budget
    by = {r.rid: r.cost for r in reqs}
    live, worst = 0, 0
    for kind, _, rids in sorted(log, key=lambda e: (e[1], e[0] == "start")):
        live += sum(by[i] for i in rids) * (1 if kind == "start" else -1)
        worst = max(worst, live)
    assert worst <= budget


def test_admission_is_in_arrival_order():
    log, lock = [], threading.Lock()
    srv = _server(log, lock, n_workers=1, max_views=3).start()
    reqs = _reqs(20)
    serve.drive(srv, reqs, np.zeros(len(reqs)))
    srv.stop()
    order = [rid for kind, _, rids in log if kind == "start" for rid in rids]
    assert order == list(range(20))
    assert max(len(rids) for kind, _, rids in log if kind == "start") <= 3


def test_requests_arriving_during_a_batch_are_batched_together():
    """Continuous batching: while one batch runs, arrivals accumulate and the
    next free worker takes them as one batch."""
    log, lock = [], threading.Lock()
    srv = _server(log, lock, n_workers=1, max_views=16, per_batch=0.05, per_view=0.0).start()
    reqs = _reqs(9)
    serve.drive(srv, reqs, np.array([0.0] + [0.005 * k for k in range(1, 9)]))
    srv.stop()
    starts = [rids for kind, _, rids in log if kind == "start"]
    assert starts[0] == [0] and starts[1] == list(range(1, 9))


def test_batches_overlap_on_several_workers():
    log, lock = [], threading.Lock()
    srv = _server(log, lock, n_workers=2, max_views=1, per_batch=0.03, per_view=0.0).start()
    reqs = _reqs(2)
    serve.drive(srv, reqs, np.zeros(2))
    srv.stop()
    (s0, s1) = [t for kind, t, _ in log if kind == "start"]
    (e0, e1) = [t for kind, t, _ in log if kind == "end"]
    assert max(s0, s1) < min(e0, e1)  # both ran at once


def test_oversized_request_is_rejected_not_deadlocked():
    log, lock = [], threading.Lock()
    cost = lambda r: 12 * r.pose.width * r.pose.height
    srv = _server(log, lock, n_workers=1, budget_bytes=cost(_reqs(2)[1]), cost=cost).start()
    reqs = _reqs(3)  # the 256^2 one does not fit
    serve.drive(srv, reqs, np.zeros(3))
    srv.stop()
    assert reqs[2].error and "budget" in reqs[2].error
    assert reqs[0].error is None and reqs[1].error is None


def test_failed_batch_fails_only_its_requests():
    log, lock = [], threading.Lock()
    srv = _server(log, lock, n_workers=1, max_views=1, fail_on=3).start()
    reqs = _reqs(6)
    serve.drive(srv, reqs, np.zeros(6))
    srv.stop()
    assert reqs[3].error and "injected" in reqs[3].error
    assert all(r.error is None for r in reqs if r.rid != 3)


def test_executor_construction_failure_is_reported():
    def bad(w):
        raise RuntimeError("no device")

    with pytest.raises(RuntimeError, match="no device"):
        serve.Server(bad, n_workers=2).start()


def test_one_per_call_baseline_and_summary():
    log, lock = [], threading.Lock()
    ex = FakeExecutor(log, lock, per_batch=0.002, per_view=0.0)
    reqs = serve.one_per_call(ex, _reqs(10), np.zeros(10))
    s = serve.summary(reqs)
    assert s["n"] == 10 and s["failed"] == 0
    # FIFO, one at a time: the k-th request waits for the k before it
    lat = [r.latency for r in reqs]
    assert all(b >= a for a, b in zip(lat, lat[1:]))
    assert s["p99_ms"] >= s["p50_ms"] >= 2.0 * 0.9
    assert 0 < s["frames_per_s"] <= 1.0 / 0.002 * 1.1


def test_request_bytes_model():
    a = serve.request_bytes(1000, 64, 32, False)
    b = serve.request_bytes(1000, 64, 32, True)
    assert a == 12 * 64 * 32 + 1000 * 48 + 4 * serve.MiB
    assert b > a
