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


def test_request_cost_model():
    """Image and workspace terms of one view: records, spans and list entries
    grow with the particle count, the composite's partial tiles with the
    list entries (sorted mode and the deterministic additive order)."""
    n, w, h = 100_000, 64, 32
    img, ws = serve.request_cost(n, w, h, False)
    entries = 2 * n
    items = entries // 1024 + 4 * 2
    assert img == 12 * w * h
    assert ws == n * 40 + 4 * entries + 16 * items + 16 * 8 + 4 * serve.MiB
    img2, ws2 = serve.request_cost(n, w, h, True)
    assert img2 == img
    assert ws2 - ws == n * 8 + 16 * entries + items * 16 * 16 * 16
    # additive in the deterministic list order: the keys and partial tiles of
    # the ordered walk, no depth record
    img3, ws3 = serve.request_cost(n, w, h, False, ordered=True)
    assert img3 == img and ws3 - ws == 16 * entries + items * 16 * 16 * 16
    # more entries per particle, more workspace
    assert serve.request_cost(n, w, h, False, entries_per_particle=4.0)[1] > ws
    assert serve.request_bytes(n, w, h, False) == img + ws


class LedgerExecutor:
    """Fake executor whose context holds workspace like the library's: it
    grows to the largest batch it rendered and is released by trim().  A
    shared ledger sums the workspace of every executor and the images of the
    requests it is rendering, so the test can check the budget at every
    moment."""

    def __init__(self, ledger, lock, per_batch=0.003):
        self.ledger, self.lock, self.per_batch = ledger, lock, per_batch
        self.held = 0

    def _note(self, delta):
        with self.lock:
            self.ledger["now"] += delta
            self.ledger["peak"] = max(self.ledger["peak"], self.ledger["now"])

    def run(self, reqs):
        need = sum(r.ws_bytes for r in reqs)
        img = sum(r.img_bytes for r in reqs)
        grow = max(need - self.held, 0)
        self._note(grow + img)
        self.held += grow
        time.sleep(self.per_batch)
        self._note(-img)
        return [None] * len(reqs), [{}] * len(reqs)

    def workspace_bytes(self):
        return self.held

    def trim(self):
        self._note(-self.held)
        self.held = 0
        with self.lock:
            self.ledger["trims"] += 1


@pytest.mark.parametrize("n_workers", [1, 2, 3])
def test_held_workspace_counts_against_the_budget(n_workers):
    """Requests with large and small workspace, a budget that holds one large
    view and a bit more: the images in flight plus every context's held workspace
    never exceed the budget, workers release workspace when the head of the
    queue does not fit, and every request completes (no deadlock)."""
    ledger, lock = {"now": 0, "peak": 0, "trims": 0}, threading.Lock()
    big, small = (1000, 40_000), (100, 4_000)
    costs = {}
    reqs = []
    for k in range(60):
        r = serve.Request(k, synth.Pose((0, 0, 2), (0, 0, 0), (0, 1, 0), 50.0, 0.01, 8, 8), 1)
        costs[k] = big if k % 5 == 0 else small
        reqs.append(r)
    budget = sum(big) + 25_000
    srv = serve.Server(lambda w: LedgerExecutor(ledger, lock), n_workers=n_workers,
                       budget_bytes=budget, max_views=4, cost=lambda r: costs[r.rid]).start()
    serve.drive(srv, reqs, np.zeros(len(reqs)))
    srv.stop()
    assert all(r.error is None for r in reqs)
    assert ledger["peak"] <= budget
    assert srv.peak_reserved <= budget
    assert srv.n_trims == ledger["trims"]


def test_workers_release_workspace_so_the_head_can_run():
    """Two workers each keep 30k of workspace from a request they rendered at
    the same time; the next request needs 45k, which fits the budget alone but
    not beside the other worker's held workspace: the worker that finds the
    head blocked releases its own, and the request runs on whichever worker
    then has room."""
    ledger, lock = {"now": 0, "peak": 0, "trims": 0}, threading.Lock()
    pose = synth.Pose((0, 0, 2), (0, 0, 0), (0, 1, 0), 50.0, 0.01, 8, 8)
    reqs = [serve.Request(k, pose, 1) for k in range(3)]
    costs = {0: (500, 30_000), 1: (500, 30_000), 2: (1000, 45_000)}
    budget = 71_000
    srv = serve.Server(lambda w: LedgerExecutor(ledger, lock, per_batch=0.05), n_workers=2,
                       budget_bytes=budget, max_views=1, cost=lambda r: costs[r.rid]).start()
    serve.drive(srv, reqs, np.array([0.0, 0.0, 0.01]))
    srv.stop()
    assert all(r.error is None for r in reqs)
    assert reqs[0].worker != reqs[1].worker
    assert srv.n_trims == ledger["trims"] >= 1
    assert ledger["peak"] <= budget


def test_a_request_larger_than_the_budget_with_workspace_is_rejected():
    ledger, lock = {"now": 0, "peak": 0, "trims": 0}, threading.Lock()
    srv = serve.Server(lambda w: LedgerExecutor(ledger, lock), n_workers=1, budget_bytes=1000,
                       cost=lambda r: (400, 700)).start()
    r = serve.Request(0, synth.Pose((0, 0, 2), (0, 0, 0), (0, 1, 0), 50.0, 0.01, 8, 8), 1)
    serve.drive(srv, [r], np.zeros(1))
    srv.stop()
    assert r.error and "budget" in r.error


class EachExecutor:
    """Fake executor that renders view by view and reports each request as
    it completes; fails at request fail_on."""

    def __init__(self, per_view=0.01, fail_on=None):
        self.per_view, self.fail_on = per_view, fail_on

    def run_each(self, reqs, done):
        for r in reqs:
            if r.rid == self.fail_on:
                raise RuntimeError("injected")
            time.sleep(self.per_view)
            done(r, f"img{r.rid}", {"rid": r.rid})


def test_requests_complete_one_by_one_inside_a_batch():
    srv = serve.Server(lambda w: EachExecutor(), n_workers=1, max_views=8).start()
    reqs = _reqs(6)
    serve.drive(srv, reqs, np.zeros(6))
    srv.stop()
    assert all(r.image == f"img{r.rid}" for r in reqs)
    one_batch = [r for r in reqs if r.batch == reqs[-1].batch]
    assert len(one_batch) > 2
    done = [r.done for r in one_batch]
    assert done == sorted(done) and done[-1] - done[0] >= 0.01 * (len(one_batch) - 1) * 0.9
    assert srv.reserved == 0 and srv.in_flight == 0


def test_a_failure_inside_a_batch_fails_only_the_unfinished_requests():
    srv = serve.Server(lambda w: EachExecutor(per_view=0.002, fail_on=3), n_workers=1,
                       max_views=8).start()
    reqs = _reqs(6)
    serve.drive(srv, reqs, np.zeros(6))
    srv.stop()
    batch_of_3 = reqs[3].batch
    for r in reqs:
        if r.batch == batch_of_3 and r.rid >= 3:
            assert r.error and "injected" in r.error
        else:
            assert r.error is None and r.image == f"img{r.rid}"
    assert srv.reserved == 0 and srv.in_flight == 0
