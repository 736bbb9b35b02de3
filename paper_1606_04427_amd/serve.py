"""Request loop for camera-view renders of one particle set resident in HBM.

Continuous batching: requests queue as they arrive.  Each of `n_workers`
workers owns one library context and one HIP stream.  Whenever a worker is
free it takes, in arrival order, the queued requests that fit its view-slot
limit and the memory budget (the head of the queue waits when it does not
fit), renders them with one `spl_render_batch` call and releases their memory
as soon as the images are ready.  With two or more workers, requests admitted
while another batch is on the GPU run beside it on the device.

The scheduler is independent of the GPU: it drives any executor with a
`run(requests) -> (images, stats)` method, so its admission and ordering logic
is tested on the CPU with a fake executor.
"""
from __future__ import annotations

import collections
import math
import threading
import time
from dataclasses import dataclass, field

import numpy as np

MiB = 1 << 20


@dataclass
class Request:
    rid: int
    pose: object          # synth.Pose (camera and image size)
    mode: int             # spl_mode
    look: int = 0         # index into the executor's bank of looks
    arrival: float = math.nan    # server clock, s
    admitted: float = math.nan
    done: float = math.nan
    batch: int = -1       # sequence number of the batch that rendered it
    worker: int = -1
    cost: int = 0         # bytes reserved while in flight
    image: object = None
    stats: dict | None = None
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def request_bytes(n_particles: int, width: int, height: int, sorted_mode: bool) -> int:
    """Device bytes one view holds while in flight: its image plus the
    per-view workspace (32 B record and 8 B span per particle, list entries;
    sorted views also hold depth records and two key buffers)."""
    img = 12 * width * height
    ws = n_particles * (32 + 8 + 8) + 4 * MiB
    if sorted_mode:
        ws += n_particles * (8 + 2 * 16)
    return img + ws


class Server:
    """Continuous-batching request loop (see the module docstring).

    make_executor(worker_index) is called once in each worker thread.
    cost(request) gives the bytes a request reserves; budget_bytes bounds
    their sum over requests in flight.  keep(request) decides whether the
    image is kept on the request after completion (dropping it frees device
    memory at once)."""

    def __init__(self, make_executor, n_workers: int = 2, budget_bytes: int = 64 << 30,
                 max_views: int = 16, cost=None, keep=None, clock=time.perf_counter):
        if n_workers < 1 or max_views < 1 or budget_bytes <= 0:
            raise ValueError("n_workers, max_views and budget_bytes must be positive")
        self.make_executor = make_executor
        self.n_workers = n_workers
        self.budget = int(budget_bytes)
        self.max_views = max_views
        self.cost = cost or (lambda r: request_bytes(0, r.pose.width, r.pose.height, False))
        self.keep = keep or (lambda r: True)
        self.clock = clock
        self.queue: collections.deque[Request] = collections.deque()
        self.cv = threading.Condition()
        self.reserved = 0
        self.peak_reserved = 0
        self.in_flight = 0
        self.n_batches = 0
        self.completed: list[Request] = []
        self.stopping = False
        self.threads: list[threading.Thread] = []
        self.errors: list[BaseException] = []
        self.ready = threading.Barrier(n_workers + 1)

    # -- public ---------------------------------------------------------------
    def start(self):
        for w in range(self.n_workers):
            t = threading.Thread(target=self._worker, args=(w,), daemon=True)
            t.start()
            self.threads.append(t)
        self.ready.wait()  # every executor is built before the first arrival
        if self.errors:
            raise RuntimeError(f"worker failed to start: {self.errors[0]!r}")
        return self

    def submit(self, r: Request):
        r.cost = int(self.cost(r))
        if math.isnan(r.arrival):
            r.arrival = self.clock()
        with self.cv:
            if r.cost > self.budget:
                r.error = f"request needs {r.cost} B, more than the {self.budget} B budget"
                r.done = self.clock()
                self.completed.append(r)
                self.cv.notify_all()
                return
            self.queue.append(r)
            self.cv.notify_all()

    def wait(self, requests, timeout: float = 600.0):
        """Waits until every request in `requests` has completed."""
        end = time.monotonic() + timeout
        with self.cv:
            while True:
                left_n = sum(1 for r in requests if math.isnan(r.done))
                if left_n == 0:
                    return
                if self.errors:
                    raise RuntimeError(f"worker failed: {self.errors[0]!r}")
                left = end - time.monotonic()
                if left <= 0:
                    raise TimeoutError(f"{left_n} of {len(requests)} requests not done")
                self.cv.wait(min(left, 1.0))

    def stop(self):
        with self.cv:
            self.stopping = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()
        if self.errors:
            raise RuntimeError(f"worker failed: {self.errors[0]!r}")

    # -- scheduling -------------------------------------------------------------
    def _take(self) -> list[Request]:
        """Admits queued requests in arrival order; caller holds the lock."""
        batch = []
        while self.queue and len(batch) < self.max_views:
            r = self.queue[0]
            if self.reserved + r.cost > self.budget:
                break
            self.queue.popleft()
            self.reserved += r.cost
            batch.append(r)
        self.peak_reserved = max(self.peak_reserved, self.reserved)
        return batch

    def _worker(self, w: int):
        try:
            ex = self.make_executor(w)
        except BaseException as e:  # reported by start()
            self.errors.append(e)
            self.ready.wait()
            return
        self.ready.wait()
        try:
            while True:
                with self.cv:
                    while True:
                        if self.errors:
                            return
                        batch = self._take()
                        if batch or (self.stopping and not self.queue):
                            break
                        self.cv.wait()
                    if not batch:
                        return
                    seq = self.n_batches
                    self.n_batches += 1
                    self.in_flight += len(batch)
                t = self.clock()
                for r in batch:
                    r.admitted, r.batch, r.worker = t, seq, w
                try:
                    images, stats = ex.run(batch)
                    err = None
                except Exception as e:  # a failed batch fails its requests only
                    images, stats, err = [None] * len(batch), [None] * len(batch), repr(e)
                t = self.clock()
                for r, im, st in zip(batch, images, stats):
                    r.stats = st
                    r.error = err
                    r.image = im if self.keep(r) else None
                with self.cv:
                    for r in batch:
                        r.done = t
                    self.reserved -= sum(r.cost for r in batch)
                    self.in_flight -= len(batch)
                    self.completed.extend(batch)
                    self.cv.notify_all()
        except BaseException as e:
            with self.cv:
                self.errors.append(e)
                self.cv.notify_all()
        finally:
            close = getattr(ex, "close", None)
            if close:
                close()


def one_per_call(executor, requests, arrivals=None, clock=time.perf_counter, keep=None):
    """The plain path: one request per call, in arrival order, on one stream,
    each finished before the next starts."""
    keep = keep or (lambda r: True)
    t0 = clock()
    for k, r in enumerate(requests):
        r.arrival = t0 + (0.0 if arrivals is None else float(arrivals[k]))
        now = clock()
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.admitted = clock()
        images, stats = executor.run([r])
        r.done = clock()
        r.image = images[0] if keep(r) else None
        r.stats = stats[0]
        r.batch, r.worker = k, 0
    return requests


def drive(server: Server, requests, arrivals, clock=time.perf_counter):
    """Submits requests at t0 + arrivals[k] (open loop) and waits for all."""
    t0 = clock()
    for k, r in enumerate(requests):
        r.arrival = t0 + float(arrivals[k])
        now = clock()
        if r.arrival > now:
            time.sleep(r.arrival - now)
        server.submit(r)
    server.wait(requests)
    return requests


def summary(requests) -> dict:
    """Latency percentiles (ms) and throughput of completed requests."""
    ok = [r for r in requests if r.error is None]
    if not ok:
        return {"n": 0}
    lat = np.array([r.latency for r in ok]) * 1e3
    span = max(r.done for r in ok) - min(r.arrival for r in ok)
    return {"n": len(ok), "failed": len(requests) - len(ok),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "frames_per_s": len(ok) / span if span > 0 else math.inf}


class GpuExecutor:
    """Renders batches through the HIP library on its own context and stream.

    bank: list of (Palettes, looks) pairs, indexed by Request.look."""

    def __init__(self, parts, bank, device: str = "cuda:0", batch_bytes: int | None = None,
                 graphs: bool = False):
        import torch

        from . import binding as B

        self.B = B
        self.parts = parts
        self.bank = bank
        self.ctx = B.Context(torch.device(device).index or 0)
        self.stream = torch.cuda.Stream(device=device)
        if batch_bytes is not None:
            self.ctx.spl_set_option(B.SPL_OPT_BATCH_BYTES, int(batch_bytes))
        self.ctx.spl_set_option(B.SPL_OPT_GRAPHS, int(graphs))
        self._params = {}

    def params(self, mode, look):
        key = (mode, look)
        if key not in self._params:
            pals, looks = self.bank[look]
            self._params[key] = self.B.make_params(mode, pals, looks)
        return self._params[key]

    def run(self, reqs):
        import torch

        with torch.cuda.stream(self.stream):
            outs, sts = self.ctx.spl_render_batch(self.parts, [r.pose for r in reqs],
                                                  [self.params(r.mode, r.look) for r in reqs])
        self.stream.synchronize()
        return outs, sts

    def close(self):
        self.stream.synchronize()
        self.ctx.close()
