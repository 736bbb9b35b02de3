"""Request loop for camera-view renders of one particle set resident in HBM.

Continuous batching: requests queue as they arrive.  Each of `n_workers`
workers owns one library context and one HIP stream.  Whenever a worker is
free it takes, in arrival order, the queued requests that fit its view-slot
limit and the memory budget (the head of the queue waits when it does not
fit), renders them (one batched call for a set small enough that one view
does not fill the device, else view by view with each request completed as
its image is ready) and releases their memory as soon as the images are
ready.  With two or more workers, requests admitted while another batch is on
the GPU run beside it on the device.

The scheduler is independent of the GPU: it drives any executor with a
`run(requests) -> (images, stats)` method, so its admission and ordering logic
is tested on the CPU with a fake executor.
"""
from __future__ import annotations

import collections
import math
import threading
import time
from dataclasses import dataclass

import numpy as np

MiB = 1 << 20


@dataclass
class Request:
    rid: int
    pose: object          # synth.Pose (camera and image size)
    mode: int             # spl_mode
    look: int = 0         # index into the executor's bank of looks
    deterministic: bool = False  # additive modes: the bit-identical list order
    arrival: float = math.nan    # server clock, s
    admitted: float = math.nan
    done: float = math.nan
    batch: int = -1       # sequence number of the batch that rendered it
    worker: int = -1
    cost: int = 0         # image + workspace bytes
    img_bytes: int = 0    # image bytes, held until the request completes
    ws_bytes: int = 0     # workspace bytes it adds to its worker's context
    image: object = None
    stats: dict | None = None
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def request_cost(n_particles: int, width: int, height: int, sorted_mode: bool,
                 entries_per_particle: float = 2.0, tile: int = 16,
                 ordered: bool = False) -> tuple[int, int]:
    """Device bytes of one view: (image, workspace).

    The image (12 B per pixel) is held from admission until the request
    completes.  The workspace is what the view adds to its worker's library
    context while it renders, and the context keeps it for later batches:
    a 32 B record and an 8 B span per particle, 4 B per tile-list entry
    (about entries_per_particle entries per particle), a 16 B work item per
    1024 entries and per tile, counts, offsets and cursors (16 B per tile) and
    fixed buffers (4 MiB).  Views drawn in list order (sorted, or additive
    with ordered = True) add two 8 B sort keys per entry and the composite's
    partial tiles (16 B per pixel of each work item's tile); sorted views also
    an 8 B depth record per particle."""
    img = 12 * width * height
    tiles = -(-width // tile) * -(-height // tile)
    entries = int(entries_per_particle * n_particles)
    items = entries // 1024 + tiles
    ws = n_particles * (32 + 8) + 4 * entries + 16 * items + 16 * tiles + 4 * MiB
    if sorted_mode or ordered:
        ws += 16 * entries + items * tile * tile * 16
    if sorted_mode:
        ws += n_particles * 8
    return img, ws


def request_bytes(n_particles: int, width: int, height: int, sorted_mode: bool, **kw) -> int:
    """Image plus workspace of one view (request_cost summed)."""
    img, ws = request_cost(n_particles, width, height, sorted_mode, **kw)
    return img + ws


class Server:
    """Continuous-batching request loop (see the module docstring).

    make_executor(worker_index) is called once in each worker thread.
    cost(request) gives either the bytes a request holds until it completes,
    or a pair (image bytes, workspace bytes).  Device memory is accounted as
    the images of requests in flight plus the workspace every worker's
    context holds (an executor with workspace_bytes() reports it after each
    batch; otherwise the largest workspace estimate of its batches is used),
    and budget_bytes bounds that sum.  A worker that is idle and cannot admit
    the head of the queue because of held workspace releases its own (the
    executor's trim(), if it has one) and tells the other workers, which then
    do the same, so the head always runs eventually.  keep(request) decides
    whether the image is kept on the request after completion (dropping it
    frees device memory at once).  max_views bounds a batch: a request that
    arrives as a batch starts waits for all of it, so small batches keep the
    tail latency down (at 100M particles, 4 views gave a p99 of about 90 ms at
    full load against about 150 ms with 8 or 16, for the same throughput)."""

    def __init__(self, make_executor, n_workers: int = 2, budget_bytes: int = 64 << 30,
                 max_views: int = 4, cost=None, keep=None, clock=time.perf_counter):
        if n_workers < 1 or max_views < 1 or budget_bytes <= 0:
            raise ValueError("n_workers, max_views and budget_bytes must be positive")
        self.make_executor = make_executor
        self.n_workers = n_workers
        self.budget = int(budget_bytes)
        self.max_views = max_views
        self.cost = cost or (lambda r: request_cost(0, r.pose.width, r.pose.height, False))
        self.keep = keep or (lambda r: True)
        self.clock = clock
        self.queue: collections.deque[Request] = collections.deque()
        self.cv = threading.Condition()
        self.reserved = 0          # images of requests in flight
        self.held = [0] * n_workers  # workspace each worker's context holds
        self.planned = [0] * n_workers  # workspace a running batch may grow to
        self.peak_reserved = 0     # largest images + workspace accounted at once
        self.in_flight = 0
        self.n_batches = 0
        self.n_trims = 0
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
        c = self.cost(r)
        r.img_bytes, r.ws_bytes = (int(c[0]), int(c[1])) if isinstance(c, tuple) else (int(c), 0)
        r.cost = r.img_bytes + r.ws_bytes
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
    def _accounted(self, w: int, extra_img: int, ws_w: int) -> int:
        """Bytes in use if worker w's workspace were ws_w and extra_img more
        image bytes were in flight; caller holds the lock."""
        others = sum(max(self.held[v], self.planned[v]) for v in range(self.n_workers) if v != w)
        return self.reserved + extra_img + others + ws_w

    def _take(self, w: int) -> list[Request]:
        """Admits queued requests in arrival order for worker w; caller holds
        the lock."""
        batch, img, ws = [], 0, 0
        while self.queue and len(batch) < self.max_views:
            r = self.queue[0]
            ws_w = max(self.held[w], ws + r.ws_bytes)
            if self._accounted(w, img + r.img_bytes, ws_w) > self.budget:
                break
            self.queue.popleft()
            batch.append(r)
            img += r.img_bytes
            ws += r.ws_bytes
        if batch:
            self.reserved += img
            self.planned[w] = max(self.held[w], ws)
            self.peak_reserved = max(self.peak_reserved, self._accounted(w, 0, self.planned[w]))
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
                        batch = self._take(w)
                        if batch or (self.stopping and not self.queue):
                            break
                        if self.queue and self.held[w] > 0:
                            # the head does not fit beside the workspace the
                            # workers hold: release this worker's and let the
                            # others reconsider
                            trim = getattr(ex, "trim", None)
                            if trim:
                                trim()
                            self.held[w] = 0
                            self.planned[w] = 0
                            self.n_trims += 1
                            self.cv.notify_all()
                            continue
                        self.cv.wait()
                    if not batch:
                        return
                    seq = self.n_batches
                    self.n_batches += 1
                    self.in_flight += len(batch)
                t = self.clock()
                for r in batch:
                    r.admitted, r.batch, r.worker = t, seq, w
                finished = set()

                def done(r, im, st):
                    # a request completes as soon as its image is ready (an
                    # executor that renders view by view reports each one)
                    t_done = self.clock()
                    r.stats = st
                    r.error = None
                    r.image = im if self.keep(r) else None
                    with self.cv:
                        r.done = t_done
                        self.reserved -= r.img_bytes
                        self.in_flight -= 1
                        self.completed.append(r)
                        finished.add(r.rid)
                        self.cv.notify_all()

                try:
                    if getattr(ex, "run_each", None):
                        ex.run_each(batch, done)
                    else:
                        images, stats = ex.run(batch)
                        for r, im, st in zip(batch, images, stats):
                            done(r, im, st)
                    err = None
                except Exception as e:  # a failed batch fails its unfinished requests only
                    err = repr(e)
                held = getattr(ex, "workspace_bytes", None)
                t = self.clock()
                with self.cv:
                    for r in batch:
                        if r.rid in finished:
                            continue
                        r.stats, r.error, r.image, r.done = None, err, None, t
                        self.reserved -= r.img_bytes
                        self.in_flight -= 1
                        self.completed.append(r)
                    self.held[w] = int(held()) if held else self.planned[w]
                    self.planned[w] = 0
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
    """Renders batches through the HIP library on its own context and stream,
    from a data set resident in device memory (binding.Dataset, shared by every
    worker).

    A set of at most `batch_particles` particles renders a batch with one
    batched call (one persistent splat launch for all its views: a view of a
    small set does not fill the device alone).  A larger set renders the
    batch's views one call each and completes every request as soon as its own
    image is ready (run_each): one view of such a set already fills the
    device, so the batched call saves nothing and would hold every result
    until the last view of the batch is done.

    bank: list of (Palettes, looks) pairs, indexed by Request.look."""

    def __init__(self, ds, bank, device: str = "cuda:0", batch_bytes: int | None = None,
                 graphs: bool = False, batch_particles: int = 32_000_000):
        import torch

        from . import binding as B

        self.B = B
        self.ds = ds
        self.bank = bank
        self.ctx = B.Context(torch.device(device).index or 0)
        self.stream = torch.cuda.Stream(device=device)
        if batch_bytes is not None:
            self.ctx.spl_set_option(B.SPL_OPT_BATCH_BYTES, int(batch_bytes))
        self.ctx.spl_set_option(B.SPL_OPT_GRAPHS, int(graphs))
        self._params = {}
        if ds.n > batch_particles:
            self.run_each = self._run_each

    def params(self, mode, look, deterministic=False):
        key = (mode, look, bool(deterministic))
        if key not in self._params:
            pals, looks = self.bank[look]
            self._params[key] = self.B.make_params(mode, pals, looks,
                                                   deterministic=int(bool(deterministic)))
        return self._params[key]

    def run(self, reqs):
        import torch

        with torch.cuda.stream(self.stream):
            if len(reqs) == 1:
                r = reqs[0]
                out, st = self.ctx.spl_render_dataset(self.ds, r.pose, self._prm(r))
                outs, sts = [out], [st]
            else:
                outs, sts = self.ctx.spl_render_batch_dataset(
                    self.ds, [r.pose for r in reqs], [self._prm(r) for r in reqs])
        self.stream.synchronize()
        return outs, sts

    def _run_each(self, reqs, done):
        import torch

        for r in reqs:
            with torch.cuda.stream(self.stream):
                out, st = self.ctx.spl_render_dataset(self.ds, r.pose, self._prm(r))
            self.stream.synchronize()
            done(r, out, st)

    def _prm(self, r):
        return self.params(r.mode, r.look, r.deterministic)

    def workspace_bytes(self) -> int:
        return self.ctx.workspace_bytes()

    def trim(self):
        self.stream.synchronize()
        self.ctx.spl_trim()

    def close(self):
        self.stream.synchronize()
        self.ctx.close()
