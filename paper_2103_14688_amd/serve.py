"""Continuous-batching query server over resident graphs.

Requests (a graph id and a compiled query) arrive at any time.  The server
keeps every graph resident in HBM and admits a request when an execution slot
is free and its estimated device footprint fits the memory budget:

  * small requests (graphs the fused kernel takes) that are waiting when a
    slot frees up are launched together as one batch: one persistent launch
    in which each workgroup drains queries from a device queue;
  * other requests run on their own slot, each slot a separate HIP stream,
    so several queries' launches overlap on the device.

Requests that arrive while others run join at the next free slot; nothing
waits for a whole batch to finish.  The "plain" mode is the baseline: one
request at a time, in arrival order, each a separate cfpq_query call.

The scheduling logic is backend-independent; ``GpuBackend`` runs requests
through the C ABI, tests substitute a fake backend.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

FUSED_MAX_N = 2048          # cfpq fused strategy limit (graph vertices)
FUSED_MAX_BOXES = 64


@dataclass
class Request:
    rid: int
    graph: object            # backend graph handle
    query: object            # backend query handle
    n: int
    n_states: int
    n_boxes: int
    arrival: float = 0.0     # seconds on the server clock
    start: float = -1.0
    done: float = -1.0
    result: object = None    # (pairs, hash, iterations)
    error: str = ""
    batched: bool = False

    @property
    def latency(self):
        return self.done - self.arrival


def footprint(n, n_states, n_boxes):
    """Estimated device bytes of one query: closure rows, two frontiers,
    nonterminal matrices and their deltas (bit-packed, padded rows)."""
    pn = (n + 63) // 64
    words = (pn + 7) // 8 * 8 if pn <= 8 else (pn + 15) // 16 * 16
    return 8 * n * words * (3 * n_states + 2 * n_boxes) + (1 << 22)


def is_small(r):
    return r.n <= FUSED_MAX_N and r.n_boxes <= FUSED_MAX_BOXES


class Server:
    def __init__(self, backend, mode="batched", slots=4, budget=64 << 30, batch_max=512):
        assert mode in ("batched", "plain")
        self.backend = backend
        self.mode = mode
        self.slots = 1 if mode == "plain" else slots
        self.budget = budget
        self.batch_max = batch_max
        self.cv = threading.Condition()
        self.pending = []          # arrived, not admitted
        self.in_use = 0            # bytes admitted
        self.busy = 0              # slots running
        self.finished = []
        self.closed = False
        self.t0 = time.perf_counter()
        self.max_concurrent = 0
        self.batches = 0
        self.workers = [threading.Thread(target=self._worker, args=(i,), daemon=True) for i in range(self.slots)]
        for w in self.workers:
            w.start()

    def now(self):
        return time.perf_counter() - self.t0

    def submit(self, req):
        with self.cv:
            req.arrival = self.now() if req.arrival <= 0 else req.arrival
            if footprint(req.n, req.n_states, req.n_boxes) > self.budget:
                req.error = "rejected: footprint exceeds the memory budget"
                req.done = self.now()
                self.finished.append(req)
                self.cv.notify_all()
                return req
            self.pending.append(req)
            self.cv.notify_all()
        return req

    def _take(self):
        """Pick work for a free slot: a batch of waiting small requests, or the
        oldest request that fits the memory budget.  Called with the lock held."""
        if not self.pending:
            return None
        head = self.pending[0]
        if self.mode == "batched" and is_small(head):
            batch, used = [], 0
            for r in self.pending:
                if not is_small(r) or len(batch) >= self.batch_max:
                    continue
                fp = footprint(r.n, r.n_states, r.n_boxes)
                if self.in_use + used + fp > self.budget:
                    break
                batch.append(r)
                used += fp
            if batch:
                for r in batch:
                    self.pending.remove(r)
                    r.batched = True
                self.in_use += used
                return batch, used
            return None
        fp = footprint(head.n, head.n_states, head.n_boxes)
        if self.in_use + fp > self.budget and self.busy > 0:
            return None                      # wait for memory to free up
        self.pending.pop(0)
        self.in_use += fp
        return [head], fp

    def _worker(self, slot):
        stream = self.backend.make_stream(slot)
        while True:
            with self.cv:
                while True:
                    if self.closed and not self.pending:
                        return
                    got = self._take()
                    if got is not None:
                        break
                    self.cv.wait(0.05)
                batch, fp = got
                self.busy += 1
                self.max_concurrent = max(self.max_concurrent, self.busy)
                if len(batch) > 1:
                    self.batches += 1
            t = self.now()
            for r in batch:
                r.start = t
            try:
                if len(batch) > 1 or batch[0].batched:
                    outs = self.backend.run_batch(batch, stream)
                else:
                    outs = [self.backend.run_one(batch[0], stream)]
                err = ""
            except Exception as e:  # report, never lose a request
                outs, err = [None] * len(batch), repr(e)
            t = self.now()
            with self.cv:
                for r, o in zip(batch, outs):
                    r.result, r.error, r.done = o, err, t
                    self.finished.append(r)
                self.in_use -= fp
                self.busy -= 1
                self.cv.notify_all()

    def drain(self, timeout=None):
        """Wait until every submitted request has finished."""
        end = None if timeout is None else time.perf_counter() + timeout
        with self.cv:
            while self.pending or self.busy:
                left = None if end is None else end - time.perf_counter()
                if left is not None and left <= 0:
                    raise TimeoutError("server did not drain")
                self.cv.wait(0.05 if left is None else min(left, 0.05))

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for w in self.workers:
            w.join()


def replay(server, requests, arrivals, report=None, every=1000):
    """Submit requests at the given arrival offsets (seconds) and wait for all;
    report(k), if given, runs after every `every` submissions."""
    t0 = server.now()
    for i, (r, a) in enumerate(zip(requests, arrivals)):
        delay = t0 + a - server.now()
        if delay > 0:
            time.sleep(delay)
        r.arrival = t0 + a
        server.submit(r)
        if report and (i + 1) % every == 0:
            report(i + 1)
    server.drain()
    return requests


def percentiles(latencies, ps=(50, 99)):
    xs = sorted(latencies)
    if not xs:
        return {p: None for p in ps}
    out = {}
    for p in ps:
        k = max(0, min(len(xs) - 1, int(round(p / 100.0 * (len(xs) - 1)))))
        out[p] = xs[k]
    return out


class GpuBackend:
    """Runs requests through the C ABI on the current device."""

    def __init__(self):
        from . import cfpq
        self.cfpq = cfpq
        self.streams = {}

    def make_stream(self, slot):
        # one stream per slot index for the backend's lifetime: the caching
        # allocator keeps freed blocks per stream, so servers that came and
        # went on fresh streams would strand their cached memory
        import torch
        torch.cuda.set_device(0)
        if slot not in self.streams:
            self.streams[slot] = torch.cuda.Stream()   # default priority
        return self.streams[slot]

    def _summ(self, res):
        it, _, _ = res.stats()
        out = (res.count(0), res.hash(0), it)
        res.close()
        return out

    def run_one(self, r, stream):
        import torch
        with torch.cuda.stream(stream):
            res = self.cfpq.query(r.graph, r.query, stream=stream.cuda_stream)
            return self._summ(res)

    def run_batch(self, rs, stream):
        import torch
        with torch.cuda.stream(stream):
            res = self.cfpq.query_batch([r.graph for r in rs], [r.query for r in rs], stream=stream.cuda_stream)
            return [self._summ(x) for x in res]
