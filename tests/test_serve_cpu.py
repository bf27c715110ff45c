"""Scheduling logic of the continuous-batching server, on the CPU with a fake
backend that sleeps instead of computing (no GPU, no oracle)."""
import threading
import time

import pytest

from paper_2103_14688_amd import serve


class FakeBackend:
    def __init__(self, server_ref, per_query=0.01, fail_rid=None):
        self.server_ref = server_ref
        self.per_query = per_query
        self.fail_rid = fail_rid
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.max_in_use = 0
        self.calls = []

    def make_stream(self, slot):
        return slot

    def _enter(self, rs):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            s = self.server_ref[0]
            self.max_in_use = max(self.max_in_use, s.in_use)
            self.calls.append([r.rid for r in rs])

    def _leave(self):
        with self.lock:
            self.running -= 1

    def run_one(self, r, stream):
        self._enter([r])
        try:
            if r.rid == self.fail_rid:
                raise RuntimeError("boom")
            time.sleep(self.per_query * (1 + r.n / 10000))
            return (r.n, r.rid, 1)
        finally:
            self._leave()

    def run_batch(self, rs, stream):
        self._enter(rs)
        try:
            time.sleep(self.per_query)
            return [(r.n, r.rid, 1) for r in rs]
        finally:
            self._leave()


def make(mode, **kw):
    ref = [None]
    fb = FakeBackend(ref, **{k: v for k, v in kw.items() if k in ("per_query", "fail_rid")})
    s = serve.Server(fb, mode=mode, **{k: v for k, v in kw.items() if k in ("slots", "budget", "batch_max")})
    ref[0] = s
    return s, fb


def reqs(ns, states=3, boxes=1):
    return [serve.Request(i, None, None, n, states, boxes) for i, n in enumerate(ns)]


def test_plain_is_one_at_a_time_in_order():
    s, fb = make("plain", per_query=0.002)
    rs = reqs([500, 5000, 700, 50000, 300])
    for r in rs:
        s.submit(r)
    s.drain(timeout=10)
    s.close()
    assert fb.max_running == 1
    assert [c[0] for c in fb.calls] == [0, 1, 2, 3, 4]
    assert all(r.result == (r.n, r.rid, 1) and not r.error for r in rs)
    assert all(r.latency >= 0 for r in rs)


def test_batched_groups_waiting_small_queries():
    s, fb = make("batched", per_query=0.02, slots=1)
    # the first small request occupies the only slot; the rest arrive meanwhile
    rs = reqs([500] * 10)
    s.submit(rs[0])
    time.sleep(0.005)
    for r in rs[1:]:
        s.submit(r)
    s.drain(timeout=10)
    s.close()
    assert len(fb.calls) <= 3
    assert max(len(c) for c in fb.calls) >= 5
    assert sorted(x for c in fb.calls for x in c) == list(range(10))
    assert all(r.batched for r in rs)


def test_large_queries_overlap_on_slots():
    s, fb = make("batched", per_query=0.03, slots=4)
    rs = reqs([50000] * 8)
    for r in rs:
        s.submit(r)
    s.drain(timeout=10)
    s.close()
    assert fb.max_running >= 3
    assert s.max_concurrent >= 3


def test_admission_respects_memory_budget():
    fp = serve.footprint(50000, 3, 1)
    s, fb = make("batched", per_query=0.01, slots=8, budget=2 * fp + 1)
    rs = reqs([50000] * 6)
    for r in rs:
        s.submit(r)
    s.drain(timeout=10)
    s.close()
    assert fb.max_in_use <= 2 * fp + 1
    assert fb.max_running <= 2
    assert all(r.result is not None for r in rs)


def test_oversized_request_is_rejected_not_queued():
    s, fb = make("batched", budget=1 << 20)
    r = reqs([200000])[0]
    s.submit(r)
    s.drain(timeout=5)
    s.close()
    assert r.error.startswith("rejected") and r.result is None


def test_failure_is_reported_and_others_complete():
    s, fb = make("plain", per_query=0.001, fail_rid=2)
    rs = reqs([10000] * 5)
    for r in rs:
        s.submit(r)
    s.drain(timeout=10)
    s.close()
    assert "boom" in rs[2].error
    assert all(r.result is not None for i, r in enumerate(rs) if i != 2)


def test_replay_and_percentiles():
    s, fb = make("batched", per_query=0.002, slots=2)
    rs = reqs([800, 30000] * 5)
    serve.replay(s, rs, [0.001 * i for i in range(len(rs))])
    s.close()
    lat = [r.latency for r in rs]
    p = serve.percentiles(lat)
    assert 0 <= p[50] <= p[99] <= max(lat)
    assert serve.percentiles([]) == {50: None, 99: None}
    assert serve.percentiles([1.0, 2.0, 3.0], (0, 50, 100)) == {0: 1.0, 50: 2.0, 100: 3.0}
