"""Serving-loop scheduling logic with a fake device backend (CPU)."""
import threading
import time

import numpy as np
import pytest

from paper_1207_0486_amd.serve import Request, Server


class FakeEntry:
    """Slots that 'converge' after a per-request number of iterations; the
    'solution' is 2 b, so results are checkable."""

    def __init__(self, key, capacity, nbytes, cost, log):
        self.key, self.capacity, self.nbytes, self.cost, self.log = key, capacity, nbytes, cost, log
        self.slots = {}
        self.closed = False

    def add(self, items):
        for slot, req in items:
            assert slot not in self.slots
            self.slots[slot] = [req, self.cost(req)]
            self.log.append(("add", self.key, slot, time.perf_counter()))

    def advance(self, iterations):
        time.sleep(0.001)
        for s in self.slots.values():
            s[1] -= iterations
        return sum(1 for s in self.slots.values() if s[1] > 0)

    def poll(self):
        states = [0] * self.capacity
        for slot, (_, left) in self.slots.items():
            states[slot] = 2 if left <= 0 else 1
        return states, [None] * self.capacity

    def take(self, slot):
        req, _ = self.slots.pop(slot)
        return 2.0 * req.b, {"slot": slot}

    def close(self):
        self.closed = True


class FakeBackend:
    def __init__(self, sizes, cost):
        self.sizes, self.cost = sizes, cost
        self.opened = []
        self.log = []
        self.lock = threading.Lock()

    def estimate_bytes(self, key, capacity):
        return self.sizes[key]

    def open(self, key, capacity):
        with self.lock:
            self.opened.append(key)
        time.sleep(0.01)  # assembly
        return FakeEntry(key, capacity, self.sizes[key], self.cost, self.log)


def _wait(futs, timeout=10.0):
    return [f.result(timeout=timeout) for f in futs]


def test_results_and_latency_accounting():
    be = FakeBackend({"a": 100, "b": 100}, cost=lambda r: 64)
    srv = Server(be, budget_bytes=1000, capacity=4, chunk=32)
    rng = np.random.default_rng(0)
    reqs = [Request(key="a" if i % 2 else "b", b=rng.standard_normal(5)) for i in range(12)]
    futs = [srv.submit(r) for r in reqs]
    res = _wait(futs)
    srv.close()
    for r, out in zip(reqs, res):
        assert np.array_equal(out.x, 2.0 * r.b) and out.key == r.key and out.latency_s >= 0
    st = srv.stats()
    assert st["completed"] == 12 and st["p50_ms"] <= st["p99_ms"]
    assert sorted(be.opened) == ["a", "b"]  # operators stay resident


def test_admission_by_footprint_and_lru_eviction():
    be = FakeBackend({"a": 400, "b": 400, "c": 400}, cost=lambda r: 32)
    srv = Server(be, budget_bytes=900, capacity=2, chunk=32)
    fa = srv.submit(Request(key="a", b=np.ones(3)))
    fb = srv.submit(Request(key="b", b=np.ones(3)))
    _wait([fa, fb])
    time.sleep(0.05)
    fc = srv.submit(Request(key="c", b=np.ones(3)))   # needs an eviction
    _wait([fc])
    srv.close()
    assert srv.peak_used <= 900
    ev = [e for e in srv.events if e[1] == "evict"]
    assert len(ev) == 1 and ev[0][2] == "a"           # least recently used goes first


def test_request_waits_for_memory_in_arrival_order():
    """While both resident operators are busy, a third operator cannot be
    admitted; its request waits and is served once one of them goes idle."""
    cost = {"a": 2000, "b": 64, "c": 32}
    be = FakeBackend({"a": 400, "b": 400, "c": 400}, cost=lambda r: cost[r.key])
    srv = Server(be, budget_bytes=900, capacity=2, chunk=32)
    fa = srv.submit(Request(key="a", b=np.ones(2)))
    fb = srv.submit(Request(key="b", b=np.ones(2)))
    fc = srv.submit(Request(key="c", b=np.ones(2)))
    rc = fc.result(timeout=10)
    rb = fb.result(timeout=10)
    ra = fa.result(timeout=10)
    srv.close()
    assert be.opened == ["a", "b", "c"]
    assert srv.peak_used <= 900
    assert rc.latency_s > rb.latency_s  # c waited for b's operator to go idle


def test_continuous_batching_join_and_leave():
    """A short request that arrives while a long one runs joins the same
    session (no new operator) and leaves first."""
    cost = lambda r: int(r.b[0])
    be = FakeBackend({"a": 100}, cost=cost)
    srv = Server(be, budget_bytes=1000, capacity=4, chunk=32)
    f_long = srv.submit(Request(key="a", b=np.array([3000.0])))
    time.sleep(0.02)
    f_short = srv.submit(Request(key="a", b=np.array([32.0])))
    r_short = f_short.result(timeout=10)
    assert not f_long.done()
    r_long = f_long.result(timeout=10)
    srv.close()
    assert be.opened == ["a"]
    adds = [e for e in be.log if e[0] == "add"]
    assert len(adds) == 2 and adds[0][2] != adds[1][2]  # two slots of one session
    assert r_short.latency_s < r_long.latency_s


def test_slots_are_reused():
    be = FakeBackend({"a": 100}, cost=lambda r: 32)
    srv = Server(be, budget_bytes=1000, capacity=2, chunk=32)
    futs = [srv.submit(Request(key="a", b=np.ones(1))) for _ in range(9)]
    _wait(futs)
    srv.close()
    slots = {e[2] for e in be.log if e[0] == "add"}
    assert slots <= {0, 1} and len([e for e in be.log if e[0] == "add"]) == 9


def test_operator_larger_than_budget_fails_its_request():
    be = FakeBackend({"big": 10_000}, cost=lambda r: 32)
    srv = Server(be, budget_bytes=1000, capacity=2)
    f = srv.submit(Request(key="big", b=np.ones(1)))
    with pytest.raises(MemoryError):
        f.result(timeout=5)
    srv.close()


class SlowAddBackend(FakeBackend):
    """Adding a request to key 'slow' takes a while (a host-to-device copy
    and the first residual on a real device)."""

    def open(self, key, capacity):
        entry = super().open(key, capacity)
        if key == "slow":
            plain_add = entry.add

            def slow_add(items):
                time.sleep(0.3)
                plain_add(items)
            entry.add = slow_add
        return entry


def test_operator_is_not_evicted_while_its_requests_are_being_added():
    """While 'slow' adds its request, it holds that request and is not idle:
    the admission of a third operator must evict the idle 'fast' one, and the
    slow request still completes."""
    be = SlowAddBackend({"slow": 400, "fast": 400, "third": 400}, cost=lambda r: 32)
    srv = Server(be, budget_bytes=900, capacity=2, chunk=32)
    f_slow = srv.submit(Request(key="slow", b=np.ones(2)))
    f_fast = srv.submit(Request(key="fast", b=np.ones(2)))
    f_fast.result(timeout=10)
    assert not f_slow.done()                      # still inside its add
    f_third = srv.submit(Request(key="third", b=np.ones(2)))
    r_slow = f_slow.result(timeout=10)
    f_third.result(timeout=10)
    srv.close()
    assert np.array_equal(r_slow.x, 2.0 * np.ones(2))
    ev = [e[2] for e in srv.events if e[1] == "evict"]
    assert ev == ["fast"]
    assert srv.peak_used <= 900 and srv.used == 0 and not srv.errors


class FailingBackend(FakeBackend):
    """The first session opened for key 'bad' fails in its advance."""

    def open(self, key, capacity):
        entry = super().open(key, capacity)
        if key == "bad" and self.opened.count("bad") == 1:
            def broken(iterations):
                raise RuntimeError("device error")
            entry.advance = broken
        return entry


def test_worker_error_fails_its_requests_and_frees_the_operator():
    be = FailingBackend({"bad": 300, "good": 300}, cost=lambda r: 32)
    srv = Server(be, budget_bytes=1000, capacity=2, chunk=32)
    f1 = srv.submit(Request(key="bad", b=np.ones(2)))
    f2 = srv.submit(Request(key="good", b=np.ones(2)))
    with pytest.raises(RuntimeError, match="device error"):
        f1.result(timeout=10)
    f2.result(timeout=10)
    # the dead operator is unregistered: a later request gets a fresh one
    r3 = srv.submit(Request(key="bad", b=np.full(2, 3.0))).result(timeout=10)
    assert np.array_equal(r3.x, np.full(2, 6.0))
    assert be.opened.count("bad") == 2
    srv.close()
    assert srv.used == 0 and len(srv.errors) == 1


def test_close_resolves_every_future():
    """Requests still running or waiting when the server closes fail with
    ServerClosed instead of hanging."""
    from paper_1207_0486_amd.serve import ServerClosed
    be = FakeBackend({"a": 600, "b": 600}, cost=lambda r: 10 ** 9)   # never finishes
    srv = Server(be, budget_bytes=1000, capacity=1, chunk=32)
    fa = srv.submit(Request(key="a", b=np.ones(1)))
    fb = srv.submit(Request(key="b", b=np.ones(1)))    # waits: a is busy
    time.sleep(0.1)
    srv.close()
    for f in (fa, fb):
        with pytest.raises(ServerClosed):
            f.result(timeout=5)
    assert srv.used == 0
    with pytest.raises(ServerClosed):
        srv.submit(Request(key="a", b=np.ones(1))).result(timeout=1)


def test_latency_by_operator():
    be = FakeBackend({"a": 100, "b": 100}, cost=lambda r: 32)
    srv = Server(be, budget_bytes=1000, capacity=2, chunk=32)
    futs = [srv.submit(Request(key=k, b=np.ones(1))) for k in "abab"]
    _wait(futs)
    srv.close()
    st = srv.stats()
    assert set(st["by_key"]) == {"a", "b"}
    assert all(v["completed"] == 2 and v["p50_ms"] <= v["p99_ms"] for v in st["by_key"].values())
