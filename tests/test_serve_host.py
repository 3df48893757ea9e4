"""Host logic of the serving form (admission, batching, latency bookkeeping)
with the device work replaced by a stand-in; no GPU needed."""
import threading
import time

import numpy as np
import pytest

from paper_1406_5687_amd import serve


class FakeServer(serve.Server):
    """Counts nothing: T of a request is its edge count and T_v its node ids;
    records the device charge in flight to check admission."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.lock = threading.Lock()
        self.inflight = 0
        self.max_inflight = 0

    def _worker_state(self):
        return {}

    def _run_batch(self, st, ws, a, b):
        arena = st["arena"]
        charge = sum(st["fp"][i] for i in range(a, b))
        with self.lock:
            self.inflight += charge
            self.max_inflight = max(self.max_inflight, self.inflight)
        time.sleep(0.0005 + 1e-9 * int(arena.eoff[b] - arena.eoff[a]))
        with self.lock:
            self.inflight -= charge
        for i in range(a, b):
            arena.tot[i] = arena.ms[i]
            arena.per_node(i)[:] = np.arange(arena.ns[i])
        return int(arena.eoff[b] - arena.eoff[a])


def make_arena(count, seed=0):
    rng = np.random.default_rng(seed)
    ns = rng.integers(2, 400, count)
    ms = rng.integers(1, 5000, count)
    ar = serve.Arena(ns, ms, pinned=False)
    for i in range(count):
        ar.put(i, rng.integers(0, ns[i], ms[i]).astype(np.int32), rng.integers(0, ns[i], ms[i]).astype(np.int32))
    return ar


def test_every_request_served_once_within_caps():
    ar = make_arena(400)
    arr = np.cumsum(np.random.default_rng(1).exponential(1 / 4000.0, ar.N))
    budget = 3 * serve.device_footprint(400, 5000)
    srv = FakeServer(streams=3, hbm_budget_bytes=budget, max_batch_edges=12000, max_batch_graphs=7)
    res = srv.run(ar, arr)
    spans = sorted(res.batches)
    assert spans[0][0] == 0 and spans[-1][1] == ar.N
    for (a, b), (c, d) in zip(spans, spans[1:]):
        assert b == c  # contiguous, each request exactly once
    for a, b in res.batches:
        assert 1 <= b - a <= 7
        if b - a > 1:
            assert ar.eoff[b] - ar.eoff[a] <= 12000
    assert srv.max_inflight <= budget
    np.testing.assert_array_equal(ar.tot[: ar.N], ar.ms)
    assert (res.latency >= 0).all() and (res.done >= arr).all()
    assert res.makespan >= arr[-1]
    assert res.m_canonical == int(ar.eoff[-1])
    # a batch never starts before its last request arrived
    for a, b in res.batches:
        assert res.done[a] >= arr[b - 1]


def test_saturated_batches_are_large():
    ar = make_arena(200)
    srv = FakeServer(streams=2, hbm_budget_bytes=1 << 40, max_batch_edges=1 << 30, max_batch_graphs=1 << 20)
    res = srv.run(ar)
    assert len(res.batches) <= 4


def test_request_larger_than_budget_runs_alone():
    ar = make_arena(20)
    fps = [serve.device_footprint(ar.ns[i], ar.ms[i]) for i in range(ar.N)]
    srv = FakeServer(streams=2, hbm_budget_bytes=max(fps) // 2, max_batch_edges=1 << 30)
    res = srv.run(ar)
    for a, b in res.batches:
        if any(fps[i] > max(fps) // 2 for i in range(a, b)):
            assert b - a == 1


def test_worker_error_is_raised():
    class Broken(FakeServer):
        def _run_batch(self, st, ws, a, b):
            raise RuntimeError("device gone")

    with pytest.raises(RuntimeError, match="device gone"):
        Broken(streams=2).run(make_arena(10))


def test_arrivals_must_follow_arena_order():
    with pytest.raises(ValueError):
        FakeServer().run(make_arena(3), [0.0, 0.2, 0.1])


def test_fingerprint_is_order_sensitive():
    a = np.array([1, 2, 3], np.int64)
    assert serve.fingerprint(a) != serve.fingerprint(a[::-1].copy())
    assert serve.fingerprint(a) == serve.fingerprint(a.copy())


class FakeHandle:
    """Stand-in for a built handle: device bytes, offsets of its packed graphs."""

    def __init__(self, ns, ms, nbytes):
        self.ns, self.nbytes = list(ns), nbytes
        self.off = np.concatenate([[0], np.cumsum(np.repeat(1, sum(ns)))]).astype(np.int64)
        self.freed = False

    def info(self):
        return {"device_bytes": self.nbytes}

    def export_offsets(self):
        return self.off

    def free(self):
        self.freed = True


def test_resident_cache_lookup_pin_and_eviction():
    c = serve.ResidentCache(250)
    h1, h2, h3 = FakeHandle([3, 2], [5, 5], 100), FakeHandle([4], [9], 100), FakeHandle([1], [1], 100)
    assert c.keep(h1, ["a", "b"], [3, 2], [5, 5]) and c.keep(h2, ["c"], [4], [9])
    assert c.has("a") and c.has("b") and c.has("c") and not c.has("d")
    ent = c.pin(["b", "a"])
    assert [(e[1], e[2]) for e in ent] == [(1, 3), (0, 0)]
    assert ent[0][0].m_of == [3, 2]  # one edge per node in the stand-in offsets
    assert c.pin(["a", "d"]) is None
    # a third handle passes the limit: the least recently used idle one goes
    assert c.keep(h3, ["e"], [1], [1])
    assert h2.freed and not h1.freed and not c.has("c")
    c.unpin(ent)
    c.clear()
    assert h1.freed and h3.freed and not c.has("a")
    # nothing is kept without a limit, or when one handle is larger than it
    assert not serve.ResidentCache(0).keep(FakeHandle([1], [1], 10), ["x"], [1], [1])
    assert not serve.ResidentCache(50).keep(FakeHandle([1], [1], 100), ["x"], [1], [1])


def test_batches_do_not_mix_resident_and_new_requests():
    ar = make_arena(30)
    ar.keys = [i % 10 for i in range(30)]
    srv = FakeServer(streams=2, hbm_budget_bytes=1 << 40, max_batch_graphs=30)
    srv.resident_bytes = 1
    srv.cache = serve.ResidentCache(1 << 30)
    for k in range(0, 10, 2):  # even keys resident
        srv.cache.where[k] = (object(), 0, 0)
    got = []
    orig = srv._run_batch

    def run_batch(st, ws, a, b):
        got.append([ar.keys[i] % 2 == 0 for i in range(a, b)])
        return orig(st, ws, a, b)

    srv._run_batch = run_batch
    srv.run(ar)
    assert all(len(set(g)) == 1 for g in got)
