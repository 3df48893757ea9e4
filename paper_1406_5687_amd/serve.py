"""Serving form: independent requests, one graph each, arrive over time and
are answered with the total T and the per-node counts T_v of their graph
(Section II definitions; the same results as a build and count of the graph
alone).

Ingest and results.  Requests land back to back, in arrival order, in a
page-locked ingest arena (src and dst arrays); results go to a page-locked
result arena (T per request, T_v per node).  Requests taken in arrival order
therefore form one contiguous range of both arenas.

Continuous batching over rotating streams.  R workers, each with its own HIP
stream, repeatedly take the longest run of arrived, not yet taken requests
that fits:

  * admission by device footprint: each request is charged an estimate of the
    device bytes its share of a packed build and count holds (input copy,
    build scratch, adjacency, counts); a batch starts only when its charge
    fits what the other in-flight batches leave of the budget;
  * the batch is one handle: its edges are copied to the device with one copy
    per endpoint array and read in place by tc_build_oriented (k graphs, one
    build); one persistent launch counts all of them (tc_count_per_node); the
    per-node counts and totals return with one copy each;
  * while one worker's batch is on the device, the others build or count
    theirs on their own streams.

Resident adjacency.  With resident_bytes > 0 the handle built for a batch
stays on the device after its results are out, up to that many device bytes
(least recently used handles are released first).  Requests carry a graph key
(by default their index): a request whose key is resident is answered from
the cached adjacency with a count launch only (tc_count_batch over the cached
handles it needs), without copying or building its edges again.  A batch is
either a run of consecutive requests none of which is resident (copied, built
and counted, then cached) or a run of consecutive resident ones (counted).

Latency of a request = completion (results in the result arena) - arrival.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import tc


def device_footprint(n: int, m: int) -> int:
    """Device bytes charged to one request in a packed batch: the input copy
    (8 B / edge), build scratch and adjacency (31 B / edge), node arrays,
    per-node counts and their staging (108 B / node)."""
    return 39 * int(m) + 108 * int(n) + 4096


def fingerprint(tv: np.ndarray) -> int:
    """Order-sensitive 64-bit digest of a per-node count array."""
    w = np.arange(1, tv.shape[0] + 1, dtype=np.uint64)
    return int((tv.astype(np.uint64) * w).sum(dtype=np.uint64))


class Arena:
    """Ingest and result arenas for N requests in arrival order.

    Request i: edges src[eoff[i]:eoff[i+1]], dst[...] (int32 node ids in
    0..ns[i]-1); results T = tot[i], T_v = out[noff[i]:noff[i+1]]."""

    def __init__(self, ns: Sequence[int], ms: Sequence[int], pinned: bool = True, keys: Optional[Sequence] = None):
        self.ns = np.asarray(ns, np.int64)
        self.ms = np.asarray(ms, np.int64)
        self.N = int(self.ns.shape[0])
        # graph identity of each request: equal keys name the same graph
        self.keys = list(range(self.N)) if keys is None else list(keys)
        if len(self.keys) != self.N:
            raise ValueError("one key per request")
        self.eoff = np.zeros(self.N + 1, np.int64)
        np.cumsum(self.ms, out=self.eoff[1:])
        self.noff = np.zeros(self.N + 1, np.int64)
        np.cumsum(self.ns, out=self.noff[1:])
        E, Nn = int(self.eoff[-1]), int(self.noff[-1])
        if pinned:
            import torch

            def alloc(count, dt):
                return torch.empty(max(count, 1), dtype=dt, pin_memory=True)

            self.t_src = alloc(E, torch.int32)
            self.t_dst = alloc(E, torch.int32)
            self.t_out = alloc(Nn, torch.int64)
            self.t_tot = alloc(self.N, torch.int64)
            self.src, self.dst = self.t_src.numpy(), self.t_dst.numpy()
            self.out, self.tot = self.t_out.numpy(), self.t_tot.numpy()
        else:
            self.t_src = self.t_dst = self.t_out = self.t_tot = None
            self.src = np.zeros(max(E, 1), np.int32)
            self.dst = np.zeros(max(E, 1), np.int32)
            self.out = np.zeros(max(Nn, 1), np.int64)
            self.tot = np.zeros(max(self.N, 1), np.int64)

    def put(self, i: int, src: np.ndarray, dst: np.ndarray):
        a, b = self.eoff[i], self.eoff[i + 1]
        if src.shape[0] != b - a or dst.shape[0] != b - a:
            raise ValueError("edge count differs from the arena layout")
        self.src[a:b] = src
        self.dst[a:b] = dst

    def edges(self, i: int) -> Tuple[np.ndarray, np.ndarray]:
        a, b = self.eoff[i], self.eoff[i + 1]
        return self.src[a:b], self.dst[a:b]

    def per_node(self, i: int) -> np.ndarray:
        return self.out[self.noff[i]:self.noff[i + 1]]

    def digests(self) -> np.ndarray:
        return np.array([fingerprint(self.per_node(i)) for i in range(self.N)], np.uint64)

    def clear_results(self):
        self.out[:] = -1
        self.tot[:] = -1


@dataclass
class ServeResult:
    latency: np.ndarray             # seconds, per request
    done: np.ndarray                # completion time, per request
    batches: List[Tuple[int, int]]  # request ranges [a, b) in start order
    m_canonical: int                # distinct edges over all requests
    makespan: float                 # seconds from the start to the last completion
    builds: int = 0                 # batches copied to the device and built
    resident_hits: int = 0          # requests answered from a resident adjacency

    def percentile_ms(self, q: float) -> float:
        return float(np.percentile(self.latency, q) * 1e3)


class _Resident:
    """A cached handle: the built adjacency of one served batch."""

    def __init__(self, graph, nbytes: int, m_of: List[int]):
        self.graph = graph
        self.nbytes = nbytes
        self.m_of = m_of      # distinct edges of each packed graph
        self.users = 0        # batches counting it right now
        self.last = 0


class ResidentCache:
    """Handles kept on the device after their batch, least recently used
    released first once their device bytes pass `limit` (0: none kept).
    key -> (handle, graph index in the handle, first node of the graph)."""

    def __init__(self, limit: int):
        self.limit = int(limit)
        self.lock = threading.Lock()
        self.where = {}
        self.handles = []
        self.bytes = 0
        self.clock = 0

    def has(self, key) -> bool:
        return self.limit > 0 and key in self.where

    def pin(self, keys):
        """(handle, graph index, first node) of every key, with the handles
        held against release; None unless every key is resident."""
        if self.limit <= 0:
            return None
        with self.lock:
            ent = [self.where.get(k) for k in keys]
            if any(e is None for e in ent):
                return None
            self.clock += 1
            for h, _, _ in ent:
                h.users += 1
                h.last = self.clock
            return ent

    def unpin(self, ent):
        with self.lock:
            for h, _, _ in ent:
                h.users -= 1
            self._evict()

    def keep(self, graph, keys, ns, ms) -> bool:
        """Caches a served batch's handle; False when nothing is kept (the
        caller frees it)."""
        if self.limit <= 0:
            return False
        nbytes = int(graph.info()["device_bytes"])
        if nbytes > self.limit:
            return False
        off = graph.export_offsets()  # degree-order labels: graph g owns a label range
        nb = np.zeros(len(keys) + 1, np.int64)
        np.cumsum(np.asarray(ns, np.int64), out=nb[1:])
        h = _Resident(graph, nbytes, [int(off[nb[g + 1]] - off[nb[g]]) for g in range(len(keys))])
        with self.lock:
            self.clock += 1
            h.last = self.clock
            first = 0
            for g, (k, n) in enumerate(zip(keys, ns)):
                self.where[k] = (h, g, first)
                first += int(n)
            self.handles.append(h)
            self.bytes += nbytes
            self._evict()
        return True

    def _evict(self):
        while self.bytes > self.limit:
            idle = [h for h in self.handles if h.users == 0]
            if not idle:
                return
            h = min(idle, key=lambda x: x.last)
            self.handles.remove(h)
            self.bytes -= h.nbytes
            for k in [k for k, e in self.where.items() if e[0] is h]:
                del self.where[k]
            h.graph.free()

    def clear(self):
        with self.lock:
            for h in self.handles:
                h.graph.free()
            self.handles, self.where, self.bytes = [], {}, 0


class Server:
    """Continuous batching of triangle-count requests on one GPU."""

    def __init__(self, *, streams: int = 4, hbm_budget_bytes: int = 32 << 30, max_batch_edges: int = 1 << 26,
                 max_batch_graphs: int = 4096, per_node: bool = True, resident_bytes: int = 0):
        if streams < 1:
            raise ValueError("streams must be >= 1")
        self.streams = streams
        self.budget = int(hbm_budget_bytes)
        self.max_batch_edges = int(max_batch_edges)
        self.max_batch_graphs = int(max_batch_graphs)
        self.per_node = per_node
        self.resident_bytes = int(resident_bytes)
        self.cache = ResidentCache(self.resident_bytes)

    # ---------------------------------------------------------- scheduling

    def _take(self, st) -> Optional[Tuple[int, int]]:
        """Next batch [a, b): arrived requests from the first one not yet taken,
        within the caps and the free budget; blocks until one is available;
        None when all are taken."""
        arena, arr, fp = st["arena"], st["arrival"], st["fp"]
        N = arena.N
        with st["cv"]:
            while True:
                if st["error"] is not None:
                    return None
                now = time.perf_counter() - st["t0"]
                while st["arrived"] < N and arr[st["arrived"]] <= now:
                    st["arrived"] += 1
                a = st["taken"]
                if a < st["arrived"]:
                    b, edges, charge = a, 0, 0
                    hit = self.cache.has(arena.keys[a])
                    while b < st["arrived"]:
                        m = int(arena.ms[b])
                        if b > a and (edges + m > self.max_batch_edges or b - a >= self.max_batch_graphs
                                      or self.cache.has(arena.keys[b]) != hit):
                            break
                        if charge + fp[b] > st["free"]:
                            # nothing else in flight: a request larger than the
                            # whole budget still runs, alone
                            if b == a and st["free"] == self.budget:
                                charge += fp[b]
                                b += 1
                            break
                        edges += m
                        charge += fp[b]
                        b += 1
                    if b > a:
                        st["taken"] = b
                        st["free"] -= charge
                        st["charge"][a] = charge
                        return a, b
                    st["cv"].wait()  # wait for a batch to finish
                    continue
                if st["taken"] >= N:
                    return None
                st["cv"].wait(timeout=max(0.0, arr[st["arrived"]] - now))

    def _release(self, st, a: int):
        with st["cv"]:
            st["free"] += st["charge"].pop(a)
            st["cv"].notify_all()

    # ---------------------------------------------------------- execution

    def _worker_state(self) -> dict:
        import torch

        torch.cuda.set_device(0)
        return {"stream": torch.cuda.Stream()}

    def _run_batch(self, st, ws, a: int, b: int) -> int:
        """Counts requests [a, b) on this worker's stream; results land in the
        arena when this returns.  Returns the batch's distinct edges."""
        arena = st["arena"]
        pinned = self.cache.pin([arena.keys[i] for i in range(a, b)])
        if pinned is not None:
            try:
                return self._run_resident(st, ws, a, b, pinned)
            finally:
                self.cache.unpin(pinned)
        return self._run_build(st, ws, a, b)

    def _run_resident(self, st, ws, a: int, b: int, entries) -> int:
        """Requests [a, b), all resident: one tc_count_batch over the cached
        handles they need (their own scratch, so handles shared with other
        workers are safe), then each request's slice of its handle's results."""
        import torch

        arena = st["arena"]
        stream = ws["stream"]
        handles = []
        slot = {}
        for h, _, _ in entries:
            if id(h) not in slot:
                slot[id(h)] = len(handles)
                handles.append(h)
        with torch.cuda.stream(stream):
            ktot = sum(h.graph.k for h in handles)
            tot = torch.empty(max(ktot, 1), dtype=torch.int64, device="cuda")
            outs = ([torch.empty(max(h.graph.n_total, 1), dtype=torch.int64, device="cuda") for h in handles]
                    if self.per_node else None)
            tc.count_batch_device([h.graph for h in handles], tot, outs, stream=stream.cuda_stream)
            kbase = np.zeros(len(handles) + 1, np.int64)
            np.cumsum([h.graph.k for h in handles], out=kbase[1:])
            tot_pin = torch.empty(max(ktot, 1), dtype=torch.int64, pin_memory=True)
            tot_pin.copy_(tot, non_blocking=True)
            out_pin = None
            if self.per_node:
                out_pin = [torch.empty(max(h.graph.n_total, 1), dtype=torch.int64, pin_memory=True) for h in handles]
                for o_p, o in zip(out_pin, outs):
                    o_p.copy_(o, non_blocking=True)
            stream.synchronize()
        m = 0
        for i, (h, g, n0) in zip(range(a, b), entries):
            j = slot[id(h)]
            arena.tot[i] = int(tot_pin[kbase[j] + g])
            if self.per_node and arena.ns[i] > 0:
                n = int(arena.ns[i])
                arena.out[arena.noff[i]:arena.noff[i] + n] = out_pin[j].numpy()[n0:n0 + n]
            m += h.m_of[g]
        with st["lock"]:
            st["hits"] += b - a
        return m

    def _run_build(self, st, ws, a: int, b: int) -> int:
        import torch

        arena = st["arena"]
        e0, e1 = int(arena.eoff[a]), int(arena.eoff[b])
        n0, n1 = int(arena.noff[a]), int(arena.noff[b])
        E, Nn, k = e1 - e0, n1 - n0, b - a
        stream = ws["stream"]
        with torch.cuda.stream(stream):
            dev = torch.empty(max(2 * E, 1), dtype=torch.int32, device="cuda")
            if E:
                dev[:E].copy_(arena.t_src[e0:e1], non_blocking=True)
                dev[E:2 * E].copy_(arena.t_dst[e0:e1], non_blocking=True)
            h = tc.build_packed_device(arena.ns[a:b], arena.ms[a:b], dev.data_ptr(), dev.data_ptr() + 4 * E,
                                       stream=stream.cuda_stream)
            try:
                m_can = h.info()["m"]
                tot = torch.empty(k, dtype=torch.int64, device="cuda")
                if self.per_node and Nn > 0:
                    out = torch.empty(Nn, dtype=torch.int64, device="cuda")
                    h.count_per_node(out=out, totals=tot)
                    arena.t_out[n0:n1].copy_(out, non_blocking=True)
                else:
                    h.count_total(out=tot)
                arena.t_tot[a:b].copy_(tot, non_blocking=True)
                stream.synchronize()
            finally:
                if not self.cache.keep(h, [arena.keys[i] for i in range(a, b)], arena.ns[a:b],
                                       arena.ms[a:b]):
                    h.free()
        with st["lock"]:
            st["builds"] += 1
        return m_can

    def _worker(self, st, wid: int):
        try:
            ws = self._worker_state()
            while True:
                got = self._take(st)
                if got is None:
                    return
                a, b = got
                try:
                    m_can = self._run_batch(st, ws, a, b)
                finally:
                    self._release(st, a)
                t_done = time.perf_counter() - st["t0"]
                with st["lock"]:
                    st["batches"].append((a, b))
                    st["m"] += m_can
                    st["done"][a:b] = t_done
        except BaseException as e:  # surfaced by run()
            with st["cv"]:
                st["error"] = e
                st["cv"].notify_all()

    def run(self, arena: Arena, arrivals: Optional[Sequence[float]] = None) -> ServeResult:
        """Serves the arena's requests, request i arriving arrivals[i] seconds
        after the start (non-decreasing; default: all at once).  Results are
        written into the arena."""
        N = arena.N
        arr = np.zeros(N) if arrivals is None else np.asarray(arrivals, float)
        if arr.shape[0] != N or (N > 1 and (np.diff(arr) < 0).any()):
            raise ValueError("arrivals must give one non-decreasing time per request (arena order)")
        st = {
            "arena": arena, "arrival": arr, "fp": [device_footprint(arena.ns[i], arena.ms[i]) for i in range(N)],
            "cv": threading.Condition(), "lock": threading.Lock(), "arrived": 0, "taken": 0,
            "free": self.budget, "charge": {}, "error": None, "done": np.zeros(N, float), "batches": [], "m": 0,
            "builds": 0, "hits": 0,
        }
        st["t0"] = time.perf_counter()
        threads = [threading.Thread(target=self._worker, args=(st, w), daemon=True) for w in range(self.streams)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if st["error"] is not None:
            raise st["error"]
        done = st["done"]
        return ServeResult(latency=done - arr, done=done, batches=st["batches"], m_canonical=int(st["m"]),
                           makespan=float(done.max(initial=0.0)), builds=st["builds"], resident_hits=st["hits"])

    def close(self):
        """Releases the resident adjacencies."""
        self.cache.clear()


def serve_alone(arena: Arena, i: int, per_node: bool = True):
    """The plain path for request i: its own build and count (host in, host
    out).  Returns (T, T_v or None, distinct edges)."""
    src, dst = arena.edges(i)
    with tc.build_oriented([(int(arena.ns[i]), src, dst)]) as h:
        m = h.info()["m"]
        if per_node:
            tv, tot = h.count_per_node()
            return int(tot[0]), tv, m
        return int(h.count_total()[0]), None, m


def run_plain(arena: Arena, per_node: bool = True) -> Tuple[float, int]:
    """Sequential plain loop over the arena's requests, back to back: one
    build and one count per request, results written into the arena.
    Returns (seconds, distinct edges)."""
    t0 = time.perf_counter()
    m = 0
    for i in range(arena.N):
        src, dst = arena.edges(i)
        with tc.build_oriented([(int(arena.ns[i]), src, dst)]) as h:
            m += h.info()["m"]
            if per_node and arena.ns[i] > 0:
                a, b = arena.noff[i], arena.noff[i + 1]
                tv, tot = h.count_per_node()
                arena.out[a:b] = tv
                arena.tot[i] = tot[0]
            else:
                arena.tot[i] = h.count_total()[0]
    return time.perf_counter() - t0, m
