"""Writes the expected results of the full-size workloads with the CPU oracle.

Test infrastructure.  The counts come from ``oracle.count`` (the node iterator
of Fig. 1 over the canonical simple graph, with T_v as defined in Section II)
and the degrees from ``oracle.orient``; the inputs come from the seeded
generators in ``graphgen``.  Nothing else is called, so no stored value comes
from the GPU library.

    python tests/golden/make_fullsize.py er pa rmat24 batch serve [--jobs J]

writes ``tests/golden/fullsize_<name>.txt``.  Independent graphs of the batch
and serve workloads are counted by J single-threaded oracle processes at once;
R-MAT scale 24 takes about 20 minutes of one core.

Digests: ``sha256`` is taken over T_v as little-endian int64 in caller ids
0..n-1; ``h64`` is the first 16 hex digits of the same digest (per graph of a
batch or per request, to keep the files small), and the whole batch or serve
stream also gets the full digest of all T_v laid end to end in graph order.
"""
from __future__ import annotations

import argparse
import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

TOP_K = 1000


def _sha(tv: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(tv, dtype="<i8").tobytes()).hexdigest()


def _header(f, name: str, what: str):
    f.write(f"# Expected results of {what}, written by tests/golden/make_fullsize.py {name}\n")
    f.write("# (CPU oracle: Fig. 1 node iterator, T_v by the Section II definition; inputs from graphgen).\n")


def single(name: str, g, what: str):
    t0 = time.time()
    T, tv, m = oracle.count(g.n, g.src, g.dst)
    t1 = time.time()
    _, _, _, deg = oracle.orient(g.n, g.src, g.dst)
    t2 = time.time()
    order = np.lexsort((np.arange(g.n), -deg.astype(np.int64)))[:TOP_K]
    path = os.path.join(HERE, f"fullsize_{name}.txt")
    with open(path, "w") as f:
        _header(f, name, what)
        f.write(f"# oracle count {t1 - t0:.1f} s, orient {t2 - t1:.1f} s (one core)\n")
        f.write(f"workload {g.name}\n")
        f.write(f"n {g.n}\nm_input {g.m}\nm {m}\nT {T}\nsha256 {_sha(tv)}\n")
        f.write(f"# the {len(order)} nodes of highest degree (ties by id): id degree T_v\n")
        for v in order:
            f.write(f"top {int(v)} {int(deg[v])} {int(tv[v])}\n")
    print(f"{name}: n={g.n} m={m} T={T} in {t1 - t0:.1f} s -> {path}", flush=True)


def _one(args):
    idx, spec = args
    g = spec.make()
    T, tv, m = oracle.count(g.n, g.src, g.dst)
    return idx, g.n, g.m, m, T, _sha(tv)[:16], np.ascontiguousarray(tv, dtype="<i8").tobytes()


def many(name: str, specs, what: str, jobs: int):
    t0 = time.time()
    rows = [None] * len(specs)
    h = hashlib.sha256()
    nxt = 0
    pending = {}
    with mp.Pool(jobs) as pool:
        for idx, n, m_in, m, T, h64, tvb in pool.imap_unordered(_one, list(enumerate(specs)), chunksize=1):
            rows[idx] = (n, m_in, m, T, h64)
            pending[idx] = tvb
            while nxt in pending:
                h.update(pending.pop(nxt))
                nxt += 1
            if idx % 500 == 0:
                print(f"{name}: {sum(r is not None for r in rows)}/{len(specs)} after {time.time() - t0:.0f} s",
                      flush=True)
    path = os.path.join(HERE, f"fullsize_{name}.txt")
    with open(path, "w") as f:
        _header(f, name, what)
        f.write(f"# {jobs} oracle processes, {time.time() - t0:.0f} s\n")
        f.write(f"count {len(specs)}\n")
        f.write(f"sum_m {sum(r[2] for r in rows)}\n")
        f.write(f"sha256 {h.hexdigest()}\n")
        f.write("# index kind n m_input m T h64\n")
        for i, (s, r) in enumerate(zip(specs, rows)):
            f.write(f"g {i} {s.kind} {r[0]} {r[1]} {r[2]} {r[3]} {r[4]}\n")
    print(f"{name}: {len(specs)} graphs in {time.time() - t0:.0f} s -> {path}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="+", choices=["er", "pa", "rmat24", "batch", "serve"])
    ap.add_argument("--jobs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    a = ap.parse_args()
    for w in a.which:
        if w == "er":
            single("er", graphgen.workload_er(1), "Erdos-Renyi G(n=10,000, m=100,000), seed 1")
        elif w == "pa":
            single("pa", graphgen.workload_pa(1), "preferential attachment PA(n=10^6, d=50), seed 1")
        elif w == "rmat24":
            single("rmat24", graphgen.workload_rmat(1), "R-MAT scale 24, edge factor 16, seed 1")
        elif w == "batch":
            many("batch4096", graphgen.batch_specs(4096, 1), "the batch of 4096 graphs, seed 1", a.jobs)
        elif w == "serve":
            many("serve20000", graphgen.serve_specs(20_000, 1), "the 20,000 serve requests, seed 1", a.jobs)


if __name__ == "__main__":
    main()
