#!/usr/bin/env python3
"""Throughput of exact triangle counting on one MI355X.

One step is the whole path on one synthetic graph whose edge list already
sits in device memory: canonical edge set, degree order, orientation and row
sort, task table (tc_build_oriented), then the persistent counting kernels
with per-node counts and their scatter back to caller labels
(tc_count_per_node).  value = oriented edges / second of whole steps.

Default workload: preferential attachment, 10^6 nodes, 50 distinct targets
per new node (49,998,725 edges), seed 1.

Prints one JSON line.  The CPU baseline is the plain oracle (single thread)
timed on a smaller graph of the same family.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name: str):
    import graphgen

    if name == "pa":
        return graphgen.workload_pa(1), "PA(n=1e6, d=50), seed 1"
    if name == "er":
        return graphgen.workload_er(1), "ER G(n=1e4, m=1e5), seed 1"
    if name == "rmat":
        return graphgen.workload_rmat(1), "R-MAT scale 24, ef 16, (0.57,0.19,0.19,0.05), seed 1"
    raise ValueError(name)


def algorithmic_bytes(off, col, n: int, per_node: bool) -> tuple[int, int]:
    """B_alg = 4 m + 4 sum_{s->t} |N_t| + 8 (n+1) + 8 n [per-node]:
    each source list once, each target list once per stored edge, the row
    offsets once and the per-node counts once.  Returns (bytes, sum |N_t|)."""
    import numpy as np

    dh = np.diff(off)
    sum_dt = int(dh[col].sum()) if len(col) else 0
    m = len(col)
    return 4 * m + 4 * sum_dt + 8 * (n + 1) + (8 * n if per_node else 0), sum_dt


def cpu_baseline(seconds_hint: float = 20.0) -> dict:
    """The oracle as it stands (single thread) on PA(2.5e5, 50): whole path,
    edge list to per-node counts."""
    import graphgen
    import oracle

    g = graphgen.preferential_attachment(250_000, 50, 1)
    t0 = time.perf_counter()
    T, tv, m = oracle.count(g.n, g.src, g.dst, per_node=True)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "oriented edges/s", "cores": 1, "kind": "oracle",
            "sample": f"PA(n=2.5e5, d=50) seed 1, m={m}: full oracle run (canonical edges, degree order, "
                      f"orientation, row sort, node iterator with per-node counts) in {dt:.2f} s"}


def bench_batch(args) -> int:
    """Packed batch: all graphs in one handle, counted by one captured
    persistent launch, against one plain count launch per graph (separate
    handles, launched back to back on one stream, one final synchronisation)."""
    import concurrent.futures as cf

    import numpy as np
    import torch

    import graphgen
    import paper_1406_5687_amd as tc
    from paper_1406_5687_amd.autotune import Autotuner
    from paper_1406_5687_amd.capture import CapturedCount

    K = args.batch_graphs
    t0 = time.time()
    specs = graphgen.batch_specs(K, seed=1)
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        graphs = list(ex.map(lambda sp: sp.make(), specs))
    m_in = sum(g.m for g in graphs)
    log(f"generated {K} graphs, {m_in} input edges in {time.time() - t0:.1f} s")
    t0 = time.time()
    h = tc.build_oriented([(g.n, g.src, g.dst) for g in graphs])
    torch.cuda.synchronize()
    info = h.info()
    m = info["m"]
    log(f"packed build: n={info['n']} m={m} tasks={info['tasks']} wide={info['wide_nodes']} in {time.time() - t0:.1f} s")
    if args.tune:
        p = Autotuner().tune(h, per_node=False)
        log(f"autotuned: {p}")
    cap = CapturedCount(h, per_node=False)
    for _ in range(args.warmup):
        cap.replay()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        cap.replay()
    ev1.record()
    torch.cuda.synchronize()
    batch_ms = ev0.elapsed_time(ev1) / args.steps
    packed = cap.totals.cpu().numpy()[:K].copy()
    h.free()
    del cap

    t0 = time.time()
    hs = [tc.build_oriented([(g.n, g.src, g.dst)]) for g in graphs]
    torch.cuda.synchronize()
    log(f"{K} separate builds in {time.time() - t0:.1f} s")
    out = torch.zeros(K, dtype=torch.int64, device="cuda")
    for i, hh in enumerate(hs):
        hh.count_total(out=out[i:i + 1])
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 3))
    ev0.record()
    for _ in range(reps):
        for i, hh in enumerate(hs):
            hh.count_total(out=out[i:i + 1])
    ev1.record()
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1) / reps
    plain = out.cpu().numpy()
    same = bool(np.array_equal(plain, packed))
    for hh in hs:
        hh.free()
    res = {
        "metric": "oriented edges/s", "value": m / (batch_ms * 1e-3), "unit": "oriented edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": batch_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32 ids, int64 counts", "data": "synthetic",
        "config": {"workload": f"batch of {K} graphs (n log-uniform 1e3..2e5; even: G(n,m) mean degree U(8,64); "
                               f"odd: Chung-Lu beta 2.1, 16n pairs), seed 1", "graphs": K, "m": m, "m_input": m_in,
                   "step": "one captured persistent count launch over the packed handle (totals)"},
        "detail": {"plain_ms": plain_ms, "batched_over_plain": plain_ms / batch_ms, "identical_counts": same,
                   "tasks": info["tasks"], "wide_nodes": info["wide_nodes"]},
    }
    print(json.dumps(res), flush=True)
    return 0 if same else 1


def bench_partitioned(args) -> int:
    """Partitioned form under device budgets: the edge list stays in host
    memory, the handle is built and counted within each budget, and the
    per-node counts must equal those of the resident form (no budget).  One
    JSON line per budget; value = oriented edges / second of the count."""
    import numpy as np
    import torch

    import paper_1406_5687_amd as tc

    t0 = time.time()
    g, wl_name = make_workload(args.workload)
    log(f"generated {wl_name}: n={g.n} input edges={g.m} in {time.time() - t0:.1f} s")
    out = torch.zeros(g.n, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    with tc.build_oriented([(g.n, src, dst)]) as h:
        h.count_per_node(out=out, totals=tot, time_kernels=True)
        res_ms = h.info()["last_count_ms"]
        m = h.info()["m"]
    del src, dst
    ref = out.clone()
    T_ref = int(tot.item())
    log(f"resident: T={T_ref} m={m} count {res_ms:.1f} ms")
    rc = 0
    for gb in args.budget_gb:
        budget = int(gb * (1 << 30))
        torch.cuda.synchronize()
        tb = time.perf_counter()
        h = tc.build_oriented([(g.n, g.src, g.dst)], hbm_budget_bytes=budget)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - tb) * 1e3
        info = h.info()
        log(f"budget {gb} GiB: P={info['partitions']} build {build_ms:.0f} ms peak {info['peak_device_bytes'] / 2**30:.3f} GiB")
        for _ in range(args.warmup):
            h.count_per_node(out=out, totals=tot, time_kernels=True)
        ms = []
        for _ in range(args.steps):
            out.fill_(-1)
            h.count_per_node(out=out, totals=tot, time_kernels=True)
            ms.append(h.info()["last_count_ms"])
        info = h.info()
        h.free()
        same = int(tot.item()) == T_ref and bool(torch.equal(out, ref))
        rc |= 0 if same else 1
        c_ms = float(np.median(ms))
        line = {
            "metric": "oriented edges/s", "value": m / (c_ms * 1e-3), "unit": "oriented edges/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": c_ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32 ids, int64 counts", "data": "synthetic",
            "config": {"workload": wl_name, "n": g.n, "m": m, "m_input": g.m, "per_node": True,
                       "hbm_budget_bytes": budget,
                       "step": "tc_count_per_node of a partitioned handle (adjacency in pinned host memory, "
                               "slices and streamed list ranges copied in per count)"},
            "detail": {"partitions": info["partitions"], "streamed_bytes": info["streamed_bytes"],
                       "peak_device_bytes": info["peak_device_bytes"], "build_ms": build_ms,
                       "resident_count_ms": res_ms, "identical_to_resident": same, "triangles": int(tot.item())},
        }
        print(json.dumps(line), flush=True)
    return rc


def profile_counts(args) -> int:
    """Short, fixed sequence of launches for hardware-counter runs."""
    import torch

    import paper_1406_5687_amd as tc

    x = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    torch.cuda.synchronize()
    y.copy_(x)  # reads and writes exactly 1 GiB
    torch.cuda.synchronize()
    del x, y
    g, name = make_workload(args.workload)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    h = tc.build_oriented([(g.n, src, dst)])
    out = torch.zeros(g.n, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    for _ in range(3):
        h.count_per_node(out=out, totals=tot)
    for _ in range(3):
        h.count_total(out=tot)
    torch.cuda.synchronize()
    log(f"{name}: T={int(tot.item())}")
    h.free()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pa", choices=["pa", "er", "rmat", "batch"])
    ap.add_argument("--batch-graphs", type=int, default=4096, help="graphs in the batch workload")
    ap.add_argument("--tune", action="store_true", help="autotune the batch schedule before timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--budget-gb", type=float, nargs="+", default=None,
                    help="partitioned form: build and count the workload under each device budget (GiB), "
                         "edge list in host memory, and compare with the resident counts")
    ap.add_argument("--profile-counts", action="store_true",
                    help="profiling target: a 1 GiB device copy (counter calibration), then one build of the "
                         "workload and three per-node and three total-only counts; prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not a measured configuration.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1406_5687_amd as tc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    tc.load()
    if args.workload == "batch":
        return bench_batch(args)
    if args.profile_counts:
        return profile_counts(args)
    if args.budget_gb:
        return bench_partitioned(args)

    t0 = time.time()
    g, wl_name = make_workload(args.workload)
    log(f"generated {wl_name}: n={g.n} input edges={g.m} in {time.time() - t0:.1f} s")
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    out = torch.zeros(g.n, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")

    # sizes for the byte model (outside the timed region)
    with tc.build_oriented([(g.n, src, dst)]) as h:
        info = h.info()
        off, col, _ = h.export_csr()
    m = info["m"]
    b_alg, sum_dt = algorithmic_bytes(off, col, g.n, per_node=True)
    del off, col
    log(f"m={m} max|N_v|={info['max_out_degree']} tasks={info['tasks']} sum|N_t|={sum_dt} B_alg={b_alg / 1e9:.3f} GB")

    def step():
        h = tc.build_oriented([(g.n, src, dst)])
        h.count_per_node(out=out, totals=tot, time_kernels=True)
        ms = h.info()["last_count_ms"]  # waits for the counting kernels
        h.free()
        return ms

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    kernel_ms = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev0.record()
    for i in range(args.steps):
        kernel_ms.append(step())
    ev1.record()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    wall_ms = (t_end - t_start) * 1e3 / args.steps
    ms_per_step = max(wall_ms, ev0.elapsed_time(ev1) / args.steps)
    T = int(tot.item())
    log(f"T={T} ms/step={ms_per_step:.3f} count kernels ms={np.mean(kernel_ms):.3f}")

    # one separate timing of the build alone and of the count alone (reported, not the metric)
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    h = tc.build_oriented([(g.n, src, dst)])
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb0) * 1e3
    h.free()

    k_ms = float(np.mean(kernel_ms))
    achieved = b_alg / (k_ms * 1e-3) / 1e9
    res = {
        "metric": "oriented edges/s",
        "value": m / (ms_per_step * 1e-3),
        "unit": "oriented edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 ids, int64 counts",
        "data": "synthetic",
        "config": {"workload": wl_name, "n": g.n, "m": m, "m_input": g.m, "per_node": True,
                   "step": "tc_build_oriented + tc_count_per_node, edge list resident in HBM"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "k_count_small (+ k_count_big when lists exceed 128)",
                     "alg_bytes_per_launch": b_alg, "kernel_ms": k_ms},
        "detail": {"triangles": T, "count_kernel_ms": k_ms, "build_ms_single": build_ms,
                   "count_only_edges_per_s": m / (k_ms * 1e-3), "sum_target_list_len": sum_dt},
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline ...")
        res["cpu_baseline"] = cpu_baseline()
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
