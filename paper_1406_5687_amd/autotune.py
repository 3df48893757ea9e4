"""Autotuner for the task schedule and the intersection: picks the rounds of
Eq. (1) (how many tasks the first half of the cost is cut into per worker), the
wave/workgroup list threshold, the task floor of Eq. (2), the cost function,
the intersection variant of one-wave lists (hash walk, binary search, or the
ratio rule between them), the longest list a workgroup keeps in LDS and the
ratio past which rows of the dense core are tested by bitmap, for a
built handle, by timing the counting kernels on the data itself, and caches
the choice per device and graph shape in a JSON file.  The search has three
stages: rounds with the other parameters at their defaults, then threshold,
floor and cost function with the best rounds, then the intersection, the LDS
cap and the bitmap ratio with the best of those.

Counts do not depend on any of these choices (Section V-D: any task split
counts every triangle once); only the time does.  The search reschedules the
handle (tc_graph_reschedule), so the adjacency is built once.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import asdict, dataclass
from typing import Callable, Iterable, Optional

from . import tc

DEFAULT_CACHE = os.environ.get("TC_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "paper_1406_5687_amd", "autotune.json"))


@dataclass(frozen=True)
class Params:
    small_max: int = 128      # lists up to this length: one wave; longer: one workgroup
    floor_div: int = 128      # min_chunk = total_cost / (workers * floor_div)
    cost_fn: int = tc.COST_PRIOR
    rounds: int = 0           # Eq. (1) with W = workers * rounds; 0 = the library's choice
    intersect: int = tc.INTERSECT_AUTO  # one-wave lists: ratio rule, hash walk only, or search only
    search_ratio: int = 0     # R of the ratio rule; 0 = the library's choice
    lds_list_max: int = 0     # longest list a workgroup hashes in LDS; 0 = the library's choice
    bitmap_ratio: int = 0     # core rows tested by bitmap past this ratio; 0 = the library's, -1 = never

    def min_chunk(self, total_cost: int, workers: int) -> int:
        return max(256, total_cost // (workers * self.floor_div + 1))


ROUNDS = (0, 1, 4, 16, 64)


def candidates(rounds: int = 0) -> list:
    """Second-stage grid (threshold, floor, cost function) at the given rounds."""
    out = []
    for cost_fn in (tc.COST_PRIOR, tc.COST_DEGREE):
        for small_max in (32, 64, 128):
            for floor_div in (16, 64, 128, 512):
                out.append(Params(small_max, floor_div, cost_fn, rounds))
    return out


def intersections(base: Params) -> list:
    """Third-stage grid: the intersection variants and LDS caps around `base`."""
    from dataclasses import replace

    out = [replace(base, intersect=tc.INTERSECT_WALK), replace(base, intersect=tc.INTERSECT_SEARCH)]
    out += [replace(base, intersect=tc.INTERSECT_AUTO, search_ratio=r) for r in SEARCH_RATIOS]
    out += [replace(base, lds_list_max=c) for c in LDS_CAPS]
    out += [replace(base, bitmap_ratio=b) for b in BITMAP_RATIOS]
    return out


SEARCH_RATIOS = (16, 32, 128, 256)
LDS_CAPS = (768, 1024, 1536)
BITMAP_RATIOS = (1, 4, 8, -1)


def features(info: dict) -> str:
    """Shape bucket of a handle (independent of its current schedule): graph
    count, log2 of nodes, edges, mean list length and longest list."""
    def lg(x):
        return int(math.log2(max(int(x), 1)))

    mean = info["m"] / max(info["n"], 1)
    return (f"k{lg(info['k'])}-n{lg(info['n'])}-m{lg(info['m'])}-a{lg(round(4 * mean))}"
            f"-d{lg(info['max_out_degree'])}")


def device_key() -> str:
    try:
        import torch

        p = torch.cuda.get_device_properties(0)
        return f"{p.name}-{p.multi_processor_count}cu"
    except Exception:
        return "unknown-device"


def kernel_time(graph: "tc.Graph", per_node: bool, reps: int = 3) -> float:
    """Minimum device time (ms) of the counting kernels over `reps` counts."""
    import torch

    best = float("inf")
    if per_node:
        out = torch.empty(max(graph.n_total, 1), dtype=torch.int64, device="cuda")
        tot = torch.empty(max(graph.k, 1), dtype=torch.int64, device="cuda")
    else:
        tot = torch.empty(max(graph.k, 1), dtype=torch.int64, device="cuda")
    for _ in range(reps):
        if per_node:
            graph.count_per_node(out=out, totals=tot, time_kernels=True)
        else:
            graph.count_total(out=tot, time_kernels=True)
        best = min(best, graph.info()["last_count_ms"])
    return best


class Autotuner:
    def __init__(self, cache_path: Optional[str] = DEFAULT_CACHE,
                 measure: Optional[Callable[["tc.Graph", bool], float]] = None,
                 space: Optional[Iterable[Params]] = None):
        self.cache_path = cache_path
        self.measure = measure or kernel_time
        # a fixed space replaces the two-stage search
        self.space = list(space) if space is not None else None
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            try:
                with open(cache_path) as fh:
                    self.cache = json.load(fh)
            except (OSError, ValueError):
                self.cache = {}

    def _key(self, info: dict, per_node: bool) -> str:
        return f"{device_key()}|{features(info)}|{'pn' if per_node else 'tot'}"

    def _apply(self, graph, p: Params):
        info = graph.info()
        graph.reschedule(workers=info["workers"], cost_fn=p.cost_fn,
                         min_chunk=p.min_chunk(info["total_cost"], info["workers"]), small_max=p.small_max,
                         rounds=p.rounds, intersect=p.intersect, search_ratio=p.search_ratio,
                         lds_list_max=p.lds_list_max, bitmap_ratio=p.bitmap_ratio)

    def tune(self, graph, per_node: bool = False, force: bool = False) -> Params:
        """Returns the chosen parameters and leaves the handle scheduled with them."""
        info = graph.info()
        key = self._key(info, per_node)
        if not force and key in self.cache:
            known = {f for f in Params.__dataclass_fields__}
            p = Params(**{k: v for k, v in self.cache[key]["params"].items() if k in known})
            self._apply(graph, p)
            return p
        best, best_t, trials = None, float("inf"), []

        def run(space):
            nonlocal best, best_t
            for p in space:
                self._apply(graph, p)
                t = self.measure(graph, per_node)
                trials.append((asdict(p), t))
                if t < best_t:
                    best, best_t = p, t

        if self.space is not None:
            run(self.space)
        else:
            run([Params(rounds=r) for r in ROUNDS])
            run([p for p in candidates(best.rounds) if p != best])
            run([p for p in intersections(best) if p != best])
        self._apply(graph, best)
        self.cache[key] = {"params": asdict(best), "ms": best_t, "trials": len(trials)}
        self._save()
        return best

    def _save(self):
        if not self.cache_path:
            return
        os.makedirs(os.path.dirname(self.cache_path) or ".", exist_ok=True)
        tmp = self.cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(self.cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)
