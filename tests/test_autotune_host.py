"""Autotuner search and cache logic on the CPU, with a fake handle and a fake
timing function (no device work)."""
import json

from paper_1406_5687_amd import autotune, tc


class FakeGraph:
    def __init__(self):
        self.calls = []
        self.sched = dict(workers=1024, cost_fn=tc.COST_PRIOR, min_chunk=0, small_max=128, rounds=0)

    def info(self):
        return {"k": 1, "n": 1 << 20, "m": 50 << 20, "max_out_degree": 77, "total_cost": 5_000_000_000,
                "workers": 1024, "wide_nodes": 0, "tasks": 9000}

    def reschedule(self, workers, cost_fn, min_chunk, small_max, rounds=0, intersect=0, search_ratio=0,
                   lds_list_max=0, bitmap_ratio=0):
        self.sched = dict(workers=workers, cost_fn=cost_fn, min_chunk=min_chunk, small_max=small_max,
                          rounds=rounds, intersect=intersect, search_ratio=search_ratio, lds_list_max=lds_list_max,
                          bitmap_ratio=bitmap_ratio)
        self.calls.append(dict(self.sched))


def fake_measure(graph, per_node):
    s = graph.sched
    # best: 16 rounds, small_max 64, prior cost, floor 64
    t = 3.0 + abs(s["small_max"] - 64) / 64 + (0.5 if s["cost_fn"] != tc.COST_PRIOR else 0)
    t += 0.0 if s["rounds"] == 16 else 0.3
    t += abs(s["min_chunk"] - autotune.Params(64, 64).min_chunk(5_000_000_000, 1024)) / 1e6
    # best intersection: the ratio rule with R = 16; LDS cap unchanged
    t += 0.0 if (s["intersect"] == tc.INTERSECT_AUTO and s["search_ratio"] == 16) else 0.2
    t += 0.0 if s["lds_list_max"] == 0 else 0.1
    return t


def test_search_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "cache.json")
    g = FakeGraph()
    at = autotune.Autotuner(cache_path=path, measure=fake_measure)
    best = at.tune(g, per_node=False)
    assert best == autotune.Params(64, 64, tc.COST_PRIOR, 16, tc.INTERSECT_AUTO, 16)
    assert g.sched["small_max"] == 64 and g.sched["cost_fn"] == tc.COST_PRIOR and g.sched["rounds"] == 16
    assert g.sched["search_ratio"] == 16 and g.sched["lds_list_max"] == 0
    # stage 1 over rounds, stage 2 over the grid (minus the point already timed), stage 3 over the
    # intersection variants and LDS caps, then the final apply
    stage3 = autotune.intersections(autotune.Params(64, 64, tc.COST_PRIOR, 16))
    assert len(g.calls) == len(autotune.ROUNDS) + (len(autotune.candidates(16)) - 1) + len(stage3) + 1
    data = json.load(open(path))
    assert len(data) == 1 and list(data.values())[0]["params"]["small_max"] == 64
    # a second tuner reads the cache and applies without measuring
    g2 = FakeGraph()
    at2 = autotune.Autotuner(cache_path=path, measure=lambda *a: (_ for _ in ()).throw(AssertionError("measured")))
    assert at2.tune(g2) == best and len(g2.calls) == 1


def test_features_do_not_depend_on_schedule():
    a = FakeGraph().info()
    b = dict(a, wide_nodes=12345, tasks=1, workers=7)
    assert autotune.features(a) == autotune.features(b)


def test_min_chunk_floor():
    assert autotune.Params(128, 16).min_chunk(10, 1024) == 256
    assert autotune.Params(128, 16).min_chunk(10**12, 1000) == 10**12 // (1000 * 16 + 1)
