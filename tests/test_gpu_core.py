"""GPU: the dense core (tc_options.bitmap_ratio).  The rows at the end of the
degree order are kept as bitmaps too, and a target row of the core that is
much longer than the list entries after its target has those entries tested
against its bitmap instead of being read (Fig. 1: the test w in N_u, turned
around).  Counts must equal the oracle's whatever the ratio, in all three
kernel tiers, per count call or set at build / reschedule time, in batches
beside handles without a core, and with the core left out (-1).  The core's
size is checked against the layout the library states: one row per core label,
each of the words (lo >> 5) .. (n - 1) >> 5 for the first core label lo.  A
graph whose core rows are all shorter than 128 entries gets no core."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_5687_amd as tcmod

    tcmod.load()
    return tcmod


def core_words(n: int, rows: int) -> int:
    """Words of the bitmaps of the last `rows` labels."""
    lo = n - rows
    return rows * (((n - 1) >> 5) - (lo >> 5) + 1)


def _workloads():
    # (name, graph, whether it gets a core)
    return [
        ("rmat15", graphgen.rmat(15, 16, seed=71), True),
        ("rmat17", graphgen.rmat(17, 16, seed=70), True),
        # hubs of degree well over 1920, lists in all three tiers; its dense
        # rows are short, so no core
        ("chung_lu", graphgen.chung_lu(30_000, 600_000, 2.0, 72), False),
        ("pa", graphgen.preferential_attachment(20_000, 24, 73), False),
    ]


@pytest.mark.parametrize("name,g,has_core", _workloads())
def test_core_ratios_equal_oracle(tc, name, g, has_core):
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    with tc.build_oriented([(g.n, g.src, g.dst)]) as h:
        info = h.info()
        assert (info["core_rows"] > 0) == has_core, name
        assert info["bitmap_ratio"] == (2 if has_core else 0)
        assert info["core_bytes"] == 4 * core_words(g.n, info["core_rows"])
        for call in ({}, {"bitmap_ratio": 1}, {"bitmap_ratio": 2}, {"bitmap_ratio": 16}, {"bitmap_ratio": -1}):
            tv, tot = h.count_per_node(**call)
            assert tot[0] == T_ref, (name, call)
            np.testing.assert_array_equal(tv, tv_ref)
            assert h.count_total(**call)[0] == T_ref, (name, call)
        h.reschedule(bitmap_ratio=1)
        assert h.info()["bitmap_ratio"] == (1 if has_core else 0)
        tv, tot = h.count_per_node()
        assert tot[0] == T_ref
        np.testing.assert_array_equal(tv, tv_ref)


def test_core_left_out_at_build(tc):
    g = graphgen.rmat(14, 16, seed=74)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    with tc.build_oriented([(g.n, g.src, g.dst)], bitmap_ratio=-1) as h:
        info = h.info()
        assert info["core_rows"] == 0 and info["core_bytes"] == 0 and info["bitmap_ratio"] == 0
        # asking for core tests without a core counts by the walk
        tv, tot = h.count_per_node(bitmap_ratio=1)
        assert tot[0] == T_ref
        np.testing.assert_array_equal(tv, tv_ref)


def test_core_with_other_intersections(tc):
    # the walk-only and search-only choices leave the core unused
    from paper_1406_5687_amd import tc as tcb

    g = graphgen.rmat(14, 16, seed=75)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    with tc.build_oriented([(g.n, g.src, g.dst)]) as h:
        for call in ({"intersect": tcb.INTERSECT_WALK}, {"intersect": tcb.INTERSECT_SEARCH},
                     {"search_ratio": 1, "bitmap_ratio": 1}):
            tv, tot = h.count_per_node(**call)
            assert tot[0] == T_ref, call
            np.testing.assert_array_equal(tv, tv_ref)


def test_core_in_batches_and_packed(tc):
    # handles with a core counted in one launch beside a packed handle (none)
    gs = [graphgen.rmat(14, 16, seed=76), graphgen.rmat(15, 16, seed=77)]
    refs = [oracle.count(g.n, g.src, g.dst) for g in gs]
    hs = [tc.build_oriented([(g.n, g.src, g.dst)]) for g in gs]
    packed = tc.build_oriented([(g.n, g.src, g.dst) for g in gs])
    try:
        assert all(h.info()["core_rows"] > 0 for h in hs)
        assert packed.info()["core_rows"] == 0
        tots, tvs = tc.count_batch(hs + [packed], per_node=True)
        for i, (T_ref, tv_ref, _) in enumerate(refs):
            assert tots[i][0] == T_ref
            np.testing.assert_array_equal(tvs[i], tv_ref)
        assert list(tots[2]) == [r[0] for r in refs]
        np.testing.assert_array_equal(tvs[2], np.concatenate([r[1] for r in refs]))
    finally:
        for h in hs + [packed]:
            h.free()


def test_core_absent_under_budget(tc):
    g = graphgen.rmat(14, 16, seed=74)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    with tc.build_oriented([(g.n, g.src, g.dst)], hbm_budget_bytes=4 << 30) as h:
        assert h.info()["core_rows"] == 0
        tv, tot = h.count_per_node()
        assert tot[0] == T_ref
        np.testing.assert_array_equal(tv, tv_ref)
