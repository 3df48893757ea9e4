"""GPU: the intersection variants of the one-wave kernel (hash walk of every
target row, binary search of the source list's candidates in every row, and
the ratio rule between them) all give the oracle's counts, resident,
partitioned, packed and in batches with per-handle choices."""
import numpy as np
import pytest

import graphgen
import oracle
from tests.graphs_small import complete, wheel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_5687_amd as tcmod

    tcmod.load()
    return tcmod


def _workloads():
    return [
        ("rmat14", graphgen.rmat(14, 16, seed=31)),
        ("rmat17", graphgen.rmat(17, 16, seed=37)),  # one-wave lists with target rows of 256+
        ("chung_lu", graphgen.chung_lu(20_000, 320_000, 2.1, 32)),
        ("pa", graphgen.preferential_attachment(20_000, 12, 33)),
        ("er", graphgen.erdos_renyi(5000, 60_000, 34)),
    ]


VARIANTS = [dict(intersect=1), dict(intersect=2), dict(intersect=0, search_ratio=1), dict(intersect=0, search_ratio=2),
            dict(intersect=0), dict(intersect=0, search_ratio=64)]


@pytest.mark.parametrize("name,g", _workloads())
def test_variants_equal_oracle(tc, name, g):
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    for kw in VARIANTS:
        with tc.build_oriented([(g.n, g.src, g.dst)], **kw) as h:
            tv, tot = h.count_per_node()
            assert tot[0] == T_ref, kw
            np.testing.assert_array_equal(tv, tv_ref)
            assert h.count_total()[0] == T_ref
            want = {1: 0, 2: -1}.get(kw["intersect"], kw.get("search_ratio", 0) or 64)
            assert h.info()["search_ratio"] == want


def test_count_time_override_and_reschedule(tc):
    g = graphgen.rmat(13, 16, seed=35)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    with tc.build_oriented([(g.n, g.src, g.dst)], intersect=1) as h:
        for kw in (dict(intersect=2), dict(search_ratio=3), dict()):
            tv, tot = h.count_per_node(**kw)
            assert tot[0] == T_ref
            np.testing.assert_array_equal(tv, tv_ref)
        h.reschedule(intersect=2)
        assert h.info()["search_ratio"] == -1
        tv, tot = h.count_per_node()
        np.testing.assert_array_equal(tv, tv_ref)


@pytest.mark.parametrize("kw", [dict(intersect=2), dict(intersect=0, search_ratio=1)])
def test_search_closed_forms_and_packed(tc, kw):
    graphs = [complete(60), wheel(40), complete(129), wheel(7), complete(300), complete(700)]
    with tc.build_oriented([(n, s, d) for n, s, d in graphs], **kw) as h:
        tv, tot = h.count_per_node()
    base = 0
    for (n, s, d), T in zip(graphs, tot):
        T_ref, tv_ref, _ = oracle.count(n, s, d)
        assert T == T_ref
        np.testing.assert_array_equal(tv[base:base + n], tv_ref)
        base += n


def test_search_partitioned(tc):
    g = graphgen.rmat(14, 16, seed=36)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    for kw in (dict(intersect=2), dict(intersect=0, search_ratio=2)):
        with tc.build_oriented([(g.n, g.src, g.dst)], partitions=5, **kw) as h:
            assert h.info()["partitions"] >= 5
            tv, tot = h.count_per_node()
        assert tot[0] == T_ref
        np.testing.assert_array_equal(tv, tv_ref)


def test_batch_with_per_handle_choices(tc):
    gs = [graphgen.chung_lu(4000, 50_000, 2.1, 40 + i) for i in range(3)]
    refs = [oracle.count(g.n, g.src, g.dst) for g in gs]
    hs = [tc.build_oriented([(g.n, g.src, g.dst)], intersect=v) for g, v in zip(gs, (0, 1, 2))]
    tots, pns = tc.count_batch(hs, per_node=True)
    for t, pn, r in zip(tots, pns, refs):
        assert t[0] == r[0]
        np.testing.assert_array_equal(pn, r[1])
    for h in hs:
        h.free()
