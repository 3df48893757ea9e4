"""GPU parity of the serving form: every request's T and T_v equal the oracle
and the same request served alone, whatever batch it landed in."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tcmod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_5687_amd as tcmod

    tcmod.load()
    return tcmod


def arena(count, seed=1, hi=2e5):
    from paper_1406_5687_amd import serve

    gs = [sp.make() for sp in graphgen.serve_specs(count, seed=seed, hi=hi)]
    ar = serve.Arena([g.n for g in gs], [g.m for g in gs])
    for i, g in enumerate(gs):
        ar.put(i, g.src, g.dst)
    return ar, gs


@pytest.mark.parametrize("rate,streams", [(0, 3), (400.0, 2), (2000.0, 4)])
def test_served_equals_oracle_and_alone(tcmod, rate, streams):
    from paper_1406_5687_amd import serve

    ar, gs = arena(48)
    arr = graphgen.poisson_arrivals(48, rate, 1) if rate else None
    srv = serve.Server(streams=streams, hbm_budget_bytes=1 << 30, max_batch_edges=1 << 21, max_batch_graphs=16)
    ar.clear_results()
    res = srv.run(ar, arr)
    assert sorted(res.batches)[0][0] == 0 and sum(b - a for a, b in res.batches) == 48
    for i, g in enumerate(gs):
        T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
        assert ar.tot[i] == T_ref
        np.testing.assert_array_equal(ar.per_node(i), tv_ref)
    for i in range(0, 48, 5):
        T, tv, _ = serve.serve_alone(ar, i)
        assert T == ar.tot[i]
        np.testing.assert_array_equal(tv, ar.per_node(i))
    assert (res.latency > 0).all()


def test_budget_smaller_than_a_request(tcmod):
    from paper_1406_5687_amd import serve

    ar, gs = arena(12, seed=3)
    small = min(serve.device_footprint(g.n, g.m) for g in gs)
    srv = serve.Server(streams=2, hbm_budget_bytes=small)  # every batch holds one request
    ar.clear_results()
    res = srv.run(ar)
    assert all(b - a == 1 for a, b in res.batches)
    for i, g in enumerate(gs):
        assert ar.tot[i] == oracle.count(g.n, g.src, g.dst, per_node=False)[0]


def test_plain_loop_matches(tcmod):
    from paper_1406_5687_amd import serve

    ar, gs = arena(10, seed=5)
    ar.clear_results()
    serve.run_plain(ar)
    for i, g in enumerate(gs):
        T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
        assert ar.tot[i] == T_ref
        np.testing.assert_array_equal(ar.per_node(i), tv_ref)


def test_packed_device_build_in_place(tcmod):
    import torch

    gs = [graphgen.rmat(10, 8, seed=s) for s in range(5)] + [graphgen.EdgeList(9, np.zeros(0, np.int32),
                                                                                np.zeros(0, np.int32))]
    ns = [g.n for g in gs]
    ms = [g.m for g in gs]
    src = torch.from_numpy(np.concatenate([g.src for g in gs])).cuda()
    dst = torch.from_numpy(np.concatenate([g.dst for g in gs])).cuda()
    with tcmod.tc.build_packed_device(ns, ms, src.data_ptr(), dst.data_ptr()) as h:
        tv, tot = h.count_per_node()
    b = 0
    for i, g in enumerate(gs):
        T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
        assert tot[i] == T_ref
        np.testing.assert_array_equal(tv[b:b + g.n], tv_ref)
        b += g.n


def test_resident_adjacency_answers_repeat_requests(tcmod):
    """Requests cycling over 12 graphs: with the adjacencies kept resident, a
    second pass over the same requests is answered by count launches only
    (no build), and every answer equals the oracle; with a budget for about
    one batch, handles are released and rebuilt, with the same answers."""
    from paper_1406_5687_amd import serve

    base = [sp.make() for sp in graphgen.serve_specs(12, seed=5, hi=2e5)]
    keys = [i % 12 for i in range(40)]
    gs = [base[k] for k in keys]
    ar = serve.Arena([g.n for g in gs], [g.m for g in gs], keys=keys)
    for i, g in enumerate(gs):
        ar.put(i, g.src, g.dst)
    refs = [oracle.count(g.n, g.src, g.dst) for g in base]

    def check():
        for i, k in enumerate(keys):
            assert ar.tot[i] == refs[k][0]
            np.testing.assert_array_equal(ar.per_node(i), refs[k][1])

    srv = serve.Server(streams=3, hbm_budget_bytes=1 << 30, max_batch_edges=1 << 21, max_batch_graphs=8,
                       resident_bytes=1 << 34)
    ar.clear_results()
    first = srv.run(ar, graphgen.poisson_arrivals(40, 200.0, 3))
    check()
    assert first.builds >= 1
    ar.clear_results()
    again = srv.run(ar)
    check()
    assert again.builds == 0 and again.resident_hits == 40
    assert again.m_canonical == first.m_canonical
    srv.close()
    small = serve.Server(streams=2, hbm_budget_bytes=1 << 30, max_batch_edges=1 << 21, max_batch_graphs=4,
                         resident_bytes=serve.device_footprint(max(g.n for g in base), max(g.m for g in base)))
    for _ in range(2):
        ar.clear_results()
        small.run(ar)
        check()
    small.close()
