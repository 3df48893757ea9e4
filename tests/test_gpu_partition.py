"""GPU parity of the partitioned form (node-range slices with streamed list
ranges, Section IV-C): results must equal the oracle and the resident form
exactly, for any number of slices (Theorem 1) and under device budgets that
force bucketed builds, several slices and several streamed batches per slice.
"""
import math

import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs_small as gs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_5687_amd as tcmod

    tcmod.load()
    return tcmod


def counts(h):
    tv, tot = h.count_per_node()
    tot2 = h.count_total()
    assert tot2[0] == tot[0]
    return int(tot[0]), tv


def check_partitioned(tc, g, P, **kw):
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    with tc.build_oriented([(g.n, g.src, g.dst)], partitions=P, **kw) as h:
        T, tv = counts(h)
        info = h.info()
    assert T == T_ref
    np.testing.assert_array_equal(tv, tv_ref)
    assert info["partitions"] >= min(P, g.n)
    return info


GRAPHS = {
    "cl3k": lambda: graphgen.chung_lu(3000, 24000, 2.1, 3),
    "er2k": lambda: graphgen.erdos_renyi(2000, 20000, 5),
    "rmat12": lambda: graphgen.rmat(12, 16, seed=7),
    "pa4k": lambda: graphgen.preferential_attachment(4000, 12, 2),
}


@pytest.mark.parametrize("P", [1, 2, 3, 7, 16])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_partition_invariance(tc, name, P):
    print(f"partitioned {name} P={P}", flush=True)
    info = check_partitioned(tc, GRAPHS[name](), P)
    assert info["streamed_bytes"] > 0


@pytest.mark.parametrize("P", [2, 5])
def test_closed_forms_partitioned(tc, P):
    for n in (4, 30, 200):
        nn, s, d = gs.complete(n)
        with tc.build_oriented([(nn, s, d)], partitions=P) as h:
            T, tv = counts(h)
        assert T == math.comb(n, 3) and (tv == math.comb(n - 1, 2)).all()
    nn, s, d = gs.wheel(101)
    with tc.build_oriented([(nn, s, d)], partitions=P) as h:
        T, tv = counts(h)
    assert T == 100 and tv[0] == 100 and (tv[1:] == 2).all()
    nn, s, d = gs.complete_bipartite(20, 30)
    with tc.build_oriented([(nn, s, d)], partitions=P) as h:
        T, tv = counts(h)
    assert T == 0 and not tv.any()


def test_partitioned_long_lists(tc):
    # K_1100: lists past 768 entries (8-wave workgroups) and, with a small
    # LDS cap, the binary-search path, all fed from streamed ranges
    nn, s, d = gs.complete(1100)
    for kw in (dict(), dict(lds_list_max=64)):
        with tc.build_oriented([(nn, s, d)], partitions=4, **kw) as h:
            T, tv = counts(h)
        assert T == math.comb(1100, 3) and (tv == math.comb(1099, 2)).all()


def test_partitioned_degenerate(tc):
    z = np.zeros(0, np.int32)
    with tc.build_oriented([(10, z, z)], partitions=3) as h:
        T, tv = counts(h)
    assert T == 0 and tv.shape == (10,) and not tv.any()
    # loops and repeats only
    s = np.array([1, 2, 2, 3, 1], np.int32)
    d = np.array([1, 3, 3, 2, 2], np.int32)
    with tc.build_oriented([(5, s, d)], partitions=2) as h:
        T, tv = counts(h)
        assert h.info()["m"] == 2
    assert T == 0 and not tv.any()
    # more slices than nodes
    nn, s, d = gs.complete(5)
    with tc.build_oriented([(nn, s, d)], partitions=16) as h:
        T, tv = counts(h)
    assert T == 10 and (tv == 6).all()
    with pytest.raises(tc.tc.IdRangeError):
        tc.build_oriented([(3, np.array([0, 3], np.int32), np.array([1, 1], np.int32))], partitions=2)


def test_partitioned_csr_equals_resident(tc):
    g = graphgen.rmat(12, 16, seed=3)
    with tc.build_oriented([(g.n, g.src, g.dst)]) as h:
        off, col, perm = h.export_csr()
    with tc.build_oriented([(g.n, g.src, g.dst)], partitions=5) as h:
        off2, col2, perm2 = h.export_csr()
        with pytest.raises(tc.tc.InvalidArgument):
            h.export_schedule()
    np.testing.assert_array_equal(off, off2)
    np.testing.assert_array_equal(col, col2)
    np.testing.assert_array_equal(perm, perm2)


def test_partitioned_device_io_and_reschedule(tc):
    import torch

    g = graphgen.chung_lu(5000, 60000, 2.1, 11)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    with tc.build_oriented([(g.n, src, dst)], partitions=3) as h:
        out = torch.full((g.n,), -7, dtype=torch.int64, device="cuda")
        tot = torch.zeros(1, dtype=torch.int64, device="cuda")
        h.count_per_node(out=out, totals=tot)
        torch.cuda.synchronize()
        assert int(tot.item()) == T_ref
        np.testing.assert_array_equal(out.cpu().numpy(), tv_ref)
        h.reschedule(workers=64, small_max=16, min_chunk=1)
        T, tv = counts(h)
        assert T == T_ref
        np.testing.assert_array_equal(tv, tv_ref)
        with pytest.raises(tc.tc.InvalidArgument):
            tc.count_batch([h])


def test_budget_forces_buckets_slices_and_batches(tc):
    # 2M input edges under a 48 MiB budget: the canonical set is built in
    # several buckets, the graph is counted in several slices, and the streamed
    # ranges of a slice come in several batches.
    g = graphgen.chung_lu(200_000, 2_000_000, 2.1, 5)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    budget = 48 << 20
    with tc.build_oriented([(g.n, g.src, g.dst)], hbm_budget_bytes=budget) as h:
        info = h.info()
        T, tv = counts(h)
        info2 = h.info()
    print("budget run:", info2, flush=True)
    assert T == T_ref
    np.testing.assert_array_equal(tv, tv_ref)
    assert info["partitions"] > 1
    assert info2["peak_device_bytes"] <= budget


def test_budget_resident_when_it_fits(tc):
    g = graphgen.rmat(11, 16, seed=4)
    with tc.build_oriented([(g.n, g.src, g.dst)], hbm_budget_bytes=1 << 30) as h:
        info = h.info()
        T, tv = counts(h)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    assert info["partitions"] == 1 and T == T_ref
    np.testing.assert_array_equal(tv, tv_ref)


def test_budget_too_small(tc):
    g = graphgen.chung_lu(200_000, 400_000, 2.1, 5)
    with pytest.raises(tc.tc.OutOfMemory):
        tc.build_oriented([(g.n, g.src, g.dst)], hbm_budget_bytes=8 << 20)


def test_partitioned_batch_form_rejects_several_graphs(tc):
    a = graphgen.rmat(8, 8, seed=1)
    with pytest.raises(tc.tc.InvalidArgument):
        tc.build_oriented([(a.n, a.src, a.dst), (a.n, a.src, a.dst)], partitions=2)


@pytest.mark.parametrize("P", [2, 5])
def test_direct_scheme_equals_surrogate(tc, P):
    # one streamed range per stored edge instead of one per slice: same counts,
    # more bytes over the host link
    g = graphgen.chung_lu(4000, 40000, 2.1, 9)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    got = {}
    for direct in (False, True):
        with tc.build_oriented([(g.n, g.src, g.dst)], partitions=P, direct=direct) as h:
            T, tv = counts(h)
            got[direct] = h.info()["streamed_bytes"]
        assert T == T_ref
        np.testing.assert_array_equal(tv, tv_ref)
    assert got[True] > got[False]
