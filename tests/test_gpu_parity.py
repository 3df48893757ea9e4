"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every comparison is exact (integer counts, labels and boundaries): tolerance 0.
"""
import math

import numpy as np
import pytest

import graphgen
import oracle
from tests import golden_io
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


def gpu_count(tc, n, src, dst, **kw):
    with tc.build_oriented([(n, src, dst)], **kw) as g:
        tv, tot = g.count_per_node()
        tot2 = g.count_total()
        assert tot2[0] == tot[0]
        return int(tot[0]), tv


def check(tc, n, src, dst, **kw):
    T_ref, tv_ref, _ = oracle.count(n, src, dst)
    T, tv = gpu_count(tc, n, src, dst, **kw)
    assert T == T_ref
    np.testing.assert_array_equal(tv, tv_ref)
    return T


# ------------------------------------------------------------ small cases

@pytest.mark.parametrize("name", golden_io.all_graphs())
def test_golden(tc, name):
    g = golden_io.graph(name)
    T, tv = gpu_count(tc, g["n"], g["src"], g["dst"])
    assert T == g["T"]
    np.testing.assert_array_equal(tv, g["Tv"])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 9, 30, 64, 65, 129, 200])
def test_complete(tc, n):
    T, tv = gpu_count(tc, *gs.complete(n))
    assert T == math.comb(n, 3)
    assert (tv == math.comb(n - 1, 2)).all()


@pytest.mark.parametrize("n", [5, 7, 100, 1000])
def test_wheel(tc, n):
    T, tv = gpu_count(tc, *gs.wheel(n))
    assert T == n - 1 and tv[0] == n - 1 and (tv[1:] == 2).all()


@pytest.mark.parametrize("g", [gs.complete_bipartite(5, 7), gs.complete_bipartite(1, 300), gs.grid(30, 40),
                               gs.hypercube(10), gs.cycle(1000)])
def test_bipartite(tc, g):
    T, tv = gpu_count(tc, *g)
    assert T == 0 and not tv.any()


def test_empty_inputs(tc):
    T, tv = gpu_count(tc, 10, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert T == 0 and tv.shape == (10,) and not tv.any()
    T, tv = gpu_count(tc, 5, np.array([1, 2, 3], np.int32), np.array([1, 2, 3], np.int32))
    assert T == 0 and not tv.any()
    with tc.build_oriented([(0, np.zeros(0, np.int32), np.zeros(0, np.int32))]) as g:
        assert g.count_total()[0] == 0


@pytest.mark.parametrize("seed", range(6))
def test_random_gnp(tc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 300))
    n, s, d = gs.gnp(n, float(rng.uniform(0.01, 0.6)), rng)
    check(tc, n, s, d)


def test_id_range_error(tc):
    with pytest.raises(tc.tc.IdRangeError):
        tc.build_oriented([(3, np.array([0, 3], np.int32), np.array([1, 1], np.int32))])
    with pytest.raises(tc.tc.IdRangeError):
        tc.build_oriented([(3, np.array([0, -1], np.int32), np.array([1, 1], np.int32))])


# ------------------------------------------------------------ workload shapes

@pytest.mark.parametrize("maker", [
    lambda: graphgen.workload_er(1),
    lambda: graphgen.workload_er(2),
    lambda: graphgen.preferential_attachment(50_000, 20, 3),
    lambda: graphgen.preferential_attachment(20_000, 50, 4),
    lambda: graphgen.rmat(14, 16, seed=5),
    lambda: graphgen.rmat(16, 16, seed=6),
    lambda: graphgen.chung_lu(40_000, 640_000, 2.1, 7),
], ids=["er1", "er2", "pa50k", "pa20k_d50", "rmat14", "rmat16", "cl40k"])
def test_workloads(tc, maker):
    g = maker()
    check(tc, g.n, g.src, g.dst)


def test_device_inputs_and_outputs(tc):
    import torch

    g = graphgen.rmat(13, 16, seed=9)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    with tc.build_oriented([(g.n, src, dst)]) as h:
        out = torch.full((g.n,), -7, dtype=torch.int64, device="cuda")
        tot = torch.zeros(1, dtype=torch.int64, device="cuda")
        h.count_per_node(out=out, totals=tot)
        t2 = torch.zeros(1, dtype=torch.int64, device="cuda")
        h.count_total(out=t2)
        torch.cuda.synchronize()
        assert int(tot.item()) == T_ref == int(t2.item())
        np.testing.assert_array_equal(out.cpu().numpy(), tv_ref)


# ------------------------------------------------------------ build parity (a1-a3)

@pytest.mark.parametrize("maker", [
    lambda: graphgen.workload_er(1),
    lambda: graphgen.rmat(12, 16, seed=2),
    lambda: graphgen.preferential_attachment(5000, 10, 3),
], ids=["er", "rmat12", "pa5k"])
def test_oriented_csr_matches_oracle(tc, maker):
    g = maker()
    m, off_o, col_o, deg = oracle.orient(g.n, g.src, g.dst)
    perm_o = oracle.degree_order(deg)
    with tc.build_oriented([(g.n, g.src, g.dst)]) as h:
        off, col, perm = h.export_csr()
        info = h.info()
    assert info["m"] == m
    np.testing.assert_array_equal(perm, perm_o)               # degree order, ties by id
    rank = np.empty(g.n, np.int64)
    rank[perm] = np.arange(g.n)
    dh = np.diff(off)
    np.testing.assert_array_equal(dh, np.diff(off_o)[perm])   # effective degrees
    for r in range(g.n):
        row = col[off[r]:off[r + 1]]
        assert (np.diff(row) > 0).all()                       # rows ascending
        expect = np.sort(rank[col_o[off_o[perm[r]]:off_o[perm[r] + 1]]])
        np.testing.assert_array_equal(row, expect)
    assert info["max_out_degree"] == int(dh.max(initial=0))


# ------------------------------------------------------------ schedule parity (a4)

@pytest.mark.parametrize("cost", [0, 1, 2, 3])
@pytest.mark.parametrize("W,floor", [(64, 1), (4096, 0), (7, 500)])
def test_schedule_matches_oracle(tc, cost, W, floor):
    g = graphgen.preferential_attachment(20_000, 8, 11)
    m, off_o, col_o, deg = oracle.orient(g.n, g.src, g.dst)
    perm = oracle.degree_order(deg)
    f_orig = oracle.costs(off_o, col_o, deg, cost)
    f = f_orig[perm].copy()
    dh = np.diff(off_o)[perm]
    f[dh > 128] = 0                       # long lists go to the workgroup kernel
    total = int(f.sum())
    min_chunk = floor if floor > 0 else max(256, total // (W * 128 + 1))
    bnd_ref = oracle.schedule(f, W, min_chunk)
    with tc.build_oriented([(g.n, g.src, g.dst)], workers=W, cost_fn=cost, min_chunk=floor) as h:
        bnd, gid = h.export_schedule()
        info = h.info()
        tv, tot = h.count_per_node()
    np.testing.assert_array_equal(bnd, bnd_ref)
    assert info["total_cost"] == total
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    assert tot[0] == T_ref
    np.testing.assert_array_equal(tv, tv_ref)


def test_schedule_rounds_matches_oracle(tc):
    # rounds R: Eq. (1)/(2) with W * R workers; the automatic floor still uses W
    g = graphgen.preferential_attachment(20_000, 8, 12)
    m, off_o, col_o, deg = oracle.orient(g.n, g.src, g.dst)
    perm = oracle.degree_order(deg)
    f = oracle.costs(off_o, col_o, deg, oracle.COST_PRIOR)[perm].copy()
    f[np.diff(off_o)[perm] > 128] = 0
    total = int(f.sum())
    W, R = 64, 5
    bnd_ref = oracle.schedule(f, W * R, max(256, total // (W * 128 + 1)))
    with tc.build_oriented([(g.n, g.src, g.dst)], workers=W, rounds=R) as h:
        bnd, _ = h.export_schedule()
        assert h.info()["rounds"] == R
    np.testing.assert_array_equal(bnd, bnd_ref)


def test_static_chunks_schedule(tc):
    # comparison schedule: W tasks of equal cost (boundary i at the first node
    # whose cost prefix reaches ceil(i * total / W))
    g = graphgen.preferential_attachment(20_000, 8, 13)
    m, off_o, col_o, deg = oracle.orient(g.n, g.src, g.dst)
    perm = oracle.degree_order(deg)
    f = oracle.costs(off_o, col_o, deg, oracle.COST_PRIOR)[perm].copy()
    f[np.diff(off_o)[perm] > 128] = 0
    F = np.concatenate([[0], np.cumsum(f)])
    total = int(F[-1])
    W = 50
    expect = [0] + [int(np.searchsorted(F, -(-(i * total) // W), side="left")) for i in range(1, W)] + [g.n]
    with tc.build_oriented([(g.n, g.src, g.dst)], workers=W, static_chunks=True) as h:
        bnd, _ = h.export_schedule()
        tv, tot = h.count_per_node(time_kernels=2)
        times = h.worker_times()
    np.testing.assert_array_equal(bnd, expect)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    assert tot[0] == T_ref
    np.testing.assert_array_equal(tv, tv_ref)
    assert times.shape[0] >= 1 and (times[:, 0] >= 0).all() and (times[:, 1] >= times[:, 0]).all()
    assert set(times[:, 2].tolist()) <= {0, 1, 2} and (times[:, 2] == 0).any()


# ------------------------------------------------------------ invariance (Section V-D)

@pytest.mark.parametrize("kw", [
    dict(workers=1), dict(workers=7), dict(workers=64), dict(workers=20000),
    dict(small_max=2), dict(small_max=16), dict(small_max=128),
    dict(lds_list_max=2), dict(lds_list_max=50), dict(small_max=4, lds_list_max=8),
    dict(cost_fn=0), dict(cost_fn=1), dict(cost_fn=3), dict(min_chunk=1), dict(min_chunk=10**12),
    dict(rounds=7), dict(rounds=64), dict(workers=3, rounds=1000),
], ids=lambda kw: ",".join(f"{k}={v}" for k, v in kw.items()))
def test_tuning_invariance(tc, kw):
    g = graphgen.rmat(13, 16, seed=13)
    check(tc, g.n, g.src, g.dst, **kw)


@pytest.mark.parametrize("n", [300, 1100, 4200])
def test_long_lists_all_paths(tc, n):
    # K_n: lists up to n-1 entries.  300 -> 4-wave workgroups; 1100 -> also the
    # 8-wave workgroups; 4200 -> also lists longer than the LDS table (binary
    # search in device memory).  Smaller lds_list_max forces the binary-search
    # path in both workgroup kernels.
    nn, s, d = gs.complete(n)
    for kw in (dict(), dict(lds_list_max=64), dict(small_max=8, lds_list_max=16)):
        if n == 4200 and kw:
            continue
        T, tv = gpu_count(tc, nn, s, d, **kw)
        assert T == math.comb(n, 3) and (tv == math.comb(n - 1, 2)).all()


# ------------------------------------------------------------ metamorphic

def test_relabel_and_input_noise(tc):
    g = graphgen.rmat(12, 16, seed=21)
    T, tv = gpu_count(tc, g.n, g.src, g.dst)
    rng = np.random.default_rng(0)
    pi = rng.permutation(g.n).astype(np.int32)
    T2, tv2 = gpu_count(tc, g.n, pi[g.src], pi[g.dst])
    assert T2 == T
    np.testing.assert_array_equal(tv2[pi], tv)
    order = rng.permutation(g.m)
    s = np.concatenate([g.dst[order], g.src[:500], np.arange(40, dtype=np.int32)])
    d = np.concatenate([g.src[order], g.dst[:500], np.arange(40, dtype=np.int32)])
    T3, tv3 = gpu_count(tc, g.n, s, d)
    assert T3 == T
    np.testing.assert_array_equal(tv3, tv)


def _complete(n):
    iu = np.triu_indices(n, 1)
    return graphgen.EdgeList(n, iu[0].astype(np.int32), iu[1].astype(np.int32), f"K{n}")


@pytest.mark.parametrize("maker,repeats", [
    (lambda: graphgen.preferential_attachment(5000, 10, 3), 1),
    (lambda: graphgen.preferential_attachment(5000, 10, 3), 37),
    (lambda: graphgen.preferential_attachment(5000, 10, 3), 4000),
    (lambda: _complete(400), 1),       # rows longer than 256: the long-row sort sees the repeat
    (lambda: _complete(400), 500),
], ids=["pa-1", "pa-37", "pa-4000", "k400-1", "k400-500"])
def test_repeated_edges_without_loops(tc, maker, repeats):
    # A simple input is built without sorting the pairs; an edge given twice
    # (here without any loop, so only the sorted rows reveal it) must send the
    # build back to the canonical path: adjacency, schedule and counts as for
    # the edges given once.
    g = maker()
    rng = np.random.default_rng(repeats)
    pick = rng.integers(0, g.m, repeats)
    flip = rng.random(repeats) < 0.5
    s = np.concatenate([g.src, np.where(flip, g.dst[pick], g.src[pick])]).astype(np.int32)
    d = np.concatenate([g.dst, np.where(flip, g.src[pick], g.dst[pick])]).astype(np.int32)
    with tc.build_oriented([(g.n, g.src, g.dst)]) as h1, tc.build_oriented([(g.n, s, d)]) as h2:
        a1, a2 = h1.export_csr(), h2.export_csr()
        for x, y in zip(a1, a2):
            np.testing.assert_array_equal(x, y)
        i1, i2 = h1.info(), h2.info()
        assert i1["m"] == i2["m"] == g.m
        assert i1["tasks"] == i2["tasks"] and i1["total_cost"] == i2["total_cost"]
        tv1, t1 = h1.count_per_node()
        tv2, t2 = h2.count_per_node()
    np.testing.assert_array_equal(tv1, tv2)
    assert t1[0] == t2[0]
    check(tc, g.n, s, d)


def test_edge_list_orders(tc):
    # Degrees of a simple input are counted from runs of equal ids when the
    # list has long runs (made from adjacency lists), else by a histogram:
    # every order of the same edges gives the same handle.
    g = graphgen.workload_er(1)
    rng = np.random.default_rng(5)
    lo, hi = np.minimum(g.src, g.dst), np.maximum(g.src, g.dst)
    o = np.lexsort((hi, lo))
    shuf = rng.permutation(g.m)
    by_hi = np.argsort(hi, kind="stable")
    orders = [
        (g.src, g.dst),           # as drawn
        (lo[o], hi[o]),           # sorted by the smaller id: long runs in src
        (hi[o], lo[o]),           # the same with the columns swapped: long runs in dst
        (lo[shuf], hi[shuf]),     # shuffled
        (hi[by_hi], lo[by_hi]),   # sorted by the larger id
    ]
    ref = None
    for s, d in orders:
        s = np.ascontiguousarray(s, dtype=np.int32)
        d = np.ascontiguousarray(d, dtype=np.int32)
        with tc.build_oriented([(g.n, s, d)]) as h:
            got = tuple(np.asarray(x) for x in h.export_csr()) + (h.count_per_node()[0],)
        if ref is None:
            ref = got
        else:
            for x, y in zip(ref, got):
                np.testing.assert_array_equal(x, y)
    check(tc, g.n, np.ascontiguousarray(lo[o], dtype=np.int32), np.ascontiguousarray(hi[o], dtype=np.int32))


# ------------------------------------------------------------ packed graphs and batches

def test_packed_handle_equals_separate(tc):
    parts = [graphgen.rmat(10, 16, seed=1), graphgen.erdos_renyi(0 + 500, 3000, 2),
             graphgen.EdgeList(0, np.zeros(0, np.int32), np.zeros(0, np.int32)),
             graphgen.preferential_attachment(3000, 12, 3), graphgen.chung_lu(2000, 30000, 2.1, 4),
             graphgen.EdgeList(7, np.zeros(0, np.int32), np.zeros(0, np.int32))]
    with tc.build_oriented([(p.n, p.src, p.dst) for p in parts]) as h:
        tv, tot = h.count_per_node()
        tot2 = h.count_total()
        bnd, gid = h.export_schedule()
    np.testing.assert_array_equal(tot, tot2)
    base = 0
    for i, p in enumerate(parts):
        T_ref, tv_ref, _ = oracle.count(p.n, p.src, p.dst)
        assert tot[i] == T_ref
        np.testing.assert_array_equal(tv[base:base + p.n], tv_ref)
        base += p.n
    # no task spans two graphs
    nb = np.cumsum([0] + [p.n for p in parts])
    for c in range(len(gid)):
        if bnd[c] < bnd[c + 1]:
            assert nb[gid[c]] <= bnd[c] and bnd[c + 1] <= nb[gid[c] + 1]


def _sparse_core(n, core_n, pendants, seed):
    # a dense core, pendant nodes hanging off it, and isolated nodes: most
    # labels of the degree order have degree 0 or 1 and come first
    core = graphgen.preferential_attachment(core_n, 6, seed)
    rng = np.random.default_rng(seed)
    pend = (core_n + rng.permutation(n - core_n)[:pendants]).astype(np.int32)
    src = np.concatenate([core.src, pend])
    dst = np.concatenate([core.dst, rng.integers(0, core_n, pendants).astype(np.int32)])
    return src, dst


@pytest.mark.parametrize("kw", [dict(workers=7), dict(workers=64), dict(workers=4096),
                                dict(workers=64, cost_fn=0), dict(workers=64, cost_fn=1),
                                dict(workers=50, static_chunks=True)])
def test_leading_low_degree_block(tc, kw):
    # tasks reaching into the leading labels of degree < 2 start their scan
    # past them; counts and the exported Eq. (1)/(2) schedule are unchanged
    n = 300_000
    src, dst = _sparse_core(n, 3000, 40_000, 31)
    T_ref, tv_ref, _ = oracle.count(n, src, dst)
    with tc.build_oriented([(n, src, dst)], **kw) as h:
        tv, tot = h.count_per_node()
        tot2 = h.count_total()
        bnd, _ = h.export_schedule()
    assert tot[0] == T_ref and tot2[0] == T_ref
    np.testing.assert_array_equal(tv, tv_ref)
    if len(kw) == 1:
        W = kw["workers"]
        m, off_o, col_o, deg = oracle.orient(n, src, dst)
        perm = oracle.degree_order(deg)
        f = oracle.costs(off_o, col_o, deg, oracle.COST_PRIOR)[perm].copy()
        f[np.diff(off_o)[perm] > 128] = 0
        total = int(f.sum())
        np.testing.assert_array_equal(bnd, oracle.schedule(f, W, max(256, total // (W * 128 + 1))))
        assert bnd[0] == 0 and (np.diff(bnd) >= 0).all()


def test_leading_low_degree_blocks_packed(tc):
    # every packed graph leads with its own block of degree < 2
    parts = [_sparse_core(n, c, p, s) for n, c, p, s in
             ((120_000, 1500, 20_000, 41), (5_000, 4000, 100, 42), (80_000, 900, 30_000, 43))]
    ns = (120_000, 5_000, 80_000)
    with tc.build_oriented([(n, s_, d_) for n, (s_, d_) in zip(ns, parts)], workers=64) as h:
        tv, tot = h.count_per_node()
        tot2 = h.count_total()
    np.testing.assert_array_equal(tot, tot2)
    base = 0
    for i, (n, (s_, d_)) in enumerate(zip(ns, parts)):
        T_ref, tv_ref, _ = oracle.count(n, s_, d_)
        assert tot[i] == T_ref
        np.testing.assert_array_equal(tv[base:base + n], tv_ref)
        base += n


def test_batch_of_handles_equals_separate(tc):
    parts = [graphgen.rmat(11, 16, seed=s) for s in range(3)] + [graphgen.erdos_renyi(800, 5000, 9)]
    hs = [tc.build_oriented([(p.n, p.src, p.dst)]) for p in parts]
    hs.append(tc.build_oriented([(p.n, p.src, p.dst) for p in parts[:2]]))
    tots, tvs = tc.count_batch(hs, per_node=True)
    tots_only, _ = tc.count_batch(hs, per_node=False)
    for h, t, t2, tv in zip(hs, tots, tots_only, tvs):
        tv1, t1 = h.count_per_node()
        np.testing.assert_array_equal(t, t1)
        np.testing.assert_array_equal(t2, t1)
        np.testing.assert_array_equal(tv, tv1)
    for h in hs:
        h.free()


# ------------------------------------------------------------ full-size workloads

@pytest.mark.slow
def test_full_er_config(tc):
    g = graphgen.workload_er(1)
    check(tc, g.n, g.src, g.dst)


@pytest.mark.slow
def test_full_pa_config(tc):
    """PA(10^6, 50) at full size, in the launch configuration the bench times:
    per-node counts compared element by element with the oracle."""
    import torch

    g = graphgen.workload_pa(1)
    T_ref, tv_ref, m = oracle.count(g.n, g.src, g.dst)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    with tc.build_oriented([(g.n, src, dst)]) as h:
        out = torch.zeros(g.n, dtype=torch.int64, device="cuda")
        tot = torch.zeros(1, dtype=torch.int64, device="cuda")
        h.count_per_node(out=out, totals=tot)
        torch.cuda.synchronize()
        assert h.info()["m"] == m
    assert int(tot.item()) == T_ref
    np.testing.assert_array_equal(out.cpu().numpy(), tv_ref)


# ------------------------------------------------------------ clustering epilogue (Section I applications)

@pytest.mark.parametrize("maker", [
    lambda: graphgen.workload_er(1),
    lambda: graphgen.rmat(13, 16, seed=3),
    lambda: graphgen.preferential_attachment(20_000, 12, 5),
    lambda: gs.wheel(50),
    lambda: gs.complete(40),
    lambda: gs.grid(20, 30),
], ids=["er", "rmat13", "pa20k", "wheel", "k40", "grid"])
def test_clustering_matches_oracle(tc, maker):
    g = maker()
    n, s, d = (g.n, g.src, g.dst) if hasattr(g, "src") else g
    coeff_ref, tr_ref, _ = oracle.clustering(n, s, d)
    T_ref, _, _ = oracle.count(n, s, d, per_node=False)
    with tc.build_oriented([(n, s, d)]) as h:
        coeff, tr, tot = h.clustering()
    # one fp64 division of the same two integers on both sides: bit-exact
    np.testing.assert_array_equal(coeff, coeff_ref)
    assert tr[0] == tr_ref and tot[0] == T_ref


def test_clustering_packed_graphs(tc):
    parts = [graphgen.rmat(10, 16, seed=1), graphgen.EdgeList(3, np.zeros(0, np.int32), np.zeros(0, np.int32)),
             graphgen.erdos_renyi(800, 6000, 2), graphgen.chung_lu(2000, 30000, 2.1, 4)]
    with tc.build_oriented([(p.n, p.src, p.dst) for p in parts]) as h:
        coeff, tr, tot = h.clustering()
    b = 0
    for i, p in enumerate(parts):
        c_ref, t_ref, _ = oracle.clustering(p.n, p.src, p.dst)
        np.testing.assert_array_equal(coeff[b:b + p.n], c_ref)
        assert tr[i] == t_ref
        b += p.n
