"""Pins for the CPU oracle: checks against facts fixed by the paper and by
mathematics, never against the oracle itself.

- brute force over all triples (the naive method, Section III-A);
- trace(A^3)/6 and diag(A^3)/2 (textbook identity);
- closed forms (complete, bipartite, wheel, friendship, tripartite graphs);
- networkx.triangles as an independent library;
- hand-derived fixtures under tests/golden/ (each cites its passage);
- invariants: sum of T_v = 3T, T_v <= C(d_v, 2), effective degree bound;
- metamorphic properties of the problem statement (Section II);
- Theorem 1 (partition invariance of Fig. 3) and Section V-D (task
  invariance of Fig. 11).
"""
import math

import numpy as np
import pytest

import graphgen
import oracle
from tests import golden_io
from tests import graphs_small as gs


def run(n, src, dst):
    T, Tv, m = oracle.count(n, src, dst)
    return T, Tv


# ------------------------------------------------------------ brute force

@pytest.mark.parametrize("seed", range(12))
def test_brute_force_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 28))
    p = float(rng.uniform(0.05, 0.9))
    n, s, d = gs.gnp(n, p, rng)
    # sprinkle loops, repeats and reversals into the input
    extra = rng.integers(0, len(s) + 1, size=min(len(s), 6)) if len(s) else []
    s2 = np.concatenate([s, d[extra[:3]] if len(s) else [], np.arange(min(n, 3))]).astype(np.int32)
    d2 = np.concatenate([d, s[extra[:3]] if len(s) else [], np.arange(min(n, 3))]).astype(np.int32)
    T, Tv = run(n, s2, d2)
    Tb, Tvb = gs.brute_force(n, s2, d2)
    assert T == Tb
    np.testing.assert_array_equal(Tv, Tvb)


def test_brute_force_hypothesis():
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies

    @hyp.settings(max_examples=150, deadline=None)
    @hyp.given(st.integers(1, 14).flatmap(
        lambda n: st.tuples(st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)),
                                                 max_size=60))))
    def check(case):
        n, pairs = case
        s = np.array([p[0] for p in pairs], np.int32)
        d = np.array([p[1] for p in pairs], np.int32)
        T, Tv = run(n, s, d)
        Tb, Tvb = gs.brute_force(n, s, d)
        assert T == Tb
        np.testing.assert_array_equal(Tv, Tvb)

    check()


# ------------------------------------------------------------ A^3 identity

@pytest.mark.parametrize("n,p,seed", [(60, 0.3, 1), (200, 0.08, 2), (400, 0.03, 3), (120, 0.7, 4)])
def test_trace_a_cubed(n, p, seed):
    rng = np.random.default_rng(seed)
    n, s, d = gs.gnp(n, p, rng)
    T, Tv = run(n, s, d)
    T3, Tv3 = gs.dense_cube(n, s, d)
    assert T == T3
    np.testing.assert_array_equal(Tv, Tv3)


def test_trace_a_cubed_power_law():
    g = graphgen.chung_lu(500, 4000, 2.1, seed=7)
    T, Tv = run(g.n, g.src, g.dst)
    T3, Tv3 = gs.dense_cube(g.n, g.src, g.dst)
    assert T == T3
    np.testing.assert_array_equal(Tv, Tv3)


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 9, 17, 30])
def test_complete_graph(n):
    T, Tv = run(*gs.complete(n))
    assert T == math.comb(n, 3)
    assert (Tv == math.comb(n - 1, 2)).all()


@pytest.mark.parametrize("g", [gs.complete_bipartite(1, 1), gs.complete_bipartite(5, 7), gs.complete_bipartite(1, 40),
                               gs.cycle(4), gs.cycle(10), gs.cycle(64), gs.grid(7, 9), gs.hypercube(6)])
def test_bipartite_is_triangle_free(g):
    T, Tv = run(*g)
    assert T == 0 and not Tv.any()


def test_random_trees_and_bipartite():
    rng = np.random.default_rng(11)
    for _ in range(5):
        assert run(*gs.random_tree(int(rng.integers(2, 300)), rng))[0] == 0
        assert run(*gs.random_bipartite(int(rng.integers(1, 40)), int(rng.integers(1, 40)), 0.4, rng))[0] == 0


@pytest.mark.parametrize("n", [5, 6, 7, 12, 101])
def test_wheel(n):
    T, Tv = run(*gs.wheel(n))
    assert T == n - 1
    assert Tv[0] == n - 1
    assert (Tv[1:] == 2).all()


def test_wheel_w4_is_k4():
    T, Tv = run(*gs.wheel(4))
    assert T == 4 and (Tv == 3).all()


def test_odd_cycle_c3():
    T, Tv = run(*gs.cycle(3))
    assert T == 1 and (Tv == 1).all()


@pytest.mark.parametrize("k", [1, 2, 5, 33])
def test_friendship(k):
    T, Tv = run(*gs.friendship(k))
    assert T == k and Tv[0] == k and (Tv[1:] == 1).all()


@pytest.mark.parametrize("a,b,c", [(1, 1, 1), (2, 3, 4), (5, 1, 7)])
def test_complete_tripartite(a, b, c):
    T, Tv = run(*gs.complete_tripartite(a, b, c))
    assert T == a * b * c
    np.testing.assert_array_equal(Tv, [b * c] * a + [a * c] * b + [a * b] * c)


def test_disjoint_union_adds():
    parts = [gs.complete(6), gs.wheel(9), gs.cycle(5), gs.friendship(4)]
    T, Tv = run(*gs.disjoint_union(*parts))
    Ts = [run(*p) for p in parts]
    assert T == sum(t for t, _ in Ts)
    np.testing.assert_array_equal(Tv, np.concatenate([tv for _, tv in Ts]))


def test_empty_and_isolated():
    assert run(0, np.zeros(0, np.int32), np.zeros(0, np.int32))[0] == 0
    T, Tv = run(10, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert T == 0 and Tv.shape == (10,) and not Tv.any()
    T, Tv = run(4, np.array([0, 1, 2], np.int32), np.array([0, 1, 2], np.int32))  # loops only
    assert T == 0 and not Tv.any()


def test_id_range_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.count(3, np.array([0, 3], np.int32), np.array([1, 1], np.int32))
    with pytest.raises(oracle.OracleError):
        oracle.count(3, np.array([-1], np.int32), np.array([1], np.int32))


# ------------------------------------------------------------ golden fixtures

@pytest.mark.parametrize("name", golden_io.all_graphs())
def test_golden_graph(name):
    g = golden_io.graph(name)
    T, Tv = run(g["n"], g["src"], g["dst"])
    assert T == g["T"]
    np.testing.assert_array_equal(Tv, g["Tv"])


@pytest.mark.parametrize("name", ["star_k1_5.orient", "cycle_c5.orient"])
def test_golden_orientation(name):
    g = golden_io.orientation(name)
    m, off, col, deg = oracle.orient(g["n"], g["src"], g["dst"])
    for v in range(g["n"]):
        assert col[off[v]:off[v + 1]].tolist() == g["rows"][v], f"row {v}"


@pytest.mark.parametrize("name", ["uniform16_w4.sched", "skewed8_w2.sched", "uniform7_w2.sched"])
def test_golden_schedule(name):
    g = golden_io.schedule(name)
    bnd = oracle.schedule(g["f"], g["W"], g["min_chunk"])
    np.testing.assert_array_equal(bnd, g["bnd"])


# ------------------------------------------------------------ independent library

@pytest.mark.parametrize("maker", [
    lambda: graphgen.erdos_renyi(3000, 30000, 5),
    lambda: graphgen.preferential_attachment(4000, 8, 6),
    lambda: graphgen.rmat(12, 8, seed=7),
    lambda: graphgen.chung_lu(5000, 40000, 2.1, 8),
])
def test_networkx(maker):
    nx = pytest.importorskip("networkx")
    g = maker()
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from((int(a), int(b)) for a, b in zip(g.src, g.dst) if a != b)
    tri = nx.triangles(G)
    T, Tv = run(g.n, g.src, g.dst)
    expect = np.array([tri[v] for v in range(g.n)], np.int64)
    np.testing.assert_array_equal(Tv, expect)
    assert T == int(expect.sum()) // 3


# ------------------------------------------------------------ invariants

@pytest.mark.parametrize("maker", [
    lambda: graphgen.preferential_attachment(20000, 10, 2),
    lambda: graphgen.rmat(13, 16, seed=3),
    lambda: graphgen.erdos_renyi(10000, 100000, 1),
])
def test_invariants(maker):
    g = maker()
    m, off, col, deg = oracle.orient(g.n, g.src, g.dst)
    T, Tv = oracle.count_oriented(g.n, off, col)
    assert Tv.sum() == 3 * T
    assert (Tv <= deg.astype(np.int64) * (deg.astype(np.int64) - 1) // 2).all()
    dhat = np.diff(off)
    assert dhat.sum() == m == deg.sum() // 2
    assert dhat.max(initial=0) <= math.isqrt(2 * m)
    # every stored pair is an edge of the input graph and each edge is stored once
    keys_in = set()
    for a, b in zip(g.src.tolist(), g.dst.tolist()):
        if a != b:
            keys_in.add((min(a, b), max(a, b)))
    stored = set()
    for v in range(g.n):
        row = col[off[v]:off[v + 1]]
        assert (np.diff(row) > 0).all()
        for u in row.tolist():
            stored.add((min(u, v), max(u, v)))
    assert stored == keys_in and len(stored) == m


def test_star_orientation_bound():
    # A leaf-to-hub orientation keeps every list at length 1; the reverse
    # direction would give the hub a list of length k > sqrt(2m).
    n, s, d = gs.star(500)
    m, off, col, deg = oracle.orient(n, s, d)
    assert off[1] - off[0] == 0 and np.diff(off).max() == 1


def test_degree_order_matches_lexsort():
    g = graphgen.preferential_attachment(3000, 5, 9)
    _, _, _, deg = oracle.orient(g.n, g.src, g.dst)
    perm = oracle.degree_order(deg)
    np.testing.assert_array_equal(perm, np.lexsort((np.arange(g.n), deg)))


def test_any_total_order_counts_once():
    # Section III-A: with any total order (here plain id order) each triangle
    # is still found exactly once.
    g = graphgen.chung_lu(3000, 20000, 2.1, 4)
    T, Tv = run(g.n, g.src, g.dst)
    s, d = g.src, g.dst
    keep = s != d
    lo = np.minimum(s[keep], d[keep]).astype(np.int64)
    hi = np.maximum(s[keep], d[keep]).astype(np.int64)
    keys = np.unique(lo * g.n + hi)
    lo, hi = (keys // g.n).astype(np.int32), (keys % g.n).astype(np.int32)
    off = np.zeros(g.n + 1, np.int64)
    np.add.at(off, lo + 1, 1)
    off = np.cumsum(off)
    T2, Tv2 = oracle.count_oriented(g.n, off, hi)  # rows of `keys` order are already sorted
    assert T2 == T
    np.testing.assert_array_equal(Tv2, Tv)


# ------------------------------------------------------------ metamorphic

def test_relabel_shuffle_reverse_duplicate():
    g = graphgen.rmat(11, 16, seed=21)
    T, Tv = run(g.n, g.src, g.dst)
    rng = np.random.default_rng(0)
    pi = rng.permutation(g.n).astype(np.int32)
    T2, Tv2 = run(g.n, pi[g.src], pi[g.dst])
    assert T2 == T
    np.testing.assert_array_equal(Tv2[pi], Tv)
    order = rng.permutation(g.m)
    flip = rng.random(g.m) < 0.5
    s = np.where(flip, g.dst, g.src)[order]
    d = np.where(flip, g.src, g.dst)[order]
    dup = rng.integers(0, g.m, 1000)
    s = np.concatenate([s, d[dup], np.arange(50, dtype=np.int32)])
    d = np.concatenate([d, s[dup], np.arange(50, dtype=np.int32)])
    T3, Tv3 = run(g.n, s, d)
    assert T3 == T
    np.testing.assert_array_equal(Tv3, Tv)


# ------------------------------------------------------------ schedule

@pytest.mark.parametrize("kind", [oracle.COST_ONE, oracle.COST_DEGREE, oracle.COST_PRIOR, oracle.COST_NEW])
@pytest.mark.parametrize("W,floor", [(1, 1), (7, 1), (64, 50), (1000, 3)])
def test_schedule_properties(kind, W, floor):
    g = graphgen.preferential_attachment(5000, 6, 12)
    m, off, col, deg = oracle.orient(g.n, g.src, g.dst)
    f = oracle.costs(off, col, deg, kind)
    bnd = oracle.schedule(f, W, floor)
    F = np.concatenate([[0], np.cumsum(f)])
    total = int(F[-1])
    H = (total + 1) // 2
    assert bnd[0] == 0 and bnd[-1] == g.n and (np.diff(bnd) >= 0).all()
    assert len(bnd) - 1 >= W
    # initial tasks: cover the first half exactly at the first reaching node
    assert F[bnd[W]] >= H and (bnd[W] == 0 or F[bnd[W] - 1] < H)
    if total:
        maxf = int(f.max())
        init_costs = np.diff(F[bnd[:W + 1]])
        assert init_costs.max() <= -(-H // W) + maxf
    # dynamic tasks shrink: each target step is ceil(remaining / W), floored
    assert len(bnd) - 1 - W <= W * (1 + math.log(max(total, 2))) + W + 2
    # Section V-D: counting task by task gives the same result
    T, Tv = oracle.count_oriented(g.n, off, col)
    T2, Tv2 = oracle.dynamic_count(off, col, bnd)
    assert T2 == T
    np.testing.assert_array_equal(Tv2, Tv)


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
def test_threaded_task_count_equals_node_iterator(threads):
    """The host-threaded task count (timing baseline only) gives the node
    iterator's T and T_v, for schedules of several sizes."""
    for g in (graphgen.rmat(12, 16, seed=21), graphgen.preferential_attachment(3000, 7, 22),
              graphgen.erdos_renyi(500, 4000, 23)):
        m, off, col, deg = oracle.orient(g.n, g.src, g.dst)
        T, Tv = oracle.count_oriented(g.n, off, col)
        f = oracle.costs(off, col, deg, oracle.COST_PRIOR)
        for W in (1, threads, 64):
            bnd = oracle.schedule(f, W, 1)
            T2, Tv2 = oracle.dynamic_count_threaded(off, col, bnd, threads)
            assert T2 == T
            np.testing.assert_array_equal(Tv2, Tv)


def test_cost_functions_closed_forms():
    # K_5: degrees all 4; ids break ties so N_v = {v+1..4}, dhat_v = 4 - v.
    n, s, d = gs.complete(5)
    m, off, col, deg = oracle.orient(n, s, d)
    dh = np.array([4, 3, 2, 1, 0])
    np.testing.assert_array_equal(np.diff(off), dh)
    np.testing.assert_array_equal(oracle.costs(off, col, deg, oracle.COST_ONE), [1] * 5)
    np.testing.assert_array_equal(oracle.costs(off, col, deg, oracle.COST_DEGREE), [4] * 5)
    # prior cost: sum over u > v of (dhat_v + dhat_u)
    prior = [sum(dh[v] + dh[u] for u in range(v + 1, 5)) for v in range(5)]
    np.testing.assert_array_equal(oracle.costs(off, col, deg, oracle.COST_PRIOR), prior)
    # new cost (Section IV-F): sum over u < v (those holding v) of (dhat_v + dhat_u)
    new = [sum(dh[v] + dh[u] for u in range(0, v)) for v in range(5)]
    np.testing.assert_array_equal(oracle.costs(off, col, deg, oracle.COST_NEW), new)
    # both cost functions spread the same total work over the edges
    assert sum(prior) == sum(new)


# ------------------------------------------------------------ Theorem 1

@pytest.mark.parametrize("P", [1, 2, 3, 7, 16])
def test_surrogate_equals_node_iterator(P):
    g = graphgen.chung_lu(4000, 30000, 2.1, 31)
    m, off, col, deg = oracle.orient(g.n, g.src, g.dst)
    T, Tv = oracle.count_oriented(g.n, off, col)
    rng = np.random.default_rng(P)
    cuts = np.sort(rng.integers(0, g.n + 1, P - 1))
    part = np.concatenate([[0], cuts, [g.n]]).astype(np.int32)
    T2, Tv2, msgs, ids = oracle.surrogate_count(off, col, part)
    assert T2 == T
    np.testing.assert_array_equal(Tv2, Tv)
    # LastProc: one message per (v, other owner among N_v), never repeated
    owner = np.searchsorted(part, np.arange(g.n), side="right") - 1
    expect_msgs, expect_ids = 0, 0
    for v in range(g.n):
        row = col[off[v]:off[v + 1]]
        others = set(owner[row].tolist()) - {int(owner[v])}
        expect_msgs += len(others)
        expect_ids += len(others) * len(row)
    assert msgs == expect_msgs and ids == expect_ids


def test_surrogate_brute_force_small():
    rng = np.random.default_rng(5)
    for trial in range(6):
        n, s, d = gs.gnp(int(rng.integers(5, 25)), 0.5, rng)
        m, off, col, deg = oracle.orient(n, s, d)
        P = int(rng.integers(1, n + 1))
        cuts = np.sort(rng.integers(0, n + 1, P - 1))
        part = np.concatenate([[0], cuts, [n]]).astype(np.int32)
        T, Tv, _, _ = oracle.surrogate_count(off, col, part)
        Tb, Tvb = gs.brute_force(n, s, d)
        assert T == Tb
        np.testing.assert_array_equal(Tv, Tvb)


# ------------------------------------------------------------ per-node definition

def test_adjacency_definition_matches():
    g = graphgen.rmat(12, 16, seed=2)
    T, Tv = run(g.n, g.src, g.dst)
    adj = oracle.Adjacency(g.n, g.src, g.dst)
    vs = np.arange(g.n, dtype=np.int32)
    np.testing.assert_array_equal(adj.triangles_at(vs), Tv)
    assert adj.m == oracle.count(g.n, g.src, g.dst, per_node=False)[2]
    adj.close()


def test_er_expected_count_band():
    # Statistical sanity (not a parity check): G(n, m) expected triangles.
    g = graphgen.workload_er(1)
    T, _, m = oracle.count(g.n, g.src, g.dst, per_node=False)
    N = g.n * (g.n - 1) // 2
    ET = math.comb(g.n, 3) * m * (m - 1) * (m - 2) / (N * (N - 1) * (N - 2))
    assert abs(T - ET) < 6 * math.sqrt(ET)


# ------------------------------------------------------------ clustering coefficients (Section I applications)

@pytest.mark.parametrize("n", [3, 4, 7, 20])
def test_clustering_complete(n):
    coeff, tr, w = oracle.clustering(*gs.complete(n))
    assert (coeff == 1.0).all() and tr == 1.0 and w == n * math.comb(n - 1, 2)


@pytest.mark.parametrize("g", [gs.complete_bipartite(3, 5), gs.grid(6, 7), gs.cycle(10), gs.star(9)])
def test_clustering_triangle_free(g):
    coeff, tr, w = oracle.clustering(*g)
    assert not coeff.any() and tr == 0.0 and w > 0


@pytest.mark.parametrize("n", [5, 8, 31])
def test_clustering_wheel(n):
    # hub: n-1 triangles over C(n-1, 2) pairs; rim: 2 triangles over 3 pairs
    coeff, tr, w = oracle.clustering(*gs.wheel(n))
    assert coeff[0] == (n - 1) / math.comb(n - 1, 2)
    assert (coeff[1:] == 2 / 3).all()
    assert w == math.comb(n - 1, 2) + 3 * (n - 1)
    assert tr == 3 * (n - 1) / w


@pytest.mark.parametrize("k", [1, 2, 6])
def test_clustering_friendship(k):
    coeff, tr, w = oracle.clustering(*gs.friendship(k))
    assert coeff[0] == 1 / (2 * k - 1) and (coeff[1:] == 1.0).all()
    assert tr == 3 * k / (math.comb(2 * k, 2) + 2 * k)


def test_clustering_isolated_and_empty():
    coeff, tr, w = oracle.clustering(5, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert coeff.shape == (5,) and not coeff.any() and tr == 0.0 and w == 0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_clustering_networkx(seed):
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(seed)
    n, s, d = gs.gnp(120, 0.15, rng)
    coeff, tr, _ = oracle.clustering(n, s, d)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(s.tolist(), d.tolist()))
    ref = nx.clustering(G)
    np.testing.assert_allclose(coeff, [ref[v] for v in range(n)], rtol=1e-13, atol=0)
    assert abs(tr - nx.transitivity(G)) <= 1e-13 * max(tr, 1e-300)
