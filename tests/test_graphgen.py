"""Seeded input generators: determinism, published RNG vectors, shapes."""
import numpy as np

import graphgen


def test_philox_known_answers():
    # Known-answer vectors published with Philox4x32-10 (Random123).
    assert graphgen.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert graphgen.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6,
                                                                          0x6D5451FD]
    assert graphgen.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == [
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_er_distinct_no_loops():
    g = graphgen.erdos_renyi(2000, 30000, 3)
    assert g.m == 30000 and (g.src != g.dst).all()
    keys = np.minimum(g.src, g.dst).astype(np.int64) * g.n + np.maximum(g.src, g.dst)
    assert np.unique(keys).shape[0] == g.m
    assert g.src.min() >= 0 and max(g.src.max(), g.dst.max()) < g.n


def test_pa_structure():
    n, d = 3000, 7
    g = graphgen.preferential_attachment(n, d, 4)
    assert g.m == d * (d - 1) // 2 + (n - d) * d
    assert (g.src != g.dst).all()
    keys = np.minimum(g.src, g.dst).astype(np.int64) * n + np.maximum(g.src, g.dst)
    assert np.unique(keys).shape[0] == g.m          # targets are distinct
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=n)
    assert deg.min() >= d - 1 and deg.max() > 10 * d  # heavy tail


def test_rmat_shape_and_skew():
    g = graphgen.rmat(14, 16, seed=9)
    assert g.n == 1 << 14 and g.m == 16 << 14
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    assert deg.max() > 50 * deg.mean()


def test_determinism_and_thread_independence(monkeypatch):
    a = graphgen.rmat(12, 8, seed=5)
    monkeypatch.setattr(graphgen, "_threads", lambda: 3)
    b = graphgen.rmat(12, 8, seed=5)
    np.testing.assert_array_equal(a.src, b.src)
    np.testing.assert_array_equal(a.dst, b.dst)
    c = graphgen.rmat(12, 8, seed=6)
    assert not np.array_equal(a.src, c.src)


def test_chung_lu_and_batch_recipe():
    g = graphgen.chung_lu(1000, 16000, 2.1, 2)
    assert g.m == 16000 and g.src.max() < 1000
    specs = graphgen.batch_specs(64, seed=1)
    ns = np.array([s.n for s in specs])
    assert ns.min() >= 1000 and ns.max() <= 200_000
    assert {s.kind for s in specs[0::2]} == {"er"} and {s.kind for s in specs[1::2]} == {"cl"}
    ks = np.array([s.param for s in specs[0::2]])
    assert ks.min() >= 8 and ks.max() <= 64


def test_serve_recipe():
    specs = graphgen.serve_specs(400, seed=1)
    assert {s.kind for s in specs[0::2]} == {"pa"} and {s.kind for s in specs[1::2]} == {"rmat"}
    sc = np.array([s.param for s in specs[1::2]])
    assert sc.min() >= 12 and sc.max() <= 20
    t = graphgen.poisson_arrivals(1000, 100.0, 1)
    assert (np.diff(t) > 0).all() and abs(t[-1] / 1000 - 0.01) < 0.002
