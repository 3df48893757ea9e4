"""GPU: task-table rescheduling, captured (HIP graph) count replays, the
autotuner, and packed batches -- all against the oracle or the plain path."""
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


def batch_graphs(count, seed=3, n_hi=20_000):
    return [s.make() for s in graphgen.batch_specs(count, seed=seed, n_lo=200, n_hi=n_hi)]


def test_reschedule_keeps_counts_and_matches_fresh_build(tc):
    g = graphgen.rmat(13, 16, seed=4)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    with tc.build_oriented([(g.n, g.src, g.dst)]) as h:
        for kw in (dict(small_max=16), dict(cost_fn=tc.COST_DEGREE, min_chunk=7), dict(workers=33),
                   dict(small_max=128, cost_fn=tc.COST_ONE), dict()):
            h.reschedule(**kw)
            tv, tot = h.count_per_node()
            assert tot[0] == T_ref
            np.testing.assert_array_equal(tv, tv_ref)
            bnd, _ = h.export_schedule()
            with tc.build_oriented([(g.n, g.src, g.dst)], **kw) as fresh:
                bnd2, _ = fresh.export_schedule()
                assert fresh.info()["wide_nodes"] == h.info()["wide_nodes"]
            np.testing.assert_array_equal(bnd, bnd2)


@pytest.mark.parametrize("per_node", [False, True])
def test_captured_replays(tc, per_node):
    import torch

    from paper_1406_5687_amd.capture import CapturedCount

    gs = batch_graphs(24)
    with tc.build_oriented([(g.n, g.src, g.dst) for g in gs]) as h:
        eager_tv, eager_tot = h.count_per_node()
        cap = CapturedCount(h, per_node=per_node)
        other = graphgen.rmat(11, 16, seed=9)
        with tc.build_oriented([(other.n, other.src, other.dst)]) as h2:
            for rep in range(5):
                cap.totals.fill_(-1)
                if per_node:
                    cap.per_node_out.fill_(-1)
                tot, pn = cap.replay()
                torch.cuda.synchronize()
                np.testing.assert_array_equal(tot.cpu().numpy(), eager_tot)
                if per_node:
                    np.testing.assert_array_equal(pn.cpu().numpy(), eager_tv)
                # unrelated eager work between replays
                h2.count_per_node()
                torch.arange(1000, device="cuda").sum().item()
    base = 0
    for i, g in enumerate(gs):
        T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
        assert eager_tot[i] == T_ref
        np.testing.assert_array_equal(eager_tv[base:base + g.n], tv_ref)
        base += g.n


def test_autotuner_on_device(tc, tmp_path):
    from paper_1406_5687_amd import autotune

    g = graphgen.chung_lu(30_000, 400_000, 2.1, 5)
    T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
    space = [autotune.Params(32, 16), autotune.Params(128, 512), autotune.Params(64, 64, tc.COST_DEGREE)]
    at = autotune.Autotuner(cache_path=str(tmp_path / "c.json"), space=space)
    with tc.build_oriented([(g.n, g.src, g.dst)]) as h:
        best = at.tune(h, per_node=True)
        assert best in space
        assert h.info()["small_max"] == best.small_max
        tv, tot = h.count_per_node()
    assert tot[0] == T_ref
    np.testing.assert_array_equal(tv, tv_ref)


def test_packed_batch_equals_plain_launches(tc):
    import torch

    gs = batch_graphs(64, seed=5)
    with tc.build_oriented([(g.n, g.src, g.dst) for g in gs]) as h:
        packed = h.count_total()
    plain = torch.zeros(len(gs), dtype=torch.int64, device="cuda")
    hs = [tc.build_oriented([(g.n, g.src, g.dst)]) for g in gs]
    for i, hh in enumerate(hs):
        hh.count_total(out=plain[i:i + 1])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(packed, plain.cpu().numpy())
    tots, _ = tc.count_batch(hs)
    np.testing.assert_array_equal(np.concatenate(tots), packed)
    for hh in hs:
        hh.free()
    for i, g in enumerate(gs):
        assert packed[i] == oracle.count(g.n, g.src, g.dst, per_node=False)[0]


def test_captured_batch_through_abi(tc):
    """tc_count_capture over three handles (one packed), per-node outputs,
    replayed on a side stream and on the current stream with eager work in
    between; every replay equals the oracle."""
    import torch

    from paper_1406_5687_amd.capture import CapturedCount

    gs = batch_graphs(6, seed=11)
    extra = graphgen.chung_lu(5000, 60_000, 2.1, 12)
    hs = [tc.build_oriented([(g.n, g.src, g.dst) for g in gs[:4]]),
          tc.build_oriented([(gs[4].n, gs[4].src, gs[4].dst)]),
          tc.build_oriented([(extra.n, extra.src, extra.dst)])]
    refs = [oracle.count(g.n, g.src, g.dst) for g in gs[:5] + [extra]]
    cap = CapturedCount(hs, per_node=True)
    side = torch.cuda.Stream()
    for rep in range(6):
        cap.totals.fill_(-1)
        for t in cap.per_node_outs:
            t.fill_(-1)
        if rep % 2:
            side.wait_stream(torch.cuda.current_stream())
            cap.replay(stream=side.cuda_stream)
            side.synchronize()
        else:
            cap.replay()
            torch.cuda.synchronize()
        tot = cap.totals.cpu().numpy()
        np.testing.assert_array_equal(tot, [r[0] for r in refs])
        tv0 = cap.per_node_outs[0].cpu().numpy()
        base = 0
        for g, r in zip(gs[:4], refs[:4]):
            np.testing.assert_array_equal(tv0[base:base + g.n], r[1])
            base += g.n
        np.testing.assert_array_equal(cap.per_node_outs[1].cpu().numpy(), refs[4][1])
        np.testing.assert_array_equal(cap.per_node_outs[2].cpu().numpy(), refs[5][1])
        hs[2].count_per_node()  # eager work on the handle's own scratch between replays
    cap.free()
    for h in hs:
        h.free()
