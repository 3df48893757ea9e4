"""GPU: tc_count_batch_static (the batch count with the library's fixed
per-GPU scratch, for callers that cannot allocate) against tc_count_batch on
the same handles, bit for bit; two calls in a row, the second smaller."""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_5687_amd as tcmod

    tcmod.load()
    return tcmod


def _run_both(tc, hs, per_node):
    import torch

    ktot = sum(h.k for h in hs)
    ref_tot = torch.full((ktot,), -1, dtype=torch.int64, device="cuda")
    st_tot = torch.full((ktot,), -1, dtype=torch.int64, device="cuda")
    ref_pn = [torch.full((h.n_total,), -1, dtype=torch.int64, device="cuda") for h in hs] if per_node else None
    st_pn = [torch.full((h.n_total,), -1, dtype=torch.int64, device="cuda") for h in hs] if per_node else None
    import ctypes
    from paper_1406_5687_amd import tc as tcb

    hp, pn = tcb._device_batch_args(hs, ref_tot, ref_pn)
    o = hs[0]._opts(outputs_on_device=True)
    tcb._raise(tcb.load().tc_count_batch(hp, len(hs), ctypes.byref(o), ctypes.c_void_p(ref_tot.data_ptr()), pn))
    tc.tc.count_batch_static(hs, st_tot, st_pn)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(st_tot.cpu().numpy(), ref_tot.cpu().numpy())
    if per_node:
        for a, b in zip(st_pn, ref_pn):
            np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    return st_tot.cpu().numpy()


@pytest.mark.parametrize("per_node", [True, False])
def test_static_scratch_equals_allocating_batch(tc, per_node):
    big = [s.make() for s in graphgen.batch_specs(12, seed=21, n_lo=500, n_hi=60_000)]
    rm = graphgen.rmat(14, 16, seed=22)
    hs = [tc.build_oriented([(g.n, g.src, g.dst) for g in big[:8]]),
          tc.build_oriented([(rm.n, rm.src, rm.dst)]),
          tc.build_oriented([(g.n, g.src, g.dst) for g in big[8:]])]
    first = _run_both(tc, hs, per_node)
    assert (first >= 0).all() and first.sum() > 0
    # a second call, smaller: the array keeps the first call's contents
    small = graphgen.erdos_renyi(3000, 30_000, seed=23)
    with tc.build_oriented([(small.n, small.src, small.dst)]) as h2:
        _run_both(tc, [h2], per_node)
    for h in hs:
        h.free()


def test_static_scratch_limits(tc):
    import torch

    g = graphgen.erdos_renyi(1000, 5000, seed=24)
    with tc.build_oriented([(g.n, g.src, g.dst)]) as h:
        tot = torch.zeros(1, dtype=torch.int64, device="cuda")
        # host outputs are refused: there is nothing to stage them through
        from paper_1406_5687_amd import tc as tcb
        import ctypes

        hp, _ = tcb._device_batch_args([h], tot, None)
        host = np.zeros(1, np.int64)
        o = h._opts(outputs_on_device=False)
        rc = tcb.load().tc_count_batch_static(hp, 1, ctypes.byref(o), ctypes.c_void_p(host.ctypes.data), None)
        assert rc == tcb.TC_ERR_INVALID_ARG
    # per-node accumulators beyond the array: refused before any launch
    n_big = tcb.STATIC_SCRATCH_BYTES // 8 + 1
    big = graphgen.erdos_renyi(n_big, 1000, seed=25)
    with tc.build_oriented([(big.n, big.src, big.dst)]) as hb:
        pn = torch.zeros(n_big, dtype=torch.int64, device="cuda")
        with pytest.raises(tcb.TcError) as ei:
            tc.tc.count_batch_static([hb], tot, [pn])
        assert ei.value.code == tcb.TC_ERR_TOO_LARGE
        # totals only still fit
        tc.tc.count_batch_static([hb], tot)
        torch.cuda.synchronize()
        assert int(tot.item()) == hb.count_total()[0]
