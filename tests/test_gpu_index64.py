"""GPU: the 64-bit row addressing path of the count kernels (an adjacency of
2^29 entries or more takes it; TC_FORCE_INDEX64=1 selects it at any size)
against the oracle: single graphs with the default and forced intersection
variants and a small LDS cap (lists probed in device memory), a packed handle
and a batch of handles.  It runs in a child process, because the switch is
read once per process."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
import torch
import graphgen
import oracle
import paper_1406_5687_amd as tc

graphs = [graphgen.rmat(17, 16, seed=51), graphgen.chung_lu(20000, 300000, 2.1, 52),
          graphgen.preferential_attachment(20000, 10, 53)]
refs = [oracle.count(g.n, g.src, g.dst) for g in graphs]
for g, (T_ref, tv_ref, _) in zip(graphs, refs):
    for kw in (dict(), dict(intersect=2), dict(intersect=0, search_ratio=1), dict(lds_list_max=64)):
        with tc.build_oriented([(g.n, g.src, g.dst)], **kw) as h:
            tv, tot = h.count_per_node()
            assert tot[0] == T_ref and np.array_equal(tv, tv_ref), (g.name, kw)
            assert h.count_total()[0] == T_ref, (g.name, kw)
with tc.build_oriented([(g.n, g.src, g.dst) for g in graphs]) as h:
    tv, tot = h.count_per_node()
base = 0
for g, (T_ref, tv_ref, _) in zip(graphs, refs):
    assert np.array_equal(tv[base:base + g.n], tv_ref), g.name
    base += g.n
assert list(tot) == [r[0] for r in refs]
hs = [tc.build_oriented([(g.n, g.src, g.dst)]) for g in graphs]
tots, pns = tc.count_batch(hs, per_node=True)
for t, pn, r in zip(tots, pns, refs):
    assert t[0] == r[0] and np.array_equal(pn, r[1])
for h in hs:
    h.free()
print("index64 ok", flush=True)
""" % ROOT


def test_index64_path_equals_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    env = dict(os.environ, TC_FORCE_INDEX64="1")
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "index64 ok" in r.stdout
