"""GPU: oriented rows longer than 256 entries are sorted in LDS by one
workgroup per row (up to 16384 entries) or, beyond that, by a radix sort of
(row, entry) keys.  Rows that long only occur above ~1.3e8 edges, so the
radix path is forced here in a child process by lowering the LDS limit
(TC_LONG_ROW_LDS, read once per process): every row must equal the oracle's
Fig. 1 row (degree order, ascending), a repeated input edge must still be
detected in a long row, and the counts must equal the oracle's."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import math, sys
sys.path.insert(0, %r)
import numpy as np
import torch
import graphgen
import oracle
from tests import graphs_small as gs
import paper_1406_5687_amd as tc

def rows_equal(n, src, dst):
    m, off_o, col_o, deg = oracle.orient(n, src, dst)
    perm_o = oracle.degree_order(deg)
    with tc.build_oriented([(n, src, dst)]) as h:
        off, col, perm = h.export_csr()
        tv, tot = h.count_per_node()
        T = int(tot[0])
    assert np.array_equal(perm, perm_o)
    rank = np.empty(n, np.int64)
    rank[perm] = np.arange(n)
    for r in np.nonzero(np.diff(off) > 0)[0]:
        row = col[off[r]:off[r + 1]]
        expect = np.sort(rank[col_o[off_o[perm[r]]:off_o[perm[r] + 1]]])
        assert np.array_equal(row, expect), r
    return T, tv

for k in (300, 700, 2500):
    n, s, d = gs.complete(k)
    T, tv = rows_equal(n, s, d)
    assert T == math.comb(k, 3) and (tv == math.comb(k - 1, 2)).all()
g = graphgen.chung_lu(20000, 400000, 2.0, 71)
T, tv = rows_equal(g.n, g.src, g.dst)
T_ref, tv_ref, _ = oracle.count(g.n, g.src, g.dst)
assert T == T_ref and np.array_equal(tv, tv_ref)
# an edge given twice (no loops): only the sorted long rows reveal it
n, s, d = gs.complete(700)
s2 = np.concatenate([s, s[:3]]).astype(np.int32)
d2 = np.concatenate([d, d[:3]]).astype(np.int32)
with tc.build_oriented([(n, s, d)]) as h1, tc.build_oriented([(n, s2, d2)]) as h2:
    for x, y in zip(h1.export_csr(), h2.export_csr()):
        assert np.array_equal(x, y)
    assert h2.info()["m"] == h1.info()["m"]
print("long rows ok", flush=True)
""" % ROOT


@pytest.mark.parametrize("limit", ["0", "1000", ""])
def test_long_row_paths_equal_oracle(limit):
    # 0: every long row by the radix sort; 1000: rows of 257..1000 entries in
    # LDS, longer ones by the radix sort; "": the default (all in LDS here)
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    env = dict(os.environ, TC_LONG_ROW_LDS=limit)
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "long rows ok" in r.stdout
