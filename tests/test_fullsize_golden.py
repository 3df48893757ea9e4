"""The full-size expected results (tests/golden/fullsize_*.txt) re-derived in
part on the CPU: the ER file whole, and sampled graphs of the batch and serve
files, with the oracle and the same seeded inputs.  Pins the writer script's
indexing and digests, not the oracle (whose pins are in test_oracle_pins)."""
import numpy as np
import pytest

import graphgen
import oracle
from tests import fullsize


def test_er_file_rederived():
    exp = fullsize.load("er")
    g = graphgen.workload_er(1)
    T, tv, m = oracle.count(g.n, g.src, g.dst)
    assert (exp["n"], exp["m_input"], exp["m"], exp["T"]) == (g.n, g.m, m, T)
    assert exp["sha256"] == fullsize.tv_sha256(tv)
    np.testing.assert_array_equal(tv[exp["top"][:, 0]], exp["top"][:, 2])


@pytest.mark.parametrize("name,specs,picks", [
    ("batch4096", lambda: graphgen.batch_specs(4096, 1), (0, 1, 2, 3, 2047, 4094, 4095)),
    ("serve20000", lambda: graphgen.serve_specs(20_000, 1), (0, 1, 2, 3, 9999, 19998, 19999)),
])
def test_many_file_rows_rederived(name, specs, picks):
    if not fullsize.available(name):
        pytest.skip(f"fullsize_{name}.txt not written")
    exp = fullsize.load(name)
    sp = specs()
    assert exp["count"] == len(sp) == len(exp["rows"])
    assert exp["sum_m"] == sum(r[3] for r in exp["rows"])
    for i in picks:
        if sp[i].m > 2_000_000 or sp[i].n > 2_000_000:
            continue
        g = sp[i].make()
        T, tv, m = oracle.count(g.n, g.src, g.dst)
        kind, n, m_in, m_exp, T_exp, h64 = exp["rows"][i]
        assert (kind, n, m_in, m_exp, T_exp) == (sp[i].kind, g.n, g.m, m, T)
        assert fullsize.tv_sha256(tv)[:16] == h64
