"""Reader of the full-size expected results in tests/golden/fullsize_*.txt
(written by tests/golden/make_fullsize.py from the CPU oracle), and the digest
they use.  Holds no counting arithmetic."""
from __future__ import annotations

import hashlib
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def tv_sha256(tv) -> str:
    """SHA-256 of per-node counts as little-endian int64, in caller ids 0..n-1."""
    return hashlib.sha256(np.ascontiguousarray(np.asarray(tv), dtype="<i8").tobytes()).hexdigest()


def path(name: str) -> str:
    return os.path.join(GOLDEN, f"fullsize_{name}.txt")


def available(name: str) -> bool:
    return os.path.exists(path(name))


def load(name: str) -> dict:
    """Single graphs (er, pa, rmat24): keys n, m_input, m, T, sha256, top
    (array of [id, degree, T_v]).  Many graphs (batch4096, serve20000): keys
    count, sum_m, sha256 and rows: a list of (kind, n, m_input, m, T, h64)."""
    out: dict = {"top": [], "rows": []}
    with open(path(name)) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            f = line.split()
            if f[0] == "top":
                out["top"].append([int(x) for x in f[1:4]])
            elif f[0] == "g":
                out["rows"].append((f[2], int(f[3]), int(f[4]), int(f[5]), int(f[6]), f[7]))
            elif f[0] in ("sha256", "workload"):
                out[f[0]] = " ".join(f[1:])
            else:
                out[f[0]] = int(f[1])
    out["top"] = np.array(out["top"], dtype=np.int64).reshape(-1, 3)
    return out
