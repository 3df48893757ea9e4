"""Readers for the hand-derived fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for ln in fh:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                yield ln


def graph(name):
    """Returns dict(n, T, Tv, src, dst) from a *.graph fixture."""
    out = {"src": [], "dst": []}
    for ln in _lines(name):
        key, *vals = ln.split()
        if key == "n":
            out["n"] = int(vals[0])
        elif key == "T":
            out["T"] = int(vals[0])
        elif key == "Tv":
            out["Tv"] = np.array([int(x) for x in vals], np.int64)
        elif key == "e":
            out["src"].append(int(vals[0]))
            out["dst"].append(int(vals[1]))
    out["src"] = np.array(out["src"], np.int32)
    out["dst"] = np.array(out["dst"], np.int32)
    return out


def orientation(name):
    """Returns dict(n, src, dst, rows) from a *.orient fixture; rows[v] = list."""
    out = {"src": [], "dst": [], "rows": {}}
    for ln in _lines(name):
        if ln.startswith("N "):
            head, _, rest = ln[2:].partition(":")
            out["rows"][int(head)] = [int(x) for x in rest.split()]
            continue
        key, *vals = ln.split()
        if key == "n":
            out["n"] = int(vals[0])
        elif key == "e":
            out["src"].append(int(vals[0]))
            out["dst"].append(int(vals[1]))
    out["src"] = np.array(out["src"], np.int32)
    out["dst"] = np.array(out["dst"], np.int32)
    return out


def schedule(name):
    out = {}
    for ln in _lines(name):
        key, *vals = ln.split()
        if key in ("W", "min_chunk"):
            out[key] = int(vals[0])
        elif key in ("f", "bnd"):
            out[key] = np.array([int(x) for x in vals], np.int64 if key == "f" else np.int32)
    return out


def all_graphs():
    return sorted(f for f in os.listdir(GOLDEN) if f.endswith(".graph"))
