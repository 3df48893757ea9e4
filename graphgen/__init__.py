"""Seeded synthetic input graphs, shared by the tests, the oracle checks and the bench.

This module produces edge lists only; it contains none of the triangle-counting
arithmetic.  The C generators (``graphgen.c``) draw from Philox4x32-10 keyed by
the seed, so the same seed yields the same graph on any machine and with any
thread count.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "_graphgen.so")
_lib = None

_I32P = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (it is plain C, no GPU code)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(
            ["gcc", "-O3", "-march=x86-64-v2", "-fPIC", "-shared", "-std=c11", "-pthread",
             "-o", tmp, _SRC, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    lib.gg_erdos_renyi.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, _I32P, _I32P]
    lib.gg_pa_edge_count.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.gg_pa_edge_count.restype = ctypes.c_int64
    lib.gg_preferential_attachment.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, _I32P, _I32P,
                                               ctypes.c_int]
    lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_uint64, _I32P, _I32P, ctypes.c_int]
    lib.gg_chung_lu.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, _I32P, _I32P,
                                ctypes.c_int]
    lib.gg_random_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, _I32P]
    lib.gg_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    lib.gg_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
    _lib = lib
    return lib


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_I32P)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"{what}: generator rejected its arguments (rc={rc})")


@dataclass
class EdgeList:
    """An undirected graph as drawn: ids 0..n-1, edges (src[e], dst[e])."""

    n: int
    src: np.ndarray
    dst: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def erdos_renyi(n: int, m: int, seed: int = 1) -> EdgeList:
    """G(n, m): m distinct uniform unordered pairs without loops."""
    lib = _load()
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    _check(lib.gg_erdos_renyi(n, m, seed, _ptr(src), _ptr(dst)), "erdos_renyi")
    return EdgeList(n, src, dst, f"ER(n={n},m={m},seed={seed})")


def preferential_attachment(n: int, d: int, seed: int = 1) -> EdgeList:
    """PA: K_d seed, then each new node links to d distinct nodes chosen with
    probability proportional to degree; ids randomly relabelled."""
    lib = _load()
    m = lib.gg_pa_edge_count(n, d)
    if m < 0:
        raise ValueError("preferential_attachment needs 1 <= d < n")
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    _check(lib.gg_preferential_attachment(n, d, seed, _ptr(src), _ptr(dst), _threads()), "pa")
    return EdgeList(n, src, dst, f"PA(n={n},d={d},seed={seed})")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1) -> EdgeList:
    """R-MAT draws (loops and repeats kept); ids randomly relabelled."""
    lib = _load()
    m = edge_factor << scale
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    _check(lib.gg_rmat(scale, edge_factor, a, b, c, seed, _ptr(src), _ptr(dst), _threads()), "rmat")
    return EdgeList(1 << scale, src, dst, f"RMAT(scale={scale},ef={edge_factor},seed={seed})")


def chung_lu(n: int, pairs: int, beta: float = 2.1, seed: int = 1) -> EdgeList:
    """Chung-Lu with power-law weights (i+1)^(-1/(beta-1)); `pairs` endpoint
    pairs drawn proportional to weight (loops and repeats kept)."""
    lib = _load()
    src = np.empty(pairs, np.int32)
    dst = np.empty(pairs, np.int32)
    _check(lib.gg_chung_lu(n, pairs, beta, seed, _ptr(src), _ptr(dst), _threads()), "chung_lu")
    return EdgeList(n, src, dst, f"CL(n={n},pairs={pairs},beta={beta},seed={seed})")


def random_permutation(n: int, seed: int) -> np.ndarray:
    lib = _load()
    p = np.empty(n, np.int32)
    _check(lib.gg_random_permutation(n, seed, _ptr(p)), "permutation")
    return p


def uniforms(seed: int, tag: int, k: int) -> np.ndarray:
    lib = _load()
    out = np.empty(k, np.float64)
    _check(lib.gg_uniforms(seed, tag, k, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "uniforms")
    return out


def philox4x32_10(ctr, key) -> list:
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib.gg_philox4x32_10(c, k, o)
    return list(o)


# ---------------------------------------------------------------- workloads

def workload_er(seed: int = 1) -> EdgeList:
    """Erdos-Renyi G(n=10,000, m=100,000)."""
    return erdos_renyi(10_000, 100_000, seed)


def workload_pa(seed: int = 1, n: int = 1_000_000, d: int = 50) -> EdgeList:
    """Preferential attachment, 10^6 nodes, 50 distinct targets per new node."""
    return preferential_attachment(n, d, seed)


def workload_rmat(seed: int = 1, scale: int = 24) -> EdgeList:
    """R-MAT scale 24, edge factor 16, (a,b,c,d) = (0.57, 0.19, 0.19, 0.05)."""
    return rmat(scale, 16, 0.57, 0.19, 0.19, seed)


@dataclass
class GraphSpec:
    kind: str          # "er", "cl", "pa", "rmat"
    n: int
    m: int             # edges (er), endpoint pairs (cl), ignored for pa/rmat
    param: float       # er: avg degree; cl: beta; pa: d; rmat: scale
    seed: int

    def make(self) -> EdgeList:
        if self.kind == "er":
            return erdos_renyi(self.n, self.m, self.seed)
        if self.kind == "cl":
            return chung_lu(self.n, self.m, self.param, self.seed)
        if self.kind == "pa":
            return preferential_attachment(self.n, int(self.param), self.seed)
        if self.kind == "rmat":
            return rmat(int(self.param), 16, 0.57, 0.19, 0.19, self.seed)
        raise ValueError(self.kind)


def batch_specs(count: int = 4096, seed: int = 1, n_lo: int = 1_000, n_hi: int = 200_000) -> list:
    """Uneven batch: n log-uniform in [n_lo, n_hi]; even index -> G(n, m) with
    average degree k ~ U(8, 64); odd index -> Chung-Lu, beta 2.1, 16n pairs
    (mean degree 32 before loops and repeats are removed)."""
    u = uniforms(seed, 0xBA7C4, 2 * count)
    specs = []
    for g in range(count):
        n = int(round(math.exp(math.log(n_lo) + u[2 * g] * (math.log(n_hi) - math.log(n_lo)))))
        gs = seed * 1_000_003 + g
        if g % 2 == 0:
            k = 8.0 + 56.0 * u[2 * g + 1]
            m = int(round(n * k / 2.0))
            specs.append(GraphSpec("er", n, m, k, gs))
        else:
            specs.append(GraphSpec("cl", n, 16 * n, 2.1, gs))
    return specs


def serve_specs(count: int = 20_000, seed: int = 1, median: float = 5e4, sigma: float = 1.5,
                lo: float = 1e3, hi: float = 2e7) -> list:
    """Serving requests: edge count log-normal (median, sigma) clipped to
    [lo, hi]; even index -> PA(d=20) with n = m/20, odd -> R-MAT with scale
    clamp(round(log2(m/16)), 12, 20), edge factor 16."""
    u = uniforms(seed, 0x5E7E, 2 * count)
    specs = []
    for i in range(count):
        # Box-Muller on two uniforms
        u1 = max(u[2 * i], 1e-300)
        z = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u[2 * i + 1])
        m = min(hi, max(lo, math.exp(math.log(median) + sigma * z)))
        gs = seed * 7_000_003 + i
        if i % 2 == 0:
            n = max(21, int(round(m / 20.0)))
            specs.append(GraphSpec("pa", n, 0, 20, gs))
        else:
            sc = int(min(20, max(12, round(math.log2(m / 16.0)))))
            specs.append(GraphSpec("rmat", 1 << sc, 16 << sc, sc, gs))
    return specs


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 1) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    u = uniforms(seed, 0xA771, count)
    gaps = -np.log1p(-u) / rate_per_s
    return np.cumsum(gaps)
