"""TEST INFRASTRUCTURE -- Python handle on the plain CPU oracle (``tc_oracle.c``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it, and it never calls the GPU library.

Every function here is a thin ctypes wrapper: the arithmetic lives in
``tc_oracle.c`` and follows the paper step by step (Fig. 1 node iterator,
Section III-A degree order, Section V-B schedule, Fig. 2/3 surrogate
algorithm, Section II definition of T_v).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tc_oracle.c")
_LIB = os.path.join(_HERE, "_tc_oracle.so")
_lib = None

_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)
_VP = ctypes.c_void_p

ERRORS = {1: "invalid argument", 2: "node id out of range", 3: "out of memory", 4: "internal check failed"}


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, single-threaded)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    lib.orc_orient.argtypes = [ctypes.c_int32, ctypes.c_int64, _I32P, _I32P, _I64P, _I64P, _I32P, _I32P]
    lib.orc_count_oriented.argtypes = [ctypes.c_int32, _I64P, _I32P, _I64P, _I64P]
    lib.orc_count.argtypes = [ctypes.c_int32, ctypes.c_int64, _I32P, _I32P, _I64P, _I64P, _I64P]
    lib.orc_degree_order.argtypes = [ctypes.c_int32, _I32P, _I32P]
    _DP = ctypes.POINTER(ctypes.c_double)
    lib.orc_clustering.argtypes = [ctypes.c_int32, ctypes.c_int64, _I32P, _I32P, _DP, _DP, _I64P]
    lib.orc_costs.argtypes = [ctypes.c_int32, _I64P, _I32P, _I32P, ctypes.c_int, _I64P]
    lib.orc_schedule.argtypes = [ctypes.c_int32, _I64P, ctypes.c_int32, ctypes.c_int64, _I32P, ctypes.c_int64,
                                 _I64P]
    lib.orc_dynamic_count.argtypes = [ctypes.c_int32, _I64P, _I32P, _I32P, ctypes.c_int64, _I64P, _I64P]
    lib.orc_dynamic_count_threaded.argtypes = [ctypes.c_int32, _I64P, _I32P, _I32P, ctypes.c_int64, ctypes.c_int32,
                                               _I64P, _I64P]
    lib.orc_surrogate_count.argtypes = [ctypes.c_int32, _I64P, _I32P, ctypes.c_int32, _I32P, _I64P, _I64P,
                                        _I64P, _I64P]
    lib.orc_adj_build.argtypes = [ctypes.c_int32, ctypes.c_int64, _I32P, _I32P]
    lib.orc_adj_build.restype = _VP
    lib.orc_adj_free.argtypes = [_VP]
    lib.orc_adj_edges.argtypes = [_VP]
    lib.orc_adj_edges.restype = ctypes.c_int64
    lib.orc_adj_degree.argtypes = [_VP, ctypes.c_int64, _I32P, _I32P]
    lib.orc_adj_tv.argtypes = [_VP, ctypes.c_int64, _I32P, _I64P]
    _lib = lib
    return lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p32(a: np.ndarray):
    return a.ctypes.data_as(_I32P)


def _p64(a: np.ndarray):
    return a.ctypes.data_as(_I64P)


def _rc(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what}: {ERRORS.get(rc, rc)}")


def count(n: int, src, dst, per_node: bool = True):
    """Fig. 1 over the canonical simple graph.  Returns (T, T_v or None, m)."""
    lib = _load()
    s, d = _i32(src), _i32(dst)
    T = np.zeros(1, np.int64)
    m = np.zeros(1, np.int64)
    Tv = np.zeros(max(n, 1), np.int64) if per_node else None
    _rc(lib.orc_count(n, s.shape[0], _p32(s), _p32(d), _p64(T), _p64(Tv) if per_node else None, _p64(m)), "count")
    return int(T[0]), (Tv[:n] if per_node else None), int(m[0])


def clustering(n: int, src, dst):
    """Local clustering coefficients T_v / C(d_v, 2) and the transitivity
    3T / sum C(d_v, 2) (Section I applications, textbook definitions), fp64.
    Returns (coeff[n], transitivity, paths of length two)."""
    lib = _load()
    s, d = _i32(src), _i32(dst)
    coeff = np.zeros(max(n, 1), np.float64)
    tr = np.zeros(1, np.float64)
    w = np.zeros(1, np.int64)
    _rc(lib.orc_clustering(n, s.shape[0], _p32(s), _p32(d), coeff.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           tr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _p64(w)), "clustering")
    return coeff[:n], float(tr[0]), int(w[0])


def orient(n: int, src, dst):
    """Oriented adjacency of Fig. 1 in original ids: (m, off[n+1], col[m], deg[n])."""
    lib = _load()
    s, d = _i32(src), _i32(dst)
    off = np.zeros(n + 1, np.int64)
    col = np.zeros(max(s.shape[0], 1), np.int32)
    deg = np.zeros(max(n, 1), np.int32)
    m = np.zeros(1, np.int64)
    _rc(lib.orc_orient(n, s.shape[0], _p32(s), _p32(d), _p64(m), _p64(off), _p32(col), _p32(deg)), "orient")
    mm = int(m[0])
    return mm, off, col[:mm].copy(), deg[:n].copy()


def count_oriented(n: int, off, col, per_node: bool = True):
    lib = _load()
    off = np.ascontiguousarray(off, np.int64)
    col = _i32(col) if len(col) else np.zeros(1, np.int32)
    T = np.zeros(1, np.int64)
    Tv = np.zeros(max(n, 1), np.int64) if per_node else None
    _rc(lib.orc_count_oriented(n, _p64(off), _p32(col), _p64(T), _p64(Tv) if per_node else None), "count_oriented")
    return int(T[0]), (Tv[:n] if per_node else None)


def degree_order(deg) -> np.ndarray:
    """perm[r] = node in place r under the degree order (ties by id)."""
    lib = _load()
    deg = _i32(deg)
    n = deg.shape[0]
    perm = np.zeros(max(n, 1), np.int32)
    _rc(lib.orc_degree_order(n, _p32(deg), _p32(perm)), "degree_order")
    return perm[:n].copy()


COST_ONE, COST_DEGREE, COST_PRIOR, COST_NEW = 0, 1, 2, 3


def costs(off, col, deg, kind: int) -> np.ndarray:
    lib = _load()
    off = np.ascontiguousarray(off, np.int64)
    n = off.shape[0] - 1
    col = _i32(col) if len(col) else np.zeros(1, np.int32)
    deg = _i32(deg) if n else np.zeros(1, np.int32)
    f = np.zeros(max(n, 1), np.int64)
    _rc(lib.orc_costs(n, _p64(off), _p32(col), _p32(deg), kind, _p64(f)), "costs")
    return f[:n].copy()


def schedule(f, W: int, min_chunk: int) -> np.ndarray:
    """Section V-B task boundaries over costs f (see tc_oracle.c for the reading)."""
    lib = _load()
    f = np.ascontiguousarray(f, np.int64)
    n = f.shape[0]
    nt = np.zeros(1, np.int64)
    fp = _p64(f) if n else None
    _rc(lib.orc_schedule(n, fp, W, min_chunk, None, 0, _p64(nt)), "schedule(size)")
    k = int(nt[0]) + 1
    bnd = np.zeros(k, np.int32)
    _rc(lib.orc_schedule(n, fp, W, min_chunk, _p32(bnd), k, _p64(nt)), "schedule")
    return bnd


def dynamic_count(off, col, bnd, per_node: bool = True):
    lib = _load()
    off = np.ascontiguousarray(off, np.int64)
    n = off.shape[0] - 1
    col = _i32(col) if len(col) else np.zeros(1, np.int32)
    bnd = _i32(bnd)
    T = np.zeros(1, np.int64)
    Tv = np.zeros(max(n, 1), np.int64) if per_node else None
    _rc(lib.orc_dynamic_count(n, _p64(off), _p32(col), _p32(bnd), bnd.shape[0] - 1, _p64(T),
                              _p64(Tv) if per_node else None), "dynamic_count")
    return int(T[0]), (Tv[:n] if per_node else None)


def dynamic_count_threaded(off, col, bnd, threads: int, per_node: bool = True):
    """dynamic_count with `threads` host threads pulling the tasks from one
    atomic counter (for timing the CPU baseline; same results)."""
    lib = _load()
    off = np.ascontiguousarray(off, np.int64)
    n = off.shape[0] - 1
    col = _i32(col) if len(col) else np.zeros(1, np.int32)
    bnd = _i32(bnd)
    T = np.zeros(1, np.int64)
    Tv = np.zeros(max(n, 1), np.int64) if per_node else None
    _rc(lib.orc_dynamic_count_threaded(n, _p64(off), _p32(col), _p32(bnd), bnd.shape[0] - 1, int(threads), _p64(T),
                                       _p64(Tv) if per_node else None), "dynamic_count_threaded")
    return int(T[0]), (Tv[:n] if per_node else None)


def surrogate_count(off, col, part, per_node: bool = True):
    """Fig. 3 with P = len(part)-1 simulated processors owning id ranges.
    Returns (T, T_v or None, messages sent, ids sent)."""
    lib = _load()
    off = np.ascontiguousarray(off, np.int64)
    n = off.shape[0] - 1
    col = _i32(col) if len(col) else np.zeros(1, np.int32)
    part = _i32(part)
    T = np.zeros(1, np.int64)
    msgs = np.zeros(1, np.int64)
    ids = np.zeros(1, np.int64)
    Tv = np.zeros(max(n, 1), np.int64) if per_node else None
    _rc(lib.orc_surrogate_count(n, _p64(off), _p32(col), part.shape[0] - 1, _p32(part), _p64(T),
                                _p64(Tv) if per_node else None, _p64(msgs), _p64(ids)), "surrogate_count")
    return int(T[0]), (Tv[:n] if per_node else None), int(msgs[0]), int(ids[0])


class Adjacency:
    """Undirected sorted adjacency for per-node T_v by the Section II definition."""

    def __init__(self, n: int, src, dst):
        lib = _load()
        s, d = _i32(src), _i32(dst)
        self._keep = (s, d)
        self._h = lib.orc_adj_build(n, s.shape[0], _p32(s), _p32(d))
        if not self._h:
            raise OracleError("adjacency build failed (bad ids or out of memory)")
        self.n = n

    @property
    def m(self) -> int:
        return int(_load().orc_adj_edges(self._h))

    def degree(self, vs) -> np.ndarray:
        vs = _i32(vs)
        out = np.zeros(max(vs.shape[0], 1), np.int32)
        _rc(_load().orc_adj_degree(self._h, vs.shape[0], _p32(vs), _p32(out)), "degree")
        return out[: vs.shape[0]]

    def triangles_at(self, vs) -> np.ndarray:
        vs = _i32(vs)
        out = np.zeros(max(vs.shape[0], 1), np.int64)
        _rc(_load().orc_adj_tv(self._h, vs.shape[0], _p32(vs), _p64(out)), "triangles_at")
        return out[: vs.shape[0]]

    def close(self):
        if self._h:
            _load().orc_adj_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
