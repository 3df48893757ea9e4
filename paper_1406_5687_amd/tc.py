"""ctypes binding of libtc.so (include/tc.h): argument marshalling only.

Every step of building and counting runs in the library's HIP kernels; this
module converts numpy arrays or torch tensors into pointers and sizes, passes
the current torch stream, and maps status codes to exceptions.  If libtc.so is
missing it raises; there is no fallback computation.
"""
from __future__ import annotations

import ctypes
import threading
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtc.so")

TC_OK, TC_ERR_INVALID_ARG, TC_ERR_ID_RANGE, TC_ERR_TOO_LARGE, TC_ERR_OUT_OF_MEMORY, TC_ERR_DEVICE = range(6)
COST_ONE, COST_DEGREE, COST_PRIOR, COST_NEW = range(4)
INTERSECT_AUTO, INTERSECT_WALK, INTERSECT_SEARCH = range(3)
HASH_AUTO, HASH_LINEAR = range(2)

EXPORTED = [
    "tc_options_default", "tc_build_oriented", "tc_count_total", "tc_count_per_node", "tc_count_batch",
    "tc_graph_info", "tc_export_csr", "tc_export_schedule", "tc_graph_free", "tc_status_str", "tc_last_error",
    "tc_graph_reschedule", "tc_worker_times", "tc_clustering", "tc_count_capture", "tc_count_replay",
    "tc_count_graph_free", "tc_count_batch_static",
]

STATIC_SCRATCH_BYTES = 32 << 20  # TC_STATIC_SCRATCH_BYTES


class TcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class IdRangeError(TcError, ValueError):
    pass


class InvalidArgument(TcError, ValueError):
    pass


class OutOfMemory(TcError, MemoryError):
    pass


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [
        ("stream", ctypes.c_void_p),
        ("inputs_on_device", ctypes.c_int32),
        ("outputs_on_device", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("alloc", _ALLOC_FN),
        ("free", _FREE_FN),
        ("alloc_ctx", ctypes.c_void_p),
        ("workers", ctypes.c_int32),
        ("cost_fn", ctypes.c_int32),
        ("min_chunk", ctypes.c_int64),
        ("small_max", ctypes.c_int32),
        ("lds_list_max", ctypes.c_int32),
        ("time_kernels", ctypes.c_int32),
        ("partitions", ctypes.c_int32),
        ("rounds", ctypes.c_int32),
        ("direct", ctypes.c_int32),
        ("static_chunks", ctypes.c_int32),
        ("intersect", ctypes.c_int32),
        ("search_ratio", ctypes.c_int32),
        ("hash", ctypes.c_int32),
        ("bitmap_ratio", ctypes.c_int32),
    ]


class Edges(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p)]


class GraphInfo(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("m_input", ctypes.c_int64),
        ("max_out_degree", ctypes.c_int32),
        ("tasks", ctypes.c_int64),
        ("total_cost", ctypes.c_int64),
        ("wide_nodes", ctypes.c_int64),
        ("device_bytes", ctypes.c_uint64),
        ("partitions", ctypes.c_int32),
        ("workers", ctypes.c_int32),
        ("last_count_ms", ctypes.c_double),
        ("small_max", ctypes.c_int32),
        ("cost_fn", ctypes.c_int32),
        ("streamed_bytes", ctypes.c_int64),
        ("peak_device_bytes", ctypes.c_uint64),
        ("rounds", ctypes.c_int32),
        ("search_ratio", ctypes.c_int32),
        ("hash", ctypes.c_int32),
        ("bitmap_ratio", ctypes.c_int32),
        ("core_rows", ctypes.c_int64),
        ("core_bytes", ctypes.c_uint64),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libtc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1406_5687_amd._build.build() "
                          "(the HIP library is required; there is no CPU path)")
    # torch brings its own HIP runtime: when torch is present it is loaded
    # first, so that the library binds to the runtime torch allocates with
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.tc_options_default.argtypes = [ctypes.POINTER(Options)]
    lib.tc_options_default.restype = None
    lib.tc_build_oriented.argtypes = [ctypes.POINTER(Edges), ctypes.c_int32, ctypes.POINTER(Options),
                                      ctypes.POINTER(P)]
    lib.tc_count_total.argtypes = [P, ctypes.POINTER(Options), P]
    lib.tc_count_per_node.argtypes = [P, ctypes.POINTER(Options), P, P]
    lib.tc_count_batch.argtypes = [ctypes.POINTER(P), ctypes.c_int32, ctypes.POINTER(Options), P,
                                   ctypes.POINTER(P)]
    lib.tc_count_batch_static.argtypes = [ctypes.POINTER(P), ctypes.c_int32, ctypes.POINTER(Options), P,
                                          ctypes.POINTER(P)]
    lib.tc_count_capture.argtypes = [ctypes.POINTER(P), ctypes.c_int32, ctypes.POINTER(Options), P,
                                     ctypes.POINTER(P), ctypes.POINTER(P)]
    lib.tc_count_replay.argtypes = [P, ctypes.POINTER(Options)]
    lib.tc_count_graph_free.argtypes = [P]
    lib.tc_count_graph_free.restype = None
    lib.tc_graph_info.argtypes = [P, ctypes.POINTER(GraphInfo)]
    lib.tc_graph_reschedule.argtypes = [P, ctypes.POINTER(Options)]
    lib.tc_export_csr.argtypes = [P, ctypes.POINTER(Options), P, P, P]
    lib.tc_export_schedule.argtypes = [P, ctypes.POINTER(Options), P, P, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64)]
    lib.tc_worker_times.argtypes = [P, ctypes.POINTER(Options), P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.tc_worker_times.restype = ctypes.c_int
    lib.tc_clustering.argtypes = [P, ctypes.POINTER(Options), P, P, P]
    lib.tc_clustering.restype = ctypes.c_int
    lib.tc_graph_free.argtypes = [P]
    lib.tc_graph_free.restype = None
    lib.tc_status_str.argtypes = [ctypes.c_int]
    lib.tc_status_str.restype = ctypes.c_char_p
    lib.tc_last_error.argtypes = []
    lib.tc_last_error.restype = ctypes.c_char_p
    for name in ("tc_build_oriented", "tc_count_total", "tc_count_per_node", "tc_count_batch", "tc_graph_info",
                 "tc_export_csr", "tc_export_schedule", "tc_graph_reschedule", "tc_count_batch_static",
                 "tc_count_capture", "tc_count_replay"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _raise(rc: int):
    if rc == TC_OK:
        return
    lib = load()
    msg = (lib.tc_last_error() or b"").decode() or lib.tc_status_str(rc).decode()
    cls = {TC_ERR_ID_RANGE: IdRangeError, TC_ERR_INVALID_ARG: InvalidArgument,
           TC_ERR_OUT_OF_MEMORY: OutOfMemory}.get(rc, TcError)
    raise cls(rc, msg)


# ------------------------------------------------------------ torch plumbing

def _torch():
    import torch
    return torch


class _TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator."""

    def __init__(self):
        torch = _torch()
        self._torch = torch

        def _alloc(nbytes, stream, ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                              stream or 0))
            except Exception:
                return 0

        def _free(ptr, nbytes, stream, ctx):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:
                # interpreter shutdown: torch is already torn down and the
                # process releases the device memory itself
                pass

        self.alloc = _ALLOC_FN(_alloc)
        self.free = _FREE_FN(_free)


_torch_alloc = None
_torch_alloc_lock = threading.Lock()


def _is_tensor(x) -> bool:
    return type(x).__module__.startswith("torch")


def make_options(*, stream=None, inputs_on_device=False, outputs_on_device=False, hbm_budget_bytes=0, workers=0,
                 cost_fn=COST_PRIOR, min_chunk=0, small_max=0, lds_list_max=0, time_kernels=False,
                 partitions=0, rounds=0, direct=False, static_chunks=False, intersect=INTERSECT_AUTO,
                 search_ratio=0, hash=HASH_AUTO, bitmap_ratio=0, torch_allocator=True) -> Options:
    global _torch_alloc
    o = Options()
    load().tc_options_default(ctypes.byref(o))
    o.inputs_on_device = int(bool(inputs_on_device))
    o.outputs_on_device = int(bool(outputs_on_device))
    o.hbm_budget_bytes = int(hbm_budget_bytes)
    o.workers = int(workers)
    o.cost_fn = int(cost_fn)
    o.min_chunk = int(min_chunk)
    o.small_max = int(small_max)
    o.lds_list_max = int(lds_list_max)
    o.time_kernels = int(time_kernels)
    o.partitions = int(partitions)
    o.rounds = int(rounds)
    o.direct = int(bool(direct))
    o.static_chunks = int(bool(static_chunks))
    o.intersect = int(intersect)
    o.search_ratio = int(search_ratio)
    o.hash = int(hash)
    o.bitmap_ratio = int(bitmap_ratio)
    if stream is None:
        try:
            torch = _torch()
            if torch.cuda.is_available():
                stream = torch.cuda.current_stream().cuda_stream
        except ImportError:
            stream = None
    o.stream = stream or None
    if torch_allocator:
        try:
            torch = _torch()
            if torch.cuda.is_available():
                if _torch_alloc is None:
                    with _torch_alloc_lock:
                        if _torch_alloc is None:
                            _torch_alloc = _TorchAllocator()
                o.alloc = _torch_alloc.alloc
                o.free = _torch_alloc.free
        except ImportError:
            pass
    return o


def _as_edge_arrays(src, dst, on_device: bool):
    """Returns (keepalive, src_ptr, dst_ptr, m)."""
    if on_device:
        torch = _torch()
        s = src.to(torch.int32).contiguous()
        d = dst.to(torch.int32).contiguous()
        if s.numel() != d.numel():
            raise ValueError("src and dst differ in length")
        return (s, d), (s.data_ptr() if s.numel() else None), (d.data_ptr() if d.numel() else None), s.numel()
    s = np.ascontiguousarray(np.asarray(src, dtype=np.int32))
    d = np.ascontiguousarray(np.asarray(dst, dtype=np.int32))
    if s.shape != d.shape:
        raise ValueError("src and dst differ in length")
    return (s, d), (s.ctypes.data if s.size else None), (d.ctypes.data if d.size else None), s.shape[0]


class Graph:
    """Handle of one build: k graphs packed together (tc_build_oriented)."""

    def __init__(self, handle, ns, options_kw):
        self._h = ctypes.c_void_p(handle)
        self.ns = list(ns)
        self._kw = options_kw

    # -- counting
    def _opts(self, **over):
        kw = dict(self._kw)
        kw.update(over)
        return make_options(**kw)

    @property
    def k(self) -> int:
        return len(self.ns)

    @property
    def n_total(self) -> int:
        return int(sum(self.ns))

    def count_total(self, out=None, **over):
        """Totals of the k graphs: numpy int64[k], or written into a device tensor `out`."""
        lib = load()
        if out is not None:
            o = self._opts(outputs_on_device=True, **over)
            _raise(lib.tc_count_total(self._h, ctypes.byref(o), ctypes.c_void_p(out.data_ptr())))
            return out
        res = np.zeros(max(self.k, 1), np.int64)
        o = self._opts(outputs_on_device=False, **over)
        _raise(lib.tc_count_total(self._h, ctypes.byref(o), ctypes.c_void_p(res.ctypes.data)))
        return res[: self.k]

    def count_per_node(self, out=None, totals=None, **over):
        """Per-node counts (packed caller labels) and totals.  Host numpy by default;
        with `out` (and optionally `totals`) device tensors, writes them asynchronously."""
        lib = load()
        if out is not None:
            o = self._opts(outputs_on_device=True, **over)
            tp = ctypes.c_void_p(totals.data_ptr()) if totals is not None else None
            _raise(lib.tc_count_per_node(self._h, ctypes.byref(o), ctypes.c_void_p(out.data_ptr()), tp))
            return out, totals
        tv = np.zeros(max(self.n_total, 1), np.int64)
        tot = np.zeros(max(self.k, 1), np.int64)
        o = self._opts(outputs_on_device=False, **over)
        _raise(lib.tc_count_per_node(self._h, ctypes.byref(o), ctypes.c_void_p(tv.ctypes.data),
                                     ctypes.c_void_p(tot.ctypes.data)))
        return tv[: self.n_total], tot[: self.k]

    def reschedule(self, workers=0, cost_fn=COST_PRIOR, min_chunk=0, small_max=0, rounds=0, static_chunks=False,
                   intersect=INTERSECT_AUTO, search_ratio=0, lds_list_max=0, hash=HASH_AUTO, bitmap_ratio=0):
        """New task table, intersection choice, LDS cap, table kind and core
        tests for the same adjacency (tc_graph_reschedule); later counts use
        them."""
        self._kw.update(workers=workers, cost_fn=cost_fn, min_chunk=min_chunk, small_max=small_max, rounds=rounds,
                        static_chunks=static_chunks, intersect=intersect, search_ratio=search_ratio,
                        lds_list_max=lds_list_max, hash=hash, bitmap_ratio=bitmap_ratio)
        o = self._opts()
        _raise(load().tc_graph_reschedule(self._h, ctypes.byref(o)))

    def clustering(self, coeff=None, transitivity=None, totals=None, **over):
        """Local clustering coefficients (caller labels) and the transitivity
        of each graph, fp64 (tc_clustering).  Host numpy by default; with device
        tensors given, written asynchronously."""
        lib = load()
        if coeff is not None or transitivity is not None:
            o = self._opts(outputs_on_device=True, **over)
            ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
            _raise(lib.tc_clustering(self._h, ctypes.byref(o), ptr(coeff), ptr(transitivity), ptr(totals)))
            return coeff, transitivity, totals
        c = np.zeros(max(self.n_total, 1), np.float64)
        t = np.zeros(max(self.k, 1), np.float64)
        tot = np.zeros(max(self.k, 1), np.int64)
        o = self._opts(outputs_on_device=False, **over)
        _raise(lib.tc_clustering(self._h, ctypes.byref(o), ctypes.c_void_p(c.ctypes.data),
                                 ctypes.c_void_p(t.ctypes.data), ctypes.c_void_p(tot.ctypes.data)))
        return c[: self.n_total], t[: self.k], tot[: self.k]

    def worker_times(self):
        """(start ns, stop ns, kind) of every worker of the last count made with
        time_kernels=2, as an int64 array of shape (workers, 3); kind 0 = node-range
        task wave, 1 / 2 = workgroup of the medium / long list tier."""
        lib = load()
        nw = ctypes.c_int64(0)
        o = self._opts()
        _raise(lib.tc_worker_times(self._h, ctypes.byref(o), None, 0, ctypes.byref(nw)))
        out = np.zeros((max(nw.value, 1), 3), np.int64)
        if nw.value:
            _raise(lib.tc_worker_times(self._h, ctypes.byref(o), ctypes.c_void_p(out.ctypes.data), nw.value,
                                       ctypes.byref(nw)))
        return out[: nw.value]

    # -- inspection
    def info(self) -> dict:
        gi = GraphInfo()
        _raise(load().tc_graph_info(self._h, ctypes.byref(gi)))
        return {f: getattr(gi, f) for f, _ in GraphInfo._fields_ if not f.startswith("reserved")}

    def export_csr(self):
        """(off[n+1], col[m], perm[n]) in degree-order labels."""
        inf = self.info()
        n, m = inf["n"], inf["m"]
        off = np.zeros(n + 1, np.int64)
        col = np.zeros(max(m, 1), np.int32)
        perm = np.zeros(max(n, 1), np.int32)
        o = self._opts()
        _raise(load().tc_export_csr(self._h, ctypes.byref(o), ctypes.c_void_p(off.ctypes.data),
                                    ctypes.c_void_p(col.ctypes.data), ctypes.c_void_p(perm.ctypes.data)))
        return off, col[:m], perm[:n]

    def export_offsets(self):
        """off[n+1]: the row offsets in degree-order labels (packed graphs
        occupy consecutive label ranges, graph after graph)."""
        n = self.info()["n"]
        off = np.zeros(n + 1, np.int64)
        o = self._opts()
        _raise(load().tc_export_csr(self._h, ctypes.byref(o), ctypes.c_void_p(off.ctypes.data), None, None))
        return off

    def export_schedule(self):
        """(bnd[tasks+1], gid[tasks])."""
        lib = load()
        nt = ctypes.c_int64(0)
        o = self._opts()
        _raise(lib.tc_export_schedule(self._h, ctypes.byref(o), None, None, 0, ctypes.byref(nt)))
        bnd = np.zeros(nt.value + 1, np.int32)
        gid = np.zeros(max(nt.value, 1), np.int32)
        _raise(lib.tc_export_schedule(self._h, ctypes.byref(o), ctypes.c_void_p(bnd.ctypes.data),
                                      ctypes.c_void_p(gid.ctypes.data), nt.value + 1, ctypes.byref(nt)))
        return bnd, gid[: nt.value]

    def free(self):
        if self._h and self._h.value:
            load().tc_graph_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


def build_oriented(graphs: Sequence, *, stream=None, hbm_budget_bytes=0, workers=0, cost_fn=COST_PRIOR, min_chunk=0,
                   small_max=0, lds_list_max=0, partitions=0, rounds=0, direct=False, static_chunks=False,
                   intersect=INTERSECT_AUTO, search_ratio=0, hash=HASH_AUTO, bitmap_ratio=0,
                   torch_allocator=True) -> Graph:
    """Builds one handle from graphs given as (n, src, dst) triples.  src/dst are
    numpy arrays (host) or torch tensors (all on the device, or all host)."""
    if not len(graphs):
        raise ValueError("at least one graph is required")
    on_dev = _is_tensor(graphs[0][1]) and graphs[0][1].is_cuda
    keep = []
    arr = (Edges * len(graphs))()
    ns = []
    for i, (n, src, dst) in enumerate(graphs):
        kp, sp, dp, m = _as_edge_arrays(src, dst, on_dev)
        keep.append(kp)
        arr[i].n = int(n)
        arr[i].m = int(m)
        arr[i].src = sp
        arr[i].dst = dp
        ns.append(int(n))
    kw = dict(stream=stream, hbm_budget_bytes=hbm_budget_bytes, workers=workers, cost_fn=cost_fn,
              min_chunk=min_chunk, small_max=small_max, lds_list_max=lds_list_max, partitions=partitions,
              rounds=rounds, direct=direct, static_chunks=static_chunks, intersect=intersect,
              search_ratio=search_ratio, hash=hash, bitmap_ratio=bitmap_ratio, torch_allocator=torch_allocator)
    o = make_options(inputs_on_device=on_dev, **kw)
    h = ctypes.c_void_p(0)
    _raise(load().tc_build_oriented(arr, len(graphs), ctypes.byref(o), ctypes.byref(h)))
    del keep
    return Graph(h.value, ns, kw)


_EDGES_DTYPE = np.dtype({"names": ["n", "m", "src", "dst"], "formats": ["<i4", "<i8", "<u8", "<u8"],
                         "offsets": [0, 8, 16, 24], "itemsize": 32})


def build_packed_device(ns, ms, src_ptr: int, dst_ptr: int, *, stream=None, workers=0, cost_fn=COST_PRIOR,
                        min_chunk=0, small_max=0, lds_list_max=0, rounds=0, intersect=INTERSECT_AUTO,
                        search_ratio=0, hash=HASH_AUTO, bitmap_ratio=0, torch_allocator=True) -> Graph:
    """Builds one handle from k graphs whose edges already lie back to back in
    two device arrays (graph i's edges start at the sum of the earlier m), read
    in place.  ns / ms: node and edge counts per graph; src_ptr / dst_ptr:
    device addresses of the int32 arrays."""
    ns = np.asarray(ns, np.int64)
    ms = np.asarray(ms, np.int64)
    k = ns.shape[0]
    if k < 1 or ms.shape[0] != k:
        raise ValueError("ns and ms must have the same, non-zero length")
    eb = np.zeros(k, np.int64)
    np.cumsum(ms[:-1], out=eb[1:])
    arr = np.zeros(k, _EDGES_DTYPE)
    arr["n"] = ns
    arr["m"] = ms
    arr["src"] = np.uint64(src_ptr) + (eb * 4).astype(np.uint64)
    arr["dst"] = np.uint64(dst_ptr) + (eb * 4).astype(np.uint64)
    kw = dict(stream=stream, workers=workers, cost_fn=cost_fn, min_chunk=min_chunk, small_max=small_max,
              lds_list_max=lds_list_max, rounds=rounds, intersect=intersect, search_ratio=search_ratio,
              hash=hash, bitmap_ratio=bitmap_ratio, torch_allocator=torch_allocator)
    o = make_options(inputs_on_device=True, **kw)
    h = ctypes.c_void_p(0)
    _raise(load().tc_build_oriented(ctypes.cast(arr.ctypes.data, ctypes.POINTER(Edges)), k, ctypes.byref(o),
                                    ctypes.byref(h)))
    return Graph(h.value, ns.tolist(), kw)


def count_batch(graphs: Sequence[Graph], per_node: bool = False, **over):
    """One launch over several handles.  Returns (totals per handle, per-node
    arrays or None), as host numpy arrays."""
    lib = load()
    ng = len(graphs)
    hs = (ctypes.c_void_p * ng)(*[g._h.value for g in graphs])
    ktot = sum(g.k for g in graphs)
    tot = np.zeros(max(ktot, 1), np.int64)
    o = graphs[0]._opts(outputs_on_device=False, **over)
    pn = None
    outs = None
    if per_node:
        outs = [np.zeros(max(g.n_total, 1), np.int64) for g in graphs]
        pn = (ctypes.c_void_p * ng)(*[a.ctypes.data for a in outs])
    _raise(lib.tc_count_batch(hs, ng, ctypes.byref(o), ctypes.c_void_p(tot.ctypes.data), pn))
    res_tot, i = [], 0
    for g in graphs:
        res_tot.append(tot[i:i + g.k].copy())
        i += g.k
    if per_node:
        outs = [a[: g.n_total] for a, g in zip(outs, graphs)]
    return res_tot, outs


def _device_batch_args(graphs, totals, per_node):
    ng = len(graphs)
    hs = (ctypes.c_void_p * ng)(*[g._h.value for g in graphs])
    if totals.numel() < sum(g.k for g in graphs):
        raise ValueError("totals holds fewer entries than the graphs of the batch")
    pn = None
    if per_node is not None:
        if len(per_node) != ng:
            raise ValueError("one per-node output (or None) per handle")
        for t, g in zip(per_node, graphs):
            if t is not None and t.numel() < g.n_total:
                raise ValueError("per-node output shorter than its handle's node count")
        pn = (ctypes.c_void_p * ng)(*[(t.data_ptr() if t is not None else None) for t in per_node])
    return hs, pn


def count_batch_device(graphs: Sequence[Graph], totals, per_node=None, **over):
    """tc_count_batch into device tensors (totals: int64[sum of k]; per_node:
    None or one int64 tensor / None per handle), asynchronous on the stream
    (default: the current one).  Uses its own scratch, so a handle may be in
    several such counts on different streams at once."""
    hs, pn = _device_batch_args(graphs, totals, per_node)
    o = graphs[0]._opts(outputs_on_device=True, **over)
    _raise(load().tc_count_batch(hs, len(graphs), ctypes.byref(o), ctypes.c_void_p(totals.data_ptr()), pn))
    return totals, per_node


def count_batch_static(graphs: Sequence[Graph], totals, per_node=None, **over):
    """tc_count_batch_static: the batch count into device tensors (totals:
    int64[sum of k]; per_node: None or one int64 tensor / None per handle),
    with the library's fixed per-GPU scratch instead of allocated memory.
    Asynchronous on the current stream."""
    hs, pn = _device_batch_args(graphs, totals, per_node)
    o = graphs[0]._opts(outputs_on_device=True, torch_allocator=False, **over)
    _raise(load().tc_count_batch_static(hs, len(graphs), ctypes.byref(o), ctypes.c_void_p(totals.data_ptr()), pn))
    return totals, per_node


def count(n, src, dst, per_node: bool = True, **kw):
    """Convenience: build and count one graph.  Returns (T, T_v or None)."""
    with build_oriented([(n, src, dst)], **kw) as g:
        if per_node:
            tv, tot = g.count_per_node()
            return int(tot[0]), tv
        return int(g.count_total()[0]), None
