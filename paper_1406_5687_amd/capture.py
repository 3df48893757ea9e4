"""Replays of a count as one captured HIP graph (tc_count_capture /
tc_count_replay of the C ABI).

The library records the count on a stream of its own: reset of its scratch,
the persistent counting kernels, the per-node scatter and the copy of the
totals.  Each replay is one graph launch on the caller's stream.  torch only
supplies the output tensors and the stream.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

from . import tc


class CapturedCount:
    """A captured count of one handle (or of several, as one batch) into device
    outputs: ``totals`` (int64[sum of k]) and, with per_node, ``per_node_out``
    (int64[n] of the first handle) or ``per_node_outs`` (one per handle)."""

    def __init__(self, graph, per_node: bool = False):
        import torch

        graphs: Sequence = list(graph) if isinstance(graph, (list, tuple)) else [graph]
        self.graphs = graphs
        self.per_node = per_node
        self.totals = torch.zeros(max(sum(g.k for g in graphs), 1), dtype=torch.int64, device="cuda")
        self.per_node_outs = ([torch.zeros(max(g.n_total, 1), dtype=torch.int64, device="cuda") for g in graphs]
                              if per_node else None)
        self.per_node_out = self.per_node_outs[0] if per_node else None
        hs, pn = tc._device_batch_args(graphs, self.totals, self.per_node_outs)
        o = graphs[0]._opts(outputs_on_device=True)
        h = ctypes.c_void_p(0)
        tc._raise(tc.load().tc_count_capture(hs, len(graphs), ctypes.byref(o), ctypes.c_void_p(self.totals.data_ptr()),
                                             pn, ctypes.byref(h)))
        self._h = h

    def replay(self, stream=None):
        """Launches the captured count on `stream` (default: the current torch
        stream); outputs are self.totals (and self.per_node_out) once the
        stream reaches them."""
        o = tc.make_options(stream=stream, torch_allocator=False)
        tc._raise(tc.load().tc_count_replay(self._h, ctypes.byref(o)))
        return self.totals, self.per_node_out

    def free(self):
        if self._h and self._h.value:
            tc.load().tc_count_graph_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
