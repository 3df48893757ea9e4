"""Replays of a handle's count as one captured HIP graph.

The count path is stream ordered and, once its per-handle scratch exists,
allocates nothing and issues no memset: reset kernels, the persistent
counting kernels, the per-node scatter and a device-to-device copy of the
totals.  Capturing it once (torch.cuda.graph drives hipStreamBeginCapture on
the library's stream) turns every later count of the same handle into a
single graph launch.
"""
from __future__ import annotations

from . import tc


class CapturedCount:
    """Captures graph.count_total / count_per_node into device outputs."""

    def __init__(self, graph: "tc.Graph", per_node: bool = False):
        import torch

        self.graph = graph
        self.per_node = per_node
        self.totals = torch.zeros(max(graph.k, 1), dtype=torch.int64, device="cuda")
        self.per_node_out = (torch.zeros(max(graph.n_total, 1), dtype=torch.int64, device="cuda")
                             if per_node else None)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._run()  # creates the handle's scratch outside the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.cuda_graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.cuda_graph):
            self._run()
        torch.cuda.synchronize()

    def _run(self):
        if self.per_node:
            self.graph.count_per_node(out=self.per_node_out, totals=self.totals)
        else:
            self.graph.count_total(out=self.totals)

    def replay(self):
        """Launches the captured count on the current stream; outputs are
        self.totals (and self.per_node_out) once the stream reaches them."""
        self.cuda_graph.replay()
        return self.totals, self.per_node_out
