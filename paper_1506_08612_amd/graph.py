"""HIP graph capture of the device-only scan launches.

A prepared batch (`api.Batch`) or a count-only single-pattern scan enqueues
nothing but kernel launches (the counters are cleared by a kernel, not a
memset), so the whole launch sequence can be captured once and replayed: a
replay costs one graph launch instead of one host call and argument check per
kernel.  The captured buffers (text, tables, workspace, counts) must stay
alive and at the same addresses for as long as the graph is replayed.
"""
from __future__ import annotations

from typing import Optional

from . import api


def _torch():
    import torch
    return torch


class GraphedBatch:
    """Capture `batch.run(text)` and replay it; counts land in `batch.counts`."""

    def __init__(self, text, batch: "api.Batch", warmup: int = 1):
        torch = _torch()
        self.text = text
        self.batch = batch
        side = torch.cuda.Stream()  # default priority
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                batch.run(text)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.out = batch.run(text)

    def replay(self):
        self.graph.replay()
        return self.out


class GraphedCount:
    """Capture a count-only single-pattern scan (dfa_count) and replay it."""

    def __init__(self, text, table, m: int, t: Optional["api.Tune"] = None, warmup: int = 1):
        torch = _torch()
        self.text, self.table, self.m, self.t = text, table, m, t
        self.count = torch.empty(1, dtype=torch.int64, device=text.device)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                api.count_async(text, table, m, self.count, t=t)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            api.count_async(text, table, m, self.count, t=t)

    def replay(self):
        self.graph.replay()
        return self.count
