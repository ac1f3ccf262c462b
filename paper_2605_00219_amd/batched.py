"""Several camera views of uneven resolution per training step, in one
persistent launch per stage, captured into a HIP graph.

One step renders all views of the set: one projection launch over all views,
one segmented sort, one persistent forward and one persistent backward launch
over every (view, tile) work item, and one projection-backward + Adam pass
that sums each Gaussian's gradient over the views.  The whole step is
captured once into a HIP graph (torch.cuda.CUDAGraph records the library's
launches on the capturing stream); each iteration then only refreshes the
camera table and the concatenated target image in their fixed buffers and
replays the graph.  Nothing in the step synchronises with the host; the
intersection-capacity status word is checked after the run.
"""
from __future__ import annotations

import numpy as np
import torch

from . import pipeline as P


class ViewSet:
    """Fixed slot resolutions; per iteration a camera goes into each slot."""

    def __init__(self, resolutions, tile: int, pixels_per_lane: int | None = None, cull: int = 0):
        self.resolutions = list(resolutions)
        self.cull = int(cull)
        self.widths = [w for w, _ in self.resolutions]
        self.heights = [h for _, h in self.resolutions]
        self.tile = tile
        self.pixels_per_lane = pixels_per_lane
        self.pixels = sum(w * h for w, h in self.resolutions)


class BatchedStep:
    """A training step over a ViewSet, optionally persistent and graph-captured.

    views_buf (V x 128 bytes) and target_buf (pixels x 3) are the fixed
    device buffers the captured launches read; `load` refreshes them."""

    def __init__(self, model: P.Model, n: int, viewset: ViewSet, capacity: int, lds_batch: int = 64,
                 persistent: bool = True, order: torch.Tensor | None = None,
                 n_groups: int | None = None, graph: bool = True, row_capacity: int | None = None):
        self.model = model
        self.viewset = viewset
        self.frame = P.Frame(n, viewset.widths, viewset.heights, viewset.tile, capacity=capacity,
                             pixels_per_lane=viewset.pixels_per_lane, cull=viewset.cull,
                             row_capacity=row_capacity)
        self.views_buf = torch.zeros(128 * len(viewset.resolutions), dtype=torch.uint8, device="cuda")
        self.target_buf = torch.zeros(viewset.pixels, 3, dtype=torch.float32, device="cuda")
        self.lds_batch = lds_batch
        self.order = order
        self.sched = self.frame.schedule(order, n_groups) if persistent else None
        self.graph = None
        self.use_graph = graph

    def load(self, views_dev_rows: torch.Tensor, target: torch.Tensor) -> None:
        self.views_buf.copy_(views_dev_rows.reshape(-1))
        self.target_buf.copy_(target.reshape(-1, 3))

    def _launch(self) -> None:
        f, m = self.frame, self.model
        P.project(m.params, f, self.views_buf)
        P.bin_sort(f)
        P.rasterize_fwd(f, self.views_buf, self.lds_batch, self.sched)
        P.rasterize_bwd(f, self.views_buf, target=self.target_buf, lds_batch=self.lds_batch,
                        sched=self.sched)
        P.project_bwd_adam(m, f, self.views_buf)

    def capture(self) -> None:
        """Record one step into a HIP graph (no optimiser state changes:
        parameters and moments are restored after the warm-up launch)."""
        saved = [t.clone() for t in (self.model.params, self.model.m, self.model.v, self.model.step)]
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._launch()      # warm-up outside capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._launch()
        torch.cuda.synchronize()
        for t, s0 in zip((self.model.params, self.model.m, self.model.v, self.model.step), saved):
            t.copy_(s0)
        self.graph = g

    def run(self) -> None:
        if self.use_graph:
            if self.graph is None:
                self.capture()
            self.graph.replay()
        else:
            self._launch()

    def status(self) -> int:
        return self.frame.status_bits()


def make_views(make_view, cams, resolutions, iteration: int):
    """Camera (8i + k) mod len(cams) in slot k at the slot's resolution."""
    k = len(resolutions)
    recs = [make_view(w, h, cams[(k * iteration + s) % len(cams)]) for s, (w, h) in enumerate(resolutions)]
    return recs
