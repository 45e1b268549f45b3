"""Many uneven boxes advanced together: every stage launch of mhd_step_batch
covers the tiles of all boxes, so small boxes fill the GPU together instead of
one after another.  A box gives the same bits alone and in a batch: both go
through the same kernel, tile by tile.

    boxes = [MHDBox(*dims, precision="fp32", stream=s) for dims in shapes]
    batch = BoxBatch(boxes)
    batch.step([20] * len(boxes))          # eager: 2 stage launches per cycle
    g = batch.capture([20] * len(boxes))   # or one hipGraph replayed at will
    g.replay()                             # on the batch's stream
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from .box import MHDBox


class BoxBatch:
    """Boxes sharing precision, solver, integrator, tile shape and stream."""

    def __init__(self, boxes: list[MHDBox]):
        if not boxes:
            raise ValueError("empty batch")
        s0 = boxes[0].stream
        for b in boxes:
            if b.stream.cuda_stream != s0.cuda_stream:
                raise ValueError("all boxes of a batch must share one stream")
        self.boxes = list(boxes)
        self.stream = s0
        self.lib = boxes[0].lib
        self._ctx = (C.c_void_p * len(boxes))(*[b.ctx.value for b in boxes])

    def step(self, nsteps):
        if isinstance(nsteps, int):
            nsteps = [nsteps] * len(self.boxes)
        if len(nsteps) != len(self.boxes):
            raise ValueError("one step count per box")
        arr = (C.c_int * len(nsteps))(*[int(n) for n in nsteps])
        L.check(self.lib.mhd_step_batch(self._ctx, arr, len(self.boxes),
                                        C.c_void_p(self.stream.cuda_stream)), "mhd_step_batch")
        return self

    def tune(self, tuner=None, force: bool = False) -> dict:
        """Choose one launch shape for the whole batch (autotune.Tuner: cached,
        else timed on the GPU) and apply it to every box."""
        from .autotune import Tuner
        tuner = tuner or Tuner()
        return tuner.tune(self.boxes, self.stream, force=force)

    def capture(self, nsteps) -> "StepGraph":
        """Record the launches of ``step(nsteps)`` into a HIP graph on the batch's
        stream (RK2 or RK3: the buffer roles of an Euler cycle alternate on the
        host).  Each replay advances every box by its step count again, with
        dt and t kept on the device."""
        for b in self.boxes:
            if b.params.integrator == L.MHD_EULER:
                raise ValueError("graph capture needs a Runge-Kutta integrator")
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=self.stream):
            self.step(nsteps)
        return StepGraph(g, self.stream)


class StepGraph:
    """A captured batch of cycles.  ``replay()`` launches it on the batch's
    stream (a bare CUDAGraph.replay() would use the caller's current stream,
    which the boxes' own copies do not wait for)."""

    def __init__(self, graph: torch.cuda.CUDAGraph, stream: torch.cuda.Stream):
        self.graph = graph
        self.stream = stream

    def replay(self):
        with torch.cuda.stream(self.stream):
            self.graph.replay()
