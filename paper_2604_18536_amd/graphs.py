"""Replayable HIP graphs of repeated time steps.

A step issues about 25 kernels; on small grids (a 64^2 or 256^2 field sits in
the 256 MB last-level cache) their launch cost, not memory, sets the rate.
``StepGraph`` records ``nsteps`` in-place steps of one solver on one buffer
into a HIP graph through torch's stream capture (the library launches on the
stream torch makes current, so its kernels are recorded) and replays them with
one launch. Nothing in a step allocates or uses memset/memcpy, so the recorded
steps are exactly the eager ones.
"""
from __future__ import annotations

import torch


class StepGraph:
    """``nsteps`` steps u <- step(u, dt) recorded once, replayed with ``replay()``."""

    def __init__(self, solver, u, dt, nsteps, scheme="rk4"):
        if not u.is_contiguous():
            raise ValueError("u must be contiguous")
        self.solver, self.u = solver, u
        # warm-up on a side stream (torch's capture recipe); the step itself allocates nothing
        side = torch.cuda.Stream(device=u.device)
        side.wait_stream(torch.cuda.current_stream(u.device))
        with torch.cuda.stream(side):
            solver.step(u.clone(), dt, scheme=scheme)
        torch.cuda.current_stream(u.device).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            for _ in range(int(nsteps)):
                solver.step(u, dt, out=u, scheme=scheme)
        # leave the library on the caller's stream again
        solver._sync_stream()

    def replay(self):
        """Advance ``u`` (in place) by the recorded steps; returns ``u``."""
        self.graph.replay()
        return self.u
