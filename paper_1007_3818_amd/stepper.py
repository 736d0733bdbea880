"""Multi-step drivers over the C ABI: a periodic uniform grid and a batch of
refinement levels, with the time step kept on the device so that a step can be
captured once in a HIP graph and replayed.

One step of ``PeriodicGrid``:
  1. ``gamer_hydro_solve_periodic``     state -> new state, per-group stats, the
                                        ghost cells read from the neighbouring
                                        groups, dt read from ``dt_dev``
     (or, with ``fused=False``: ``gamer_pack_periodic`` into a padded copy, then
     ``gamer_hydro_solve_batched``; bitwise the same in FP64, to rounding in FP32)
  2. ``gamer_step_reduce``              stats -> next dt (CFL) and totals
plus a device-side time accumulator.  Nothing synchronises with the host.
"""
from __future__ import annotations

import torch

from . import hydro

NI, NP, NV = 16, 20, 5


class PeriodicGrid:
    """A uniform periodic grid of gx x gy x gz groups, advanced on the GPU."""

    def __init__(self, state: torch.Tensor, gx: int, gy: int, gz: int, dh: float, gamma: float,
                 cfl: float = 0.5, theta: float | None = None, variant: int | None = None,
                 grid: int | None = None, fused: bool = True):
        if not state.is_cuda:
            raise ValueError("state must live on the GPU")
        self.gx, self.gy, self.gz = gx, gy, gz
        self.n = gx * gy * gz
        self.gamma, self.cfl, self.theta = gamma, cfl, theta
        self.variant, self.grid = variant, grid
        dev, dt_ = state.device, state.dtype
        self.state = [state.contiguous().clone(), torch.empty_like(state)]
        self.cur = 0
        self.fused = fused
        self.padded = None if fused else torch.empty((self.n, NV, NP, NP, NP), dtype=dt_, device=dev)
        self.stats = torch.empty((self.n, 8), dtype=torch.float64, device=dev)
        self.dh_dev = torch.full((1,), dh, dtype=torch.float64, device=dev)
        self.dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
        self.totals = torch.empty(7, dtype=torch.float64, device=dev)
        self.t_dev = torch.zeros(1, dtype=torch.float64, device=dev)
        self.graph = None
        # initial time step from the initial state
        hydro.group_stats(self.state[0], gamma, out=self.stats)
        hydro.step_reduce(self.stats, None, self.dh_dev, cfl, dt_out=self.dt_dev, totals_out=self.totals)

    @property
    def current(self) -> torch.Tensor:
        return self.state[self.cur]

    def _step(self, src: int):
        dst = 1 - src
        if self.fused:
            hydro.hydro_solve_periodic(self.state[src], self.gx, self.gy, self.gz, self.dt_dev,
                                       self.dh_dev, self.gamma, out=self.state[dst],
                                       group_stats=self.stats, theta=self.theta,
                                       variant=self.variant, grid=self.grid)
        else:
            hydro.pack_periodic(self.state[src], self.gx, self.gy, self.gz, out=self.padded)
            hydro.hydro_solve_batched(self.padded, None, self.dt_dev, self.dh_dev, self.gamma,
                                      out=self.state[dst], group_stats=self.stats, theta=self.theta,
                                      variant=self.variant, grid=self.grid)
        self.t_dev += self.dt_dev
        hydro.step_reduce(self.stats, None, self.dh_dev, self.cfl, dt_out=self.dt_dev,
                          totals_out=self.totals)
        return dst

    def step(self, n: int = 1):
        """Advance n steps (eagerly, or by graph replays when captured)."""
        if self.graph is not None:
            if n % 2:
                raise ValueError("a captured grid advances in pairs of steps")
            for _ in range(n // 2):
                self.graph.replay()
            return
        for _ in range(n):
            self.cur = self._step(self.cur)

    def capture(self):
        """Capture two steps (state A -> B -> A) in one HIP graph.  One eager pair of
        steps runs first to warm up the launch path."""
        if self.cur != 0:
            raise ValueError("capture from the initial buffer")
        self.step(2)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self._step(self._step(0))
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g
        return self

    def time(self) -> float:
        return float(self.t_dev.item())
