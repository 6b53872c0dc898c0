"""Launch-shape autotuning and hipGraph capture of the SSPRK step.

``autotune`` times ``grmhd_rk_step`` for every compiled stage-kernel tile shape
and both schedules (one workgroup per tile, persistent workgroups over per-XCD
tile queues) on scratch copies of the state, and returns the fastest
``grmhd_params``.  Results are cached per domain and method.

``StepGraph`` captures one ``grmhd_rk_step`` (its 7 kernels; no memsets) into a
graph and replays it.
"""
from __future__ import annotations

import ctypes

import torch

from . import grmhd as G

_CACHE = {}
NTILE = G.GRMHD_NTILE


def _key(dom, par):
    boxes = tuple((tuple(b.n), b.ng, tuple(b.bc), b.cell_off, b.vert_off) for b in dom._boxes)
    return (boxes, dom.cell_stride, par.recon, par.precision, par.wenoz_p)


def _with(par, tile, schedule):
    p = G.grmhd_params()
    ctypes.memmove(ctypes.byref(p), ctypes.byref(par), ctypes.sizeof(p))
    p.tile = tile
    p.schedule = schedule
    return p


def autotune(dom, par, met, U, P, dt, reps=3, verbose=False):
    """Fastest (tile, schedule) for grmhd_rk_step on this domain; returns (params, timings_ms)."""
    k = _key(dom, par)
    if k in _CACHE:
        return _with(par, *_CACHE[k][0]), _CACHE[k][1]
    Us, Ps = U.clone(), P.clone()
    ws = torch.empty(G.grmhd_workspace_bytes(dom, par) // 8 + 1, dtype=torch.float64, device=U.device)
    times = {}
    for tile in range(NTILE):
        for sched in (G.GRMHD_SCHED_GRID, G.GRMHD_SCHED_QUEUE):
            p = _with(par, tile, sched)
            Us.copy_(U)
            Ps.copy_(P)
            G.grmhd_rk_step(dom, p, met, Us, Ps, dt, ws=ws)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                G.grmhd_rk_step(dom, p, met, Us, Ps, dt, ws=ws)
            b.record()
            b.synchronize()
            times[(tile, sched)] = a.elapsed_time(b) / reps
            if verbose:
                print(f"autotune tile={tile} schedule={sched}: {times[(tile, sched)]:.3f} ms/step")
    best = min(times, key=times.get)
    _CACHE[k] = (best, times)
    return _with(par, *best), times


class StepGraph:
    """One grmhd_rk_step captured in a graph over fixed U, P, workspace and scalars."""

    def __init__(self, dom, par, met, U, P, dt, scheme=G.GRMHD_SSPRK3, max_rate=None, n_fail=None):
        self.ws = torch.empty(G.grmhd_workspace_bytes(dom, par, scheme) // 8 + 1, dtype=torch.float64,
                              device=U.device)
        self.graph = torch.cuda.CUDAGraph()
        self._keep = (dom, par, met, U, P, max_rate, n_fail)
        torch.cuda.synchronize()
        with torch.cuda.graph(self.graph):
            G.grmhd_rk_step(dom, par, met, U, P, dt, scheme, None, max_rate, n_fail, ws=self.ws)
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()
