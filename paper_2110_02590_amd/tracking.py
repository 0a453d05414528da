"""Batched real-time tracking (Section IV-C) over many grids of uneven size.

Each instance owns a grid handle and device state (u, x, y); one tracking
update per instance and step runs entirely on the device
(`rpf_track_step`).  The updates of all instances for one step are either
launched eagerly one instance after the other, or captured once into a HIP
graph with the instances spread over several streams (fork/join), which is
then replayed every step.  This module only routes tensors; all arithmetic
is in the HIP library.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import torch

from .problem import Problem


@dataclasses.dataclass
class TrackingItem:
    """One instance: grid dict, AL point dict (rho, y, sigma_f, sigma_c),
    constraint bounds, per-step load factors [steps, nb]."""
    grid: dict
    point: dict
    s_lo: np.ndarray
    s_hi: np.ndarray
    factors: np.ndarray


class _Inst:
    def __init__(self, item: TrackingItem, max_batch: int):
        self.pr = pr = Problem(item.grid, max_batch=max_batch)
        dev = "cuda"
        self.u = pr.u0.clone()
        self.x = pr.flat_x()
        st, _ = pr.grid.pf_solve(self.u, pr.pd, pr.qd, self.x)
        if int(st[1]) != 1:
            raise RuntimeError("base power flow did not converge")
        ep = item.point
        self.rho = float(ep["rho"])
        self.y = torch.tensor(np.asarray(ep["y"], float), device=dev)
        self.sigma = torch.tensor(np.concatenate([[ep["sigma_f"]], np.asarray(ep["sigma_c"], float)]),
                                  device=dev)
        self.s_lo = torch.tensor(np.asarray(item.s_lo, float), device=dev)
        self.s_hi = torch.tensor(np.asarray(item.s_hi, float), device=dev)
        lo, hi = pr.u_bounds()
        self.u_lo = torch.tensor(lo, device=dev)
        self.u_hi = torch.tensor(hi, device=dev)
        self.status = torch.zeros(5, dtype=torch.int32, device=dev)
        self.delta = self._shift(item)

    def _shift(self, item) -> float:
        """Inertia-control shift at the base point: the smallest value of the
        ladder 0, 1e-8 max(1, max|diag H|) * 10^k for which the Cholesky
        succeeds, times 10 (loads move between steps)."""
        pr = self.pr
        g = pr.grid
        s = torch.clamp(torch.tensor(np.asarray(item.point["s"], float), device="cuda"), self.s_lo, self.s_hi)
        grad, _ = g.reduced_gradient(self.x, self.u, pr.pd, pr.qd, s, self.y, self.rho, self.sigma)
        H = g.reduced_hessian(batch=min(g.max_batch, pr.nu))
        base = 1e-8 * max(1.0, float(torch.diagonal(H).abs().max()))
        delta = 0.0
        for _ in range(40):
            _, info = g.factor_solve(H.clone(), grad, delta=delta)
            if int(info) == 0:
                return max(10.0 * delta, base)
            delta = base if delta == 0.0 else 10.0 * delta
        raise RuntimeError("no positive definite shift found")


class TrackingBatch:
    def __init__(self, items: List[TrackingItem], max_batch: int = 256, pf_iters: int = 6,
                 max_halvings: int = 4, tol: float = 1e-10, nstreams: int = 8):
        self.items = items
        self.inst = [_Inst(it, max_batch) for it in items]
        self.pf_iters, self.max_halvings, self.tol = pf_iters, max_halvings, tol
        sizes = [int(it.grid["nb"]) for it in items]
        self.offs = np.concatenate([[0], np.cumsum(sizes)])
        steps = min(it.factors.shape[0] for it in items)
        self.steps = steps
        self.fac_all = torch.tensor(np.concatenate([it.factors[:steps] for it in items], axis=1), device="cuda")
        self.cur = torch.empty(int(self.offs[-1]), dtype=torch.float64, device="cuda")
        self.nstreams = max(1, nstreams)
        self.streams = [torch.cuda.Stream() for _ in range(self.nstreams)]
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    def _launch(self, k: int):
        it = self.inst[k]
        pr = it.pr
        fac = self.cur[int(self.offs[k]):int(self.offs[k + 1])]
        pr.grid.track_step(it.u, it.x, it.y, pr.pd, pr.qd, fac, it.s_lo, it.s_hi, it.u_lo, it.u_hi, it.rho,
                           it.sigma, it.delta, self.pf_iters, self.max_halvings, self.tol, status=it.status)

    def set_step(self, t: int):
        self.cur.copy_(self.fac_all[t])

    def step_eager(self, t: int):
        """All instances, one after the other on the current stream."""
        self.set_step(t)
        for k in range(len(self.inst)):
            self._launch(k)

    def _forked(self):
        main = torch.cuda.current_stream()
        ev = torch.cuda.Event()
        ev.record(main)
        for j, st in enumerate(self.streams):
            st.wait_event(ev)
        for k in range(len(self.inst)):
            st = self.streams[k % self.nstreams]
            with torch.cuda.stream(st):
                self._launch(k)
        for st in self.streams:
            main.wait_stream(st)

    def capture(self):
        """Capture one step of every instance into a HIP graph (fork/join
        over the streams).  The captured step reads the loads of `self.cur`;
        state lives in the instances' tensors."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._forked()
        torch.cuda.synchronize()
        self.graph = g

    def step_graph(self, t: int):
        self.set_step(t)
        self.graph.replay()

    def state(self):
        return [(i.u.clone(), i.x.clone(), i.y.clone(), i.status.clone()) for i in self.inst]

    def load_state(self, st):
        for i, (u, x, y, s) in zip(self.inst, st):
            i.u.copy_(u)
            i.x.copy_(x)
            i.y.copy_(y)
            i.status.copy_(s)
