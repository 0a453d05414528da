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
    def __init__(self, item: TrackingItem, max_batch: int, mode: str = "newton"):
        self.mode = mode
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
        if mode == "qp":
            # slack at the base point: the constraints clipped into their box
            pr_s = torch.zeros(pr.m, dtype=torch.float64, device=dev)
            _, c = pr.grid.al_objective(self.x, self.u, pr.pd, pr.qd, pr_s, self.y, self.rho, self.sigma)
            self.s = torch.minimum(torch.maximum(c, self.s_lo), self.s_hi).contiguous()
            self.J = torch.empty((pr.m, pr.nu), dtype=torch.float64, device=dev)
            self.status = torch.zeros(8, dtype=torch.int32, device=dev)
            self.delta = self._qp_shift()
        else:
            self.s = None
            self.status = torch.zeros(5, dtype=torch.int32, device=dev)
            self.delta = self._shift(item)

    def _qp_shift(self) -> float:
        """Shift of the exact step's QP: at the base point, 1.5 times the most
        negative eigenvalue of H_uu = H - rho J^T D_c^2 J (the curvature the
        penalty does not supply) plus 1e-2 makes the QP strictly convex; ten
        times that keeps it convex while the loads move (the inertia control
        of the interior-point method covers the rest)."""
        pr = self.pr
        g = pr.grid
        lo, hi = pr.u_bounds()
        ulo = torch.tensor(lo, device="cuda")
        uhi = torch.tensor(hi, device="cuda")
        out = g.qp_step(self.x, self.u, pr.pd, pr.qd, self.s, self.y, self.rho, self.sigma, 0.0, ulo, uhi,
                        self.s_lo, self.s_hi, max_iter=0, J=self.J)
        H, J = out["H"], out["J"]
        sc2 = self.sigma[1:] ** 2
        Huu = H - self.rho * (J.T.contiguous() @ (sc2[:, None] * J))
        lam = float(torch.linalg.eigvalsh(0.5 * (Huu + Huu.T)).min())
        return 10.0 * (1.5 * max(0.0, -lam) + 1e-2)

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
    """mode "newton": the shifted Newton step (rpf_track_step); mode "qp":
    the exact step, the bounded QP by the interior-point method
    (rpf_track_step_qp, qp_iters and qp_tol)."""

    def __init__(self, items: List[TrackingItem], max_batch: int = 256, pf_iters: int = 6,
                 max_halvings: int = 4, tol: float = 1e-10, nstreams: int = 8, mode: str = "newton",
                 qp_iters: int = 50, qp_tol: float = 1e-10, redispatch: bool = False):
        if mode not in ("newton", "qp"):
            raise ValueError("mode must be 'newton' or 'qp'")
        self.items = items
        self.mode = mode
        self.qp_iters, self.qp_tol = qp_iters, qp_tol
        # exact step only: at a change of the total load the PV dispatch is
        # scaled by the ratio of total loads before the update
        self.redispatch = redispatch and mode == "qp"
        self.t = 0
        self.inst = [_Inst(it, max_batch, mode) for it in items]
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
        if self.mode == "qp":
            pr.grid.track_step_qp(it.u, it.s, it.x, it.y, pr.pd, pr.qd, fac, it.s_lo, it.s_hi, it.u_lo, it.u_hi,
                                  it.rho, it.sigma, it.delta, self.pf_iters, self.max_halvings, self.tol,
                                  self.qp_iters, self.qp_tol, J=it.J, status=it.status,
                                  dispatch_scale=self.dispatch_scale(k, self.t))
            return
        pr.grid.track_step(it.u, it.x, it.y, pr.pd, pr.qd, fac, it.s_lo, it.s_hi, it.u_lo, it.u_hi, it.rho,
                           it.sigma, it.delta, self.pf_iters, self.max_halvings, self.tol, status=it.status)

    def dispatch_scale(self, k: int, t: int) -> float:
        """Ratio of instance k's total load at step t to that at step t - 1
        when redispatching (1.0 otherwise): host figures of the scenario's
        load factors."""
        if not self.redispatch or t == 0:
            return 1.0
        it = self.items[k]
        pd0 = np.asarray(it.grid["pd"], float)
        a = float(pd0 @ it.factors[t])
        b = float(pd0 @ it.factors[t - 1])
        return 1.0 if a == b else a / b

    def set_step(self, t: int):
        self.t = t
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
        return [(i.u.clone(), i.x.clone(), i.y.clone(), i.status.clone(),
                 None if i.s is None else i.s.clone()) for i in self.inst]

    def save(self, path, t: int):
        """The tracking state between steps as a .npz: per instance u, x, y,
        the status words, the slack s (exact step), rho and the step's shift;
        the index t of the next step; the step mode; and the content hash of
        each instance's grid (gridgen.fingerprint), which `load` checks.  The
        load factors are not stored: they come from the instances' items."""
        import gridgen
        arrs = {"t": np.array(int(t)), "mode": np.array(self.mode), "n": np.array(len(self.inst)),
                "fingerprint": np.array([gridgen.fingerprint(it.grid) for it in self.items])}
        for k, i in enumerate(self.inst):
            arrs[f"u{k}"] = i.u.cpu().numpy()
            arrs[f"x{k}"] = i.x.cpu().numpy()
            arrs[f"y{k}"] = i.y.cpu().numpy()
            arrs[f"status{k}"] = i.status.cpu().numpy()
            arrs[f"param{k}"] = np.array([i.rho, i.delta])
            if i.s is not None:
                arrs[f"s{k}"] = i.s.cpu().numpy()
        np.savez(path, **arrs)

    def load(self, path) -> int:
        """Restore a state written by `save` into the instances' tensors (in
        place, so a captured graph stays valid) and return the index of the
        next step.  The file must come from a batch of the same grids (by
        content hash), mode, AL penalty and shifts."""
        import gridgen
        with np.load(path, allow_pickle=False) as z:
            if str(z["mode"]) != self.mode or int(z["n"]) != len(self.inst):
                raise ValueError("saved state is for another mode or number of instances")
            fp = [gridgen.fingerprint(it.grid) for it in self.items]
            if [str(v) for v in z["fingerprint"]] != fp:
                raise ValueError("saved state is for other grids")
            for k, i in enumerate(self.inst):
                rho, delta = (float(v) for v in z[f"param{k}"])
                if rho != i.rho or delta != i.delta:
                    raise ValueError(f"instance {k}: saved with another penalty or shift")
                for name, dst in (("u", i.u), ("x", i.x), ("y", i.y), ("status", i.status), ("s", i.s)):
                    if dst is None:
                        continue
                    src = z[f"{name}{k}"]
                    if src.shape != tuple(dst.shape):
                        raise ValueError(f"instance {k}: {name} has shape {src.shape}, expected {tuple(dst.shape)}")
                    dst.copy_(torch.from_numpy(src).to(dst.device))
            return int(z["t"])

    def load_state(self, st):
        for i, (u, x, y, stt, sv) in zip(self.inst, st):
            i.u.copy_(u)
            i.x.copy_(x)
            i.y.copy_(y)
            i.status.copy_(stt)
            if sv is not None:
                i.s.copy_(sv)
