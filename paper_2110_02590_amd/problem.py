"""Device-side inputs for one grid: the control vector in the paper's order
u = (v_ref, v_pv, p_pv) built from generator setpoints, loads, and the AL
parameters (rho, y, s, sigma), as float64 tensors on the current device.
Marshalling only; all arithmetic of the method runs in the HIP library."""
from __future__ import annotations

import numpy as np

from .binding import Grid

PQ, PV, REF = 0, 1, 2


class Problem:
    def __init__(self, g: dict, max_batch: int = 256, pack_tile=None):
        """pack_tile: (columns, staged) of the batched pack solves' tiles --
        (16, False), (8, True) or (8, False), as `tune.best_config` picks
        them; None keeps the library's choice (the first that fits in LDS)."""
        import os

        import torch
        self.torch = torch
        self.g = g
        env = {}
        if pack_tile is not None:
            tw, sv = int(pack_tile[0]), bool(pack_tile[1])
            if (tw, sv) not in ((16, False), (8, True), (8, False)):
                raise ValueError("pack_tile must be (16, False), (8, True) or (8, False)")
            env = {"RPF_PACK_TW": str(tw), "RPF_PACK_SV": "1" if sv else "0"}
        old = {k: os.environ.get(k) for k in env}
        os.environ.update(env)
        try:
            # the handle reads the tile choice when it is created
            self.grid = Grid(g, max_batch=max_batch)
        finally:
            for k, v in old.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        bt = np.asarray(g["bus_type"])
        self.ref = int(np.flatnonzero(bt == REF)[0])
        self.pv = np.flatnonzero(bt == PV)
        self.pq = np.flatnonzero(bt == PQ)
        genat = np.full(g["nb"], -1)
        genat[np.asarray(g["gen_bus"])] = np.arange(g["ng"])
        self.gen_ref = int(genat[self.ref])
        self.gen_pv = genat[self.pv]
        self.nx, self.nu, self.m, self.nb = self.grid.nx, self.grid.nu, self.grid.m, self.grid.nb
        dev = "cuda"
        self.pd = torch.tensor(np.asarray(g["pd"], float), device=dev)
        self.qd = torch.tensor(np.asarray(g["qd"], float), device=dev)
        self.u0 = torch.tensor(self.u_from_setpoints(g["vg0"], g["pg0"]), device=dev)

    def u_from_setpoints(self, vg, pg) -> np.ndarray:
        vg = np.asarray(vg, float); pg = np.asarray(pg, float)
        return np.concatenate([[vg[self.gen_ref]], vg[self.gen_pv], pg[self.gen_pv]])

    def u_bounds(self):
        g = self.g
        lo = np.concatenate([[g["vmin"][self.ref]], g["vmin"][self.pv], g["pmin"][self.gen_pv]])
        hi = np.concatenate([[g["vmax"][self.ref]], g["vmax"][self.pv], g["pmax"][self.gen_pv]])
        return lo, hi

    def flat_x(self):
        t = self.torch
        npv, npq = self.pv.size, self.pq.size
        return t.cat([t.zeros(npv + npq, dtype=t.float64, device="cuda"),
                      t.ones(npq, dtype=t.float64, device="cuda")])

    def point(self, ep: dict):
        """(s, y, rho, sigma) device tensors from an evaluation-point dict."""
        t = self.torch
        s = t.tensor(np.asarray(ep["s"], float), device="cuda")
        y = t.tensor(np.asarray(ep["y"], float), device="cuda")
        sigma = t.tensor(np.concatenate([[ep["sigma_f"]], np.asarray(ep["sigma_c"], float)]), device="cuda")
        return s, y, float(ep["rho"]), sigma
