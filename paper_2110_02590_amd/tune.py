"""Batch-width tuner for the Hessian-vector products: times the full
reduced Hessian for candidate widths on the device and caches the best per
(grid fingerprint, device name) in a JSON file next to the package.  A
committed table of earlier tuning results (tune_table.json, same keys) is
consulted after the local cache and before any sweep."""
from __future__ import annotations

import json
import os
import time

_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")
CANDIDATES = (128, 256, 512, 1024)


def _key(g):
    """(grid fingerprint, GPU architecture) -- the architecture rather than
    the marketing name, which tools that wrap the runtime may report
    differently."""
    import gridgen
    import torch
    arch = str(getattr(torch.cuda.get_device_properties(0), "gcnArchName", "")).split(":")[0]
    return f"{gridgen.fingerprint(g)[:16]}|{arch or torch.cuda.get_device_name(0)}"


def _load(path=_CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def best_batch(g, ep, candidates=CANDIDATES, reps=2, use_cache=True) -> int:
    import torch

    from .problem import Problem
    key = _key(g)
    cache = _load()
    if use_cache and key in cache:
        return int(cache[key]["batch"])
    table = _load(_TABLE)
    if use_cache and key in table:
        return int(table[key]["batch"])
    nu = 1 + 2 * int((g["bus_type"] == 1).sum())
    cands = sorted({min(c, nu) for c in candidates})
    times = {}
    for B in cands:
        # one handle per candidate, created as a caller with this batch width
        # creates it (the handle's stream count depends on its max_batch)
        pr = Problem(g, max_batch=B)
        x = pr.flat_x()
        pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
        s, y, rho, sigma = pr.point(ep)
        pr.grid.reduced_gradient(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma)
        H = torch.empty((pr.nu, pr.nu), dtype=torch.float64, device="cuda")
        pr.grid.reduced_hessian(batch=B, H=H)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pr.grid.reduced_hessian(batch=B, H=H)
        torch.cuda.synchronize()
        times[B] = (time.perf_counter() - t0) / reps
        pr.grid.close()
        del pr, H
    best = min(times, key=times.get)
    cache[key] = {"batch": best, "ms": {str(k): round(v * 1e3, 3) for k, v in times.items()}}
    try:
        with open(_CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    return best
