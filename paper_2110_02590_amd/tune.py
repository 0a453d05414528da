"""Tuner of the Hessian-vector products' launch shape: times the full
reduced Hessian on the device for each batch width and each tile variant of
the batched pack solves (16 columns; 8 columns with the factor values
staged in LDS; 8 columns without), and caches the fastest per (grid
fingerprint, device architecture) in a JSON file next to the package.  A
committed table of earlier tuning results (tune_table.json, same keys) is
consulted after the local cache and before any sweep."""
from __future__ import annotations

import json
import os
import time

_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")
CANDIDATES = (128, 256, 512, 1024, 2048, 4096)   # capped at n_u: one batch of every column
TILES = ((16, False), (8, True), (8, False))


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


def _entry_ok(e) -> bool:
    return isinstance(e, dict) and "batch" in e and "pack_tw" in e and "pack_sv" in e


def best_config(g, ep, candidates=CANDIDATES, tiles=TILES, reps=2, use_cache=True) -> dict:
    """{"batch": B, "pack_tw": columns, "pack_sv": staged} of the fastest full
    reduced Hessian, with the timings of every pair under "ms"."""
    import torch

    from .problem import Problem
    key = _key(g)
    cache = _load()
    if use_cache and _entry_ok(cache.get(key)):
        return cache[key]
    table = _load(_TABLE)
    if use_cache and _entry_ok(table.get(key)):
        return table[key]
    nu = 1 + 2 * int((g["bus_type"] == 1).sum())
    cands = sorted({min(c, nu) for c in candidates})
    times = {}
    for tile in tiles:
        for B in cands:
            # one handle per pair, created as a caller with this batch width
            # and tile creates it
            try:
                pr = Problem(g, max_batch=B, pack_tile=tile)
            except Exception:   # the tile does not fit this grid's packs
                continue
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
            times[(tile, B)] = (time.perf_counter() - t0) / reps
            pr.grid.close()
            del pr, H
    (tw, sv), best = min(times, key=times.get)
    entry = {"batch": best, "pack_tw": tw, "pack_sv": bool(sv),
             "ms": {f"{t[0]}{'s' if t[1] else ''}/{b}": round(v * 1e3, 3) for (t, b), v in times.items()}}
    cache[key] = entry
    try:
        with open(_CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    return entry


def best_batch(g, ep, candidates=CANDIDATES, reps=2, use_cache=True) -> int:
    """The batch width of `best_config`."""
    return int(best_config(g, ep, candidates=candidates, reps=reps, use_cache=use_cache)["batch"])


def main(argv=None):
    """python -m paper_2110_02590_amd.tune WORKLOAD ... [--out PATH]: sweep
    the named synthetic workloads on this device and write their entries
    into the committed table (tune_table.json) or PATH."""
    import argparse

    import gridgen
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+")
    ap.add_argument("--out", default=_TABLE, help="table to write (default: the committed table)")
    a = ap.parse_args(argv)
    table = _load(_TABLE)
    for name in a.workloads:
        g = gridgen.grid(name)
        e = best_config(g, gridgen.eval_point(g), use_cache=False)
        table[_key(g)] = e
        print(name, _key(g), {k: e[k] for k in ("batch", "pack_tw", "pack_sv")}, flush=True)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)


if __name__ == "__main__":
    main()
