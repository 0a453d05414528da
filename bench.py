"""Benchmark of the reduced-space hot path on one MI355X.

One step = one pass of the whole path on the 9241-bus synthetic grid (the
PEGASE9241 shape: n_x = 17036, n_u = 2889, m = 41340) for one set of
perturbed loads: warm-started Newton power flow, AL value, reduced gradient
(adjoint), the full reduced Hessian by n_u batched Hessian-vector products
(adjoint-adjoint), and the Cholesky step of the shifted reduced Hessian.

value = reduced-Hessian HVPs per second of the whole path
      = n_u * steps / (timed seconds); ms_per_step is the full reduced-
Hessian time including the Cholesky step.  Inputs are resident on the GPU
before the timed region.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="syn9241")
    ap.add_argument("--batch", type=int, default=0, help="HVP batch width, 0 = tuned")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-cols", type=int, default=512)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--quick", action="store_true", help="skip the comparison passes")
    ap.add_argument("--tracking", action="store_true",
                    help="batched real-time tracking: 64 grids, one tracking update per step")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--track-steps", type=int, default=50)
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is "
                                   "described in DESIGN.md and not implemented", "n_gpus": a.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import gridgen
    from paper_2110_02590_amd import Problem
    from paper_2110_02590_amd import tune

    if a.tracking:
        return tracking_bench(a)

    torch.cuda.set_device(0)
    g = gridgen.grid(a.workload)
    ep = gridgen.eval_point(g)
    B = a.batch if a.batch > 0 else tune.best_batch(g, ep)
    pr = Problem(g, max_batch=B)
    grid = pr.grid
    nu, nx = pr.nu, pr.nx
    s, y, rho, sigma = pr.point(ep)

    steps, warm = a.steps, a.warmup
    fac = gridgen.tracking_factors(gridgen.WORKLOADS[a.workload].seed if a.workload in gridgen.WORKLOADS
                                   else 0, steps + warm, pr.nb)
    PD = [pr.pd * torch.tensor(fac[k], device="cuda") for k in range(steps + warm)]
    QD = [pr.qd * torch.tensor(fac[k], device="cuda") for k in range(steps + warm)]
    x = pr.flat_x()
    st, _ = grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
    H = torch.empty((nu, nu), dtype=torch.float64, device="cuda")
    K = torch.empty_like(H)

    # shift for the Cholesky step: smallest ladder value that factorizes the
    # base point's reduced Hessian, times 10 (loads move between steps)
    grad, lam = grid.reduced_gradient(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma)
    grid.reduced_hessian(batch=B, H=H)
    base = 1e-8 * max(1.0, float(torch.diagonal(H).abs().max()))
    delta = 0.0
    for _ in range(25):
        K.copy_(H)
        _, info = grid.factor_solve(K, grad, delta=delta)
        if int(info) == 0:
            break
        delta = base if delta == 0.0 else 10.0 * delta
    delta = max(10.0 * delta, base)

    infos = []

    def step(k, xw):
        grid.pf_solve(pr.u0, PD[k], QD[k], xw)
        phi, c = grid.al_objective(xw, pr.u0, PD[k], QD[k], s, y, rho, sigma)
        gr, _ = grid.reduced_gradient(xw, pr.u0, PD[k], QD[k], s, y, rho, sigma, grad=grad, lam=lam)
        grid.reduced_hessian(batch=B, H=H)
        K.copy_(H)
        stp, info = grid.factor_solve(K, gr, delta=delta)
        infos.append(info)
        return stp

    for k in range(warm):
        step(k, x)
    torch.cuda.synchronize()
    grid.profile(True)
    grid.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warm, warm + steps):
        step(k, x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = grid.profile_read(reset=True)
    grid.profile(False)
    ok = all(int(i) == 0 for i in infos)
    ms_step = (t1 - t0) * 1e3 / steps
    value = nu * steps / (t1 - t0)

    # dominant kernel: batched level-scheduled triangular solves
    S = grid.structure()
    nnz_strict = (S["nnz_lu"] - nx) // 2
    bytes_per_launch = 12 * nnz_strict + 6 * nx + 8 * (nx + 1) + 16 * nx * B
    ms_trsv, n_trsv = prof["trsv_batch"]
    avg_us = ms_trsv * 1e3 / max(n_trsv, 1)
    achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9
    # launches of one reduced Hessian: 4 per batch
    cols_per_launch = [min(B, nu - j0) for j0 in range(0, nu, B)]
    alg_bytes = sum(12 * nnz_strict + 6 * nx + 8 * (nx + 1) + 16 * nx * c for c in cols_per_launch) * 4
    achieved_avg = alg_bytes / (ms_trsv * 1e-3 / steps) / 1e9

    out = {
        "metric": "reduced-Hessian HVPs/sec and full reduced-Hessian time, 9241-bus grid, FP64",
        "value": round(value, 1),
        "unit": "HVPs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {pr.nb} buses, {g['nl']} branches, n_x={nx}, n_u={nu}, "
                               f"m={pr.m}; step = warm power flow at perturbed loads + AL value + "
                               f"reduced gradient + {nu} HVPs + Cholesky step",
                   "hvp_batch": B, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved_avg, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved_avg / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_trsv_batch (level-scheduled triangular solves, all 4 per batch)",
                     "avg_launch_us": round(avg_us, 2),
                     "bytes_per_launch_full_batch": int(bytes_per_launch)},
        "breakdown_ms_per_step": {k: round(v[0] / steps, 4) for k, v in prof.items()},
        "cholesky_ok": ok,
        "cholesky_shift": delta,
    }

    if not a.quick:
        # Hessian products alone (point prepared), batched
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            grid.reduced_hessian(batch=B, H=H)
        torch.cuda.synchronize()
        out["hvp_only_hvps_per_s"] = round(nu * reps / (time.perf_counter() - t0), 1)
        # plain one-direction-at-a-time path: B = 1, eager launches
        nd = 64
        E = torch.zeros((nu, 1), dtype=torch.float64, device="cuda")
        HV1 = torch.empty((nu, 1), dtype=torch.float64, device="cuda")
        grid.hessian_batch(E, HV1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(nd):
            E.zero_()
            E[j, 0] = 1.0
            grid.hessian_batch(E, HV1)
        torch.cuda.synchronize()
        out["b1_eager_hvps_per_s"] = round(nd / (time.perf_counter() - t0), 1)
        out["batched_over_b1"] = round(out["hvp_only_hvps_per_s"] / out["b1_eager_hvps_per_s"], 1)

    if a.copy_probe:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 8

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, ep, a.cpu_sample_cols)

    print(json.dumps(out), flush=True)


def tracking_bench(a):
    """64 synthetic grids (n_b ~ U[300, 2000], seeds 100..163), each tracking
    per-step load perturbations with one device-resident reduced-Hessian
    Newton AL update; eager per-instance launches vs. one HIP graph per step
    (instances forked over streams)."""
    import numpy as np
    import torch

    import gridgen
    from paper_2110_02590_amd.tracking import TrackingBatch, TrackingItem

    torch.cuda.set_device(0)
    steps = a.track_steps
    items = []
    for sd in gridgen.TRACKING_SEEDS[:a.instances]:
        g = gridgen.make_grid(gridgen.tracking_workload(sd))
        ep = gridgen.eval_point(g, seed=sd + 1000)
        lo, hi = gridgen.constraint_bounds(g)
        items.append(TrackingItem(g, ep, lo, hi, gridgen.tracking_factors(sd, steps, g["nb"])))
    t0 = time.perf_counter()
    tb = TrackingBatch(items, max_batch=256, nstreams=8)
    setup_s = time.perf_counter() - t0
    n = len(items)

    def run(fn):
        lat = []
        torch.cuda.synchronize()
        T0 = time.perf_counter()
        for t in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn(t)
            e1.record()
            e1.synchronize()
            lat.append(e0.elapsed_time(e1))
        torch.cuda.synchronize()
        return time.perf_counter() - T0, np.array(lat)

    s0 = tb.state()
    tb.step_eager(0)                      # warm-up
    torch.cuda.synchronize()
    tb.load_state(s0)
    te, le = run(tb.step_eager)
    st_e = [i.status.cpu().numpy().copy() for i in tb.inst]
    tb.load_state(s0)
    tb.capture()
    tb.load_state(s0)
    tg, lg = run(tb.step_graph)
    st_g = [i.status.cpu().numpy().copy() for i in tb.inst]
    acc = np.array([s[1] for s in st_g])
    out = {
        "metric": "batched real-time tracking: instances/s and step latency (64 grids, FP64)",
        "value": round(n * steps / tg, 1), "unit": "instances/s", "n_gpus": 1, "steps": steps,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{n} grids, n_b in [{min(int(i.grid['nb']) for i in items)}, "
                               f"{max(int(i.grid['nb']) for i in items)}], one tracking update per grid "
                               f"and step (power flow, gradient, full reduced Hessian, Cholesky step, "
                               f"halving on power-flow failure, multiplier update)",
                   "streams": tb.nstreams},
        "graph": {"instances_per_s": round(n * steps / tg, 1), "p50_ms": round(float(np.percentile(lg, 50)), 3),
                  "p99_ms": round(float(np.percentile(lg, 99)), 3)},
        "eager_per_instance": {"instances_per_s": round(n * steps / te, 1),
                               "p50_ms": round(float(np.percentile(le, 50)), 3),
                               "p99_ms": round(float(np.percentile(le, 99)), 3)},
        "graph_over_eager": round(te / tg, 2),
        "last_step_accepted_full_step": int((acc == 0).sum()), "last_step_no_step": int((acc < 0).sum()),
        "setup_s": round(setup_s, 1),
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(g, ep, ncols):
    """The oracle on the host: power flow, reduced gradient and `ncols`
    reduced-Hessian columns by its adjoint-adjoint products."""
    import numpy as np
    import threadpoolctl

    import oracle
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    P = oracle.Point.from_dict(ep)
    threads = threadpoolctl.threadpool_info()
    nthr = max([t.get("num_threads", 1) for t in threads] or [1])
    t0 = time.perf_counter()
    pf = oracle.solve_pf(M, u, g["pd"], g["qd"])
    _, lam = oracle.reduced_gradient(M, pf.x, u, g["pd"], g["qd"], P)
    t1 = time.perf_counter()
    W = np.eye(M.nu)[:, :ncols]
    oracle.hvp_adjoint_adjoint(M, pf.x, u, g["pd"], g["qd"], P, lam, W)
    t2 = time.perf_counter()
    return {"value": round(ncols / (t2 - t1), 2), "unit": "HVPs/s", "cores": int(nthr), "kind": "oracle",
            "sample": f"{g['name']}: power flow + reduced gradient ({t1 - t0:.2f} s) then {ncols} of "
                      f"{M.nu} reduced-Hessian columns by adjoint-adjoint products with SciPy SuperLU "
                      f"({t2 - t1:.2f} s); value = columns / column time"}


if __name__ == "__main__":
    main()
