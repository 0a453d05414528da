"""Benchmark of the reduced-space hot path on one MI355X.

One step = one pass of the whole path on the 9241-bus synthetic grid (the
PEGASE9241 shape: n_x = 17036, n_u = 2889, m = 41340) for one set of
perturbed loads: warm-started Newton power flow, AL value, reduced gradient
(adjoint), the full reduced Hessian by n_u batched Hessian-vector products
(adjoint-adjoint), and the Cholesky step of the shifted reduced Hessian.

value = reduced-Hessian HVPs per second of the whole path
      = n_u * steps / (timed seconds); ms_per_step is the full reduced-
Hessian time including the Cholesky step.  The timed steps are one HIP
graph per step (captured once, replayed with each step's loads; --no-graph:
eager launches); an eager pass over the same steps with the library's
per-kernel event timing gives the roofline and breakdown figures.  Inputs
are resident on the GPU before the timed region.

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
PF_ITERS = 6
FP64_PEAK_TFLOPS = 78.6

# HBM traffic per launch from two rocprofv3 --pmc passes over this bench at
# batch 1024 (FETCH_SIZE scaled by 2.0 and WRITE_SIZE by 1.0: what the two
# counters read for a 1 GiB streaming kernel; KiB per dispatch averaged over
# the four forward/backward x J_x/J_x^T variants).  Valid only for the kernel
# source it was measured on (sha1 of the kernel's text and of the device
# functions it calls, in kernels.hpp) and for the batch width it was
# measured at; reported as null otherwise.
# Figures and commands: profiles/pack_solve_t_syn9241_traffic.txt.
TRAFFIC = {
    "pack_solve": {"kernel": "k_pack_solve_t", "helpers": ["tail_apply", "tail_apply_mfma", "tail_apply_any",
                                                           "stage_1d", "sum_xor16", "sum_xor32", "lds_barrier"],
                   "batch": 2889, "bytes_per_launch": 729805842,
                   "source_sha1": "eaf8998a300b58a3b1574444071592faf783b206"},
}


def _func_text(src, name):
    """Text of a function definition in the kernel header: from its
    __global__ / __device__ line (with a template line before it) to the
    closing brace at column 0."""
    import re
    m = re.search(r"\n((?:template <[^\n]*>\n)?__(?:global|device)__[^\n]*[ *&]" + re.escape(name) + r"\()", src)
    if m is None:
        raise KeyError(name)
    j = src.index("\n}\n", m.start(1)) + 3
    return src[m.start(1):j]


def _kernel_sha1(name, helpers=()):
    """sha1 of a kernel's text and of the listed device functions' texts in
    the library's kernel header."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2110_02590_amd", "csrc", "kernels.hpp")).read()
    h = hashlib.sha1(_func_text(src, name).encode())
    for f in helpers:
        h.update(_func_text(src, f).encode())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="syn9241")
    ap.add_argument("--batch", type=int, default=0, help="HVP batch width, 0 = tuned")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--quick", action="store_true", help="skip the comparison passes")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-captured leg")
    ap.add_argument("--tracking", action="store_true",
                    help="batched real-time tracking: 64 grids, one tracking update per step")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--track-steps", type=int, default=50)
    ap.add_argument("--tracking-mode", default="newton", choices=["newton", "qp"])
    ap.add_argument("--static-opf", action="store_true", help="static OPF on --workload only")
    ap.add_argument("--max-outer", type=int, default=40)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the exact-step, load-drop and 64-grid tracking legs of the default run")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "one GPU only: the column blocks of the reduced Hessian would shard "
                                   "over GPUs, but no multi-GPU path is implemented", "n_gpus": a.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import gridgen
    from paper_2110_02590_amd import Problem
    from paper_2110_02590_amd import tune

    if a.tracking:
        return tracking_bench(a)
    if a.static_opf:
        torch.cuda.set_device(0)
        print(json.dumps(static_opf_leg(a.workload, a.max_outer)), flush=True)
        return

    torch.cuda.set_device(0)
    g = gridgen.grid(a.workload)
    ep = gridgen.eval_point(g)
    if a.batch > 0:
        B, tile = a.batch, None
    else:
        cfg = tune.best_config(g, ep)
        B, tile = int(cfg["batch"]), (int(cfg["pack_tw"]), bool(cfg["pack_sv"]))
    pr = Problem(g, max_batch=B, pack_tile=tile)
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

    # the workload's grids are scaled so that Newton's method meets 1e-10
    # within PF_ITERS steps from a flat start; the device loop is predicated
    # on convergence, so steps past convergence launch but do no work
    pf_st = []

    def step(k, xw):
        pst, _ = grid.pf_solve(pr.u0, PD[k], QD[k], xw, max_iter=PF_ITERS)
        pf_st.append(pst)
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
    prof = grid.profile_read(reset=True, busy=True)
    grid.profile(False)
    ok = all(int(i) == 0 for i in infos)
    pf_ok = all(int(p[1]) == 1 for p in pf_st)
    ms_eager = (t1 - t0) * 1e3 / steps
    value_eager = nu * steps / (t1 - t0)

    # the headline: the same steps as one captured HIP graph, replayed (the
    # eager pass above, with the library's per-kernel event timing on, gives
    # the roofline figures: one stream, the same kernels)
    graph = None if a.no_graph else graph_leg(grid, pr, PD, QD, s, y, rho, sigma, B, delta, steps, warm)
    if graph is not None and graph["last_step_ok"]:
        value, ms_step, form = graph["hvps_per_s"], graph["ms_per_step"], "graph"
    else:
        value, ms_step, form = value_eager, ms_eager, "eager"

    rl, rl_all = roofline(g, pr, prof, B, steps)
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
                   "hvp_batch": B, "pack_tile": ("library default" if tile is None else
                                                   f"{tile[0]} columns{', values staged' if tile[1] else ''}"),
                   "parallelism": "single GPU",
                   "form": "one HIP graph per step, captured once and replayed" if form == "graph"
                   else "eager launches"},
        "eager": {"hvps_per_s": round(value_eager, 1), "ms_per_step": round(ms_eager, 3),
                  "note": "the same steps launched eagerly with per-kernel event timing on (the roofline "
                          "and breakdown figures come from this pass)"},
        "roofline": rl,
        "roofline_other_kernels": rl_all,
        "breakdown_ms_per_step": {k: round(v[0] / steps, 4) for k, v in prof.items()},
        "breakdown_busy_ms_per_step": {k: round(v[2] / steps, 4) for k, v in prof.items()},
        "cholesky_ok": ok,
        "power_flow_converged": pf_ok,
        "power_flow_max_iter": PF_ITERS,
        "cholesky_shift": delta,
    }

    if graph is not None:
        out["graph"] = graph

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

    if not a.no_extras:
        out["rt_qp"] = rt_qp_leg(g, ep, pr)
        out["load_drop_tracking"] = load_drop_leg()
        out["tracking_64"] = tracking_leg(a.instances, a.track_steps, 10)
        out["static_opf"] = static_opf_leg()

    if a.copy_probe:
        # a plain streaming kernel of known size for scaling the HBM byte
        # counters: 3 launches of dst = src + 0 over 1 GiB (1 GiB read and
        # 1 GiB written per launch)
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            torch.add(src, 0.0, out=dst)
        torch.cuda.synchronize()
        out["copy_probe_bytes_read_per_launch"] = src.numel() * 8
        out["copy_probe_bytes_written_per_launch"] = src.numel() * 8

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, ep)

    print(json.dumps(out), flush=True)


def graph_leg(grid, pr, PD, QD, s, y, rho, sigma, B, delta, steps, warm):
    """The same step captured once into a HIP graph and replayed: the loads
    of each step are copied into the captured input buffers before the
    replay (inside the timed region).  Under capture the library runs the
    Hessian batches on the caller's stream only."""
    import torch
    nu, nx = pr.nu, pr.nx
    f64 = dict(dtype=torch.float64, device="cuda")
    i32 = dict(dtype=torch.int32, device="cuda")
    pd = PD[0].clone()
    qd = QD[0].clone()
    x = pr.flat_x()
    grid.pf_solve(pr.u0, pd, qd, x)
    st = torch.empty(3, **i32)
    res = torch.empty(1, **f64)
    c = torch.empty(pr.m, **f64)
    gr = torch.empty(nu, **f64)
    lam = torch.empty(nx, **f64)
    ginfo = torch.empty(1, **i32)
    H = torch.empty((nu, nu), **f64)
    K = torch.empty((nu, nu), **f64)
    keep = {}

    def body():
        grid.pf_solve(pr.u0, pd, qd, x, max_iter=PF_ITERS, status=st, resid=res)
        keep["phi"], _ = grid.al_objective(x, pr.u0, pd, qd, s, y, rho, sigma, c=c)
        grid.reduced_gradient(x, pr.u0, pd, qd, s, y, rho, sigma, grad=gr, lam=lam, info=ginfo)
        grid.reduced_hessian(batch=B, H=H)
        K.copy_(H)
        keep["step"], keep["info"] = grid.factor_solve(K, gr, delta=delta)

    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        body()
    torch.cuda.synchronize()
    for k in range(warm):
        pd.copy_(PD[k])
        qd.copy_(QD[k])
        graph.replay()
    torch.cuda.synchronize()
    ok = True
    t0 = time.perf_counter()
    for k in range(warm, warm + steps):
        pd.copy_(PD[k])
        qd.copy_(QD[k])
        graph.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ok = int(st[1]) == 1 and int(ginfo) == 0 and int(keep["info"]) == 0
    return {"hvps_per_s": round(nu * steps / (t1 - t0), 1), "ms_per_step": round((t1 - t0) * 1e3 / steps, 3),
            "last_step_ok": ok,
            "note": "one HIP graph per step (captured once, replayed per step), loads copied into the "
                    "captured inputs before each replay (inside the timed region)"}


def _ju_row_counts(g, perm):
    """Entries of J_u in each row of the library's state order (perm maps a
    row to its index in x = (theta_pv, theta_pq, v_pq); a row is the P or Q
    balance of that bus).  The balance of bus i depends on the voltage
    magnitudes of the REF and PV buses among i and its neighbours, and the P
    balance of a PV bus on its own p_pv."""
    import numpy as np

    import gridgen
    bt, nb = g["bus_type"], g["nb"]
    pv = np.flatnonzero(bt == gridgen.PV)
    pq = np.flatnonzero(bt == gridgen.PQ)
    ctrl = bt != gridgen.PQ
    nbr = [{i} for i in range(nb)]
    for f, t in zip(g["br_from"], g["br_to"]):
        nbr[f].add(int(t))
        nbr[t].add(int(f))
    nv = np.array([sum(1 for j in nbr[i] if ctrl[j]) for i in range(nb)])
    npv, npq = pv.size, pq.size
    perm = np.asarray(perm)
    bus = np.where(perm < npv, pv[np.minimum(perm, npv - 1)],
                   pq[np.clip(np.where(perm < npv + npq, perm - npv, perm - npv - npq), 0, npq - 1)])
    return nv[bus] + (perm < npv)


def roofline(g, pr, prof, B, steps):
    """Roofline figures of the batched kernels from the library's HIP-event
    timings (events recorded on the launch stream around each launch).

    Algorithmic bytes (each factor entry read once as 8 B value + 4 B index,
    row pointers 4 B, reciprocal pivots 8 B, every right-hand-side element
    read and written once, 16 B), per launch with ncols columns:
      pack solve (k_pack_solve_t), pack rows [0, t0), pack-local entries:
        forward  12 nnz(L_pack) + 4 (t0 + 1) + 16 t0 ncols
        backward 12 nnz(U_pack, pack columns) + 4 (t0 + 1) + 8 t0 + 16 t0 ncols
        (nnz(U_pack, pack columns) = nnz(L_pack) by symmetry of the pattern;
        with J_x^T the unit and non-unit factors swap);
        the forward launch of J_x forms its right-hand side R = -J_u V
        itself: its R read is replaced by 12 nnz(J_u, pack rows) + 8 n_u
        ncols (V read once); every backward launch subtracts the pack rows'
        top-column products itself: + 12 nnz(U, pack rows, top columns)
        + 8 n_top ncols (the solved top part read once);
      top solve (k_top_rhs_w + k_top_inv_apply), one per solve pair (the
      dense top inverse read once):
        12 nnz(L, top rows, pack columns) + 8 ncols #(pack columns read)
        + 8 n_top^2 + 16 n_top ncols;
      refactorization (per call): LU values read and written (16 B each),
        update targets 4 B each, update pointers 8 B per entry.
    The dense Cholesky group is priced in FLOPs: n_u^3/3 + 2 n_u^2."""
    import numpy as np
    from paper_2110_02590_amd import binding
    info = binding.presolve_info(g)
    _, ptr, col = binding.presolve_pattern(g)
    nx, ntop = info["nx"], info["ntop"]
    t0 = nx - ntop
    rows = np.repeat(np.arange(nx), np.diff(ptr))
    pack = rows < t0
    nnz_lp = int(np.sum(pack & (col < rows)))
    topl = (rows >= t0) & (col < t0)
    nnz_tl = int(np.sum(topl))
    ncol_tl = int(np.unique(col[topl]).size)
    packtop = pack & (col >= t0)
    nnz_pt = int(np.sum(packtop))
    nrow_pt = int(np.unique(rows[packtop]).size)
    nu = pr.nu
    ju_rows = _ju_row_counts(g, binding.presolve_pattern(g)[0])
    nnz_ju_pack = int(ju_rows[:t0].sum())
    if int(ju_rows.sum()) != info["nnz_ju"]:
        raise RuntimeError("J_u pattern count disagrees with the library's")
    cols = [min(B, nu - j0) for j0 in range(0, nu, B)]   # one reduced Hessian
    # per batch: two solve pairs (J_x and J_x^T), each one forward and one
    # backward pack launch and one top solve
    pack_bytes = sum(2 * (12 * 2 * nnz_lp + 8 * (t0 + 1) + 8 * t0 + 32 * t0 * c)
                     - 8 * t0 * c + 12 * nnz_ju_pack + 8 * nu * c
                     + 2 * (12 * nnz_pt + 8 * ntop * c) for c in cols)
    top_bytes = sum(2 * (12 * nnz_tl + 8 * c * ncol_tl + 8 * ntop * ntop + 16 * ntop * c) for c in cols)
    pack_launches, top_launches = 4 * len(cols), 2 * len(cols)
    rf_bytes = 16 * info["nnz_lu"] + 4 * info["refactor_updates"] + 8 * info["nnz_lu"]
    chol_flops = nu ** 3 / 3.0 + 2.0 * nu * nu
    ent = {}

    def add(name, kernel, cls, alg_per_launch, bound, peak, unit, per_unit, launches_per_step=None):
        ms, n, busy = prof[cls]
        if n == 0:
            return
        scale = 1e9 if unit == "GB/s" else 1e12
        avg_us = ms * 1e3 / n
        achieved = alg_per_launch / (avg_us * 1e-6) / scale
        # launches of one class may overlap on the library's concurrent
        # streams; the busy figure counts overlapped time once
        ach_busy = alg_per_launch * n / (busy * 1e-3) / scale if busy > 0 else 0.0
        ent[name] = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
                     "frac": round(achieved / peak, 5), "traffic": None, "kernel": kernel,
                     "avg_launch_us": round(avg_us, 2), "launches_per_step": n // steps,
                     "ms_per_step": round(ms / steps, 3),
                     "busy_ms_per_step": round(busy / steps, 3),
                     "achieved_busy": round(ach_busy, 2), "frac_busy": round(ach_busy / peak, 5),
                     "algorithmic_per_launch": round(alg_per_launch, 1), "per_unit": per_unit}

    add("pack_solve", "k_pack_solve_t (batched triangular solves in the subtree packs)", "pack_batch",
        pack_bytes / pack_launches, "hbm", HBM_PEAK_GBS, "GB/s",
        f"bytes; nnz(L_pack)={nnz_lp}, t0={t0}, nnz(J_u,pack rows)={nnz_ju_pack}, "
        f"nnz(U_pack,top cols)={nnz_pt}, B={B}")
    add("top_solve", "k_top_rhs_w + k_top_inv_apply (top rows of the batched solves)",
        "top_batch",
        top_bytes / top_launches, "hbm", HBM_PEAK_GBS, "GB/s",
        f"bytes; nnz(L_top,pack cols)={nnz_tl}, n_top={ntop}, B={B}")
    add("refactor", "LU refactorization (k_rf_pack_lds, k_rf_top_ext, dense top LU)", "refactor",
        rf_bytes, "hbm", HBM_PEAK_GBS, "GB/s",
        f"bytes; nnz(L+U)={info['nnz_lu']}, updates={info['refactor_updates']}")
    # sparse products of a batch (4 launches): R = -J_u V (n_x rows), T = G D
    # (rank-one rows), Y = K D + G^T diag(kappa) T (all variables), HV = Y_u +
    # J_u^T Psi (n_u rows): each entry 12 B, each operand row read and each
    # result row written once (8 B per column)
    nvar, nr1 = nx + nu, 2 + (nu - 1) // 2     # rank-one rows: p_ref, q_ref, q at each PV bus
    # (R only on the top rows: the pack rows are formed in the pack solve)
    spmm_bytes = sum(12 * (2 * info["nnz_ju"] - nnz_ju_pack + 2 * info["nnz_g"] + info["nnz_k"])
                     + 8 * c * ((nu + ntop) + (nvar + nr1) + (2 * nvar + nr1) + (nx + 2 * nu)) for c in cols)
    add("spmm", "k_spmm (top rows of J_u V, G D, K D + G^T diag(kappa) T, J_u^T Psi)", "spmm",
        spmm_bytes / (4 * len(cols)),
        "hbm", HBM_PEAK_GBS, "GB/s",
        f"bytes; nnz(J_u)={info['nnz_ju']}, nnz(K)={info['nnz_k']}, nnz(G)={info['nnz_g']}, B={B}")
    add("cholesky", "dense Cholesky group (k_symmetrize, k_blk_*<true>, k_chol_fwd/bwd)", "dense",
        chol_flops, "mfma", FP64_PEAK_TFLOPS, "TFLOP/s", f"flops n_u^3/3 + 2 n_u^2, n_u={nu}")
    for name, tr in TRAFFIC.items():
        if name in ent and _kernel_sha1(tr["kernel"], tr["helpers"]) == tr["source_sha1"] and tr["batch"] == B:
            ent[name]["traffic"] = tr["bytes_per_launch"]
    if not ent:
        return None, {}
    dom = max(ent, key=lambda k: ent[k]["ms_per_step"])
    return ent[dom], {k: v for k, v in ent.items() if k != dom}


def tracking_leg(instances, steps, eager_steps, mode="newton", qp_iters=40):
    """64 synthetic grids (n_b ~ U[300, 2000], seeds 100..163), each tracking
    per-step load perturbations with one device-resident update per step
    (mode "newton": shifted Newton step; "qp": exact step by the bounded
    QP): one HIP graph per step (instances forked over 8 streams, captured
    once, replayed every step) timed over `steps` steps, and eager
    per-instance launches over `eager_steps` steps."""
    import numpy as np
    import torch

    import gridgen
    from paper_2110_02590_amd.tracking import TrackingBatch, TrackingItem

    items = []
    for sd in gridgen.TRACKING_SEEDS[:instances]:
        g = gridgen.make_grid(gridgen.tracking_workload(sd))
        ep = gridgen.eval_point(g, seed=sd + 1000)
        lo, hi = gridgen.constraint_bounds(g)
        items.append(TrackingItem(g, ep, lo, hi, gridgen.tracking_factors(sd, max(steps, eager_steps), g["nb"])))
    t0 = time.perf_counter()
    tb = TrackingBatch(items, max_batch=256, nstreams=8, mode=mode, qp_iters=qp_iters)
    setup_s = time.perf_counter() - t0
    n = len(items)

    def run(fn, nsteps):
        lat = []
        torch.cuda.synchronize()
        T0 = time.perf_counter()
        for t in range(nsteps):
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
    te, le = run(tb.step_eager, eager_steps)
    tb.load_state(s0)
    tb.capture()
    tb.load_state(s0)
    tg, lg = run(tb.step_graph, steps)
    st_g = np.array([i.status.cpu().numpy().copy() for i in tb.inst])
    out = {
        "workload": f"{n} grids, n_b in [{min(int(i.grid['nb']) for i in items)}, "
                    f"{max(int(i.grid['nb']) for i in items)}], one tracking update per grid and step "
                    + ("(power flow, gradient, full reduced Hessian, Cholesky step, halving on power-flow "
                       "failure, multiplier update)" if mode == "newton" else
                       "(power flow, reduced Hessian and Jacobian, bounded QP by the interior-point method, "
                       "halving on power-flow failure, multiplier update)"),
        "mode": mode, "steps": steps, "streams": tb.nstreams,
        "graph": {"instances_per_s": round(n * steps / tg, 1), "p50_ms": round(float(np.percentile(lg, 50)), 3),
                  "p99_ms": round(float(np.percentile(lg, 99)), 3)},
        "eager_per_instance": {"steps": eager_steps, "instances_per_s": round(n * eager_steps / te, 1),
                               "p50_ms": round(float(np.percentile(le, 50)), 3),
                               "p99_ms": round(float(np.percentile(le, 99)), 3)},
        "graph_over_eager": round((te / eager_steps) / (tg / steps), 2),
        "last_step_accepted_full_step": int((st_g[:, 1] == 0).sum()),
        "last_step_no_step": int((st_g[:, 1] < 0).sum()),
        "setup_s": round(setup_s, 1),
    }
    if mode == "qp":
        out["last_step_qp_converged"] = int(st_g[:, 3].sum())
    return out


def tracking_bench(a):
    import torch
    torch.cuda.set_device(0)
    r = tracking_leg(a.instances, a.track_steps, a.track_steps, mode=a.tracking_mode)
    out = {
        "metric": "batched real-time tracking: instances/s and step latency (64 grids, FP64)",
        "value": r["graph"]["instances_per_s"], "unit": "instances/s", "n_gpus": 1, "steps": a.track_steps,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": r.pop("workload"), "streams": r.pop("streams")},
    }
    out.update(r)
    print(json.dumps(out), flush=True)


def rt_qp_leg(g, ep, pr, reps=3, iters=60, tol=1e-10):
    """The exact real-time step (the bounded QP of eq. qp_rto) at the
    workload's evaluation point, timed like the paper's real-time table: the
    QP data alone (power flow state given; reduced gradient, Hessian and
    Jacobian from the identity batches) and the whole step with its
    interior-point iterations.  The shift is the one that makes the QP
    strictly convex at this point (1.5 |most negative eigenvalue of
    H - rho J^T D^2 J| + 1e-2)."""
    import numpy as np
    import torch

    import gridgen
    nu, m = pr.nu, pr.m
    s, y, rho, sigma = pr.point(ep)
    x = pr.flat_x()
    pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
    sz = torch.zeros(m, dtype=torch.float64, device="cuda")
    _, c = pr.grid.al_objective(x, pr.u0, pr.pd, pr.qd, sz, y, rho, sigma)
    lo, hi = gridgen.constraint_bounds(g)
    slo = torch.tensor(lo, device="cuda")
    shi = torch.tensor(hi, device="cuda")
    s = torch.minimum(torch.maximum(c, slo), shi).contiguous()
    ul, uh = pr.u_bounds()
    ulo = torch.tensor(ul, device="cuda")
    uhi = torch.tensor(uh, device="cuda")
    H = torch.empty((nu, nu), dtype=torch.float64, device="cuda")
    J = torch.empty((m, nu), dtype=torch.float64, device="cuda")
    q = pr.grid.qp_step(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma, 0.0, ulo, uhi, slo, shi, max_iter=0, H=H, J=J)
    Huu = H - rho * (J.T.contiguous() @ ((sigma[1:] ** 2)[:, None] * J))
    delta = 1.5 * max(0.0, -float(torch.linalg.eigvalsh(0.5 * (Huu + Huu.T)).min())) + 1e-2
    del Huu

    def timed(max_iter):
        ts = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = pr.grid.qp_step(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma, delta, ulo, uhi, slo, shi,
                                max_iter=max_iter, tol=tol, H=H, J=J)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts[1:])) * 1e3, r

    t_data, _ = timed(0)
    t_all, r = timed(iters)
    st = r["status"].cpu().numpy()
    return {"what": "exact real-time step at the evaluation point: QP data (reduced gradient, Hessian, "
                    "Jacobian) + bounded QP by the interior-point method with Schur-complement solves",
            "n": nu + m, "delta": delta, "iterations": int(st[0]), "factorizations": int(st[5]),
            "converged": bool(st[1]), "kkt": float(r["kkt"][0]),
            "qp_data_ms": round(t_data, 3), "qp_iterations_ms": round(t_all - t_data, 3),
            "total_ms": round(t_all, 3),
            "ms_per_iteration": round((t_all - t_data) / max(1, int(st[5])), 3)}


def load_drop_leg(name="syn2000", steps=60, t_drop=2, drop=0.2, qp_iters=60):
    """Tracking with the exact step through a sudden load drop (the paper's
    real-time experiment): all loads at their base values, then (1 - drop)
    times them from step t_drop on, the PV dispatch scaled with the total
    load at the drop; eager, one grid."""
    import numpy as np
    import torch

    import gridgen
    from paper_2110_02590_amd.tracking import TrackingBatch, TrackingItem

    g = gridgen.grid(name)
    ep = gridgen.eval_point(g)
    lo, hi = gridgen.constraint_bounds(g)
    it = TrackingItem(g, ep, lo, hi, gridgen.load_drop_factors(g["nb"], steps=steps, t_drop=t_drop, drop=drop))
    tb = TrackingBatch([it], max_batch=256, nstreams=1, mode="qp", qp_iters=qp_iters, redispatch=True)
    inst = tb.inst[0]
    lat, stat = [], []
    for t in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        tb.step_eager(t)
        e1.record()
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
        stat.append(inst.status.cpu().numpy().copy())
    stat = np.array(stat)
    # constraint violation at the final point (host check of the device state)
    pr = inst.pr
    fac = torch.tensor(it.factors[-1], device="cuda")
    _, c = pr.grid.al_objective(inst.x, inst.u, pr.pd * fac, pr.qd * fac, inst.s, inst.y, inst.rho, inst.sigma)
    c = c.cpu().numpy()
    viol = float(np.max(np.maximum(0.0, np.maximum(c - hi, lo - c))))
    lat = np.array(lat)
    return {"workload": f"{name}: {g['nb']} buses, {steps} steps, loads x{1 - drop:.2f} from step {t_drop}",
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "drop_step_ms": round(float(lat[t_drop]), 3),
            "steps_power_flow_converged": int(stat[:, 0].sum()),
            "steps_full_step_accepted": int((stat[:, 1] == 0).sum()),
            "steps_qp_converged": int(stat[:, 3].sum()),
            "qp_iterations_p50": float(np.percentile(stat[:, 2], 50)),
            "final_max_violation": viol}


def static_opf_leg(name="syn300", max_outer=40):
    """The static OPF by the augmented-Lagrangian method from the base
    dispatch (multipliers 0, penalty 10, unit constraint scaling): wall
    time, outer iterations, subproblem QPs, final infeasibility and cost."""
    import numpy as np
    import torch

    import gridgen
    from paper_2110_02590_amd import Problem
    g = gridgen.grid(name)
    ep = gridgen.eval_point(g, sigma="ones")
    pr = Problem(g, max_batch=256)
    s0, y0, rho, sigma = pr.point(ep)
    x = pr.flat_x()
    pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
    lo, hi = gridgen.constraint_bounds(g)
    slo = torch.tensor(lo, device="cuda")
    shi = torch.tensor(hi, device="cuda")
    _, c = pr.grid.al_objective(x, pr.u0, pr.pd, pr.qd, s0, y0, rho, sigma)
    s = torch.minimum(torch.maximum(c, slo), shi).contiguous()
    y = torch.zeros(pr.m, dtype=torch.float64, device="cuda")
    ul, uh = pr.u_bounds()
    u = pr.u0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, rho_f = pr.grid.static_opf(x, u, s, y, pr.pd, pr.qd, 10.0, sigma, torch.tensor(ul, device="cuda"),
                                     torch.tensor(uh, device="cuda"), slo, shi, max_outer=max_outer)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    last = hist[-1]
    return {"workload": f"{name}: {g['nb']} buses, static OPF from the base dispatch",
            "seconds": round(dt, 3), "outer_iterations": int(len(hist)), "qps": int(hist[:, 1].sum()),
            "converged": bool(last[6]), "final_infeasibility": float(last[2]),
            "final_projected_gradient": float(last[3]), "cost": float(last[4]), "final_rho": rho_f,
            "seconds_per_outer": round(dt / len(hist), 4)}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, ep):
    """The oracle on the host: power flow, reduced gradient and the full
    reduced Hessian in its dense Schur-complement form (SuperLU with n_u
    right-hand sides, the sparse Lagrangian Hessian times Z, one dense
    GEMM), timed with the BLAS pool at all usable cores and at one thread.
    value = n_u / reduced-Hessian time at all cores."""
    import numpy as np  # noqa: F401
    import threadpoolctl

    import oracle
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    P = oracle.Point.from_dict(ep)
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    runs = {}
    for label, lim in (("all", ncpu), ("one", 1)):
        with threadpoolctl.threadpool_limits(lim):
            nthr = max([t.get("num_threads", 1) for t in threadpoolctl.threadpool_info()] or [1])
            t0 = time.perf_counter()
            pf = oracle.solve_pf(M, u, g["pd"], g["qd"])
            _, lam = oracle.reduced_gradient(M, pf.x, u, g["pd"], g["qd"], P)
            t1 = time.perf_counter()
            oracle.reduced_hessian(M, pf.x, u, g["pd"], g["qd"], P, lam)
            t2 = time.perf_counter()
        runs[label] = dict(threads=int(nthr), pf_grad_s=round(t1 - t0, 3), hessian_s=round(t2 - t1, 3),
                           hvps_per_s=round(M.nu / (t2 - t1), 2))
    return {"value": runs["all"]["hvps_per_s"], "unit": "HVPs/s", "cores": runs["all"]["threads"],
            "kind": "oracle", "nproc": ncpu, "cpu_model": _cpu_model(),
            "one_thread": runs["one"],
            "sample": f"{g['name']}: the full {M.nu}-column reduced Hessian once per run (dense Schur "
                      f"form: SciPy SuperLU with {M.nu} right-hand sides, sparse Lagrangian Hessian "
                      f"product, dense GEMM), after power flow and reduced gradient "
                      f"({runs['all']['pf_grad_s']} s, not counted); all cores: "
                      f"{runs['all']['hessian_s']} s, one thread: {runs['one']['hessian_s']} s"}


if __name__ == "__main__":
    main()
