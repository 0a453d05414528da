"""Tracking steps on the GPU (device-resident, graph-capturable) against the
oracle's tracking update, and graph replay against eager launches."""
import dataclasses

import numpy as np
import pytest

import gridgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEEDS = [100, 101]
STEPS = 3


def _items(seeds, steps):
    from paper_2110_02590_amd.tracking import TrackingItem
    out = []
    for sd in seeds:
        w = gridgen.tracking_workload(sd)
        g = gridgen.make_grid(w)
        ep = gridgen.eval_point(g, seed=sd + 1000)
        lo, hi = gridgen.constraint_bounds(g)
        out.append(TrackingItem(g, ep, lo, hi, gridgen.tracking_factors(sd, steps, g["nb"])))
    return out


def test_tracking_matches_oracle():
    from paper_2110_02590_amd.tracking import TrackingBatch
    print("[case] tracking seeds", SEEDS, flush=True)
    items = _items(SEEDS, STEPS)
    tb = TrackingBatch(items, max_batch=256, nstreams=1)
    for k, (it, inst) in enumerate(zip(items, tb.inst)):
        g = it.grid
        M = oracle.Model(g)
        u = M.u_from_setpoints(g["vg0"], g["pg0"])
        x = oracle.solve_pf(M, u, g["pd"], g["qd"]).x
        y = np.asarray(it.point["y"], float)
        P = oracle.Point.from_dict(it.point)
        for t in range(STEPS):
            u, x, y, info = oracle.tracking_step(M, u, x, y, g["pd"], g["qd"], it.factors[t], P, it.s_lo,
                                                 it.s_hi, inst.delta, pf_iters=6, max_halvings=4)
            tb.set_step(t)
            tb._launch(k)
            torch.cuda.synchronize()
            st = inst.status.cpu().numpy()
            assert st[0] == int(info["pf_converged"]) and st[1] == info["accepted"] and st[2] == info["info"]
            ug, yg, xg = inst.u.cpu().numpy(), inst.y.cpu().numpy(), inst.x.cpu().numpy()
            assert np.linalg.norm(ug - u) <= 1e-9 * np.linalg.norm(u), (k, t)
            assert np.linalg.norm(xg - x) <= 1e-9 * np.linalg.norm(x), (k, t)
            assert np.linalg.norm(yg - y) <= 1e-8 * max(1.0, np.linalg.norm(y)), (k, t)


def test_graph_replay_equals_eager():
    from paper_2110_02590_amd.tracking import TrackingBatch
    items = _items(SEEDS, 2)
    tb = TrackingBatch(items, max_batch=256, nstreams=2)
    s0 = tb.state()
    tb.step_eager(0)
    tb.step_eager(1)
    torch.cuda.synchronize()
    eager = tb.state()
    tb.load_state(s0)
    tb.capture()
    tb.load_state(s0)
    torch.cuda.synchronize()
    for rep in range(2):
        tb.step_graph(rep)
        torch.cuda.synchronize()
    graph = tb.state()
    for a, b in zip(eager, graph):
        for va, vb in zip(a, b):
            assert torch.equal(va, vb)
