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
# eight grids of the 64-grid workload: the smallest (307 buses) and the
# largest (1982 buses) bus counts, and six in between
PARITY_SEEDS = [108, 161, 100, 101, 120, 136, 147, 155]


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


def _run_against_oracle(tb, items, steps, pf_iters=6, max_halvings=4):
    for k, (it, inst) in enumerate(zip(items, tb.inst)):
        g = it.grid
        M = oracle.Model(g)
        u = M.u_from_setpoints(g["vg0"], g["pg0"])
        x = oracle.solve_pf(M, u, g["pd"], g["qd"]).x
        y = np.asarray(it.point["y"], float)
        P = oracle.Point.from_dict(it.point)
        for t in range(steps):
            u, x, y, info = oracle.tracking_step(M, u, x, y, g["pd"], g["qd"], it.factors[t], P, it.s_lo,
                                                 it.s_hi, inst.delta, pf_iters=pf_iters,
                                                 max_halvings=max_halvings)
            tb.set_step(t)
            tb._launch(k)
            torch.cuda.synchronize()
            st = inst.status.cpu().numpy()
            assert st[0] == int(info["pf_converged"]) and st[1] == info["accepted"] and st[2] == info["info"], \
                (k, t, st, info["accepted"], info["info"])
            assert st[4] == 0
            ug, yg, xg = inst.u.cpu().numpy(), inst.y.cpu().numpy(), inst.x.cpu().numpy()
            assert np.linalg.norm(ug - u) <= 1e-9 * np.linalg.norm(u), (k, t)
            assert np.linalg.norm(xg - x) <= 1e-9 * np.linalg.norm(x), (k, t)
            assert np.linalg.norm(yg - y) <= 1e-8 * max(1.0, np.linalg.norm(y)), (k, t)
    return


def test_tracking_matches_oracle():
    from paper_2110_02590_amd.tracking import TrackingBatch
    print("[case] tracking seeds", SEEDS, flush=True)
    items = _items(SEEDS, STEPS)
    tb = TrackingBatch(items, max_batch=256, nstreams=1)
    _run_against_oracle(tb, items, STEPS)


@pytest.mark.parametrize("seed", PARITY_SEEDS)
def test_tracking_grid_matches_oracle(seed):
    """Two tracking updates of one grid of the 64-grid workload against the
    oracle's tracking step (Section IV-C, steps 1-3 with the shifted Newton
    step)."""
    from paper_2110_02590_amd.tracking import TrackingBatch
    print("[case] tracking seed", seed, flush=True)
    items = _items([seed], 2)
    tb = TrackingBatch(items, max_batch=256, nstreams=1)
    _run_against_oracle(tb, items, 2)


def _small_item():
    from paper_2110_02590_amd.tracking import TrackingItem
    w = gridgen.tracking_workload(100)
    g = gridgen.make_grid(dataclasses.replace(w, nb=300, nl=480, ng=81))
    ep = gridgen.eval_point(g, seed=1100)
    lo, hi = gridgen.constraint_bounds(g)
    return TrackingItem(g, ep, lo, hi, np.ones((2, g["nb"])))


@pytest.mark.parametrize("delta,pf_iters,accepted", [(40.0, 2, 3), (10.0, 1, -1), (1e-3, 6, 0)])
def test_tracking_branches_match_oracle(delta, pf_iters, accepted):
    """The step-halving branch (two Newton steps per power flow: the full
    step's power flow fails, the third halving converges), the no-trial
    branch (one Newton step: nothing converges, u and x stay) and the failed
    Cholesky (shift 1e-3 on an indefinite reduced Hessian: zero step), each
    against the oracle, whose branches the CPU tests pin."""
    from paper_2110_02590_amd.tracking import TrackingBatch
    print("[case] tracking branch", delta, pf_iters, flush=True)
    items = [_small_item()]
    tb = TrackingBatch(items, max_batch=256, nstreams=1, pf_iters=pf_iters)
    tb.inst[0].delta = delta
    it = items[0]
    g = it.grid
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    x = oracle.solve_pf(M, u, g["pd"], g["qd"]).x
    P = oracle.Point.from_dict(it.point)
    uo, xo, yo, info = oracle.tracking_step(M, u, x, P.y, g["pd"], g["qd"], it.factors[0], P, it.s_lo, it.s_hi,
                                            delta, pf_iters=pf_iters, max_halvings=4)
    assert info["accepted"] == accepted
    tb.set_step(0)
    tb._launch(0)
    torch.cuda.synchronize()
    inst = tb.inst[0]
    st = inst.status.cpu().numpy()
    assert st[1] == accepted and st[2] == info["info"] and (st[2] == 0) == (info["info"] == 0)
    assert np.linalg.norm(inst.u.cpu().numpy() - uo) <= 1e-9 * np.linalg.norm(uo)
    assert np.linalg.norm(inst.x.cpu().numpy() - xo) <= 1e-9 * np.linalg.norm(xo)
    assert np.linalg.norm(inst.y.cpu().numpy() - yo) <= 1e-8 * max(1.0, np.linalg.norm(yo))


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
            assert (va is None and vb is None) or torch.equal(va, vb)


def test_saved_state_resumes_bitwise(tmp_path):
    """A state saved between steps and loaded back resumes the same
    trajectory bit for bit; a file from other grids is refused."""
    from paper_2110_02590_amd.tracking import TrackingBatch
    print("[case] tracking save/load seeds 108 101", flush=True)
    items = _items([108, 101], 4)
    tb = TrackingBatch(items, max_batch=256, nstreams=2)
    for t in range(2):
        tb.step_eager(t)
    path = str(tmp_path / "track.npz")
    tb.save(path, 2)
    tb.step_eager(2)
    tb.step_eager(3)
    torch.cuda.synchronize()
    ref = [tuple(v.cpu().numpy() for v in st[:4]) for st in tb.state()]
    assert tb.load(path) == 2
    tb.step_eager(2)
    tb.step_eager(3)
    torch.cuda.synchronize()
    got = [tuple(v.cpu().numpy() for v in st[:4]) for st in tb.state()]
    for a, b in zip(ref, got):
        for va, vb in zip(a, b):
            assert np.array_equal(va, vb)
    other = TrackingBatch(_items([108, 100], 2), max_batch=256, nstreams=2)
    with pytest.raises(ValueError):
        other.load(path)
