"""Static OPF on the GPU (rpf_static_opf: the augmented-Lagrangian method of
Section IV-B.3 with the tolerances of Section V-B; each subproblem by bounded
QPs through the device interior-point method and a line search on L_rho)
against the oracle's static OPF (oracle.static_opf): the same sequence of
decisions (penalty, subproblem QPs, multiplier updates) and the same final
point."""
import numpy as np
import pytest

import gridgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(name, max_outer):
    from paper_2110_02590_amd import Problem
    g = gridgen.grid(name)
    ep = gridgen.eval_point(g, sigma="ones")
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    x = oracle.solve_pf(M, u, g["pd"], g["qd"]).x
    P = oracle.Point.from_dict(ep)
    lo, hi = gridgen.constraint_bounds(g)
    s = np.clip(M.constraints(x, u, g["pd"], g["qd"]), lo, hi)
    y = np.zeros(M.m)
    uo, so, xo, yo, rho_o, hist_o = oracle.static_opf(M, u, s, y, g["pd"], g["qd"], P, lo, hi, rho=10.0,
                                                      max_outer=max_outer)
    pr = Problem(g, max_batch=256)
    t = lambda a: torch.tensor(np.asarray(a, float), device="cuda")
    xg, ug, sg, yg = t(x), t(u), t(s), t(y)
    ulo, uhi = pr.u_bounds()
    sig = t(np.concatenate([[P.sigma_f], P.sigma_c]))
    hist_g, rho_g = pr.grid.static_opf(xg, ug, sg, yg, pr.pd, pr.qd, 10.0, sig, t(ulo), t(uhi), t(lo), t(hi),
                                       max_outer=max_outer)
    torch.cuda.synchronize()
    return (uo, so, xo, yo, rho_o, hist_o), (ug.cpu().numpy(), sg.cpu().numpy(), xg.cpu().numpy(),
                                              yg.cpu().numpy(), rho_g, hist_g)


def _compare(o, gpu, tol_state):
    uo, so, xo, yo, rho_o, hist_o = o
    ug, sg, xg, yg, rho_g, hist_g = gpu
    assert len(hist_g) == len(hist_o)
    for k, (ho, hg) in enumerate(zip(hist_o, hist_g)):
        print(f"outer {k}: rho {hg[0]:g} QPs {int(hg[1])} theta {hg[2]:.3e} pg {hg[3]:.3e} f {hg[4]:.6f} "
              f"(oracle QPs {ho['inner']}, theta {ho['theta']:.3e})", flush=True)
        assert hg[0] == ho["rho"] and int(hg[1]) == ho["inner"], (k, hg, ho)
        assert bool(hg[5]) == ho["updated"] and bool(hg[6]) == ho["converged"], (k, hg, ho)
        assert abs(hg[4] - ho["f"]) <= 1e-9 * abs(ho["f"]), (k, hg[4], ho["f"])
        assert abs(hg[2] - ho["theta"]) <= 1e-6 * max(ho["theta"], 1e-6), (k, hg[2], ho["theta"])
    assert rho_g == rho_o
    for name, a, b in (("u", ug, uo), ("s", sg, so), ("x", xg, xo), ("y", yg, yo)):
        err = np.linalg.norm(a - b) / max(1.0, np.linalg.norm(b))
        assert err <= tol_state, (name, err)


def test_static_opf_tiny10_matches_oracle():
    """tiny10 to convergence (ten outer iterations, both updates of the
    method taken)."""
    print("[case] static OPF tiny10", flush=True)
    o, gpu = _run("tiny10", 30)
    assert o[5][-1]["converged"]
    _compare(o, gpu, 1e-8)


def test_static_opf_syn300_first_iterations_match_oracle():
    """syn300, the first two outer iterations (eleven subproblem QPs)."""
    print("[case] static OPF syn300, two outer iterations", flush=True)
    o, gpu = _run("syn300", 2)
    _compare(o, gpu, 1e-8)
