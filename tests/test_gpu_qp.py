"""Exact real-time step on the GPU (rpf_qp_step): the bounded QP of eq.
(qp_rto) by the device interior-point method through the Schur complement of
Proposition 3, against the oracle's interior-point method on the full
(n_u + m) system (oracle.rt_step_qp).

Parity: the same algorithm run for a fixed number of iterations gives the
same iterate (tol = 0 on both sides); run to convergence both give the QP's
solution.  At the 9241-bus size, where the oracle's dense system does not
fit, the GPU's answer is checked through the KKT conditions of the QP built
from its own H and J (both checked against the oracle elsewhere)."""
import dataclasses

import numpy as np
import pytest

import gridgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(name, seed=7, max_batch=256):
    """Point, slack inside its box, and a shift delta that makes the QP
    strictly convex (as the oracle's own QP tests choose it)."""
    from paper_2110_02590_amd import Problem
    g = gridgen.grid(name)
    ep = gridgen.eval_point(g, seed=seed)
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    x = oracle.solve_pf(M, u, g["pd"], g["qd"], tol=1e-12).x
    P = oracle.Point.from_dict(ep)
    lo, hi = gridgen.constraint_bounds(g)
    s = np.clip(M.constraints(x, u, g["pd"], g["qd"]), lo, hi)
    pr = Problem(g, max_batch=max_batch)
    return g, ep, M, u, x, P, s, lo, hi, pr


def _delta(M, u, x, g, P, s):
    Pt = dataclasses.replace(P, s=s)
    H = oracle.reduced_hessian(M, x, u, g["pd"], g["qd"], Pt)
    J = oracle.reduced_jacobian(M, x, u)
    Huu = 0.5 * (H + H.T) - P.rho * (J.T * P.sigma_c ** 2) @ J
    return 1.5 * max(0.0, -float(np.linalg.eigvalsh(Huu).min())) + 1e-2


def _gpu(pr, x, u, s, P, lo, hi, delta, iters, tol, batch=0):
    t = lambda a: torch.tensor(np.asarray(a, float), device="cuda")
    ulo, uhi = pr.u_bounds()
    sig = np.concatenate([[P.sigma_f], P.sigma_c])
    out = pr.grid.qp_step(t(x), t(u), pr.pd, pr.qd, t(s), t(P.y), P.rho, t(sig), delta, t(ulo), t(uhi), t(lo),
                          t(hi), max_iter=iters, tol=tol, batch=batch)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("name,iters", [("tiny10", 1), ("tiny10", 4), ("syn300", 2), ("syn300", 6)])
def test_fixed_iterations_match_oracle(name, iters):
    """tol = 0: both sides take exactly `iters` predictor-corrector
    iterations from the same start; the iterates agree."""
    print(f"[case] qp fixed {name} iters={iters}", flush=True)
    g, ep, M, u, x, P, s, lo, hi, pr = _case(name)
    delta = _delta(M, u, x, g, P, s)
    ulo, uhi = M.u_bounds()
    du, ds, info = oracle.rt_step_qp(M, u, s, x, P.y, g["pd"], g["qd"], P, ulo, uhi, lo, hi, delta, iters=iters,
                                     tol=0.0)
    assert info["iters"] == iters
    r = _gpu(pr, x, u, s, P, lo, hi, delta, iters, 0.0, batch=64)
    st = r["status"]
    assert st[0] == iters and st[2] == 0 and st[3] == 0 and st[4] == 0 and st[5] == iters, st
    assert info["reg"]["slots"] == iters and info["reg"]["w"] == 0.0
    d = np.concatenate([du, ds])
    assert np.linalg.norm(r["dw"] - d) <= 1e-9 * np.linalg.norm(d), np.linalg.norm(r["dw"] - d) / np.linalg.norm(d)
    # the QP data the GPU built: reduced gradient and symmetrised H, J
    np.testing.assert_allclose(r["grad"], info["grad"], rtol=0, atol=1e-10 * np.abs(info["grad"]).max())
    Ho = 0.5 * (info["H"] + info["H"].T)
    assert np.linalg.norm(r["H"] - Ho) <= 1e-9 * np.linalg.norm(Ho)
    assert np.linalg.norm(r["J"] - info["J"]) <= 1e-9 * np.linalg.norm(info["J"])


@pytest.mark.parametrize("name", ["tiny10", "syn300"])
def test_converged_step_matches_oracle(name):
    """Both sides to convergence (KKT error < 1e-12): the same solution of
    the QP, within what the stopping test allows, in about as many
    iterations, with bounds that are active at the solution."""
    print(f"[case] qp converged {name}", flush=True)
    g, ep, M, u, x, P, s, lo, hi, pr = _case(name)
    delta = _delta(M, u, x, g, P, s)
    ulo, uhi = M.u_bounds()
    du, ds, info = oracle.rt_step_qp(M, u, s, x, P.y, g["pd"], g["qd"], P, ulo, uhi, lo, hi, delta, iters=80,
                                     tol=1e-12)
    r = _gpu(pr, x, u, s, P, lo, hi, delta, 80, 1e-12, batch=64)
    st = r["status"]
    assert st[1] == 1 and st[2] == 0, st
    assert abs(int(st[0]) - info["iters"]) <= 1, (st, info["iters"])
    assert r["kkt"][0] < 1e-12
    d = np.concatenate([du, ds])
    assert np.linalg.norm(r["dw"] - d) <= 1e-8 * np.linalg.norm(d)
    n = d.size
    wlo = np.concatenate([ulo - u, lo - s])
    whi = np.concatenate([uhi - u, hi - s])
    # inside the box up to the rounding of d = lo + t_l at an active bound
    eps = 1e-13 * np.maximum(1.0, np.abs(wlo) + np.abs(whi))
    assert np.all(r["dw"] >= wlo - eps) and np.all(r["dw"] <= whi + eps)
    assert np.all(r["zw"] > 0)
    active = np.sum((d <= wlo + 1e-8) | (d >= whi - 1e-8))
    assert active > 0


def _kkt_blocks(H, J, grad, P, c, s, delta, d, nu):
    """r = Hw d + g, with Hw and g in block form (no dense Hw)."""
    sc2 = P.sigma_c ** 2
    du, ds = d[:nu], d[nu:]
    gs = -P.sigma_c * (P.y + P.rho * P.sigma_c * (c - s))
    ru = H @ du + delta * du - P.rho * (J.T @ (sc2 * ds)) + grad
    rs = P.rho * sc2 * (ds - J @ du) + gs
    return np.concatenate([ru, rs]), np.concatenate([grad, gs])


def test_largest_workload_kkt_certificate():
    """9241 buses in the benchmark's launch configuration (one batch of all 2889 columns):
    the GPU step satisfies the QP's KKT conditions, built in NumPy from the
    GPU's own H and J, to the stopping tolerance; the multipliers are
    positive and the step lies inside its box."""
    print("[case] qp syn9241", flush=True)
    g, ep, M, u, x, P, s, lo, hi, pr = _case("syn9241", max_batch=2889)
    ulo, uhi = M.u_bounds()
    # the QP data alone (no iteration), then the shift that makes the QP
    # strictly convex: H_uu = H - rho J^T D^2 J + delta I positive definite
    r0 = _gpu(pr, x, u, s, P, lo, hi, 0.0, 0, 1e-10, batch=2889)
    Ht = torch.tensor(r0["H"], device="cuda")
    Jt = torch.tensor(r0["J"], device="cuda")
    sc2 = torch.tensor(P.sigma_c ** 2, device="cuda")
    Huu = (Ht - P.rho * (Jt.T.contiguous() @ (sc2[:, None] * Jt))).cpu().numpy()
    delta = 1.5 * max(0.0, -float(np.linalg.eigvalsh(0.5 * (Huu + Huu.T)).min())) + 1e-2
    del Ht, Jt
    r = _gpu(pr, x, u, s, P, lo, hi, delta, 60, 1e-10, batch=2889)
    st = r["status"]
    print("status", st.tolist(), "kkt", float(r["kkt"][0]), flush=True)
    assert st[1] == 1 and st[2] == 0 and st[4] == 0, st
    nu, m = M.nu, M.m
    d, zw = r["dw"], r["zw"]
    zl, zu = zw[:nu + m], zw[nu + m:]
    c = M.constraints(x, u, g["pd"], g["qd"])
    res, gw = _kkt_blocks(r["H"], r["J"], r["grad"], P, c, s, delta, d, nu)
    wlo = np.concatenate([ulo - u, lo - s])
    whi = np.concatenate([uhi - u, hi - s])
    stat = np.max(np.abs(res - zl + zu)) / (1.0 + np.max(np.abs(gw)))
    comp = max(np.max((d - wlo) * zl), np.max((whi - d) * zu))
    assert stat < 1e-9 and comp < 1e-9, (stat, comp)
    assert np.all(zl > 0) and np.all(zu > 0)
    eps = 1e-13 * np.maximum(1.0, np.abs(wlo) + np.abs(whi))
    assert np.all(d >= wlo - eps) and np.all(d <= whi + eps)
    # the reduced gradient the QP used is the oracle's
    Pt = dataclasses.replace(P, s=s)
    go, _ = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], Pt)
    assert np.linalg.norm(r["grad"] - go) <= 1e-10 * np.linalg.norm(go)


@pytest.mark.parametrize("slots", [3, 12])
def test_inertia_control_matches_oracle(slots):
    """delta = 0 leaves the QP indefinite (H_uu has negative eigenvalues at
    this point), so the first Cholesky of S fails and the regularisation
    w I engages (Section IV-B.2).  Both sides take the same decisions: the
    same iterations and factorization attempts in `slots` slots, and the
    same iterate."""
    print(f"[case] qp inertia control syn300 slots={slots}", flush=True)
    g, ep, M, u, x, P, s, lo, hi, pr = _case("syn300")
    assert _delta(M, u, x, g, P, s) > 1.0        # H_uu is indefinite here
    ulo, uhi = M.u_bounds()
    du, ds, info = oracle.rt_step_qp(M, u, s, x, P.y, g["pd"], g["qd"], P, ulo, uhi, lo, hi, 0.0, iters=slots,
                                     tol=0.0)
    r = _gpu(pr, x, u, s, P, lo, hi, 0.0, slots, 0.0, batch=64)
    st = r["status"]
    print("status", st.tolist(), "oracle", info["iters"], info["reg"], "gpu w", float(r["wreg"][0]), flush=True)
    assert st[5] == slots and st[0] == info["iters"] and st[0] < slots, (st, info["iters"])
    assert st[2] == 0 and st[3] == 0
    d = np.concatenate([du, ds])
    assert np.linalg.norm(r["dw"] - d) <= 1e-9 * np.linalg.norm(d)
    assert abs(float(r["wreg"][0]) - info["reg"]["w"]) <= 1e-12 * max(1.0, info["reg"]["w"])
