"""Oracle, part 4: the static OPF by the augmented-Lagrangian method
(Section IV-B.3, the algorithm of the textbook it cites: bound-constrained
Lagrangian method), with the stopping tolerances of Section V-B.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.

The problem is eq. (problem_algo) in w = (u, s) with the scaled AL of
Section IV-A.2.  Outer iteration k, at multipliers y and penalty rho:
  1. solve the subproblem eq. (auglag_subproblem) -- min L_rho(w; y) over the
     box -- approximately, warm-started from the current w: repeated bounded
     QPs of eq. (qp_rto) at the current point (the second-order model of
     L_rho in w, solved by the interior-point method of rt_step_qp), each
     followed by a backtracking (Armijo) line search on L_rho whose trial
     points carry a power flow; stop once the projected-gradient measure
     ||w - clip(w - grad L_rho, w_lo, w_hi)||_inf is below omega_k;
  2. primal infeasibility theta = ||c(u) - s||_inf:
     theta <= eta_k: converged if theta <= ETA_PRIMAL and the subproblem's
     measure <= ETA_DUAL; else y <- y + rho D_c (c - s), eta_k <- eta_k /
     rho^0.9, omega_k <- omega_k / rho;
     theta > eta_k: rho <- RHO_UP rho, eta_k <- 1 / rho^0.1, omega_k <- 1 / rho.
The subproblem's QP uses no shift (delta = 0): the interior point's inertia
control keeps its Newton matrices positive definite.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .model import Model
from .reduced import Point, al_objective, solve_pf
from .rtqp import rt_step_qp

#: stopping tolerances of Section V-B
ETA_PRIMAL = 1e-5
ETA_DUAL = 1e-4
RHO_UP = 10.0
ARMIJO = 1e-4
MAX_HALVINGS = 10


def projected_gradient(w, g, lo, hi):
    """||w - clip(w - g, lo, hi)||_inf, zero exactly at a stationary point of
    the box-constrained problem."""
    return float(np.max(np.abs(w - np.clip(w - g, lo, hi))))


def static_opf(M: Model, u, s, y, pd, qd, P: Point, s_lo, s_hi, rho=10.0, max_outer=30, max_inner=20,
               qp_iters=60, qp_tol=1e-10, pf_iters=20, tol=1e-10):
    """Returns (u, s, x, y, rho, history) with one history dict per outer
    iteration: rho, inner iterations, theta, the subproblem's projected
    gradient, the objective f and whether the multipliers were updated."""
    u = np.asarray(u, float).copy()
    s = np.asarray(s, float).copy()
    y = np.asarray(y, float).copy()
    ulo, uhi = M.u_bounds()
    wlo = np.concatenate([ulo, s_lo])
    whi = np.concatenate([uhi, s_hi])
    x = solve_pf(M, u, pd, qd, tol=tol, max_iter=pf_iters).x
    omega, eta = 1.0 / rho, 1.0 / rho ** 0.1
    hist = []
    for _ in range(max_outer):
        Pk = dataclasses.replace(P, rho=rho)
        inner, pg = 0, np.inf
        for inner in range(max_inner + 1):
            du, ds, info = rt_step_qp(M, u, s, x, y, pd, qd, Pk, ulo, uhi, s_lo, s_hi, 0.0, iters=qp_iters,
                                      tol=qp_tol)
            w = np.concatenate([u, s])
            g = info["g"]
            pg = projected_gradient(w, g, wlo, whi)
            if pg <= omega or inner == max_inner:
                break
            d = np.concatenate([du, ds])
            slope = float(g @ d)
            if not slope < 0.0:
                break
            phi0, _ = al_objective(M, x, u, pd, qd, dataclasses.replace(Pk, y=y, s=s))
            step = None
            a = 1.0
            for _h in range(MAX_HALVINGS + 1):
                ut, st = u + a * du, s + a * ds
                pf = solve_pf(M, ut, pd, qd, x0=x, tol=tol, max_iter=pf_iters, raise_on_fail=False)
                if pf.converged:
                    phi, _ = al_objective(M, pf.x, ut, pd, qd, dataclasses.replace(Pk, y=y, s=st))
                    if phi <= phi0 + ARMIJO * a * slope:
                        step = (ut, st, pf.x)
                        break
                a *= 0.5
            if step is None:
                break
            u, s, x = step
        c = M.constraints(x, u, pd, qd)
        theta = float(np.max(np.abs(c - s)))
        f = M.cost(M.gen_p(x, u, pd))
        rec = dict(rho=rho, inner=inner, theta=theta, pg=pg, f=f, updated=False, converged=False)
        if theta <= eta:
            if theta <= ETA_PRIMAL and pg <= ETA_DUAL:
                rec["converged"] = True
                hist.append(rec)
                break
            y = y + rho * P.sigma_c * (c - s)
            eta, omega = eta / rho ** 0.9, omega / rho
            rec["updated"] = True
        else:
            rho = RHO_UP * rho
            eta, omega = 1.0 / rho ** 0.1, 1.0 / rho
        hist.append(rec)
    return u, s, x, y, rho, hist
