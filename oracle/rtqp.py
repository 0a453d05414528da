"""Oracle, part 3: the exact real-time step (Section IV-C) -- the bounded QP
of eq. (qp_rto) in w = (u, s), solved by a primal-dual interior-point method
(Section IV-B.1/2, eq. ipm_subproblem, eq. ipm_firstorderconditions,
eq. ipm_kkt_reduced) -- and the tracking update built on it.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

The QP's data are the AL derivatives in w (eq. gradient_auglag,
eq. hessian_auglag, with the scalings of Section IV-A.2):
  g = (grad_u L, -D_c (y + rho D_c (c - s)))
  H = [[H_red + delta I, -rho J^T D_c^2], [-rho D_c^2 J, rho D_c^2]]
with H_red the reduced Hessian of the scaled AL in u at fixed s (it already
holds rho J^T D_c^2 J), J = grad_u c the reduced Jacobian and delta the
inertia-control shift of the u block.  The oracle solves every Newton system
(H + Sigma) dw = -grad psi of eq. (ipm_kkt_reduced) as one dense
(n_u + m) x (n_u + m) system; it does not use the Schur complement of
Proposition 3.  Small grids only.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .model import Model
from .reduced import Point, reduced_gradient, reduced_hessian, reduced_jacobian, solve_pf

#: interior-point parameters shared with the device implementation: the
#: starting point is pushed KAPPA of the way into the box, the duals start at
#: MU0 / slack, every step stops TAU of the way to the boundary
KAPPA = 1e-2
MU0 = 1.0
TAU = 0.995
#: inertia control (Section IV-B.2: the regularisation keeps the Newton
#: matrix positive definite): first regularisation REG_BASE * max(1, max
#: |diag H_uu block|), raised REG_UP times per failed factorisation; an
#: iteration starts from the last successful value / REG_DOWN (0 if it was
#: 0); beyond REG_MAX the method gives up
REG_BASE = 1e-4
REG_UP = 8.0
REG_DOWN = 4.0
REG_MAX = 1e30


def qp_data(H_red, J, grad_u, c, P: Point, delta):
    """Gradient and Hessian of the scaled AL in w = (u, s) at w_t
    (eq. gradient_auglag, eq. hessian_auglag)."""
    nu = H_red.shape[0]
    d2 = P.sigma_c ** 2
    g = np.concatenate([grad_u, -P.sigma_c * (P.y + P.rho * P.sigma_c * (c - P.s))])
    Hw = np.block([[H_red + delta * np.eye(nu), -P.rho * (J.T * d2)],
                   [-P.rho * (d2[:, None] * J), P.rho * np.diag(d2)]])
    return g, Hw


def box_qp_ipm(Hw, g, lo, hi, iters=50, tol=1e-10, nreg=None):
    """min g^T d + 1/2 d^T Hw d subject to lo <= d <= hi (lo < hi), by a
    primal-dual interior-point method with Mehrotra's predictor-corrector.

    Slacks t_l = d - lo, t_u = hi - d and duals z_l, z_u stay positive; with
    Sigma = z_l / t_l + z_u / t_u every iteration solves (eq. ipm_kkt_reduced)
      (Hw + Sigma + w P) dd = -(Hw d + g) + r_l / t_l - r_u / t_u
    twice with one factorization, where P is the identity on the first nreg
    variables (the controls) and zero elsewhere, and w the inertia-control
    regularisation: with nreg given, each iteration factorizes by Cholesky,
    first with w = 0 if the last successful w was 0, else max(w0, w_last /
    REG_DOWN), then w0, then REG_UP w after each failure (w0 = REG_BASE
    max(1, max |diag Hw[:nreg, :nreg]|)); every factorization attempt uses
    one of the `iters` slots.  Without nreg (the default) w = 0 and any
    nonsingular Hw + Sigma is solved by LU:
      predictor: r_l = r_u = 0, dz_l = -z_l - z_l/t_l dd, dz_u = -z_u + z_u/t_u dd;
        the largest steps to the boundary give the complementarity mu_a they
        would reach, and the centring target is mu = (mu_a / mu_c)^3 mu_c,
        mu_c = (t_l.z_l + t_u.z_u) / 2n;
      corrector: r_l = mu - dd_a dz_la, r_u = mu + dd_a dz_ua,
        dz_l = r_l / t_l - z_l - z_l/t_l dd, dz_u = r_u / t_u - z_u + z_u/t_u dd.
    Primal and dual steps stop TAU of the way to the boundary.  Stops when
    kkt_error < tol or after `iters` slots.  Returns (d, z_l, z_u,
    iterations) -- with nreg, (d, z_l, z_u, iterations, info) where info
    holds the last w, the factorization attempts and `failed` (the
    regularisation passed REG_MAX)."""
    Hw = np.asarray(Hw, float)
    g = np.asarray(g, float)
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    n = g.size
    kap = KAPPA * (hi - lo)
    d = np.clip(np.zeros(n), lo + kap, hi - kap)
    tl, tu = d - lo, hi - d
    zl, zu = MU0 / tl, MU0 / tu
    it = 0
    slots = 0
    w0 = REG_BASE * max(1.0, float(np.max(np.abs(np.diag(Hw)[:nreg])))) if nreg else 0.0
    wlast, w, failed = 0.0, None, False
    while slots < iters:
        if w is None:
            # a new iteration: convergence test, barrier terms, first w
            if _kkt(Hw, g, d, zl, zu, tl, tu) < tol:
                break
            Sig = zl / tl + zu / tu
            base = -(Hw @ d + g)
            w = 0.0 if wlast == 0.0 else max(w0, wlast / REG_DOWN)
        slots += 1
        A = Hw + np.diag(Sig)
        if nreg:
            A[:nreg, :nreg] += w * np.eye(nreg)
            try:
                np.linalg.cholesky(A)
            except np.linalg.LinAlgError:
                w = w0 if w == 0.0 else REG_UP * w
                if w > REG_MAX:
                    failed = True
                    break
                continue
            wlast, w = w, None
        else:
            w = None
        # predictor
        dda = np.linalg.solve(A, base)
        dzla = -zl - (zl / tl) * dda
        dzua = -zu + (zu / tu) * dda
        ap = min(_step(tl, dda, 1.0), _step(tu, -dda, 1.0))
        ad = min(_step(zl, dzla, 1.0), _step(zu, dzua, 1.0))
        muc = (tl @ zl + tu @ zu) / (2 * n)
        mua = ((tl + ap * dda) @ (zl + ad * dzla) + (tu - ap * dda) @ (zu + ad * dzua)) / (2 * n)
        mu = (mua / muc) ** 3 * muc
        # corrector
        rl = mu - dda * dzla
        ru = mu + dda * dzua
        dd = np.linalg.solve(A, base + rl / tl - ru / tu)
        dzl = rl / tl - zl - (zl / tl) * dd
        dzu = ru / tu - zu + (zu / tu) * dd
        ap = min(_step(tl, dd, TAU), _step(tu, -dd, TAU))
        ad = min(_step(zl, dzl, TAU), _step(zu, dzu, TAU))
        d = d + ap * dd
        tl = tl + ap * dd
        tu = tu - ap * dd
        zl = zl + ad * dzl
        zu = zu + ad * dzu
        it += 1
    if nreg:
        return d, zl, zu, it, dict(w=wlast, slots=slots, failed=failed)
    return d, zl, zu, it


def _step(v, dv, tau):
    """Largest a <= 1 with v + a dv >= (1 - tau) v (v > 0)."""
    neg = dv < 0
    if not np.any(neg):
        return 1.0
    return min(1.0, float(np.min(-tau * v[neg] / dv[neg])))


def _kkt(Hw, g, d, zl, zu, tl, tu):
    r = Hw @ d + g - zl + zu
    comp = max(float(np.max(tl * zl)), float(np.max(tu * zu)))
    return max(float(np.max(np.abs(r))) / (1.0 + float(np.max(np.abs(g)))), comp)


def kkt_error(Hw, g, lo, hi, d, zl, zu):
    """Scaled KKT error of the box QP: dual residual relative to (1 + |g|),
    largest complementarity product of either bound."""
    return _kkt(Hw, g, d, zl, zu, d - lo, hi - d)


def rt_step_qp(M: Model, u, s, x, y, pd, qd, P: Point, u_lo, u_hi, s_lo, s_hi, delta, iters=50, tol=1e-10):
    """The QP of eq. (qp_rto) at w_t = (u, s) for loads (pd, qd) with the
    state x solving the power flow there, by box_qp_ipm with inertia control
    on the control block: returns (du, ds, info dict)."""
    Pt = dataclasses.replace(P, s=s, y=y)
    c = M.constraints(x, u, pd, qd)
    grad, lam = reduced_gradient(M, x, u, pd, qd, Pt)
    H = reduced_hessian(M, x, u, pd, qd, Pt, lam)
    J = reduced_jacobian(M, x, u)
    g, Hw = qp_data(0.5 * (H + H.T), J, grad, c, Pt, delta)
    lo = np.concatenate([u_lo - u, s_lo - s])
    hi = np.concatenate([u_hi - u, s_hi - s])
    d, zl, zu, it, reg = box_qp_ipm(Hw, g, lo, hi, iters=iters, tol=tol, nreg=M.nu)
    return d[:M.nu], d[M.nu:], dict(iters=it, kkt=kkt_error(Hw, g, lo, hi, d, zl, zu), grad=grad, H=H, J=J,
                                    g=g, Hw=Hw, lo=lo, hi=hi, zl=zl, zu=zu, reg=reg)


def tracking_step_qp(M: Model, u, s, x, y, pd0, qd0, factor, P: Point, s_lo, s_hi, delta, pf_iters=6,
                     max_halvings=4, tol=1e-10, qp_iters=50, qp_tol=1e-10):
    """One exact real-time update (Section IV-C, steps 1-3): loads
    (pd0, qd0) * factor; power flow at u from x; the QP of eq. (qp_rto) at
    (u, s, y); w <- w + dw / 2^k for the first k <= max_halvings whose power
    flow converges (w unchanged if none); y <- y + rho D_c (c(u) - s).
    Returns (u, s, x, y, info)."""
    pd = pd0 * factor
    qd = qd0 * factor
    pf = solve_pf(M, u, pd, qd, x0=x, tol=tol, max_iter=pf_iters, raise_on_fail=False)
    x = pf.x
    ulo, uhi = M.u_bounds()
    du, ds, qinfo = rt_step_qp(M, u, s, x, y, pd, qd, P, ulo, uhi, s_lo, s_hi, delta, iters=qp_iters,
                                tol=qp_tol)
    accepted = -1
    for k in range(max_halvings + 1):
        ut = u + du / 2.0 ** k
        pf2 = solve_pf(M, ut, pd, qd, x0=x, tol=tol, max_iter=pf_iters, raise_on_fail=False)
        if pf2.converged:
            u, s, x, accepted = ut, s + ds / 2.0 ** k, pf2.x, k
            break
    c = M.constraints(x, u, pd, qd)
    y = y + P.rho * P.sigma_c * (c - s)
    return u, s, x, y, dict(pf_converged=pf.converged, pf_iters=pf.iters, accepted=accepted, du=du, ds=ds,
                            qp=qinfo)
