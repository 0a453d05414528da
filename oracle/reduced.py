"""Oracle, part 2: the reduced-space quantities, computed by their plain
definitions with SciPy's SuperLU and dense linear algebra.  FP64.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

* Newton-Raphson power flow, stop on ||g||_2 < tol: Section III-A,
  eq. (projection:newtonraphson), stopping rule of Section V-A.1.
* AL value with scalings: Section IV-A.1 (L_rho) and IV-A.2 (sigma_f, D_c).
* Reduced gradient by the adjoint: Proposition 1, eq. (reduced_gradient).
* Reduced Jacobian of the constraints by the direct (forward) sensitivities:
  Section III-C.
* Reduced Hessian: the dense Schur-complement form Z^T (grad^2 l) Z with
  Z = [-J_x^{-1} J_u; I], which equals Proposition 2's adjoint-adjoint
  products column by column (eq. hessvecprod, eq. socadjoint).
* Dense step: Cholesky of the symmetrised, shifted Hessian, Section IV-B.2
  (inertia control makes the matrix positive definite).
* Tracking step: Section IV-C steps 1-3, with the bounded QP replaced by one
  regularised Newton step (the closed-form slack minimiser and the
  multiplier update are kept).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .model import Model, term_hessian


class PowerFlowError(RuntimeError):
    pass


@dataclasses.dataclass
class PFResult:
    x: np.ndarray
    iters: int
    resid: float
    converged: bool


def solve_pf(M: Model, u, pd, qd, x0=None, tol=1e-10, max_iter=20, raise_on_fail=True):
    """x_{k+1} = x_k - J_x^{-1} g_k until ||g||_2 < tol (eq. projection:newtonraphson)."""
    x = M.flat_x() if x0 is None else np.array(x0, dtype=float)
    it = 0
    while True:
        g = M.residual(x, u, pd, qd)
        r = float(np.linalg.norm(g))
        if not np.isfinite(r):
            break
        if r < tol:
            return PFResult(x, it, r, True)
        if it >= max_iter:
            break
        Jx, _ = M.jacobians(x, u)
        x = x - spla.spsolve(Jx.tocsc(), g)
        it += 1
    if raise_on_fail:
        raise PowerFlowError(f"power flow did not converge: ||g|| = {r:.3e} after {it} steps")
    return PFResult(x, it, r, False)


@dataclasses.dataclass
class Point:
    """AL parameters: penalty rho, multipliers y, slacks s, scalings."""
    rho: float
    y: np.ndarray
    s: np.ndarray
    sigma_f: float
    sigma_c: np.ndarray

    @classmethod
    def from_dict(cls, d):
        return cls(float(d["rho"]), np.asarray(d["y"], float), np.asarray(d["s"], float),
                   float(d["sigma_f"]), np.asarray(d["sigma_c"], float))


def al_objective(M: Model, x, u, pd, qd, P: Point):
    """phi = sigma_f f + y^T D_c (c - s) + rho/2 ||D_c (c - s)||^2 and c."""
    c = M.constraints(x, u, pd, qd)
    f = M.cost(M.gen_p(x, u, pd))
    r = P.sigma_c * (c - P.s)
    phi = P.sigma_f * f + float(P.y @ r) + 0.5 * P.rho * float(r @ r)
    return phi, c


def _al_weights(M, x, u, pd, qd, P):
    c = M.constraints(x, u, pd, qd)
    # d phi / d c_k
    w = P.sigma_c * P.y + P.rho * P.sigma_c ** 2 * (c - P.s)
    return c, w


def full_gradient(M: Model, x, u, pd, qd, P: Point):
    """Gradient of phi w.r.t. z = (theta, v, p_pv)."""
    c, w = _al_weights(M, x, u, pd, qd, P)
    Jc = M.constraint_jac_full(x, u)
    gz = Jc.T @ w
    pg = M.gen_p(x, u, pd)
    d1 = M.cost_d1(pg)
    # cost: PV generators directly on p_pv, slack through P_ref(theta, v)
    gz[2 * M.nb:] += P.sigma_f * d1[M.gen_pv]
    gz += P.sigma_f * d1[M.gen_ref] * _pref_grad(M, x, u)
    return gz


def _pref_grad(M, x, u):
    th, v, _ = M.full(x, u)
    dSa, dSv = M.dS_dV(M.Y, th, v)
    out = np.zeros(M.nz)
    out[:M.nb] = dSa.real[[M.ref]].toarray().ravel()
    out[M.nb:2 * M.nb] = dSv.real[[M.ref]].toarray().ravel()
    return out


def reduced_gradient(M: Model, x, u, pd, qd, P: Point):
    """Proposition 1: J_x^T lambda = -(d_x phi)^T, grad = d_u phi + lambda^T J_u."""
    gz = full_gradient(M, x, u, pd, qd, P)
    Jx, Ju = M.jacobians(x, u)
    lam = spla.spsolve(Jx.T.tocsc(), -gz[M.ix])
    grad = gz[M.iu] + Ju.T @ lam
    return grad, lam


def lagrangian_hessian_full(M: Model, x, u, pd, qd, P: Point, lam):
    """Hessian of l = phi + lambda^T g w.r.t. z = (theta, v, p_pv), sparse.

    phi's Hessian is sigma_f grad^2 f + sum_k w_k grad^2 c_k
    + rho Jc^T D_c^2 Jc, with w_k = d phi / d c_k.  Second derivatives of
    injections and branch flows come from ``term_hessian``."""
    nb, nl = M.nb, M.nl
    th, v, _ = M.full(x, u)
    c, w = _al_weights(M, x, u, pd, qd, P)
    pg = M.gen_p(x, u, pd)
    d1 = M.cost_d1(pg)
    d2 = M.cost_d2()

    # weights on P_i and Q_i of the bus injections
    a = np.zeros(nb)
    b = np.zeros(nb)
    a[M.pv] += lam[:M.npv]
    a[M.pq] += lam[M.npv:M.npv + M.npq]
    b[M.pq] += lam[M.npv + M.npq:]
    o = 2 * nl + M.npq
    a[M.ref] += P.sigma_f * d1[M.gen_ref] + w[o]
    b[M.ref] += w[o + 1]
    b[M.pv] += w[o + 2:]
    # S_i = sum_k v_i v_k conj(Y_ik) e^{j(th_i - th_k)}, weighted by (a - jb)
    Yc = M.Y.tocoo()
    mu = a - 1j * b
    Hs = term_hessian(nb, Yc.row, Yc.col, mu[Yc.row] * np.conj(Yc.data), th, v)

    # branch flows: h = P^2 + Q^2, grad^2 h = 2(dP dP^T + dQ dQ^T) + 2P grad^2 P + 2Q grad^2 Q
    Sf, St = M.branch_flows(th, v)
    wf, wt = w[:nl], w[nl:2 * nl]
    f, t = M.f, M.t
    ia = np.concatenate([f, f, t, t])
    ib = np.concatenate([f, t, t, f])
    # S_f = v_f^2 conj(Yff) + v_f v_t conj(Yft) e^{j(th_f-th_t)}, likewise S_t
    kf = wf * 2.0 * (Sf.real - 1j * Sf.imag)
    kt = wt * 2.0 * (St.real - 1j * St.imag)
    coef = np.concatenate([kf * np.conj(M.Yff), kf * np.conj(M.Yft),
                           kt * np.conj(M.Ytt), kt * np.conj(M.Ytf)])
    Hb = term_hessian(nb, ia, ib, coef, th, v)
    # the 2 w (dP dP^T + dQ dQ^T) part, from the branch-flow Jacobians
    Hg = sp.csr_matrix((2 * nb, 2 * nb))
    for Yb, C, wk in ((M.Yf, M.Cf, wf), (M.Yt, M.Ct, wt)):
        da, dv = M.dS_dV(Yb, th, v, C)
        dS = sp.hstack([da, dv]).tocsr()
        Wd = sp.diags(2.0 * wk)
        Hg = Hg + dS.real.T @ Wd @ dS.real + dS.imag.T @ Wd @ dS.imag

    n2 = 2 * nb
    Hz = sp.block_diag([Hs + Hb + Hg, sp.csr_matrix((M.npv, M.npv))]).tocsr()

    # rank terms rho Jc^T D_c^2 Jc
    Jc = M.constraint_jac_full(x, u)
    Hz = Hz + P.rho * (Jc.T @ sp.diags(P.sigma_c ** 2) @ Jc)
    # cost curvature: PV generators on p_pv, slack through P_ref
    gref = _pref_grad(M, x, u)
    Hz = Hz + sp.diags(np.concatenate([np.zeros(n2), P.sigma_f * d2[M.gen_pv]]))
    gr = sp.csr_matrix(gref)
    Hz = Hz + P.sigma_f * d2[M.gen_ref] * (gr.T @ gr)
    return sp.csr_matrix(Hz)


def reduced_hessian(M: Model, x, u, pd, qd, P: Point, lam=None, return_parts=False):
    """H = Z^T (grad^2 l) Z with Z = [-J_x^{-1} J_u; I] (dense, n_u x n_u)."""
    if lam is None:
        _, lam = reduced_gradient(M, x, u, pd, qd, P)
    Hz = lagrangian_hessian_full(M, x, u, pd, qd, P, lam).tocsc()
    Hxx = Hz[M.ix][:, M.ix]
    Hxu = Hz[M.ix][:, M.iu]
    Hux = Hz[M.iu][:, M.ix]
    Huu = Hz[M.iu][:, M.iu]
    Jx, Ju = M.jacobians(x, u)
    lu = spla.splu(Jx.tocsc())
    S = -lu.solve(Ju.toarray())                        # sensitivity dx/du, [nx, nu]
    H = S.T @ (Hxx @ S + Hxu.toarray()) + Hux @ S + Huu.toarray()
    if return_parts:
        return H, dict(S=S, Hxx=Hxx, Hxu=Hxu, Hux=Hux, Huu=Huu, Jx=Jx, Ju=Ju)
    return H


def reduced_jacobian(M: Model, x, u):
    """Reduced Jacobian of the constraints, grad_u c(x(u), u) = (d_x c) S +
    d_u c with the sensitivity S = dx/du = -J_x^{-1} J_u (Section III-C,
    reduced Jacobian), dense [m, n_u]."""
    Jc = M.constraint_jac_full(x, u).tocsc()
    Jx, Ju = M.jacobians(x, u)
    S = -spla.splu(Jx.tocsc()).solve(Ju.toarray())
    return Jc[:, M.ix] @ S + Jc[:, M.iu].toarray()


def hvp_adjoint_adjoint(M: Model, x, u, pd, qd, P: Point, lam, W):
    """Proposition 2 applied to the columns of W: two sparse solves each.
    Used to check the Schur form; same Hessian blocks."""
    Hz = lagrangian_hessian_full(M, x, u, pd, qd, P, lam).tocsc()
    Hxx = Hz[M.ix][:, M.ix]; Hxu = Hz[M.ix][:, M.iu]
    Hux = Hz[M.iu][:, M.ix]; Huu = Hz[M.iu][:, M.iu]
    Jx, Ju = M.jacobians(x, u)
    lu = spla.splu(Jx.tocsc())
    z = lu.solve(-(Ju @ W))
    psi = lu.solve(-(Hxu @ W) - Hxx @ z, trans="T")
    return Huu @ W + Hux @ z + Ju.T @ psi


def cholesky_lower(K):
    """Lower Cholesky factor; returns (L, info) with info = first failing
    column (1-based) or 0.  Plain right-looking column algorithm."""
    K = np.array(K, dtype=float)
    n = K.shape[0]
    L = np.zeros_like(K)
    A = np.tril(K).copy()
    for j in range(n):
        d = A[j, j] - L[j, :j] @ L[j, :j]
        if not d > 0.0:
            return L, j + 1
        L[j, j] = np.sqrt(d)
        if j + 1 < n:
            L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L, 0


def factor_solve(H, diag=None, delta=0.0, rhs=None):
    """K = (H + H^T)/2 + diag(Sigma) + delta I = L L^T, d = -K^{-1} rhs."""
    H = np.asarray(H, dtype=float)
    K = 0.5 * (H + H.T)
    if diag is not None:
        K = K + np.diag(diag)
    K = K + delta * np.eye(K.shape[0])
    L, info = cholesky_lower(K)
    d = None
    if rhs is not None and info == 0:
        yv = sla.solve_triangular(L, -np.asarray(rhs, float), lower=True)
        d = sla.solve_triangular(L.T, yv, lower=False)
    return L, info, d


def delta_ladder(H, max_tries=20):
    """Regularisation that makes (H + H^T)/2 + delta I positive definite:
    delta = 0, then 1e-8 max(1, max|diag H|), times 10 per failure."""
    H = np.asarray(H, float)
    K = 0.5 * (H + H.T)
    base = 1e-8 * max(1.0, float(np.max(np.abs(np.diag(K)))))
    delta = 0.0
    for _ in range(max_tries + 1):
        try:
            np.linalg.cholesky(K + delta * np.eye(K.shape[0]))
            return delta
        except np.linalg.LinAlgError:
            delta = base if delta == 0.0 else 10.0 * delta
    raise RuntimeError("no positive definite shift found")


def slack_minimiser(c, P: Point, lo, hi):
    """argmin_s of the scaled AL in s: s = clip(c + y / (rho sigma_c), lo, hi)."""
    return np.clip(c + P.y / (P.rho * P.sigma_c), lo, hi)


def tracking_step(M: Model, u, x, y, pd0, qd0, factor, P: Point, s_lo, s_hi, delta,
                  pf_iters=6, max_halvings=4, tol=1e-10):
    """One tracking update at new loads (Section IV-C, steps 1-3), with the
    bounded QP replaced by a shifted Newton step:
    loads pd0*factor, qd0*factor; power flow at u (at most pf_iters Newton
    steps from x); s = clip(c + y/(rho sigma), lo, hi); reduced gradient and
    Hessian at (u, s, y); d = -((H+H^T)/2 + delta I)^{-1} grad (0 when the
    Cholesky fails); u <- clip(u + d/2^k) for the first k <= max_halvings whose
    power flow converges; s = clip(c(u) + y/(rho sigma)); y <- y + rho D_c(c - s).
    Returns (u, x, y, info dict)."""
    pd = pd0 * factor
    qd = qd0 * factor
    pf = solve_pf(M, u, pd, qd, x0=x, tol=tol, max_iter=pf_iters, raise_on_fail=False)
    x = pf.x
    c = M.constraints(x, u, pd, qd)
    s = slack_minimiser(c, dataclasses.replace(P, y=y), s_lo, s_hi)
    Pt = dataclasses.replace(P, s=s, y=y)
    grad, lam = reduced_gradient(M, x, u, pd, qd, Pt)
    H = reduced_hessian(M, x, u, pd, qd, Pt, lam)
    _, info, d = factor_solve(H, None, delta, grad)
    if info != 0:
        d = np.zeros(M.nu)
    ulo, uhi = M.u_bounds()
    accepted = -1
    for k in range(max_halvings + 1):
        ut = np.clip(u + d / 2.0 ** k, ulo, uhi)
        pf2 = solve_pf(M, ut, pd, qd, x0=x, tol=tol, max_iter=pf_iters, raise_on_fail=False)
        if pf2.converged:
            u, x, accepted = ut, pf2.x, k
            break
    c = M.constraints(x, u, pd, qd)
    s = slack_minimiser(c, dataclasses.replace(P, y=y), s_lo, s_hi)
    y = y + P.rho * P.sigma_c * (c - s)
    return u, x, y, dict(pf_converged=pf.converged, pf_iters=pf.iters, accepted=accepted, info=info,
                         grad=grad, step=d, s=s)
