"""Pins of the CPU oracle against facts fixed outside it: Table I sizes, a
closed-form two-bus power flow, 50-digit reference derivatives, an autograd
Hessian, finite differences, Taylor remainders and physical invariants."""
import dataclasses
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import gridgen
import oracle
from tests import smallgrids
from tests.mpref import MPGrid


def _setup(g, seed=7, sigma="random", rho=10.0, tol=1e-12):
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    pf = oracle.solve_pf(M, u, g["pd"], g["qd"], tol=tol)
    P = oracle.Point.from_dict(smallgrids.point_for(g, seed=seed, rho=rho, sigma=sigma))
    return M, u, pf.x, P


# ---------------------------------------------------------------- Table I
def _table1():
    here = os.path.join(os.path.dirname(__file__), "golden", "table1_sizes.csv")
    rows = []
    for line in open(here):
        if line.strip() and not line.startswith("#"):
            name, *vals = line.strip().split(",")
            rows.append((name, *map(int, vals)))
    return rows


@pytest.mark.parametrize("row", _table1(), ids=lambda r: r[0])
def test_table1_dimensions(row):
    """Table I: (n_x, n_u, m) of the PEGASE cases follow from (n_b, n_l) and
    n_pv = (n_u - 1) / 2 through the state/control split and the count m."""
    name, nb, nl, nx, nu, m = row
    npv = (nu - 1) // 2
    w = gridgen.Workload("t", nb, nl, npv + 1, 5, "geometric")
    M = oracle.Model(gridgen.make_grid(w))
    assert (M.nx, M.nu, M.m) == (nx, nu, m)


def test_workload_dimensions():
    M = oracle.Model(gridgen.grid("tiny10"))
    assert (M.nx, M.nu, M.m) == (16, 5, 37)
    M = oracle.Model(gridgen.grid("syn300"))
    assert (M.nx, M.nu) == (530, 137)
    M = oracle.Model(gridgen.grid("syn2000"))
    assert (M.nu,) == (1079,)


# ------------------------------------------------------ two-bus closed form
def test_two_bus_closed_form():
    """Slack V1 feeding P + jQ over r + jx: v2^4 + (2(rP + xQ) - v1^2) v2^2
    + (r^2 + x^2)(P^2 + Q^2) = 0 (larger root), theta2 = -atan2(xP - rQ,
    v2^2 + rP + xQ)."""
    r, x, P, Q, v1 = 0.03, 0.12, 1.1, 0.45, 1.03
    g = smallgrids.two_bus(r=r, x=x, P=P, Q=Q, v1=v1)
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    pf = oracle.solve_pf(M, u, g["pd"], g["qd"])
    bq = 2 * (r * P + x * Q) - v1 ** 2
    cq = (r * r + x * x) * (P * P + Q * Q)
    v2sq = (-bq + np.sqrt(bq * bq - 4 * cq)) / 2
    th2 = -np.arctan2(x * P - r * Q, v2sq + r * P + x * Q)
    assert pf.converged and pf.resid < 1e-10
    np.testing.assert_allclose(pf.x, [th2, np.sqrt(v2sq)], rtol=0, atol=1e-13)
    # slack generation = load + series loss r (P^2 + Q^2) / v2^2
    pg = M.gen_p(pf.x, u, g["pd"])
    np.testing.assert_allclose(pg[0], P + r * (P * P + Q * Q) / v2sq, rtol=1e-13)


# -------------------------------------------- 50-digit reduced derivatives
@pytest.mark.parametrize("which", ["two_bus", "two_bus_charging", "three_bus"])
def test_reduced_derivatives_vs_mpmath(which):
    """Prop. 1 gradient and the Schur-form Hessian against 50-digit
    numerical derivatives of the closed-loop phi(u)."""
    if which == "two_bus":
        g = smallgrids.two_bus()
    elif which == "two_bus_charging":
        g = smallgrids.two_bus(b=0.08)
    else:
        g = smallgrids.three_bus()
    M, u, x, P = _setup(g, seed=11, tol=1e-14)
    grad, lam = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], P)
    H = oracle.reduced_hessian(M, x, u, g["pd"], g["qd"], P, lam)
    pt = smallgrids.point_for(g, seed=11)
    ref = MPGrid(g, pt, dps=40)
    gm, Hm = ref.derivatives(list(u))
    gm = np.array([float(v) for v in gm])
    Hm = np.array([[float(v) for v in row] for row in Hm])
    np.testing.assert_allclose(grad, gm, rtol=1e-11, atol=1e-11 * np.abs(gm).max())
    np.testing.assert_allclose(H, Hm, rtol=1e-10, atol=1e-10 * np.abs(Hm).max())
    phi, _ = oracle.al_objective(M, x, u, g["pd"], g["qd"], P)
    assert abs(phi - float(ref.phi([mp.mpf(v) for v in u]))) <= 1e-12 * max(1.0, abs(phi))


def test_cost_only_special_case():
    """rho = 0, y = 0, sigma_f = 1: the reduced Hessian is that of the cost
    f(x(u), u) alone."""
    g = smallgrids.three_bus()
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    x = oracle.solve_pf(M, u, g["pd"], g["qd"], tol=1e-14).x
    pt = smallgrids.point_for(g)
    pt = dict(pt, rho=0.0, y=np.zeros_like(pt["y"]), sigma_f=1.0)
    P = oracle.Point.from_dict(pt)
    grad, lam = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], P)
    H = oracle.reduced_hessian(M, x, u, g["pd"], g["qd"], P, lam)
    ref = MPGrid(g, pt, dps=40)
    gm, Hm = ref.derivatives(list(u))
    np.testing.assert_allclose(grad, [float(v) for v in gm], rtol=1e-11)
    Hm = np.array([[float(v) for v in r] for r in Hm])
    np.testing.assert_allclose(H, Hm, rtol=1e-10, atol=1e-10 * np.abs(Hm).max())


# ------------------------------------------------- autograd Hessian of l
def _torch_lagrangian(M, g, pd, qd, P, lam):
    """l(z) = phi(z) + lambda^T g(z), z = (theta, v, p_pv), in plain torch."""
    nb = M.nb
    Y = torch.tensor(M.Y.toarray())
    Yf = torch.tensor(M.Yf.toarray())
    Yt = torch.tensor(M.Yt.toarray())
    f_idx = torch.tensor(M.f)
    t_idx = torch.tensor(M.t)
    pd_t = torch.tensor(pd)
    qd_t = torch.tensor(qd)
    lam_t = torch.tensor(lam)
    y = torch.tensor(P.y)
    s = torch.tensor(P.s)
    sc = torch.tensor(P.sigma_c)
    c2 = torch.tensor(g["c2"])
    c1 = torch.tensor(g["c1"])
    base = g["base_mva"]
    pv = torch.tensor(M.pv)
    pq = torch.tensor(M.pq)

    def ell(z):
        th, v, ppv = z[:nb], z[nb:2 * nb], z[2 * nb:]
        V = torch.polar(v, th)
        S = V * torch.conj(Y @ V)
        Sf = V[f_idx] * torch.conj(Yf @ V)
        St = V[t_idx] * torch.conj(Yt @ V)
        gvec = torch.cat([S.real[pv] - ppv + pd_t[pv], S.real[pq] + pd_t[pq], S.imag[pq] + qd_t[pq]])
        pref = S.real[M.ref] + pd_t[M.ref]
        qnet = S.imag + qd_t
        c = torch.cat([Sf.real ** 2 + Sf.imag ** 2, St.real ** 2 + St.imag ** 2, v[pq],
                       pref.reshape(1), qnet[M.ref].reshape(1), qnet[pv]])
        pg = torch.zeros(M.ng, dtype=torch.float64)
        pg = pg.index_put((torch.tensor(M.gen_pv),), ppv)
        pg = pg.index_put((torch.tensor([M.gen_ref]),), pref.reshape(1))
        f = torch.sum(c2 * (base * pg) ** 2 + c1 * base * pg)
        r = sc * (c - s)
        return P.sigma_f * f + y @ r + 0.5 * P.rho * r @ r + lam_t @ gvec

    return ell


@pytest.mark.parametrize("name", ["tiny10", "three_bus"])
def test_lagrangian_hessian_vs_autograd(name):
    g = gridgen.grid(name) if name != "three_bus" else smallgrids.three_bus()
    M, u, x, P = _setup(g)
    grad, lam = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], P)
    Hz = oracle.lagrangian_hessian_full(M, x, u, g["pd"], g["qd"], P, lam).toarray()
    th, v, ppv = M.full(x, u)
    z = torch.tensor(np.concatenate([th, v, ppv]))
    ell = _torch_lagrangian(M, g, g["pd"], g["qd"], P, lam)
    Ht = torch.autograd.functional.hessian(ell, z).numpy()
    np.testing.assert_allclose(Hz, Ht, rtol=0, atol=1e-12 * np.abs(Ht).max())
    # first derivatives: d phi/dz (without lambda^T g) against autograd
    ell0 = _torch_lagrangian(M, g, g["pd"], g["qd"], P, np.zeros_like(lam))
    gt = torch.autograd.functional.jacobian(ell0, z).numpy()
    gz = oracle.full_gradient(M, x, u, g["pd"], g["qd"], P)
    np.testing.assert_allclose(gz, gt, rtol=0, atol=1e-12 * np.abs(gt).max())


# ----------------------------------------- Schur form == adjoint-adjoint
@pytest.mark.parametrize("name", ["tiny10", "syn300"])
def test_schur_equals_adjoint_adjoint(name):
    """Proposition 2 applied to the identity equals Z^T (grad^2 l) Z."""
    g = gridgen.grid(name)
    M, u, x, P = _setup(g)
    grad, lam = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], P)
    H = oracle.reduced_hessian(M, x, u, g["pd"], g["qd"], P, lam)
    Ha = oracle.hvp_adjoint_adjoint(M, x, u, g["pd"], g["qd"], P, lam, np.eye(M.nu))
    assert np.linalg.norm(H - Ha) <= 1e-12 * np.linalg.norm(H)


# ------------------------------------------------ finite differences, Taylor
def _reduced_phi(M, u, g, P, x0):
    x = oracle.solve_pf(M, u, g["pd"], g["qd"], x0=x0, tol=1e-13).x
    return oracle.al_objective(M, x, u, g["pd"], g["qd"], P)[0], x


@pytest.mark.parametrize("name", ["tiny10", "syn300"])
def test_hessian_vs_fd_of_gradient(name):
    g = gridgen.grid(name)
    M, u, x, P = _setup(g)
    grad, lam = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], P)
    H = oracle.reduced_hessian(M, x, u, g["pd"], g["qd"], P, lam)
    rng = np.random.default_rng(3)
    cols = range(M.nu) if M.nu <= 8 else rng.choice(M.nu, 8, replace=False)
    for k in cols:
        h = 1e-6 * max(1.0, abs(u[k]))
        gs = []
        for sgn in (1, -1):
            up = u.copy(); up[k] += sgn * h
            xp = oracle.solve_pf(M, up, g["pd"], g["qd"], x0=x, tol=1e-13).x
            gs.append(oracle.reduced_gradient(M, xp, up, g["pd"], g["qd"], P)[0])
        fd = (gs[0] - gs[1]) / (2 * h)
        assert np.linalg.norm(fd - H[:, k]) <= 1e-6 * max(1.0, np.linalg.norm(H[:, k]))


def test_gradient_vs_fd_of_phi():
    g = gridgen.grid("tiny10")
    M, u, x, P = _setup(g)
    grad, _ = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], P)
    for k in range(M.nu):
        h = 1e-6
        up = u.copy(); up[k] += h
        um = u.copy(); um[k] -= h
        fd = (_reduced_phi(M, up, g, P, x)[0] - _reduced_phi(M, um, g, P, x)[0]) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-7 * max(1.0, abs(grad[k]))


def test_taylor_remainder_is_cubic():
    """|phi(u + t d) - phi - t g.d - t^2/2 d^T H d| = O(t^3): log-log slopes
    near 3 (a wrong Hessian gives 2), well above the rounding floor."""
    g = gridgen.grid("tiny10")
    M, u, x, P = _setup(g)
    phi0, _ = oracle.al_objective(M, x, u, g["pd"], g["qd"], P)
    grad, lam = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], P)
    H = oracle.reduced_hessian(M, x, u, g["pd"], g["qd"], P, lam)
    d = np.random.default_rng(5).standard_normal(M.nu)
    d /= np.linalg.norm(d)
    ts = np.array([4e-3, 2e-3, 1e-3, 5e-4])
    rem = []
    for t in ts:
        ph, _ = _reduced_phi(M, u + t * d, g, P, x)
        rem.append(abs(ph - phi0 - t * grad @ d - 0.5 * t * t * d @ H @ d))
    slopes = np.diff(np.log(rem)) / np.diff(np.log(ts))
    assert np.all((slopes > 2.8) & (slopes < 3.5)), slopes
    assert min(rem) > 1e3 * np.finfo(float).eps * abs(phi0)


# -------------------------------------------------------------- invariants
@pytest.mark.parametrize("name", ["tiny10", "syn300", "syn2000"])
def test_invariants(name):
    g = gridgen.grid(name)
    M, u, x, P = _setup(g)
    gres = M.residual(x, u, g["pd"], g["qd"])
    assert np.linalg.norm(gres) < 1e-10
    th, v, _ = M.full(x, u)
    Sf, St = M.branch_flows(th, v)
    pg = M.gen_p(x, u, g["pd"])
    # generation = load + losses (active); reactive incl. line charging
    assert abs(pg.sum() - g["pd"].sum() - np.sum(Sf.real + St.real)) < 1e-10
    S = M.injections(th, v)
    qnet = S.imag + g["qd"]
    assert abs(qnet[g["gen_bus"]].sum() - g["qd"].sum() - np.sum(Sf.imag + St.imag)) < 1e-10
    # adjoint identity <lambda, J_x z> = -<d_x phi, z>
    grad, lam = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], P)
    Jx, Ju = M.jacobians(x, u)
    gz = oracle.full_gradient(M, x, u, g["pd"], g["qd"], P)
    z = np.random.default_rng(1).standard_normal(M.nx)
    assert abs(lam @ (Jx @ z) + gz[M.ix] @ z) <= 1e-10 * np.abs(gz[M.ix] @ z) + 1e-12
    if M.nu <= 200:
        H = oracle.reduced_hessian(M, x, u, g["pd"], g["qd"], P, lam)
        assert np.linalg.norm(H - H.T) <= 1e-12 * np.linalg.norm(H)


@pytest.mark.slow
def test_largest_workload_power_flow_within_six_steps():
    """The 9241-bus workload's base power flow converges in <= 6 Newton
    steps from a flat start to ||g||_2 < 1e-10."""
    g = gridgen.grid("syn9241")
    M = oracle.Model(g)
    assert (M.nx, M.nu, M.m) == (17036, 2889, 41340)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    pf = oracle.solve_pf(M, u, g["pd"], g["qd"], max_iter=6)
    assert pf.converged and pf.iters <= 6


# ---------------------------------------------------------------- Cholesky
def test_cholesky_matches_lapack_and_reconstructs():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 40))
    K = A @ A.T + 40 * np.eye(40)
    L, info = oracle.cholesky_lower(K)
    assert info == 0
    assert np.linalg.norm(L @ L.T - K) <= 1e-14 * np.linalg.norm(K)
    np.testing.assert_allclose(L, np.linalg.cholesky(K), rtol=1e-12, atol=1e-13)


def test_cholesky_reports_first_failing_column():
    K = np.diag([4.0, 1.0, -2.0, 3.0])
    L, info = oracle.cholesky_lower(K)
    assert info == 3


def test_factor_solve_symmetrises_and_solves():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((12, 12))
    H = A @ A.T + 0.3 * rng.standard_normal((12, 12))     # not symmetric
    diag = rng.uniform(0.5, 1.0, 12)
    rhs = rng.standard_normal(12)
    L, info, d = oracle.factor_solve(H, diag, 2.0, rhs)
    K = 0.5 * (H + H.T) + np.diag(diag) + 2.0 * np.eye(12)
    assert info == 0
    np.testing.assert_allclose(K @ d, -rhs, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------ tracking bits
def test_slack_minimiser_minimises_the_al_in_s():
    g = gridgen.grid("tiny10")
    M, u, x, P = _setup(g)
    _, c = oracle.al_objective(M, x, u, g["pd"], g["qd"], P)
    lo, hi = gridgen.constraint_bounds(g)
    s = oracle.slack_minimiser(c, P, lo, hi)
    # per-coordinate objective -sigma y s + rho/2 sigma^2 (c - s)^2 on a grid
    for k in range(0, len(c), 5):
        grid = np.linspace(lo[k], hi[k], 20001)
        obj = P.sigma_c[k] * P.y[k] * (c[k] - grid) + 0.5 * P.rho * (P.sigma_c[k] * (c[k] - grid)) ** 2
        best = grid[np.argmin(obj)]
        assert abs(best - s[k]) <= (hi[k] - lo[k]) / 20000 + 1e-12


def _tracking_setup(seed=100):
    w = gridgen.tracking_workload(seed)
    g = gridgen.make_grid(dataclasses.replace(w, nb=300, nl=480, ng=81))
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    x = oracle.solve_pf(M, u, g["pd"], g["qd"]).x
    ep = gridgen.eval_point(g, seed=seed + 1000)
    lo, hi = gridgen.constraint_bounds(g)
    return g, M, u, x, ep, lo, hi


def test_tracking_multiplier_update_vanishes_inside_bounds():
    """y_new = y + rho sigma (c - clip(c + y/(rho sigma))): for constraints
    whose shifted value stays strictly inside the bounds, y_new = 0."""
    g, M, u, x, ep, lo, hi = _tracking_setup()
    P = oracle.Point.from_dict(ep)
    fac = np.ones(g["nb"])
    un, xn, yn, info = oracle.tracking_step(M, u, x, P.y, g["pd"], g["qd"], fac, P, lo, hi, delta=1e6)
    c = M.constraints(xn, un, g["pd"], g["qd"])
    z = c + P.y / (P.rho * P.sigma_c)
    inside = (z > lo + 1e-9) & (z < hi - 1e-9)
    assert inside.sum() > 0
    assert np.max(np.abs(yn[inside])) < 1e-9
    out = ~inside
    assert np.allclose(yn[out], P.y[out] + P.rho * P.sigma_c[out] * (c[out] - np.clip(z[out], lo[out], hi[out])))


def test_tracking_huge_shift_keeps_the_control():
    """With delta -> infinity the Newton step vanishes: u stays put and the
    first trial is accepted."""
    g, M, u, x, ep, lo, hi = _tracking_setup()
    P = oracle.Point.from_dict(ep)
    fac = np.ones(g["nb"])
    ulo, uhi = M.u_bounds()
    un, xn, yn, info = oracle.tracking_step(M, u, x, P.y, g["pd"], g["qd"], fac, P, lo, hi, delta=1e15)
    assert info["accepted"] == 0
    assert np.allclose(un, np.clip(u, ulo, uhi), atol=1e-9)


def test_tracking_step_is_a_descent_direction():
    """The shifted Newton step d = -(H + delta I)^{-1} grad has grad.d < 0."""
    g, M, u, x, ep, lo, hi = _tracking_setup()
    P = oracle.Point.from_dict(ep)
    fac = gridgen.tracking_factors(100, 1, g["nb"])[0]
    H0 = None
    un, xn, yn, info = oracle.tracking_step(M, u, x, P.y, g["pd"], g["qd"], fac, P, lo, hi, delta=1e3)
    assert info["info"] == 0
    assert float(info["grad"] @ info["step"]) < 0


# ------------------------------------------------------- inertia-control ladder
def _rotated(eigs, seed=3):
    """Q diag(eigs) Q^T with a random orthogonal Q: the eigenvalues, hence the
    first positive definite rung of the shift ladder, are known exactly."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((len(eigs), len(eigs))))
    return (Q * np.asarray(eigs, float)) @ Q.T


def test_delta_ladder_positive_definite_needs_no_shift():
    assert oracle.delta_ladder(np.diag([3.0, 1e-9, 2.0])) == 0.0
    assert oracle.delta_ladder(_rotated([5.0, 0.5, 1e-3, 2.0])) == 0.0


def test_delta_ladder_rung_from_the_eigenvalues():
    """delta = 0, then base = 1e-8 max(1, max|diag K|), times 10 per failure:
    the first rung above -lambda_min is returned.
    diag(5, -2e-6, 1): base 5e-8, rungs 5e-8, 5e-7, 5e-6 -> 5e-6."""
    d = oracle.delta_ladder(np.diag([5.0, -2e-6, 1.0]))
    assert d == pytest.approx(5e-6, rel=1e-12)
    # max|diag| below one: base = 1e-8; lambda_min = -3e-5 -> rung 1e-4
    d = oracle.delta_ladder(np.diag([0.5, -3e-5, 0.25]))
    assert d == pytest.approx(1e-4, rel=1e-12)
    # rotated: eigenvalues (40, 7, -0.02, 1) -> max|diag K| unknown a priori,
    # so recompute the base from the diagonal and count rungs by hand
    K = _rotated([40.0, 7.0, -0.02, 1.0])
    base = 1e-8 * max(1.0, float(np.max(np.abs(np.diag(K)))))
    k = int(np.ceil(np.log10(0.02 / base) - 1e-12))
    if base * 10.0 ** k <= 0.02:
        k += 1
    assert oracle.delta_ladder(K) == pytest.approx(base * 10.0 ** k, rel=1e-12)


def test_delta_ladder_uses_the_symmetric_part():
    """Only (H + H^T)/2 matters: a large skew part changes nothing."""
    S = np.diag([2.0, -1e-3, 1.0])
    A = np.array([[0.0, 50.0, -3.0], [-50.0, 0.0, 7.0], [3.0, -7.0, 0.0]])
    assert oracle.delta_ladder(S + A) == oracle.delta_ladder(S)


# ------------------------------------------- tracking: halving and failed step
def test_tracking_step_halving_takes_the_first_converging_trial():
    """With two Newton steps allowed per power flow, the full Newton step's
    power flow fails and the step is halved (Section IV-C with the step-halving
    safeguard): the accepted k is the first whose power flow converges within
    pf_iters from the previous state, and u, x are that trial's."""
    g, M, u, x, ep, lo, hi = _tracking_setup()
    P = oracle.Point.from_dict(ep)
    fac = np.ones(g["nb"])
    pd, qd = g["pd"], g["qd"]
    un, xn, yn, info = oracle.tracking_step(M, u, x, P.y, pd, qd, fac, P, lo, hi, delta=40.0, pf_iters=2)
    k = info["accepted"]
    assert k >= 1
    ulo, uhi = M.u_bounds()
    x0 = oracle.solve_pf(M, u, pd, qd, x0=x, max_iter=2, raise_on_fail=False).x
    for j in range(k):
        ut = np.clip(u + info["step"] / 2.0 ** j, ulo, uhi)
        r = oracle.solve_pf(M, ut, pd, qd, x0=x0, max_iter=2, raise_on_fail=False)
        assert not r.converged
    np.testing.assert_array_equal(un, np.clip(u + info["step"] / 2.0 ** k, ulo, uhi))
    assert np.linalg.norm(M.residual(xn, un, pd, qd)) < 1e-10
    # more Newton steps let the full step through
    un3, _, _, info3 = oracle.tracking_step(M, u, x, P.y, pd, qd, fac, P, lo, hi, delta=40.0, pf_iters=3)
    assert info3["accepted"] == 0
    np.testing.assert_array_equal(un3, np.clip(u + info3["step"], ulo, uhi))


def test_tracking_step_no_trial_converges_keeps_u_and_x():
    """One Newton step per power flow: no trial converges, so u and the state
    stay at the first power flow's, and y is still updated at them."""
    g, M, u, x, ep, lo, hi = _tracking_setup()
    P = oracle.Point.from_dict(ep)
    fac = np.ones(g["nb"])
    un, xn, yn, info = oracle.tracking_step(M, u, x, P.y, g["pd"], g["qd"], fac, P, lo, hi, delta=10.0,
                                            pf_iters=1)
    assert info["accepted"] == -1
    np.testing.assert_array_equal(un, u)
    c = M.constraints(xn, un, g["pd"], g["qd"])
    z = np.clip(c + P.y / (P.rho * P.sigma_c), lo, hi)
    np.testing.assert_allclose(yn, P.y + P.rho * P.sigma_c * (c - z), rtol=0, atol=1e-12)


def test_tracking_step_failed_cholesky_gives_zero_step():
    """A shift too small for the indefinite reduced Hessian makes the Cholesky
    fail (info > 0): the step is zero, the unchanged control is accepted at
    k = 0, and only the multipliers move."""
    g, M, u, x, ep, lo, hi = _tracking_setup()
    P = oracle.Point.from_dict(ep)
    fac = np.ones(g["nb"])
    # the reduced Hessian at this point is indefinite: its smallest eigenvalue
    # is below -1e-3, so the shift 1e-3 cannot make it positive definite
    s = oracle.slack_minimiser(M.constraints(x, u, g["pd"], g["qd"]), P, lo, hi)
    Pt = dataclasses.replace(P, s=s)
    H = oracle.reduced_hessian(M, x, u, g["pd"], g["qd"], Pt)
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() < -1e-3
    un, xn, yn, info = oracle.tracking_step(M, u, x, P.y, g["pd"], g["qd"], fac, P, lo, hi, delta=1e-3)
    assert info["info"] > 0 and info["accepted"] == 0
    assert not np.any(info["step"])
    ulo, uhi = M.u_bounds()
    np.testing.assert_array_equal(un, np.clip(u, ulo, uhi))


def test_zero_voltage_makes_the_jacobian_singular():
    """Every entry of the theta_i column of J_x carries v_i (dS_k/dtheta_i =
    j v_k v_i conj(Y_ki) e^{j(theta_k - theta_i)} and dS_i/dtheta_i likewise),
    so v_i = 0 at a PQ bus zeroes that column: J_x is singular and Newton's
    step is undefined; the oracle reports a failed power flow."""
    import warnings
    g = gridgen.grid("syn300")
    M, u, x, P = _setup(g)
    k = 5
    x0 = x.copy()
    x0[M.npv + M.npq + k] = 0.0
    Jx, _ = M.jacobians(x0, u)
    col = Jx.tocsc()[:, M.npv + k]
    assert col.nnz == 0 or abs(col).sum() == 0.0
    assert np.linalg.matrix_rank(Jx.toarray()) == M.nx - 1
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        r = oracle.solve_pf(M, u, g["pd"], g["qd"], x0=x0, raise_on_fail=False)
    assert not r.converged


# ------------------------------------------------------------ reduced Jacobian
def test_reduced_jacobian_vs_central_differences():
    """grad_u c(x(u), u) against central differences of c along every control,
    with the power flow re-solved at u +- h e_i (h = 1e-6 max(1, |u_i|))."""
    g = gridgen.grid("tiny10")
    M, u, x, P = _setup(g, tol=1e-13)
    J = oracle.reduced_jacobian(M, x, u)
    assert J.shape == (M.m, M.nu)
    for i in range(M.nu):
        h = 1e-6 * max(1.0, abs(u[i]))
        e = np.zeros(M.nu)
        e[i] = h
        cp = M.constraints(oracle.solve_pf(M, u + e, g["pd"], g["qd"], x0=x, tol=1e-14).x, u + e, g["pd"], g["qd"])
        cm = M.constraints(oracle.solve_pf(M, u - e, g["pd"], g["qd"], x0=x, tol=1e-14).x, u - e, g["pd"], g["qd"])
        fd = (cp - cm) / (2 * h)
        assert np.linalg.norm(J[:, i] - fd) <= 1e-6 * max(1.0, np.linalg.norm(fd)), i


@pytest.mark.parametrize("name", ["tiny10", "syn300"])
def test_reduced_jacobian_transpose_is_the_adjoint_gradient(name):
    """With sigma_f = 0 and rho = 0, phi = y^T D_c (c - s), so its reduced
    gradient by the adjoint (Proposition 1: one transposed solve) must equal
    J^T D_c y from the direct sensitivities (n_u forward solves)."""
    g = gridgen.grid(name)
    M, u, x, P = _setup(g)
    P0 = dataclasses.replace(P, sigma_f=0.0, rho=0.0)
    grad, _ = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], P0)
    J = oracle.reduced_jacobian(M, x, u)
    want = J.T @ (P.sigma_c * P.y)
    assert np.linalg.norm(grad - want) <= 1e-11 * np.linalg.norm(want)


def test_reduced_jacobian_state_rows_are_sensitivity_rows():
    """v at a PQ bus is a state, so its row of the reduced Jacobian is that
    state's row of dx/du = -J_x^{-1} J_u (here from spsolve, not SuperLU's
    factor object)."""
    g = gridgen.grid("syn300")
    M, u, x, P = _setup(g)
    J = oracle.reduced_jacobian(M, x, u)
    Jx, Ju = M.jacobians(x, u)
    S = -spla.spsolve(Jx.tocsc(), Ju.toarray())
    o = 2 * M.nl
    np.testing.assert_allclose(J[o:o + M.npq], S[M.npv + M.npq:], rtol=0, atol=1e-12)


# ------------------------------------------------ real-time QP (interior point)
def _rt_qp_case(name, seed=7):
    g = gridgen.grid(name)
    M, u, x, P = _setup(g, seed=seed)
    lo, hi = gridgen.constraint_bounds(g)
    s = np.clip(M.constraints(x, u, g["pd"], g["qd"]), lo, hi)
    Pt = dataclasses.replace(P, s=s)
    H = oracle.reduced_hessian(M, x, u, g["pd"], g["qd"], Pt)
    J = oracle.reduced_jacobian(M, x, u)
    Huu = 0.5 * (H + H.T) - P.rho * (J.T * P.sigma_c ** 2) @ J
    delta = 1.5 * max(0.0, -float(np.linalg.eigvalsh(Huu).min())) + 1e-2
    return g, M, u, x, P, s, lo, hi, delta


@pytest.mark.parametrize("name", ["tiny10", "syn300"])
def test_rt_qp_matches_an_active_set_solver(name):
    """The interior-point solution of the bounded QP of eq. (qp_rto) equals
    the solution of the same strictly convex QP by scipy's bounded-variable
    least squares (an active-set method): with Hw = R^T R,
    g^T d + 1/2 d^T Hw d = 1/2 |R d + R^{-T} g|^2 + const."""
    from scipy.optimize import lsq_linear
    import scipy.linalg as sla
    g, M, u, x, P, s, lo, hi, delta = _rt_qp_case(name)
    ulo, uhi = M.u_bounds()
    du, ds, info = oracle.rt_step_qp(M, u, s, x, P.y, g["pd"], g["qd"], P, ulo, uhi, lo, hi, delta, tol=1e-14,
                                     iters=60)
    Hw, gw, l, h = info["Hw"], info["g"], info["lo"], info["hi"]
    R = np.linalg.cholesky(0.5 * (Hw + Hw.T)).T
    ref = lsq_linear(R, -sla.solve_triangular(R.T, gw, lower=True), bounds=(l, h), method="bvls",
                     tol=1e-15, max_iter=100000).x
    d = np.concatenate([du, ds])
    active = np.sum((ref <= l + 1e-12) | (ref >= h - 1e-12))
    assert active > 0                         # bounds matter in this QP
    assert np.linalg.norm(d - ref) <= 1e-9 * np.linalg.norm(ref)
    assert info["iters"] <= 30


def test_box_qp_closed_forms():
    """Diagonal Hessian: the minimiser is the clipped Newton point
    clip(-g_i / H_ii, lo_i, hi_i) coordinate by coordinate; a box that no
    bound touches gives the unconstrained Newton step -Hw^{-1} g."""
    rng = np.random.default_rng(5)
    n = 40
    hd = rng.uniform(0.5, 5.0, n)
    gv = rng.standard_normal(n) * 3.0
    lo = -rng.uniform(0.1, 1.0, n)
    hi = rng.uniform(0.1, 1.0, n)
    d, zl, zu, it = oracle.box_qp_ipm(np.diag(hd), gv, lo, hi, tol=1e-14, iters=80)
    want = np.clip(-gv / hd, lo, hi)
    assert np.max(np.abs(d - want)) <= 1e-10
    A = rng.standard_normal((n, n))
    Hw = A @ A.T / n + np.eye(n)
    x0 = np.linalg.solve(Hw, -gv)
    d, zl, zu, it = oracle.box_qp_ipm(Hw, gv, x0 - 10.0, x0 + 10.0, tol=1e-14, iters=80)
    assert np.linalg.norm(d - x0) <= 1e-10 * np.linalg.norm(x0)


def test_box_qp_inertia_control_convex_case_unchanged():
    """On a strictly convex QP the inertia control never regularises: the
    first factorization of every iteration succeeds with w = 0 and the
    iterates are those of the unregularised method."""
    rng = np.random.default_rng(11)
    n = 30
    A = rng.standard_normal((n, n))
    Hw = A @ A.T / n + 0.1 * np.eye(n)
    gv = rng.standard_normal(n)
    lo, hi = -rng.uniform(0.05, 0.5, n), rng.uniform(0.05, 0.5, n)
    d0, zl0, zu0, it0 = oracle.box_qp_ipm(Hw, gv, lo, hi, tol=1e-13, iters=80)
    d1, zl1, zu1, it1, info = oracle.box_qp_ipm(Hw, gv, lo, hi, tol=1e-13, iters=80, nreg=n)
    assert it1 == it0 and info["slots"] == it1 and info["w"] == 0.0 and not info["failed"]
    assert np.max(np.abs(d1 - d0)) <= 1e-13


def test_box_qp_inertia_control_reaches_a_local_minimiser():
    """Separable indefinite QP (diagonal Hw, ten negative entries): the
    regularised iteration ends at a local minimiser, checked coordinate by
    coordinate -- a positive-curvature coordinate at its clipped Newton point
    clip(-g_i / h_i, lo_i, hi_i), a negative-curvature one at a bound where
    the derivative g_i + h_i d_i points outward (strict local minimum of a
    concave parabola on an interval).  The first factorization fails, so the
    regularisation was used."""
    rng = np.random.default_rng(12)
    n = 30
    hd = rng.uniform(0.5, 5.0, n)
    hd[:10] = -rng.uniform(0.5, 5.0, 10)
    gv = rng.standard_normal(n)
    lo, hi = -rng.uniform(0.1, 1.0, n), rng.uniform(0.1, 1.0, n)
    d, zl, zu, it, info = oracle.box_qp_ipm(np.diag(hd), gv, lo, hi, tol=1e-12, iters=300, nreg=n)
    assert not info["failed"] and info["slots"] > it
    assert oracle.kkt_error(np.diag(hd), gv, lo, hi, d, zl, zu) < 1e-12
    np.testing.assert_allclose(d[10:], np.clip(-gv[10:] / hd[10:], lo[10:], hi[10:]), rtol=0, atol=1e-9)
    for i in range(10):
        slope = gv[i] + hd[i] * d[i]
        at_lo, at_hi = abs(d[i] - lo[i]) < 1e-9, abs(d[i] - hi[i]) < 1e-9
        assert (at_lo and slope > 0) or (at_hi and slope < 0), (i, d[i], lo[i], hi[i], slope)


def test_rt_qp_kkt_certificate_and_slack_coupling():
    """At the interior-point solution the bound multipliers are non-negative,
    complementary to the active bounds, and the s block of the stationarity
    condition gives d_s in closed form from d_u (Proposition 3: the slack
    direction depends linearly on the control direction)."""
    g, M, u, x, P, s, lo, hi, delta = _rt_qp_case("syn300")
    ulo, uhi = M.u_bounds()
    du, ds, info = oracle.rt_step_qp(M, u, s, x, P.y, g["pd"], g["qd"], P, ulo, uhi, lo, hi, delta, tol=1e-13,
                                     iters=60)
    assert info["kkt"] < 1e-13 * 10
    # inside the s box: rho D^2 (ds - J du) + g_s = 0 for the free slacks
    c = M.constraints(x, u, g["pd"], g["qd"])
    gs = -P.sigma_c * (P.y + P.rho * P.sigma_c * (c - s))
    free = (ds > (lo - s) + 1e-7) & (ds < (hi - s) - 1e-7)
    want = info["J"][free] @ du - gs[free] / (P.rho * P.sigma_c[free] ** 2)
    np.testing.assert_allclose(ds[free], want, rtol=0, atol=1e-8 * max(1.0, np.abs(want).max()))


# ------------------------------------------- static OPF (augmented Lagrangian)
def _static_case(name):
    g = gridgen.grid(name)
    ep = gridgen.eval_point(g, sigma="ones")
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    x = oracle.solve_pf(M, u, g["pd"], g["qd"]).x
    P = oracle.Point.from_dict(ep)
    lo, hi = gridgen.constraint_bounds(g)
    s = np.clip(M.constraints(x, u, g["pd"], g["qd"]), lo, hi)
    return g, M, u, x, P, lo, hi, s


def test_static_opf_matches_a_full_space_nlp_solver():
    """The augmented-Lagrangian method (Section IV-B.3) on tiny10 stops
    within the tolerances of Section V-B, at the optimum that a general NLP
    solver finds for the full-space problem eq. (acopf) -- SciPy's SLSQP over
    (x, u) with the power flow as equalities and the operational constraints
    and control bounds as inequalities: objectives within 1e-5 relative (the
    AL point is feasible only to 1e-5), controls within 1e-3."""
    from scipy.optimize import minimize
    g, M, u, x, P, lo, hi, s = _static_case("tiny10")
    u2, s2, x2, y2, rho, hist = oracle.static_opf(M, u, s, np.zeros(M.m), g["pd"], g["qd"], P, lo, hi)
    assert hist[-1]["converged"] and hist[-1]["theta"] <= 1e-5 and hist[-1]["pg"] <= 1e-4
    assert any(h["updated"] for h in hist) and rho > 10.0      # both updates of the method were taken
    nx = M.nx
    pd, qd = g["pd"], g["qd"]
    ulo, uhi = M.u_bounds()
    split = lambda z: (z[:nx], z[nx:])
    cons = [dict(type="eq", fun=lambda z: M.residual(*split(z), pd, qd)),
            dict(type="ineq", fun=lambda z: M.constraints(*split(z), pd, qd) - lo),
            dict(type="ineq", fun=lambda z: hi - M.constraints(*split(z), pd, qd))]
    ref = minimize(lambda z: M.cost(M.gen_p(*split(z), pd)) / 1e4, np.concatenate([x, u]), method="SLSQP",
                   constraints=cons, bounds=[(None, None)] * nx + list(zip(ulo, uhi)),
                   options=dict(maxiter=500, ftol=1e-12))
    assert ref.success
    f_al = M.cost(M.gen_p(x2, u2, pd))
    assert abs(f_al - 1e4 * ref.fun) <= 1e-5 * abs(f_al)
    np.testing.assert_allclose(u2, ref.x[nx:], rtol=0, atol=1e-3)
    # the AL's final point solves the power flow and keeps u in its box
    assert np.linalg.norm(M.residual(x2, u2, pd, qd)) < 1e-9
    assert np.all(u2 >= ulo - 1e-12) and np.all(u2 <= uhi + 1e-12)


def test_projected_gradient_measure():
    """Zero exactly at a stationary point of a box-constrained problem:
    interior points with zero gradient, and bound points whose gradient
    points outward; positive otherwise."""
    lo, hi = np.zeros(3), np.ones(3)
    w = np.array([0.5, 0.0, 1.0])
    assert oracle.projected_gradient(w, np.array([0.0, 2.0, -3.0]), lo, hi) == 0.0
    assert oracle.projected_gradient(w, np.array([0.1, 0.0, 0.0]), lo, hi) == pytest.approx(0.1)
    assert oracle.projected_gradient(w, np.array([0.0, -0.2, 0.0]), lo, hi) == pytest.approx(0.2)
