"""Oracle, part 1: the polar AC model, written bus-wise with the complex
bus admittance matrix.  Plain and slow on purpose; FP64 throughout.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

Definitions followed:
* grid, polar variables, loads, generation: Section II-A, eq. (acopf);
* control / state split u = (v_ref, v_pv, p_pv), x = (theta_pv, theta_pq,
  v_pq): Section II-B, eq. (statecontrol);
* operational constraints c = (h, r), r = (v_pq, p_ref, q_ref^net,
  q_pv^net), m = 2 n_l + n_pq + n_pv + 2: eq. (acopf_controlstate);
* the lower bound 0 on h (Section IV-A) makes h the squared apparent flow;
* AL functional with scalings sigma_f, D_c: Section IV-A.2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

PQ, PV, REF = 0, 1, 2


class Model:
    """Index maps and admittances of one grid (a dict from ``gridgen``)."""

    def __init__(self, g: dict):
        self.g = g
        nb, nl = g["nb"], g["nl"]
        self.nb, self.nl, self.ng = nb, nl, g["ng"]
        self.base = float(g["base_mva"])
        bt = np.asarray(g["bus_type"])
        refs = np.flatnonzero(bt == REF)
        if refs.size != 1:
            raise ValueError("exactly one REF bus is required")
        self.ref = int(refs[0])
        self.pv = np.flatnonzero(bt == PV)
        self.pq = np.flatnonzero(bt == PQ)
        self.npv, self.npq = self.pv.size, self.pq.size
        genat = np.full(nb, -1)
        genat[np.asarray(g["gen_bus"])] = np.arange(self.ng)
        if np.any(genat[self.pv] < 0) or genat[self.ref] < 0:
            raise ValueError("every PV/REF bus needs a generator")
        self.gen_ref = int(genat[self.ref])
        self.gen_pv = genat[self.pv]
        # sizes (Section II-B and eq. acopf_controlstate)
        self.nx = self.npv + 2 * self.npq
        self.nu = 1 + 2 * self.npv
        self.m = 2 * nl + self.npq + self.npv + 2

        # full variable vector z = (theta[nb], v[nb], p_pv[npv])
        self.nz = 2 * nb + self.npv
        self.ix = np.concatenate([self.pv, self.pq, nb + self.pq])
        self.iu = np.concatenate([[nb + self.ref], nb + self.pv, 2 * nb + np.arange(self.npv)])

        # pi-model admittances, no taps or shifts
        f = np.asarray(g["br_from"]); t = np.asarray(g["br_to"])
        self.f, self.t = f, t
        ys = 1.0 / (np.asarray(g["br_r"]) + 1j * np.asarray(g["br_x"]))
        bc = 1j * np.asarray(g["br_b"]) / 2.0
        self.Yff = ys + bc
        self.Ytt = ys + bc
        self.Yft = -ys
        self.Ytf = -ys
        rows = np.concatenate([f, t, f, t])
        cols = np.concatenate([f, t, t, f])
        vals = np.concatenate([self.Yff, self.Ytt, self.Yft, self.Ytf])
        self.Y = sp.csr_matrix((vals, (rows, cols)), shape=(nb, nb))
        li = np.arange(nl)
        self.Yf = sp.csr_matrix((np.concatenate([self.Yff, self.Yft]),
                                 (np.concatenate([li, li]), np.concatenate([f, t]))), shape=(nl, nb))
        self.Yt = sp.csr_matrix((np.concatenate([self.Ytf, self.Ytt]),
                                 (np.concatenate([li, li]), np.concatenate([f, t]))), shape=(nl, nb))
        self.Cf = sp.csr_matrix((np.ones(nl), (li, f)), shape=(nl, nb))
        self.Ct = sp.csr_matrix((np.ones(nl), (li, t)), shape=(nl, nb))

    # ---------------------------------------------------------------- vectors
    def u_from_setpoints(self, vg: np.ndarray, pg: np.ndarray) -> np.ndarray:
        """u = (v_ref, v_pv, p_pv) from per-generator setpoints."""
        return np.concatenate([[vg[self.gen_ref]], vg[self.gen_pv], pg[self.gen_pv]])

    def u_bounds(self):
        g = self.g
        lo = np.concatenate([[g["vmin"][self.ref]], g["vmin"][self.pv], g["pmin"][self.gen_pv]])
        hi = np.concatenate([[g["vmax"][self.ref]], g["vmax"][self.pv], g["pmax"][self.gen_pv]])
        return lo, hi

    def flat_x(self) -> np.ndarray:
        return np.concatenate([np.zeros(self.npv + self.npq), np.ones(self.npq)])

    def full(self, x: np.ndarray, u: np.ndarray):
        """(theta, v, p_pv) over all buses from (x, u); theta_ref = 0."""
        nb = self.nb
        z = np.zeros(self.nz)
        z[nb:2 * nb] = 1.0
        z[self.ix] = x
        z[self.iu] = u
        z[self.ref] = 0.0
        return z[:nb], z[nb:2 * nb], z[2 * nb:]

    # ----------------------------------------------------------- power flows
    def injections(self, th, v):
        V = v * np.exp(1j * th)
        return V * np.conj(self.Y @ V)

    def branch_flows(self, th, v):
        V = v * np.exp(1j * th)
        Sf = (self.Cf @ V) * np.conj(self.Yf @ V)
        St = (self.Ct @ V) * np.conj(self.Yt @ V)
        return Sf, St

    def residual(self, x, u, pd, qd):
        """g(x, u): active balance at PV and PQ buses, reactive at PQ buses."""
        th, v, ppv = self.full(x, u)
        S = self.injections(th, v)
        gp_pv = S.real[self.pv] - ppv + pd[self.pv]
        gp_pq = S.real[self.pq] + pd[self.pq]
        gq_pq = S.imag[self.pq] + qd[self.pq]
        return np.concatenate([gp_pv, gp_pq, gq_pq])

    # ------------------------------------------------- first derivatives
    def dS_dV(self, Ybus, th, v, Cside=None):
        """Polar derivatives of S = V_side * conj(Ybus V) w.r.t. (theta, v).
        With Cside None the side is the bus itself (square Ybus)."""
        V = v * np.exp(1j * th)
        E = np.exp(1j * th)
        I = Ybus @ V
        if Cside is None:
            Vs = V
            dIa = sp.diags(np.conj(I)) @ sp.diags(1j * V)
            dIv = sp.diags(np.conj(I)) @ sp.diags(E)
        else:
            Vs = Cside @ V
            dIa = sp.diags(np.conj(I)) @ Cside @ sp.diags(1j * V)
            dIv = sp.diags(np.conj(I)) @ Cside @ sp.diags(E)
        dSa = dIa + sp.diags(Vs) @ (Ybus @ sp.diags(1j * V)).conj()
        dSv = dIv + sp.diags(Vs) @ (Ybus @ sp.diags(E)).conj()
        return sp.csr_matrix(dSa), sp.csr_matrix(dSv)

    def jac_full(self, x, u):
        """Jacobian of g w.r.t. z = (theta, v, p_pv), shape [nx, nz]."""
        th, v, _ = self.full(x, u)
        dSa, dSv = self.dS_dV(self.Y, th, v)
        dS = sp.hstack([dSa, dSv, sp.csr_matrix((self.nb, self.npv))]).tocsr()
        P = dS.real
        Q = dS.imag
        gpv = P[self.pv] - sp.hstack([sp.csr_matrix((self.npv, 2 * self.nb)), sp.identity(self.npv)])
        return sp.vstack([gpv, P[self.pq], Q[self.pq]]).tocsr()

    def jacobians(self, x, u):
        Jz = self.jac_full(x, u).tocsc()
        return Jz[:, self.ix].tocsr(), Jz[:, self.iu].tocsr()

    # ---------------------------------------------------- constraints, cost
    def constraints(self, x, u, pd, qd):
        """c(x, u) = (|S_f|^2, |S_t|^2, v_pq, p_ref, q_ref^net, q_pv^net)."""
        th, v, _ = self.full(x, u)
        Sf, St = self.branch_flows(th, v)
        S = self.injections(th, v)
        pref = S.real[self.ref] + pd[self.ref]
        qnet = S.imag + qd
        return np.concatenate([np.abs(Sf) ** 2, np.abs(St) ** 2, v[self.pq], [pref],
                               [qnet[self.ref]], qnet[self.pv]])

    def constraint_jac_full(self, x, u):
        """Jacobian of c w.r.t. z, shape [m, nz]."""
        th, v, _ = self.full(x, u)
        Sf, St = self.branch_flows(th, v)
        zer = sp.csr_matrix((self.nl, self.npv))
        blocks = []
        for Yb, C, Sb in ((self.Yf, self.Cf, Sf), (self.Yt, self.Ct, St)):
            da, dv = self.dS_dV(Yb, th, v, C)
            dS = sp.hstack([da, dv, zer]).tocsr()
            # d|S|^2 = 2 Re(conj(S) dS)
            blocks.append((sp.diags(2.0 * np.conj(Sb)) @ dS).real)
        nb = self.nb
        ev = sp.csr_matrix((np.ones(self.npq), (np.arange(self.npq), nb + self.pq)),
                           shape=(self.npq, self.nz))
        dSa, dSv = self.dS_dV(self.Y, th, v)
        dS = sp.hstack([dSa, dSv, sp.csr_matrix((nb, self.npv))]).tocsr()
        rows = np.concatenate([[self.ref], self.pv])
        blocks += [ev, dS.real[[self.ref]], dS.imag[rows]]
        return sp.vstack(blocks).tocsr()

    def gen_p(self, x, u, pd):
        """Active generation per generator (slack from the balance at REF)."""
        th, v, ppv = self.full(x, u)
        S = self.injections(th, v)
        p = np.zeros(self.ng)
        p[self.gen_pv] = ppv
        p[self.gen_ref] = S.real[self.ref] + pd[self.ref]
        return p

    def cost(self, pg):
        """Quadratic generation cost on MW, over all generators."""
        pmw = self.base * pg
        return float(np.sum(self.g["c2"] * pmw ** 2 + self.g["c1"] * pmw + self.g["c0"]))

    def cost_d1(self, pg):
        return self.base * (2.0 * self.g["c2"] * self.base * pg + self.g["c1"])

    def cost_d2(self):
        return 2.0 * self.g["c2"] * self.base ** 2


def term_hessian(nn, ia, ib, coef, th, v):
    """Hessian in (theta[nn], v[nn]) of sum_k v_a v_b Re(coef_k e^{j(theta_a - theta_b)})
    over terms k with a = ia[k], b = ib[k].  Terms with a == b are v_a^2 Re(coef).
    Every bus injection and branch flow is a sum of such terms, so weighted
    sums of their real/imaginary parts use complex weights folded into coef."""
    ia = np.asarray(ia); ib = np.asarray(ib); coef = np.asarray(coef, dtype=complex)
    same = ia == ib
    d = ~same
    a, b, c = ia[d], ib[d], coef[d]
    E = c * np.exp(1j * (th[a] - th[b]))
    A, B = E.real, E.imag
    va, vb = v[a], v[b]
    ta, tb, wa, wb = a, b, nn + a, nn + b
    r = []; cc = []; val = []

    def add(i, j, x):
        r.append(i); cc.append(j); val.append(x)
        r.append(j); cc.append(i); val.append(x)

    def add_diag(i, x):
        r.append(i); cc.append(i); val.append(x)

    add_diag(ta, -va * vb * A)
    add_diag(tb, -va * vb * A)
    add(ta, tb, va * vb * A)
    add(ta, wa, -vb * B)
    add(ta, wb, -va * B)
    add(tb, wa, vb * B)
    add(tb, wb, va * B)
    add(wa, wb, A)
    s = ia[same]
    add_diag(nn + s, 2.0 * coef[same].real)
    r = np.concatenate(r); cc = np.concatenate(cc); val = np.concatenate(val)
    return sp.csr_matrix((val, (r, cc)), shape=(2 * nn, 2 * nn))
