"""50-digit reference for tiny grids, written directly from the model's
definitions with mpmath (no code shared with the oracle): the power flow is
solved with mpmath.findroot from a flat start and the reduced AL function
phi(u) = phi(x(u), u) is differentiated numerically at high precision."""
import mpmath as mp

REF, PV, PQ = 2, 1, 0


class MPGrid:
    def __init__(self, g, point, dps=50):
        mp.mp.dps = dps
        self.g = g
        self.nb = g["nb"]
        bt = [int(t) for t in g["bus_type"]]
        self.ref = bt.index(REF)
        self.pv = [i for i in range(self.nb) if bt[i] == PV]
        self.pq = [i for i in range(self.nb) if bt[i] == PQ]
        self.genat = {int(b): k for k, b in enumerate(g["gen_bus"])}
        self.br = []
        for k in range(g["nl"]):
            ys = 1 / mp.mpc(mp.mpf(g["br_r"][k]), mp.mpf(g["br_x"][k]))
            sh = mp.mpc(0, mp.mpf(g["br_b"][k]) / 2)
            self.br.append((int(g["br_from"][k]), int(g["br_to"][k]), ys + sh, -ys, -ys, ys + sh))
        self.pd = [mp.mpf(v) for v in g["pd"]]
        self.qd = [mp.mpf(v) for v in g["qd"]]
        self.pt = point

    def voltages(self, th, v):
        return [v[i] * mp.expj(th[i]) for i in range(self.nb)]

    def injections(self, V):
        I = [mp.mpc(0)] * self.nb
        for f, t, yff, yft, ytf, ytt in self.br:
            I[f] += yff * V[f] + yft * V[t]
            I[t] += ytf * V[f] + ytt * V[t]
        return [V[i] * mp.conj(I[i]) for i in range(self.nb)]

    def unpack(self, x, u):
        npv, npq = len(self.pv), len(self.pq)
        th = [mp.mpf(0)] * self.nb
        v = [mp.mpf(1)] * self.nb
        for k, i in enumerate(self.pv):
            th[i] = x[k]
        for k, i in enumerate(self.pq):
            th[i] = x[npv + k]
            v[i] = x[npv + npq + k]
        v[self.ref] = u[0]
        for k, i in enumerate(self.pv):
            v[i] = u[1 + k]
        ppv = list(u[1 + npv:])
        return th, v, ppv

    def residual(self, x, u):
        th, v, ppv = self.unpack(x, u)
        S = self.injections(self.voltages(th, v))
        out = [S[i].real - ppv[k] + self.pd[i] for k, i in enumerate(self.pv)]
        out += [S[i].real + self.pd[i] for i in self.pq]
        out += [S[i].imag + self.qd[i] for i in self.pq]
        return out

    def solve(self, u):
        npv, npq = len(self.pv), len(self.pq)
        x0 = [mp.mpf(0)] * (npv + npq) + [mp.mpf(1)] * npq
        sol = mp.findroot(lambda *x: self.residual(list(x), u), x0, solver="mdnewton",
                          tol=mp.mpf(10) ** (-2 * mp.mp.dps + 10), maxsteps=200)
        if not hasattr(sol, "rows"):
            return [sol]
        return [sol[k] for k in range(sol.rows)]

    def phi(self, u):
        """Reduced AL objective at control u (list of mpf)."""
        g, P = self.g, self.pt
        x = self.solve(u)
        th, v, ppv = self.unpack(x, u)
        V = self.voltages(th, v)
        S = self.injections(V)
        hf, ht = [], []
        for f, t, yff, yft, ytf, ytt in self.br:
            sf = V[f] * mp.conj(yff * V[f] + yft * V[t])
            st = V[t] * mp.conj(ytf * V[f] + ytt * V[t])
            hf.append(abs(sf) ** 2)
            ht.append(abs(st) ** 2)
        pref = S[self.ref].real + self.pd[self.ref]
        c = hf + ht + [v[i] for i in self.pq] + [pref, S[self.ref].imag + self.qd[self.ref]]
        c += [S[i].imag + self.qd[i] for i in self.pv]
        base = mp.mpf(g["base_mva"])
        pg = {self.genat[self.ref]: pref}
        for k, i in enumerate(self.pv):
            pg[self.genat[i]] = ppv[k]
        f = mp.mpf(0)
        for k, p in pg.items():
            pm = base * p
            f += mp.mpf(g["c2"][k]) * pm ** 2 + mp.mpf(g["c1"][k]) * pm + mp.mpf(g["c0"][k])
        phi = mp.mpf(P["sigma_f"]) * f
        rho = mp.mpf(P["rho"])
        for k in range(len(c)):
            r = mp.mpf(P["sigma_c"][k]) * (c[k] - mp.mpf(P["s"][k]))
            phi += mp.mpf(P["y"][k]) * r + rho / 2 * r * r
        return phi

    def derivatives(self, u):
        """(gradient, Hessian) of phi at u by high-precision differentiation."""
        u = [mp.mpf(v) for v in u]
        n = len(u)
        f = lambda *a: self.phi(list(a))
        grad = [mp.diff(f, u, tuple(1 if j == i else 0 for j in range(n))) for i in range(n)]
        H = [[None] * n for _ in range(n)]
        for i in range(n):
            for j in range(i, n):
                order = [0] * n
                order[i] += 1
                order[j] += 1
                H[i][j] = H[j][i] = mp.diff(f, u, tuple(order))
        return grad, H
