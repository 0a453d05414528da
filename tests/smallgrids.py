"""Hand-made tiny grids for the pins, in the same dict layout as ``gridgen``."""
import numpy as np

import gridgen


def make(bus_type, branches, gens, pd, qd, vg=None, pg=None, name="hand"):
    """branches: list of (f, t, r, x, b); gens: list of (bus, c2, c1)."""
    nb = len(bus_type)
    br = np.array(branches, dtype=float)
    ng = len(gens)
    gen_bus = np.array([g[0] for g in gens], dtype=np.int32)
    pd = np.asarray(pd, float)
    qd = np.asarray(qd, float)
    d = dict(
        name=name, nb=nb, nl=len(branches), ng=ng, base_mva=gridgen.BASE_MVA,
        bus_type=np.asarray(bus_type, np.int32), br_from=br[:, 0].astype(np.int32),
        br_to=br[:, 1].astype(np.int32), br_r=br[:, 2], br_x=br[:, 3], br_b=br[:, 4],
        br_rate=np.full(len(branches), 2.0), gen_bus=gen_bus,
        c2=np.array([g[1] for g in gens], float), c1=np.array([g[2] for g in gens], float),
        c0=np.zeros(ng), vmin=np.full(nb, 0.94), vmax=np.full(nb, 1.06),
        pmin=np.zeros(ng), pmax=np.full(ng, 3.0), qmin=np.full(ng, -1.5), qmax=np.full(ng, 1.5),
        pd=pd, qd=qd,
        vg0=np.ones(ng) if vg is None else np.asarray(vg, float),
        pg0=np.full(ng, pd.sum() / ng) if pg is None else np.asarray(pg, float),
    )
    return d


def two_bus(r=0.02, x=0.1, b=0.0, P=0.8, Q=0.3, v1=1.02):
    """REF bus 0 feeding a PQ load P + jQ at bus 1 over one line."""
    return make([gridgen.REF, gridgen.PQ], [(0, 1, r, x, b)], [(0, 0.02, 20.0)],
                [0.0, P], [0.0, Q], vg=[v1], pg=[P])


def three_bus(b=0.04):
    """REF bus 0, PV bus 1, PQ bus 2, meshed triangle."""
    return make([gridgen.REF, gridgen.PV, gridgen.PQ],
                [(0, 1, 0.01, 0.08, b), (1, 2, 0.02, 0.12, b), (2, 0, 0.015, 0.1, b)],
                [(0, 0.02, 20.0), (1, 0.03, 25.0)],
                [0.0, 0.3, 0.9], [0.0, 0.1, 0.35], vg=[1.03, 1.01], pg=[0.6, 0.7])


def point_for(g, seed=7, rho=10.0, sigma="random"):
    return gridgen.eval_point(g, seed=seed, rho=rho, sigma=sigma)
