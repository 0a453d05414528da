"""Seeded synthetic transmission grids and evaluation points.

This module only draws random inputs (topology, impedances, loads, costs,
limits, multipliers, slacks, directions).  It contains none of the
reduced-space method's arithmetic: no AC power flow, no derivatives, no
adjoints.  Both the CPU oracle and the GPU library consume its output, each
with its own code.

Grid data follow the polar AC-OPF model of the paper (Section II-A): buses
with types REF/PV/PQ (Section II-B), pi-model branches with series r + jx
and total line charging b, one generator per generator bus, quadratic costs
on MW.  The paper's PGLIB PEGASE instances (Section V-A, Table I) are not
available; these grids stand in for them with the same sizes
(n_b, n_l, n_pv).

Recipe (all draws from ``numpy.random.default_rng(seed)`` in a fixed order):

* topology: ``tree_chords`` = random recursive spanning tree plus random
  chords; ``geometric`` = points uniform in the unit square, Euclidean
  minimum spanning tree of the Delaunay graph, then nearest-neighbour chords
  (buses in random order each add their shortest Delaunay edge that is not
  yet a branch, round after round) until n_l branches; each branch
  orientation flipped with probability 1/2.
* r ~ U(0.001, 0.05), x ~ U(0.01, 0.3), b ~ U(0, 0.1) (p.u.).
* generator buses: farthest-first traversal in branch hops from a random
  start bus (ties broken by a random priority), so that every load bus lies
  a few hops from a generator; the bus of least hop eccentricity among them
  is the slack (REF), the others PV; all other buses are PQ and carry the
  loads.
* p_d ~ lognormal with distribution mean 0.3 p.u. and sigma 0.5,
  q_d = p_d * U(0.1, 0.4), both times a per-workload load scale alpha.
* c2 ~ U(0.001, 0.05), c1 ~ U(10, 40), c0 = 0 (cost on MW, base 100 MVA).
* |V| bounds [0.94, 1.06]; initial setpoints v = 1.0 at generator buses;
  each load bus is served by the generator bus nearest in branch hops (ties
  to the generator placed first) and p_g0 is the load it serves plus an
  estimate of nearby branch losses r (F_p^2 + F_q^2), F_p and F_q the
  branch flows of two linear (1/x-weighted Laplacian) networks: active
  injections with the slack grounded, and line charging minus reactive load
  with the generator buses grounded.  The slack thus carries only the error
  of that estimate.  pmin = 0, pmax = 2 max(p_g0, 0.1), q bounds +-0.5 pmax.
* line rating = 1.5 * max(hypot(F_p, F_q), 0.1).  Only the slack bounds of
  the flow constraints depend on it.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.sparse.linalg as spla
from scipy.spatial import Delaunay

PQ, PV, REF = 0, 1, 2
BASE_MVA = 100.0


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nb: int
    nl: int
    ng: int
    seed: int
    topology: str
    load_scale: float = 1.0


# Workloads of the benchmark: sizes, seeds and topology method.  The 9241-bus
# case takes PEGASE9241's exact shape (n_l = 16049, n_g = 1445 -> n_pv = 1444).
# load_scale is the largest 0.9^k for which a flat-start Newton power flow
# reaches ||g||_2 < 1e-10 within 6 steps (checked by the test suite).
WORKLOADS: Dict[str, Workload] = {
    "tiny10": Workload("tiny10", 10, 13, 3, 0, "tree_chords"),
    "syn300": Workload("syn300", 300, 410, 69, 1, "geometric"),
    "syn2000": Workload("syn2000", 2000, 3200, 540, 2, "geometric"),
    "syn9241": Workload("syn9241", 9241, 16049, 1445, 3, "geometric", 0.9 ** 10),
    # PEGASE1354 / PEGASE2869 shapes (Table I), context only
    "syn1354": Workload("syn1354", 1354, 1991, 260, 11, "geometric", 0.9 ** 6),
    "syn2869": Workload("syn2869", 2869, 4582, 510, 12, "geometric", 0.9 ** 4),
}

TRACKING_SEEDS = list(range(100, 164))
TRACKING_LOAD_SCALE = 0.8


def tracking_workload(seed: int) -> Workload:
    """One instance of the 64-grid tracking batch: n_b ~ U[300, 2000],
    n_l = 1.6 n_b, n_g = 0.27 n_b, loads at 0.8 (every instance then
    converges from flat start within 6 Newton steps)."""
    rng = np.random.default_rng(seed)
    nb = int(rng.integers(300, 2001))
    return Workload(f"track{seed}", nb, int(round(1.6 * nb)), int(round(0.27 * nb)),
                    seed, "geometric", TRACKING_LOAD_SCALE)


def _tree_chords(rng, nb, nl):
    perm = rng.permutation(nb)
    edges = set()
    out = []
    for k in range(1, nb):
        p = int(rng.integers(0, k))
        a, b = int(perm[k]), int(perm[p])
        out.append((a, b))
        edges.add((min(a, b), max(a, b)))
    while len(out) < nl:
        a, b = (int(v) for v in rng.integers(0, nb, size=2))
        if a == b or (min(a, b), max(a, b)) in edges:
            continue
        edges.add((min(a, b), max(a, b)))
        out.append((a, b))
    return np.array(out, dtype=np.int64)


def _geometric(rng, nb, nl):
    pts = rng.random((nb, 2))
    tri = Delaunay(pts)
    e = set()
    for s in tri.simplices:
        for i in range(3):
            a, b = int(s[i]), int(s[(i + 1) % 3])
            e.add((min(a, b), max(a, b)))
    e = np.array(sorted(e), dtype=np.int64)
    length = np.hypot(*(pts[e[:, 0]] - pts[e[:, 1]]).T)
    g = sp.coo_matrix((length, (e[:, 0], e[:, 1])), shape=(nb, nb)).tocsr()
    mst = csgraph.minimum_spanning_tree(g).tocoo()
    tree = {(min(a, b), max(a, b)) for a, b in zip(mst.row.tolist(), mst.col.tolist())}
    if len(tree) != nb - 1:
        raise RuntimeError("Delaunay graph is not connected")
    # nearest-neighbour chords: buses in random order each take their
    # shortest Delaunay edge that is not yet a branch, round after round
    nbr = [[] for _ in range(nb)]
    for k in np.lexsort((e[:, 1], e[:, 0], length)).tolist():
        a, b = int(e[k, 0]), int(e[k, 1])
        nbr[a].append(b)
        nbr[b].append(a)
    have = set(tree)
    out = sorted(tree)
    need = nl - (nb - 1)
    ptr = [0] * nb
    while need > 0:
        added = 0
        for a in rng.permutation(nb).tolist():
            while ptr[a] < len(nbr[a]):
                b = nbr[a][ptr[a]]
                ptr[a] += 1
                key = (min(a, b), max(a, b))
                if key not in have:
                    have.add(key)
                    out.append(key)
                    need -= 1
                    added += 1
                    break
            if need == 0:
                break
        if added == 0:
            raise ValueError(f"cannot place {nl} branches on {nb} buses")
    return np.array(out, dtype=np.int64)


def _adjacency(nb, f, t):
    adj = [[] for _ in range(nb)]
    for a, b in zip(f.tolist(), t.tolist()):
        adj[a].append(b)
        adj[b].append(a)
    return [sorted(x) for x in adj]


def _bfs(adj, src, dist=None):
    """Hop distances from ``src``; with ``dist`` given, only improves it."""
    if dist is None:
        dist = np.full(len(adj), np.iinfo(np.int64).max, dtype=np.int64)
    parent = {src: -1}
    dist[src] = 0
    frontier = [src]
    while frontier:
        nxt = []
        for a in frontier:
            da = dist[a] + 1
            for b in adj[a]:
                if da < dist[b]:
                    dist[b] = da
                    parent[b] = a
                    nxt.append(b)
        frontier = nxt
    return dist, parent


def _spread_generators(rng, nb, f, t, ng):
    """Farthest-first generator placement; the first entry is the slack, the
    chosen bus nearest to the middle of a double-sweep diameter path."""
    adj = _adjacency(nb, f, t)
    prio = rng.random(nb)
    start = int(rng.integers(0, nb))
    chosen = [start]
    dist, _ = _bfs(adj, start)
    for _ in range(ng - 1):
        far = np.flatnonzero(dist == dist.max())
        k = int(far[np.argmax(prio[far])])
        chosen.append(k)
        _bfs(adj, k, dist)
    d0, _ = _bfs(adj, start)
    a = int(np.argmax(d0))
    d1, par = _bfs(adj, a)
    path = [int(np.argmax(d1))]
    while par[path[-1]] >= 0:
        path.append(par[path[-1]])
    dc, _ = _bfs(adj, path[len(path) // 2])
    chosen = np.array(chosen, dtype=np.int32)
    slack = int(np.argmin(dc[chosen]))
    return np.concatenate([chosen[slack:slack + 1], np.delete(chosen, slack)]).astype(np.int32)


def _nearest_generator(nb, f, t, gen_bus):
    """Index of the generator nearest to every bus in branch hops
    (multi-source breadth-first search, generators in drawn order)."""
    adj = _adjacency(nb, f, t)
    owner = np.full(nb, -1, dtype=np.int64)
    frontier = []
    for k, bus in enumerate(gen_bus.tolist()):
        owner[bus] = k
        frontier.append(bus)
    while frontier:
        nxt = []
        for a in frontier:
            for b in adj[a]:
                if owner[b] < 0:
                    owner[b] = owner[a]
                    nxt.append(b)
        frontier = nxt
    return owner


def _laplacian(nb, f, t, w):
    return sp.coo_matrix((np.concatenate([w, w, -w, -w]),
                          (np.concatenate([f, t, f, t]), np.concatenate([f, t, t, f]))),
                         shape=(nb, nb)).tocsc()


def _linear_flows(nb, f, t, x, inj, grounded):
    """Branch flows (phi_f - phi_t)/x of the linear network L phi = inj with
    phi = 0 on the ``grounded`` buses (L the 1/x-weighted Laplacian)."""
    L = _laplacian(nb, f, t, 1.0 / x)
    keep = np.setdiff1d(np.arange(nb), grounded)
    phi = np.zeros(nb)
    phi[keep] = spla.spsolve(L[keep][:, keep], inj[keep])
    return (phi[f] - phi[t]) / x


def make_grid(w: Workload) -> dict:
    """Draw the grid of workload ``w``.  Returns a dict of numpy arrays."""
    rng = np.random.default_rng(w.seed)
    nb, nl, ng = w.nb, w.nl, w.ng
    if ng < 1 or ng > nb:
        raise ValueError("need 1 <= n_g <= n_b")
    if w.topology == "tree_chords":
        e = _tree_chords(rng, nb, nl)
    elif w.topology == "geometric":
        e = _geometric(rng, nb, nl)
    else:
        raise ValueError(w.topology)
    flip = rng.random(nl) < 0.5
    f = np.where(flip, e[:, 1], e[:, 0]).astype(np.int32)
    t = np.where(flip, e[:, 0], e[:, 1]).astype(np.int32)
    r = rng.uniform(0.001, 0.05, nl)
    x = rng.uniform(0.01, 0.3, nl)
    b = rng.uniform(0.0, 0.1, nl)

    gen_bus = _spread_generators(rng, nb, f, t, ng)
    bus_type = np.full(nb, PQ, dtype=np.int32)
    bus_type[gen_bus] = PV
    bus_type[gen_bus[0]] = REF
    is_pq = bus_type == PQ

    sig = 0.5
    mu = np.log(0.3) - 0.5 * sig * sig
    pd = np.where(is_pq, rng.lognormal(mu, sig, nb), 0.0) * w.load_scale
    qd = pd * rng.uniform(0.1, 0.4, nb)

    c2 = rng.uniform(0.001, 0.05, ng)
    c1 = rng.uniform(10.0, 40.0, ng)
    c0 = np.zeros(ng)

    # dispatch: served load plus an estimate of the losses of the branches
    # around each generator (linear active flows with the slack grounded,
    # linear reactive flows of charging and reactive load with the
    # generator buses grounded; loss r (F_p^2 + F_q^2), half to the
    # generator serving each end)
    owner = _nearest_generator(nb, f, t, gen_bus)
    pinj = -pd.copy()
    np.add.at(pinj, gen_bus, np.bincount(owner, weights=pd, minlength=ng))
    fp = _linear_flows(nb, f, t, x, pinj, [int(gen_bus[0])])
    qinj = -qd.copy()
    np.add.at(qinj, f, 0.5 * b)
    np.add.at(qinj, t, 0.5 * b)
    fq = _linear_flows(nb, f, t, x, qinj, gen_bus)
    loss = r * (fp ** 2 + fq ** 2)
    pg0 = np.bincount(owner, weights=pd, minlength=ng) \
        + 0.5 * np.bincount(owner[f], weights=loss, minlength=ng) \
        + 0.5 * np.bincount(owner[t], weights=loss, minlength=ng)
    vg0 = np.ones(ng)
    pmin = np.zeros(ng)
    pmax = 2.0 * np.maximum(pg0, 0.1)
    qmax = 0.5 * pmax
    qmin = -qmax
    vmin = np.full(nb, 0.94)
    vmax = np.full(nb, 1.06)

    rate = 1.5 * np.maximum(np.hypot(fp, fq), 0.1)

    return dict(
        name=w.name, nb=nb, nl=nl, ng=ng, base_mva=BASE_MVA,
        bus_type=bus_type, br_from=f, br_to=t, br_r=r, br_x=x, br_b=b, br_rate=rate,
        gen_bus=gen_bus, c2=c2, c1=c1, c0=c0, vmin=vmin, vmax=vmax,
        pmin=pmin, pmax=pmax, qmin=qmin, qmax=qmax, pd=pd, qd=qd,
        vg0=vg0, pg0=pg0,
    )


def grid(name: str) -> dict:
    return make_grid(WORKLOADS[name])


def constraint_bounds(g: dict):
    """Bounds of the m operational constraints, in the order
    (h at from ends, h at to ends, v at PQ buses, p^g at REF, q^net at REF,
    q^net at PV buses), buses ascending.  h is the squared apparent flow, so
    its lower bound is 0 and its upper bound the squared rating."""
    bt = g["bus_type"]
    pq = np.flatnonzero(bt == PQ)
    pv = np.flatnonzero(bt == PV)
    genat = np.full(g["nb"], -1)
    genat[g["gen_bus"]] = np.arange(g["ng"])
    ref_gen = genat[np.flatnonzero(bt == REF)[0]]
    pv_gen = genat[pv]
    r2 = g["br_rate"] ** 2
    lo = np.concatenate([np.zeros(2 * g["nl"]), g["vmin"][pq], [g["pmin"][ref_gen]],
                         [g["qmin"][ref_gen]], g["qmin"][pv_gen]])
    hi = np.concatenate([r2, r2, g["vmax"][pq], [g["pmax"][ref_gen]],
                         [g["qmax"][ref_gen]], g["qmax"][pv_gen]])
    return lo, hi


def eval_point(g: dict, seed: Optional[int] = None, rho: float = 10.0,
               sigma: str = "random") -> dict:
    """AL evaluation point: penalty rho, multipliers y ~ U(-1, 1), slacks s
    uniform inside their bounds, objective scaling sigma_f = 1/(100 max c1)
    and constraint scalings sigma_c ~ U(0.5, 2) (or all ones)."""
    if seed is None:
        seed = WORKLOADS[g["name"]].seed + 1000 if g["name"] in WORKLOADS else 1000
    rng = np.random.default_rng(seed)
    lo, hi = constraint_bounds(g)
    m = lo.size
    y = rng.uniform(-1.0, 1.0, m)
    s = lo + rng.random(m) * (hi - lo)
    sigma_c = rng.uniform(0.5, 2.0, m) if sigma == "random" else np.ones(m)
    sigma_f = 1.0 / (BASE_MVA * float(np.max(g["c1"])))
    return dict(rho=float(rho), y=y, s=s, sigma_f=sigma_f, sigma_c=sigma_c, s_lo=lo, s_hi=hi)


def directions(nu: int, nbatch: int, seed: int) -> np.ndarray:
    """Random unit directions, shape [nu, nbatch] (columns normalised)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((nu, nbatch))
    return v / np.linalg.norm(v, axis=0, keepdims=True)


def tracking_factors(seed: int, steps: int, nb: int, sd: float = 0.02) -> np.ndarray:
    """Load factors 1 + N(0, sd) per step and bus, relative to the base loads."""
    rng = np.random.default_rng(seed + 5000)
    return 1.0 + sd * rng.standard_normal((steps, nb))


def load_drop_factors(nb: int, steps: int = 60, t_drop: int = 2, drop: float = 0.2) -> np.ndarray:
    """Load factors of the load-drop scenario: every load at its base value
    before step t_drop and at (1 - drop) times it from t_drop on (all loads
    drop together, as in the paper's real-time experiment)."""
    f = np.ones((steps, nb))
    f[t_drop:] = 1.0 - drop
    return f


def fingerprint(g: dict) -> str:
    h = hashlib.sha256()
    for k in sorted(g):
        v = g[k]
        if isinstance(v, np.ndarray):
            h.update(k.encode())
            h.update(np.ascontiguousarray(v).tobytes())
        else:
            h.update(f"{k}={v}".encode())
    return h.hexdigest()
