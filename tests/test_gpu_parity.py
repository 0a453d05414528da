"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Tolerances: x 1e-12, phi and c 1e-12, gradient and
lambda 1e-10, reduced Hessian 1e-9 (relative Frobenius), Cholesky factor
and step 1e-9 relative."""
import numpy as np
import pytest

import gridgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


class Case:
    def __init__(self, name, max_batch=256):
        from paper_2110_02590_amd import Problem
        print(f"[case] {name} max_batch={max_batch}", flush=True)
        self.name = name
        self.g = gridgen.grid(name)
        self.ep = gridgen.eval_point(self.g)
        self.pr = Problem(self.g, max_batch=max_batch)
        self.M = oracle.Model(self.g)
        self.u = self.M.u_from_setpoints(self.g["vg0"], self.g["pg0"])
        self.P = oracle.Point.from_dict(self.ep)
        self._o = _ORACLE.setdefault(name, {})   # oracle results shared by a grid's handles

    def oracle(self, what):
        if what not in self._o:
            g, M, u, P = self.g, self.M, self.u, self.P
            if what == "pf":
                self._o[what] = oracle.solve_pf(M, u, g["pd"], g["qd"])
            elif what == "grad":
                x = self.oracle("pf").x
                self._o[what] = oracle.reduced_gradient(M, x, u, g["pd"], g["qd"], P)
            elif what == "H":
                x = self.oracle("pf").x
                self._o[what] = oracle.reduced_hessian(M, x, u, g["pd"], g["qd"], P, self.oracle("grad")[1])
        return self._o[what]

    def gpu_point(self):
        pr = self.pr
        x = pr.flat_x()
        st, res = pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
        s, y, rho, sigma = pr.point(self.ep)
        grad, lam = pr.grid.reduced_gradient(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma)
        torch.cuda.synchronize()
        return x, st, res, grad, lam


_cases = {}
_ORACLE = {}


def case(name, max_batch=256):
    key = (name, max_batch)
    if key not in _cases:
        _cases[key] = Case(name, max_batch)
    return _cases[key]


SMALL = ["tiny10", "syn300", "syn2000"]


@pytest.mark.parametrize("name", SMALL + ["syn9241"])
def test_power_flow(name):
    c = case(name)
    pr = c.pr
    x = pr.flat_x()
    st, res = pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
    torch.cuda.synchronize()
    o = c.oracle("pf")
    assert int(st[1]) == 1 and float(res) < 1e-10 and int(st[2]) == 0
    assert abs(int(st[0]) - o.iters) <= 1
    assert _rel(x.cpu().numpy(), o.x) < 1e-12


@pytest.mark.parametrize("name", SMALL + ["syn9241"])
def test_al_objective(name):
    c = case(name)
    pr = c.pr
    x = torch.tensor(c.oracle("pf").x, device="cuda")
    s, y, rho, sigma = pr.point(c.ep)
    phi, cv = pr.grid.al_objective(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma)
    torch.cuda.synchronize()
    phio, co = oracle.al_objective(c.M, c.oracle("pf").x, c.u, c.g["pd"], c.g["qd"], c.P)
    assert abs(float(phi) - phio) <= 1e-12 * abs(phio)
    assert _rel(cv.cpu().numpy(), co) < 1e-12


@pytest.mark.parametrize("name", SMALL + ["syn9241"])
def test_reduced_gradient(name):
    c = case(name)
    x, st, res, grad, lam = c.gpu_point()
    go, lo = c.oracle("grad")
    assert _rel(grad.cpu().numpy(), go) < 1e-10
    assert _rel(lam.cpu().numpy(), lo) < 1e-10


@pytest.mark.parametrize("name,batch", [("tiny10", 0), ("syn300", 64), ("syn300", 16), ("syn2000", 256)])
def test_reduced_hessian_full(name, batch):
    c = case(name)
    c.gpu_point()
    H = c.pr.grid.reduced_hessian(batch=batch)
    torch.cuda.synchronize()
    Ho = c.oracle("H")
    Hg = H.cpu().numpy()
    assert _rel(Hg, Ho) < 1e-9
    assert np.linalg.norm(Hg - Hg.T) <= 1e-11 * np.linalg.norm(Hg)


def test_batch_width_one_equals_batched():
    c = case("syn300")
    c.gpu_point()
    pr = c.pr
    V = torch.tensor(gridgen.directions(pr.nu, 5, 2005), device="cuda")
    HV = pr.grid.hessian_batch(V.contiguous())
    cols = [pr.grid.hessian_batch(V[:, k:k + 1].contiguous()) for k in range(5)]
    torch.cuda.synchronize()
    one = torch.cat(cols, dim=1).cpu().numpy()
    assert _rel(one, HV.cpu().numpy()) < 1e-13
    Ho = c.oracle("H")
    assert _rel(HV.cpu().numpy(), Ho @ V.cpu().numpy()) < 1e-9


def test_random_directions_linear():
    c = case("syn2000")
    c.gpu_point()
    pr = c.pr
    V = torch.tensor(gridgen.directions(pr.nu, 33, 2002), device="cuda")   # ragged width
    HV = pr.grid.hessian_batch(V)
    W = (2.0 * V[:, :7] - 0.5 * V[:, 7:14]).contiguous()
    HW = pr.grid.hessian_batch(W)
    torch.cuda.synchronize()
    lin = 2.0 * HV[:, :7] - 0.5 * HV[:, 7:14]
    assert _rel(HW.cpu().numpy(), lin.cpu().numpy()) < 1e-12
    assert _rel(HV.cpu().numpy(), c.oracle("H") @ V.cpu().numpy()) < 1e-9


@pytest.mark.parametrize("max_batch", [512, 1024, 2889])
def test_largest_workload_full_hessian(max_batch):
    """9241-bus grid: all 2889 columns of the reduced Hessian against the
    oracle's Schur form Z^T (grad^2 l) Z within 1e-9 relative Frobenius error
    (Proposition 2).  2889 is the benchmark's launch configuration (one batch
    of every column); 1024 gives three batches, the last one 841 columns, and
    512 six, the last one 329 columns.  Every column is also compared on
    its own, so that no batch can hide behind the whole matrix's norm."""
    c = case("syn9241", max_batch=max_batch)
    c.gpu_point()
    H = c.pr.grid.reduced_hessian(batch=max_batch)
    torch.cuda.synchronize()
    Hg = H.cpu().numpy()
    Ho = c.oracle("H")
    assert _rel(Hg, Ho) < 1e-9
    colerr = np.linalg.norm(Hg - Ho, axis=0) / np.maximum(np.linalg.norm(Ho, axis=0), 1e-300)
    assert colerr.max() < 1e-8, (int(colerr.argmax()), float(colerr.max()))
    for j0 in range(0, c.M.nu, max_batch):
        blk = slice(j0, min(j0 + max_batch, c.M.nu))
        assert _rel(Hg[:, blk], Ho[:, blk]) < 1e-9, j0
    assert np.linalg.norm(Hg - Hg.T) <= 1e-11 * np.linalg.norm(Hg)


@pytest.mark.parametrize("name,batch", [("tiny10", 0), ("syn300", 64), ("syn2000", 256)])
def test_reduced_jacobian(name, batch):
    """grad_u c = (d_x c) Z + d_u c from the V = I batches (Section III-C)
    against the oracle's direct sensitivities, and the Hessian of the same
    call equal to rpf_reduced_hessian's bit for bit."""
    c = case(name)
    c.gpu_point()
    H, J = c.pr.grid.reduced_derivatives(batch=batch)
    H2 = c.pr.grid.reduced_hessian(batch=batch)
    _, J2 = c.pr.grid.reduced_derivatives(batch=batch, want_H=False)
    torch.cuda.synchronize()
    Jo = oracle.reduced_jacobian(c.M, c.oracle("pf").x, c.u)
    assert _rel(J.cpu().numpy(), Jo) < 1e-9
    assert torch.equal(H, H2) and torch.equal(J, J2)


def test_reduced_jacobian_largest_workload():
    """The 41340 x 2889 reduced Jacobian of the 9241-bus grid in the
    benchmark's launch configuration (one batch of all 2889 columns),
    together with the Hessian, against the oracle; per constraint block
    (line flows, voltages, slack and PV reactive rows) as well."""
    c = case("syn9241", max_batch=2889)
    c.gpu_point()
    H, J = c.pr.grid.reduced_derivatives(batch=2889)
    torch.cuda.synchronize()
    Jg = J.cpu().numpy()
    del J
    Jo = oracle.reduced_jacobian(c.M, c.oracle("pf").x, c.u)
    assert _rel(Jg, Jo) < 1e-9
    nl, npq = c.M.nl, c.M.npq
    for a, b in [(0, 2 * nl), (2 * nl, 2 * nl + npq), (2 * nl + npq, c.M.m)]:
        assert _rel(Jg[a:b], Jo[a:b]) < 1e-9, (a, b)
    assert _rel(H.cpu().numpy(), c.oracle("H")) < 1e-9


def test_singular_jacobian_is_reported():
    """A state with v = 0 at a PQ bus makes the theta column of that bus in
    J_x exactly zero (every term of dS/dtheta_i carries v_i), so the static
    pivot of theta_i is zero.  The power flow must stop unconverged and
    report that pivot; the reduced gradient reports it in its info word
    (Section V-A.1: refactorization with the presolve's pivots)."""
    c = case("syn300", max_batch=64)
    pr = c.pr
    M = c.M
    k = 5
    x0 = c.oracle("pf").x.copy()
    x0[M.npv + M.npq + k] = 0.0
    ith = M.npv + k                       # x index of theta at that bus
    Jx, _ = M.jacobians(x0, c.u)
    assert abs(Jx.tocsc()[:, ith]).sum() == 0.0
    x = torch.tensor(x0, device="cuda")
    st, res = pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x, max_iter=10)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert st[1] == 0 and st[2] == ith + 1, st
    assert not np.isfinite(float(res)) or float(res) >= 1e-10
    s, y, rho, sigma = pr.point(c.ep)
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    pr.grid.reduced_gradient(torch.tensor(x0, device="cuda"), pr.u0, pr.pd, pr.qd, s, y, rho, sigma, info=info)
    torch.cuda.synchronize()
    assert int(info) == ith + 1
    # a regular point right after: the words start clear again
    x = pr.flat_x()
    st, res = pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
    pr.grid.reduced_gradient(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma, info=info)
    torch.cuda.synchronize()
    assert int(st[1]) == 1 and int(st[2]) == 0 and int(info) == 0
    assert _rel(x.cpu().numpy(), c.oracle("pf").x) < 1e-12


def test_factor_solve_matches_lapack():
    c = case("syn300")
    x, st, res, grad, lam = c.gpu_point()
    H = c.pr.grid.reduced_hessian(batch=64)
    Hn = H.cpu().numpy()
    delta = oracle.delta_ladder(Hn)
    delta = max(delta, 1.0)
    diag = torch.tensor(np.linspace(0.1, 0.5, c.pr.nu), device="cuda")
    K = H.clone()
    step, info = c.pr.grid.factor_solve(K, grad, diag=diag, delta=delta)
    torch.cuda.synchronize()
    Lo, io, so = oracle.factor_solve(Hn, diag.cpu().numpy(), delta, grad.cpu().numpy())
    assert int(info) == 0 and io == 0
    Lg = np.tril(K.cpu().numpy())
    assert _rel(Lg, Lo) < 1e-11
    assert _rel(step.cpu().numpy(), so) < 1e-9


def test_factor_solve_full_size():
    """The Cholesky step at the 9241-bus grid's n_u = 2889 (45 blocks of 64,
    ragged last block), shifted as the benchmark shifts it, against the
    oracle's column Cholesky and triangular solves."""
    c = case("syn9241", max_batch=512)
    x, st, res, grad, lam = c.gpu_point()
    H = c.pr.grid.reduced_hessian(batch=512)
    Hn = H.cpu().numpy()
    delta = 10.0 * max(oracle.delta_ladder(Hn), 1e-8 * max(1.0, float(np.abs(np.diag(Hn)).max())))
    K = H.clone()
    step, info = c.pr.grid.factor_solve(K, grad, delta=delta)
    torch.cuda.synchronize()
    Lo, io, so = oracle.factor_solve(Hn, None, delta, grad.cpu().numpy())
    assert int(info) == 0 and io == 0
    assert _rel(np.tril(K.cpu().numpy()), Lo) < 1e-11
    assert _rel(step.cpu().numpy(), so) < 1e-9


@pytest.mark.parametrize("n", [1, 63, 64, 65, 128, 129, 200, 191 + 64 * 3, 700, 1500])
def test_factor_sizes_match_oracle(n):
    """The blocked dense Cholesky and its triangular solves at orders from
    one 64-column block to 24 blocks (full and ragged last blocks), on
    seeded SPD matrices, against the oracle's column Cholesky and
    triangular solves; the upper triangle is not touched."""
    c = case("syn9241", max_batch=512)
    print(f"[case] factor n={n}", flush=True)
    rng = np.random.default_rng(1000 + n)
    A = rng.standard_normal((n, n))
    K = A @ A.T / n + np.eye(n)
    K = 0.5 * (K + K.T)                  # exactly symmetric
    Kt = torch.tensor(K, device="cuda")
    rhs = rng.standard_normal(n)
    step, info = c.pr.grid.factor_solve(Kt, torch.tensor(rhs, device="cuda"))
    torch.cuda.synchronize()
    Lo, io, so = oracle.factor_solve(K, None, 0.0, rhs)
    assert int(info) == 0 and io == 0
    assert _rel(np.tril(Kt.cpu().numpy()), Lo) < 1e-12
    assert _rel(step.cpu().numpy(), so) < 1e-11
    # the upper triangle is left as it was
    iu = np.triu_indices(n, 1)
    assert np.array_equal(Kt.cpu().numpy()[iu], K[iu])


def test_concurrent_batches_match_one_stream():
    """Batches on three handle-owned streams (RPF_HVP_STREAMS=3) give the
    same reduced Hessian, bit for bit, as one stream (each batch has its own
    workspace; no floating-point atomics)."""
    import os
    from paper_2110_02590_amd import Problem
    g = gridgen.grid("syn2000")
    ep = gridgen.eval_point(g)
    out = []
    for streams in ("1", "3"):
        old = os.environ.pop("RPF_HVP_STREAMS", None)
        if streams:
            os.environ["RPF_HVP_STREAMS"] = streams
        try:
            pr = Problem(g, max_batch=512)
        finally:
            os.environ.pop("RPF_HVP_STREAMS", None)
            if old is not None:
                os.environ["RPF_HVP_STREAMS"] = old
        x = pr.flat_x()
        pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
        s, y, rho, sigma = pr.point(ep)
        pr.grid.reduced_gradient(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma)
        H = pr.grid.reduced_hessian(batch=96)   # several batches, ragged last
        torch.cuda.synchronize()
        out.append(H.cpu().numpy())
        pr.grid.close()
    assert np.array_equal(out[0], out[1])


def test_factor_reports_first_bad_pivot():
    c = case("tiny10")
    n = 100
    rng = np.random.default_rng(4)
    A = rng.standard_normal((n, n)) * 1e-3
    K = np.diag(np.full(n, 2.0)) + A + A.T
    K[70, 70] = -1.0
    Kt = torch.tensor(K, device="cuda")
    rhs = torch.ones(n, dtype=torch.float64, device="cuda")
    grid = c.pr.grid
    from paper_2110_02590_amd import RpfError
    with pytest.raises(RpfError):
        grid.factor_solve(Kt, rhs)          # n above n_u of this grid
    big = case("syn300")
    step, info = big.pr.grid.factor_solve(Kt, rhs)
    torch.cuda.synchronize()
    _, io = oracle.cholesky_lower(K)
    assert int(info) == io == 71


def test_call_order_and_size_errors():
    from paper_2110_02590_amd import Problem, RpfError
    from paper_2110_02590_amd.binding import RPF_ESIZE, RPF_ESTATE
    g = gridgen.grid("tiny10")
    pr = Problem(g, max_batch=4)
    V = torch.zeros((pr.nu, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(RpfError) as e:
        pr.grid.hessian_batch(V)
    assert e.value.code == RPF_ESTATE
    x = pr.flat_x()
    pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
    s, y, rho, sigma = pr.point(gridgen.eval_point(g))
    pr.grid.reduced_gradient(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma)
    V5 = torch.zeros((pr.nu, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(RpfError) as e:
        pr.grid.hessian_batch(V5)
    assert e.value.code == RPF_ESIZE


def test_power_flow_divergence_is_reported():
    c = case("syn300")
    pr = c.pr
    x = pr.flat_x()
    st, res = pr.grid.pf_solve(pr.u0, pr.pd * 8.0, pr.qd * 8.0, x, max_iter=8)
    torch.cuda.synchronize()
    o = oracle.solve_pf(c.M, c.u, c.g["pd"] * 8.0, c.g["qd"] * 8.0, max_iter=8, raise_on_fail=False)
    assert int(st[1]) == 0 and not o.converged


def test_trace_lines(capfd):
    """RPF_TRACE: each compute call on a handle created with it set writes
    one JSON line with its device time once it has completed (the last ones
    when the handle is destroyed); a handle created without it writes
    nothing."""
    import json
    import os
    from paper_2110_02590_amd import Problem
    g = gridgen.grid("syn300")
    ep = gridgen.eval_point(g)
    old = os.environ.get("RPF_TRACE")
    os.environ["RPF_TRACE"] = "1"
    try:
        pr = Problem(g, max_batch=64)
    finally:
        if old is None:
            os.environ.pop("RPF_TRACE")
        else:
            os.environ["RPF_TRACE"] = old
    x = pr.flat_x()
    pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
    s, y, rho, sigma = pr.point(ep)
    pr.grid.reduced_gradient(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma)
    pr.grid.reduced_hessian(batch=64)
    torch.cuda.synchronize()
    pr.grid.close()
    err = capfd.readouterr().err
    recs = [json.loads(l) for l in err.splitlines() if l.startswith('{"rpf_trace"')]
    names = [r["rpf_trace"] for r in recs]
    assert names == ["rpf_pf_solve", "rpf_reduced_gradient", "rpf_reduced_derivatives"], names
    assert all(r["ms"] > 0.0 for r in recs)
    assert recs[2]["arg"] == 64
    quiet = Problem(g, max_batch=64)
    quiet.grid.pf_solve(quiet.u0, quiet.pd, quiet.qd, quiet.flat_x())
    torch.cuda.synchronize()
    quiet.grid.close()
    assert '"rpf_trace"' not in capfd.readouterr().err


@pytest.mark.parametrize("env", [
    {"RPF_PACK_TW": "8", "RPF_PACK_SV": "1"},
    {"RPF_PACK_TW": "8", "RPF_PACK_SV": "0"},
    {"RPF_TAIL_MAX": "0"},
    {"RPF_TAIL_MAX": "32"},
    {"RPF_SUBTREE_MAX": "256"},
    {"RPF_SUBTREE_MAX": "512", "RPF_PACK_THREADS": "512"},
    {"RPF_SUBTREE_MAX": "1536"},
    {"RPF_SUBTREE_MAX": "1792"},
    {"RPF_SUBTREE_MAX": "2048"},
], ids=lambda e: ",".join(f"{k}={v}" for k, v in e.items()))
def test_solve_variants_match_default(env):
    """The other batched-solve variants -- 8-column tiles with and without
    staged factor values, packs without dense tails or with small ones,
    smaller packs (also with 512-thread workgroups), and larger packs (past the LDS-resident refactorization:
    its global-memory version; at 1792 rows the largest pack, 1769 rows with
    8757 entries and a level of 300 rows, takes the single right-hand side
    solve's second staging passes and a level of two passes; at 2048 that
    solve's level records no longer fit in LDS and the solve without them
    runs) -- give the default handle's power flow,
    gradient and full reduced Hessian (syn2000, 1e-10 relative; the
    orderings differ, so not bit for bit).  A pack too large for any of the
    solves is refused at handle creation with an error."""
    import os
    from paper_2110_02590_amd import Problem
    print(f"[case] solve variant {env}", flush=True)
    g = gridgen.grid("syn2000")
    ep = gridgen.eval_point(g)

    from paper_2110_02590_amd import RpfError

    def run(extra):
        old = {k: os.environ.get(k) for k in extra}
        os.environ.update(extra)
        try:
            pr = Problem(g, max_batch=256)
        except RpfError as e:
            assert "does not fit in LDS" in str(e)
            pytest.skip(f"refused at creation: {e}")
        finally:
            for k, v in old.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        x = pr.flat_x()
        st, _ = pr.grid.pf_solve(pr.u0, pr.pd, pr.qd, x)
        s, y, rho, sigma = pr.point(ep)
        grad, _ = pr.grid.reduced_gradient(x, pr.u0, pr.pd, pr.qd, s, y, rho, sigma)
        H = pr.grid.reduced_hessian(batch=256)
        torch.cuda.synchronize()
        out = (st.cpu().numpy(), x.cpu().numpy(), grad.cpu().numpy(), H.cpu().numpy())
        pr.grid.close()
        return out

    st0, x0, g0, H0 = run({})
    st1, x1, g1, H1 = run(env)
    assert st1[1] == 1 and st1[0] == st0[0], (st0, st1)
    assert _rel(x1, x0) < 1e-12
    assert _rel(g1, g0) < 1e-10
    assert _rel(H1, H0) < 1e-10
