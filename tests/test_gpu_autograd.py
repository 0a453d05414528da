"""The reduced AL objective as a torch.autograd.Function on the 2000-bus
workload: backward (adjoint kernels) against central finite differences of
phi, and the forward-over-reverse HVP (adjoint-adjoint kernels) against
finite differences of the gradient, on 20 seeded unit control directions;
both against the oracle."""
import numpy as np
import pytest

import gridgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_reduced_al_autograd_fd_and_oracle():
    from paper_2110_02590_amd import Problem
    from paper_2110_02590_amd.autograd import ReducedAL, ReducedALGrad, _Ctx
    print("[case] syn2000 autograd", flush=True)
    g = gridgen.grid("syn2000")
    ep = gridgen.eval_point(g)
    pr = Problem(g, max_batch=4)
    s, y, rho, sigma = pr.point(ep)
    C = _Ctx(pr, s, y, rho, sigma, tol=1e-12, max_iter=30)
    u = pr.u0.clone().requires_grad_(True)
    phi = ReducedAL.apply(u, C)
    (grad,) = torch.autograd.grad(phi, u, create_graph=True)
    D = torch.tensor(gridgen.directions(pr.nu, 20, 2020), device="cuda")
    h = 1e-5

    def phi_at(v):
        return float(ReducedAL.apply(v.detach(), C))

    def grad_at(v):
        x = C.solve(v.detach())
        return ReducedALGrad.apply(v.detach(), x, C)

    M = oracle.Model(g)
    uo = M.u_from_setpoints(g["vg0"], g["pg0"])
    P = oracle.Point.from_dict(ep)
    xo = oracle.solve_pf(M, uo, g["pd"], g["qd"], tol=1e-12).x
    go, lo = oracle.reduced_gradient(M, xo, uo, g["pd"], g["qd"], P)
    Ho = oracle.reduced_hessian(M, xo, uo, g["pd"], g["qd"], P, lo)
    gg = grad.detach().cpu().numpy()
    assert np.linalg.norm(gg - go) <= 1e-10 * np.linalg.norm(go)

    for k in range(20):
        d = D[:, k].contiguous()
        gd = float(grad.detach() @ d)
        fd = (phi_at(u + h * d) - phi_at(u - h * d)) / (2 * h)
        assert abs(fd - gd) <= 1e-5 * max(1.0, abs(gd)), (k, fd, gd)
        (hv,) = torch.autograd.grad(grad, u, grad_outputs=d, retain_graph=True)
        fdg = (grad_at(u + h * d) - grad_at(u - h * d)) / (2 * h)
        hvn = hv.detach().cpu().numpy()
        assert np.linalg.norm(hvn - fdg.cpu().numpy()) <= 1e-5 * max(1.0, np.linalg.norm(hvn)), k
        ho = Ho @ d.cpu().numpy()
        assert np.linalg.norm(hvn - ho) <= 1e-9 * np.linalg.norm(ho), k
