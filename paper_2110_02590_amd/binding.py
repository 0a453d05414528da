"""ctypes binding of the C ABI in include/rpf.h.

Argument marshalling only: every computation runs in the HIP library
(librpf.so, built in-tree for gfx950).  Device buffers are torch tensors on
the current device, float64 and contiguous; calls are enqueued on torch's
current stream.  The import fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpf.so")

RPF_OK, RPF_EINVAL, RPF_ENOMEM, RPF_EHIP, RPF_ESTATE, RPF_ESIZE = 0, -1, -2, -3, -4, -5
_NAMES = {RPF_EINVAL: "EINVAL", RPF_ENOMEM: "ENOMEM", RPF_EHIP: "EHIP", RPF_ESTATE: "ESTATE",
          RPF_ESIZE: "ESIZE"}


class RpfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rpf error {_NAMES.get(code, code)}: {msg}")
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("nb", ctypes.c_int32), ("nl", ctypes.c_int32), ("ng", ctypes.c_int32),
        ("base_mva", ctypes.c_double),
        ("bus_type", ctypes.c_void_p), ("br_from", ctypes.c_void_p), ("br_to", ctypes.c_void_p),
        ("br_r", ctypes.c_void_p), ("br_x", ctypes.c_void_p), ("br_b", ctypes.c_void_p),
        ("gen_bus", ctypes.c_void_p), ("c2", ctypes.c_void_p), ("c1", ctypes.c_void_p),
        ("c0", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64p, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double
        sig = {
            "rpf_grid_create": [vp, i32, vp],
            "rpf_grid_destroy": [vp],
            "rpf_dims": [vp, vp, vp, vp],
            "rpf_structure": [vp, i64p],
            "rpf_pf_solve": [vp, vp, vp, vp, vp, dbl, i32, vp, vp, vp],
            "rpf_al_objective": [vp, vp, vp, vp, vp, vp, vp, dbl, vp, vp, vp, vp],
            "rpf_reduced_gradient": [vp, vp, vp, vp, vp, vp, vp, dbl, vp, vp, vp, vp, vp],
            "rpf_reduced_hessian_batch": [vp, vp, i32, i32, vp, i32, vp],
            "rpf_reduced_hessian": [vp, vp, i32, vp],
            "rpf_reduced_derivatives": [vp, vp, vp, i32, vp],
            "rpf_factor_solve": [vp, i32, vp, vp, dbl, vp, vp, vp, vp],
            "rpf_factor_solve_noalloc": [i32, vp, vp, dbl, vp, vp, vp, vp],
            "rpf_presolve_info": [vp, i64p],
            "rpf_profile_enable": [vp, i32],
            "rpf_track_step": [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, dbl, vp, dbl, i32, i32, dbl, vp, vp],
            "rpf_track_step_qp": [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, dbl, vp, dbl, i32, i32, dbl,
                                  i32, dbl, i32, dbl, vp, vp, vp],
            "rpf_static_opf": [vp, vp, vp, vp, vp, vp, vp, dbl, vp, vp, vp, vp, vp, i32, i32, i32, dbl, i32, dbl,
                               vp, vp, vp, vp, vp],
            "rpf_qp_step": [vp, vp, vp, vp, vp, vp, vp, dbl, vp, dbl, vp, vp, vp, vp, i32, dbl, i32, vp, vp, vp,
                            vp, vp, vp, vp, vp, vp],
            "rpf_profile_read": [vp, vp, vp, i32],
            "rpf_profile_read_busy": [vp, vp, vp, vp, i32],
            "rpf_presolve_pattern": [vp, vp, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None if name == "rpf_grid_destroy" else ctypes.c_int
        L.rpf_last_error.argtypes = []
        L.rpf_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != RPF_OK:
        raise RpfError(rc, lib().rpf_last_error().decode())


NOALLOC_MAX_N = 4096   # RPF_NOALLOC_MAX_N


def factor_solve_noalloc(K, rhs, step, info, diag=None, delta=0.0):
    """rpf_factor_solve_noalloc: the dense step without a handle and without
    allocation.  K [n, n] (in: H, out: L in the lower triangle), rhs [n],
    step [n] (out), info int32 [1] (out), diag [n] or None: caller-owned
    device tensors."""
    torch = _torch()
    n = int(K.shape[0])
    dptr = _dev(diag, n, "diag") if diag is not None else None
    _check(lib().rpf_factor_solve_noalloc(n, _dev(K, n * n, "K"), dptr, float(delta), _dev(rhs, n, "rhs"),
                                          _dev(step, n, "step"), _dev(info, 1, "info", torch.int32),
                                          _stream()))


class _HostDesc:
    """Grid description with its host arrays kept alive."""

    def __init__(self, g: dict):
        self._keep = {
            "bus_type": np.ascontiguousarray(g["bus_type"], dtype=np.int32),
            "br_from": np.ascontiguousarray(g["br_from"], dtype=np.int32),
            "br_to": np.ascontiguousarray(g["br_to"], dtype=np.int32),
            "br_r": np.ascontiguousarray(g["br_r"], dtype=np.float64),
            "br_x": np.ascontiguousarray(g["br_x"], dtype=np.float64),
            "br_b": np.ascontiguousarray(g["br_b"], dtype=np.float64),
            "gen_bus": np.ascontiguousarray(g["gen_bus"], dtype=np.int32),
            "c2": np.ascontiguousarray(g["c2"], dtype=np.float64),
            "c1": np.ascontiguousarray(g["c1"], dtype=np.float64),
            "c0": np.ascontiguousarray(g["c0"], dtype=np.float64),
        }
        k = self._keep
        self.desc = GridDesc(int(g["nb"]), int(g["nl"]), int(g["ng"]), float(g["base_mva"]),
                             *[k[n].ctypes.data for n in ("bus_type", "br_from", "br_to", "br_r",
                                                          "br_x", "br_b", "gen_bus", "c2", "c1", "c0")])

    def ref(self):
        return ctypes.byref(self.desc)


def presolve_info(g: dict) -> dict:
    """Host-only presolve figures (no GPU needed)."""
    d = _HostDesc(g)
    out = np.zeros(20, dtype=np.int64)
    _check(lib().rpf_presolve_info(d.ref(), out.ctypes.data))
    keys = ["nx", "nu", "m", "nnz_jx", "nnz_lu", "nlev_lo", "nlev_up", "max_lu_row",
            "refactor_updates", "nnz_ju", "nnz_k", "nnz_g", "npacks", "ntop", "max_pack_levels",
            "top_levels", "max_tail_fwd_levels", "max_tail_bwd_levels", "tail_rows", "tail_max"]
    return dict(zip(keys, out.tolist()))


def presolve_pattern(g: dict):
    """(perm, lu_ptr, lu_col) of the symbolic LU, host-only."""
    info = presolve_info(g)
    d = _HostDesc(g)
    perm = np.zeros(info["nx"], dtype=np.int32)
    ptr = np.zeros(info["nx"] + 1, dtype=np.int32)
    col = np.zeros(info["nnz_lu"], dtype=np.int32)
    _check(lib().rpf_presolve_pattern(d.ref(), perm.ctypes.data, ptr.ctypes.data, col.ctypes.data))
    return perm, ptr, col


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, n: Optional[int] = None, name: str = "tensor", dtype=None):
    torch = _torch()
    dtype = dtype or torch.float64
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Grid:
    """A grid handle on the current HIP device (rpf_grid_create)."""

    def __init__(self, g: dict, max_batch: int = 256):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.g = g
        self._d = _HostDesc(g)
        h = ctypes.c_void_p()
        _check(lib().rpf_grid_create(self._d.ref(), int(max_batch), ctypes.byref(h)))
        self._h = h
        nx, nu, m = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().rpf_dims(h, ctypes.byref(nx), ctypes.byref(nu), ctypes.byref(m)))
        self.nx, self.nu, self.m = nx.value, nu.value, m.value
        self.nb = int(g["nb"])
        self.max_batch = int(max_batch)

    def close(self):
        if getattr(self, "_h", None):
            lib().rpf_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def structure(self) -> dict:
        out = np.zeros(10, dtype=np.int64)
        _check(lib().rpf_structure(self._h, out.ctypes.data))
        keys = ["nnz_jx", "nnz_lu", "nlev_lo", "nlev_up", "max_lu_row", "refactor_updates",
                "nnz_ju", "nnz_k", "nnz_g", "max_batch"]
        return dict(zip(keys, out.tolist()))

    PROF_CLASSES = ["pack_batch", "trsv_single", "refactor", "spmm", "dense", "top_batch"]

    def profile(self, enable: bool = True):
        _check(lib().rpf_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self, reset: bool = True, busy: bool = False) -> dict:
        """{class: (summed ms, launches)}, or with busy (summed ms, launches,
        ms of the union of the launch intervals)."""
        ms = np.zeros(len(self.PROF_CLASSES), dtype=np.float64)
        n = np.zeros(len(self.PROF_CLASSES), dtype=np.int64)
        if not busy:
            _check(lib().rpf_profile_read(self._h, ms.ctypes.data, n.ctypes.data, 1 if reset else 0))
            return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.PROF_CLASSES)}
        bz = np.zeros(len(self.PROF_CLASSES), dtype=np.float64)
        _check(lib().rpf_profile_read_busy(self._h, ms.ctypes.data, n.ctypes.data, bz.ctypes.data,
                                           1 if reset else 0))
        return {k: (float(ms[i]), int(n[i]), float(bz[i])) for i, k in enumerate(self.PROF_CLASSES)}

    def _empty(self, n, dtype=None):
        torch = _torch()
        return torch.empty(n, dtype=dtype or torch.float64, device="cuda")

    # --------------------------------------------------------------- calls
    def pf_solve(self, u, pd, qd, x, tol=1e-10, max_iter=20, status=None, resid=None):
        """Newton power flow; x is updated in place.  Returns (status, resid)
        device tensors: status = (steps, converged, tiny pivot: 1-based x
        index or 0)."""
        torch = _torch()
        status = self._empty(3, torch.int32) if status is None else status
        resid = self._empty(1) if resid is None else resid
        _check(lib().rpf_pf_solve(self._h, _dev(u, self.nu, "u"), _dev(pd, self.nb, "pd"),
                                  _dev(qd, self.nb, "qd"), _dev(x, self.nx, "x"), float(tol),
                                  int(max_iter), _dev(status, 3, "status", torch.int32),
                                  _dev(resid, 1, "resid"), _stream()))
        return status, resid

    def al_objective(self, x, u, pd, qd, s, y, rho, sigma, c=None):
        phi = self._empty(1)
        c = self._empty(self.m) if c is None else c
        _check(lib().rpf_al_objective(self._h, _dev(x, self.nx, "x"), _dev(u, self.nu, "u"),
                                      _dev(pd, self.nb, "pd"), _dev(qd, self.nb, "qd"),
                                      _dev(s, self.m, "s"), _dev(y, self.m, "y"), float(rho),
                                      _dev(sigma, 1 + self.m, "sigma"), _dev(phi, 1, "phi"),
                                      _dev(c, self.m, "c"), _stream()))
        return phi, c

    def reduced_gradient(self, x, u, pd, qd, s, y, rho, sigma, grad=None, lam=None, info=None):
        """Proposition 1.  Returns (grad, lambda); `info` (int32 device
        tensor [1]), when given, receives the tiny-pivot word of J_x's
        factorization at x (1-based x index, 0 = none)."""
        torch = _torch()
        grad = self._empty(self.nu) if grad is None else grad
        lam = self._empty(self.nx) if lam is None else lam
        iptr = _dev(info, 1, "info", torch.int32) if info is not None else None
        _check(lib().rpf_reduced_gradient(self._h, _dev(x, self.nx, "x"), _dev(u, self.nu, "u"),
                                          _dev(pd, self.nb, "pd"), _dev(qd, self.nb, "qd"),
                                          _dev(s, self.m, "s"), _dev(y, self.m, "y"), float(rho),
                                          _dev(sigma, 1 + self.m, "sigma"), _dev(grad, self.nu, "grad"),
                                          _dev(lam, self.nx, "lambda"), iptr, _stream()))
        return grad, lam

    def hessian_batch(self, V, HV=None):
        """H V for V of shape [n_u, nbatch] (row-major)."""
        if V.dim() != 2 or V.shape[0] != self.nu:
            raise ValueError("V must be [n_u, nbatch]")
        nbatch = V.shape[1]
        HV = self._empty(V.numel()).view(self.nu, nbatch) if HV is None else HV
        _check(lib().rpf_reduced_hessian_batch(self._h, _dev(V, None, "V"), int(nbatch), int(nbatch),
                                               _dev(HV, self.nu * nbatch, "HV"), int(nbatch),
                                               _stream()))
        return HV

    def reduced_hessian(self, batch=0, H=None):
        H = self._empty(self.nu * self.nu).view(self.nu, self.nu) if H is None else H
        _check(lib().rpf_reduced_hessian(self._h, _dev(H, self.nu * self.nu, "H"), int(batch), _stream()))
        return H

    def reduced_derivatives(self, batch=0, H=None, J=None, want_H=True, want_J=True):
        """Dense reduced Hessian [n_u, n_u] and reduced constraint Jacobian
        [m, n_u] at the cached point (either may be skipped)."""
        if want_H and H is None:
            H = self._empty(self.nu * self.nu).view(self.nu, self.nu)
        if want_J and J is None:
            J = self._empty(self.m * self.nu).view(self.m, self.nu)
        hp = _dev(H, self.nu * self.nu, "H") if want_H else None
        jp = _dev(J, self.m * self.nu, "J") if want_J else None
        _check(lib().rpf_reduced_derivatives(self._h, hp, jp, int(batch), _stream()))
        return (H if want_H else None), (J if want_J else None)

    def track_step(self, u, x, y, pd0, qd0, factor, s_lo, s_hi, u_lo, u_hi, rho, sigma, delta,
                   pf_iters=6, max_halvings=4, tol=1e-10, status=None):
        """One device-resident tracking update; u, x, y updated in place.
        Returns the status tensor (first PF converged, accepted halving,
        Cholesky info, Newton steps, tiny pivot of the factorization behind
        the gradient and Hessian)."""
        torch = _torch()
        status = self._empty(5, torch.int32) if status is None else status
        _check(lib().rpf_track_step(self._h, _dev(u, self.nu, "u"), _dev(x, self.nx, "x"), _dev(y, self.m, "y"),
                                    _dev(pd0, self.nb, "pd0"), _dev(qd0, self.nb, "qd0"),
                                    _dev(factor, self.nb, "factor"), _dev(s_lo, self.m, "s_lo"),
                                    _dev(s_hi, self.m, "s_hi"), _dev(u_lo, self.nu, "u_lo"),
                                    _dev(u_hi, self.nu, "u_hi"), float(rho), _dev(sigma, 1 + self.m, "sigma"),
                                    float(delta), int(pf_iters), int(max_halvings), float(tol),
                                    _dev(status, 5, "status", torch.int32), _stream()))
        return status

    def factor_solve(self, K, rhs, diag=None, delta=0.0):
        """In place: K (holding H) becomes L in its lower triangle.  Returns
        (step, info) device tensors."""
        torch = _torch()
        n = K.shape[0]
        step = self._empty(n)
        info = self._empty(1, torch.int32)
        dptr = _dev(diag, n, "diag") if diag is not None else None
        _check(lib().rpf_factor_solve(self._h, int(n), _dev(K, n * n, "K"), dptr, float(delta),
                                      _dev(rhs, n, "rhs"), _dev(step, n, "step"),
                                      _dev(info, 1, "info", torch.int32), _stream()))
        return step, info

    def qp_step(self, x, u, pd, qd, s, y, rho, sigma, delta, u_lo, u_hi, s_lo, s_hi, max_iter=50, tol=1e-10,
                batch=0, H=None, J=None, grad=None, dw=None, zw=None, kkt=None, wreg=None, status=None):
        """Exact real-time step: the bounded QP of eq. (qp_rto) in w = (u, s)
        at the point (x, u, s, y) by the device interior-point method.
        Returns a dict of device tensors: dw [n_u + m] (du, ds), zw [2 (n_u +
        m)] (z_l, z_u), kkt [1], wreg [1] (last regularisation), status int32
        [6] (iterations, converged, Cholesky info of the Schur complement,
        done word, tiny pivot word, factorization attempts), H [n_u, n_u]
        (symmetrised reduced Hessian), J [m, n_u], grad [n_u]."""
        torch = _torch()
        nu, m = self.nu, self.m
        n = nu + m
        H = self._empty(nu * nu).view(nu, nu) if H is None else H
        J = self._empty(m * nu).view(m, nu) if J is None else J
        grad = self._empty(nu) if grad is None else grad
        dw = self._empty(n) if dw is None else dw
        zw = self._empty(2 * n) if zw is None else zw
        kkt = self._empty(1) if kkt is None else kkt
        wreg = self._empty(1) if wreg is None else wreg
        status = self._empty(6, torch.int32) if status is None else status
        _check(lib().rpf_qp_step(self._h, _dev(x, self.nx, "x"), _dev(u, nu, "u"), _dev(pd, self.nb, "pd"),
                                 _dev(qd, self.nb, "qd"), _dev(s, m, "s"), _dev(y, m, "y"), float(rho),
                                 _dev(sigma, 1 + m, "sigma"), float(delta), _dev(u_lo, nu, "u_lo"),
                                 _dev(u_hi, nu, "u_hi"), _dev(s_lo, m, "s_lo"), _dev(s_hi, m, "s_hi"),
                                 int(max_iter), float(tol), int(batch), _dev(H, nu * nu, "H"),
                                 _dev(J, m * nu, "J"), _dev(grad, nu, "grad"), _dev(dw, n, "dw"),
                                 _dev(zw, 2 * n, "zw"), _dev(kkt, 1, "kkt"), _dev(wreg, 1, "wreg"),
                                 _dev(status, 6, "status", torch.int32), _stream()))
        return dict(dw=dw, zw=zw, kkt=kkt, wreg=wreg, status=status, H=H, J=J, grad=grad)

    def track_step_qp(self, u, s, x, y, pd0, qd0, factor, s_lo, s_hi, u_lo, u_hi, rho, sigma, delta,
                      pf_iters=6, max_halvings=4, tol=1e-10, qp_iters=50, qp_tol=1e-10, batch=0, J=None,
                      status=None, dispatch_scale=1.0):
        """One device-resident tracking update with the exact QP step; u, s,
        x, y updated in place (p_pv scaled by dispatch_scale first).
        Returns (status int32 [8], J)."""
        torch = _torch()
        J = self._empty(self.m * self.nu).view(self.m, self.nu) if J is None else J
        status = self._empty(8, torch.int32) if status is None else status
        _check(lib().rpf_track_step_qp(self._h, _dev(u, self.nu, "u"), _dev(s, self.m, "s"), _dev(x, self.nx, "x"),
                                       _dev(y, self.m, "y"), _dev(pd0, self.nb, "pd0"), _dev(qd0, self.nb, "qd0"),
                                       _dev(factor, self.nb, "factor"), _dev(s_lo, self.m, "s_lo"),
                                       _dev(s_hi, self.m, "s_hi"), _dev(u_lo, self.nu, "u_lo"),
                                       _dev(u_hi, self.nu, "u_hi"), float(rho), _dev(sigma, 1 + self.m, "sigma"),
                                       float(delta), int(pf_iters), int(max_halvings), float(tol), int(qp_iters),
                                       float(qp_tol), int(batch), float(dispatch_scale),
                                       _dev(J, self.m * self.nu, "J"),
                                       _dev(status, 8, "status", torch.int32), _stream()))
        return status, J

    def static_opf(self, x, u, s, y, pd, qd, rho, sigma, u_lo, u_hi, s_lo, s_hi, max_outer=30, max_inner=20,
                   qp_iters=60, qp_tol=1e-10, pf_iters=20, tol=1e-10, J=None):
        """Static OPF by the augmented-Lagrangian method; x, u, s, y updated
        in place.  Returns (history rows [n, 8] as a NumPy array: rho, QPs,
        theta, projected gradient, cost, multipliers updated, converged,
        L_rho; final rho)."""
        J = self._empty(self.m * self.nu).view(self.m, self.nu) if J is None else J
        hist = np.zeros((max_outer, 8), dtype=np.float64)
        nh = ctypes.c_int32(0)
        rho_out = ctypes.c_double(0.0)
        _check(lib().rpf_static_opf(self._h, _dev(x, self.nx, "x"), _dev(u, self.nu, "u"), _dev(s, self.m, "s"),
                                    _dev(y, self.m, "y"), _dev(pd, self.nb, "pd"), _dev(qd, self.nb, "qd"),
                                    float(rho), _dev(sigma, 1 + self.m, "sigma"), _dev(u_lo, self.nu, "u_lo"),
                                    _dev(u_hi, self.nu, "u_hi"), _dev(s_lo, self.m, "s_lo"),
                                    _dev(s_hi, self.m, "s_hi"), int(max_outer), int(max_inner), int(qp_iters),
                                    float(qp_tol), int(pf_iters), float(tol), _dev(J, self.m * self.nu, "J"),
                                    hist.ctypes.data, ctypes.byref(nh), ctypes.byref(rho_out), _stream()))
        return hist[:nh.value].copy(), rho_out.value
