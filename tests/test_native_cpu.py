"""Host-side checks of the native library (no GPU): it loads, exports every
symbol declared in include/rpf.h, and its presolve (index maps, ordering,
symbolic LU) is right."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg as sla

import gridgen
import oracle
from tests import smallgrids

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "rpf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rpf_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2110_02590_amd import binding
    L = ctypes.CDLL(binding.LIB_PATH)
    syms = _declared_symbols()
    assert len(syms) >= 10
    for s in syms:
        assert hasattr(L, s), s


@pytest.mark.parametrize("name", ["tiny10", "syn300", "syn2000"])
def test_presolve_dimensions_match_oracle(name):
    from paper_2110_02590_amd import presolve_info
    g = gridgen.grid(name)
    info = presolve_info(g)
    M = oracle.Model(g)
    assert (info["nx"], info["nu"], info["m"]) == (M.nx, M.nu, M.m)


def test_presolve_table1_dimensions():
    from paper_2110_02590_amd import presolve_info
    w = gridgen.Workload("t", 9241, 16049, 1445, 5, "geometric")
    info = presolve_info(gridgen.make_grid(w))
    assert (info["nx"], info["nu"], info["m"]) == (17036, 2889, 41340)


@pytest.mark.parametrize("name", ["tiny10", "syn300"])
def test_symbolic_lu_contains_numeric_fill(name):
    """Factor the oracle's J_x without pivoting in the library's order: the
    factors' nonzeros lie inside the symbolic pattern and pivots are sound."""
    from paper_2110_02590_amd import presolve_pattern
    g = gridgen.grid(name)
    M = oracle.Model(g)
    u = M.u_from_setpoints(g["vg0"], g["pg0"])
    x = oracle.solve_pf(M, u, g["pd"], g["qd"]).x
    Jx = M.jacobians(x, u)[0].toarray()
    perm, ptr, col = presolve_pattern(g)
    assert sorted(perm.tolist()) == list(range(M.nx))
    A = Jx[np.ix_(perm, perm)]
    n = A.shape[0]
    pat = np.zeros((n, n), bool)
    for i in range(n):
        pat[i, col[ptr[i]:ptr[i + 1]]] = True
        assert np.all(np.diff(col[ptr[i]:ptr[i + 1]]) > 0)
    assert np.all(pat[A != 0])
    # right-looking LU without pivoting
    LU = A.copy()
    for k in range(n):
        assert abs(LU[k, k]) > 1e-8 * np.abs(LU[k]).max()
        LU[k + 1:, k] /= LU[k, k]
        LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k + 1:])
    assert np.all(pat[np.abs(LU) > 1e-300])
    P, L, U = sla.lu(A)
    # reconstruct from the no-pivot factors
    Lf = np.tril(LU, -1) + np.eye(n)
    Uf = np.triu(LU)
    assert np.linalg.norm(Lf @ Uf - A) <= 1e-12 * np.linalg.norm(A)


def test_presolve_rejects_bad_grids():
    from paper_2110_02590_amd import RpfError, presolve_info
    g = smallgrids.three_bus()
    bad = dict(g, bus_type=np.array([2, 2, 0], np.int32))
    with pytest.raises(RpfError):
        presolve_info(bad)
    bad = dict(g, gen_bus=np.array([0, 2], np.int32))        # generator at a PQ bus
    with pytest.raises(RpfError):
        presolve_info(bad)
    bad = dict(g, br_to=np.array([1, 2, 2], np.int32))       # branch 2 -> 2
    with pytest.raises(RpfError):
        presolve_info(bad)


def test_profile_class_count_matches_header():
    """The binding's timing arrays are as long as the library writes."""
    import re
    from paper_2110_02590_amd.binding import Grid
    txt = open(os.path.join(ROOT, "include", "rpf.h")).read()
    n = int(re.search(r"#define\s+RPF_PROF_CLASSES\s+(\d+)", txt).group(1))
    assert len(Grid.PROF_CLASSES) == n
