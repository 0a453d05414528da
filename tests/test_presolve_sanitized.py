"""The host presolve under AddressSanitizer and UndefinedBehaviorSanitizer:
presolve.cpp and a checking driver (tests/presolve_check.cpp) built with
g++ for the host only, run on each synthetic grid.  The driver validates
every solve schedule (a row reads only rows of earlier levels, or of its
pack's dense tail in the backward program) and the staged entries of each
pack program; its statistics must equal the library's own presolve
(rpf_presolve_info).  Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import gridgen

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
GRIDS = ["tiny10", "syn300", "syn2000", "syn9241"]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    out = str(tmp_path_factory.mktemp("presolve_san") / "presolve_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(HERE, "presolve_check.cpp"),
           os.path.join(ROOT, "paper_2110_02590_amd", "csrc", "presolve.cpp"), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return out


def _write_grid(g, path):
    with open(path, "wb") as f:
        np.array([g["nb"], g["nl"], g["ng"]], dtype="<i4").tofile(f)
        np.array([g.get("base_mva", 100.0)], dtype="<f8").tofile(f)
        for k in ("bus_type", "br_from", "br_to", "gen_bus"):
            np.ascontiguousarray(g[k], dtype="<i4").tofile(f)
        for k in ("br_r", "br_x", "br_b", "c2", "c1", "c0"):
            np.ascontiguousarray(g[k], dtype="<f8").tofile(f)


@pytest.mark.parametrize("name", GRIDS)
def test_presolve_under_sanitizers(checker, name, tmp_path):
    from paper_2110_02590_amd import binding
    g = gridgen.grid(name)
    path = str(tmp_path / f"{name}.bin")
    _write_grid(g, path)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env.pop("RPF_SUBTREE_MAX", None)
    env.pop("RPF_TAIL_MAX", None)
    res = subprocess.run([checker, path], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
    got = [int(v) for v in res.stdout.split()]
    old = {k: os.environ.pop(k) for k in ("RPF_SUBTREE_MAX", "RPF_TAIL_MAX") if k in os.environ}
    try:
        info = binding.presolve_info(g)
    finally:
        os.environ.update(old)
    want = [info[k] for k in ("nx", "nu", "m", "nnz_lu", "nlev_lo", "nlev_up", "npacks", "ntop",
                              "max_tail_fwd_levels", "max_tail_bwd_levels", "tail_rows", "refactor_updates")]
    assert got == want, (got, want)
