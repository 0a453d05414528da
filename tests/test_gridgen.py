"""The input generator is deterministic and produces the stated shapes."""
import numpy as np
import pytest

import gridgen


@pytest.mark.parametrize("name", ["tiny10", "syn300", "syn2000"])
def test_deterministic(name):
    assert gridgen.fingerprint(gridgen.grid(name)) == gridgen.fingerprint(gridgen.grid(name))


@pytest.mark.parametrize("name", ["tiny10", "syn300", "syn2000"])
def test_shapes_and_types(name):
    w = gridgen.WORKLOADS[name]
    g = gridgen.grid(name)
    assert g["nb"] == w.nb and g["br_from"].size == w.nl and g["gen_bus"].size == w.ng
    bt = g["bus_type"]
    assert (bt == gridgen.REF).sum() == 1
    assert (bt == gridgen.PV).sum() == w.ng - 1
    assert bt[g["gen_bus"][0]] == gridgen.REF
    assert np.all(g["br_from"] != g["br_to"])
    pairs = {(min(a, b), max(a, b)) for a, b in zip(g["br_from"], g["br_to"])}
    assert len(pairs) == w.nl                       # no parallel branches
    assert np.all(g["pd"][bt != gridgen.PQ] == 0)   # loads at PQ buses only
    assert np.all((g["br_r"] >= 0.001) & (g["br_r"] <= 0.05))
    assert np.all((g["br_x"] >= 0.01) & (g["br_x"] <= 0.3))


def test_eval_point_inside_bounds():
    g = gridgen.grid("syn300")
    p = gridgen.eval_point(g)
    lo, hi = gridgen.constraint_bounds(g)
    m = 2 * g["nl"] + int((g["bus_type"] == 0).sum()) + int((g["bus_type"] == 1).sum()) + 2
    assert p["y"].size == m and np.all((p["s"] >= lo) & (p["s"] <= hi))


def test_directions_unit_columns():
    V = gridgen.directions(17, 5, 3)
    np.testing.assert_allclose(np.linalg.norm(V, axis=0), 1.0, rtol=1e-14)


def test_fingerprints_match_stored():
    """The generator's draws are pinned by the stored sha256 of every array
    (tests/golden/grid_fingerprints.json, written by make_fingerprints.py)."""
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden", "grid_fingerprints.json")
    want = json.load(open(here))
    for name in ["tiny10", "syn300", "syn2000", "syn9241"]:
        assert gridgen.fingerprint(gridgen.grid(name)) == want[name], name
    for seed in (100, 163):
        g = gridgen.make_grid(gridgen.tracking_workload(seed))
        assert gridgen.fingerprint(g) == want[f"tracking{seed}"], seed
