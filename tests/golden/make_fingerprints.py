"""Writes grid_fingerprints.json: the sha256 of every array of the seeded
synthetic grids (gridgen.fingerprint), so that a change in the generator's
draws fails tests/test_gridgen.py.  Calls only the input generator.

    python tests/golden/make_fingerprints.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gridgen  # noqa: E402

NAMES = ["tiny10", "syn300", "syn2000", "syn9241"]


def main():
    out = {n: gridgen.fingerprint(gridgen.grid(n)) for n in NAMES}
    for seed in (100, 163):
        g = gridgen.make_grid(gridgen.tracking_workload(seed))
        out[f"tracking{seed}"] = gridgen.fingerprint(g)
    with open(os.path.join(HERE, "grid_fingerprints.json"), "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
