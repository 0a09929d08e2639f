"""Write the oracle's results for small seeded grids to text fixtures.

    python tests/golden/make_golden.py

Calls only the CPU oracle (oracle/) and the seeded input generators; no
value here comes from the GPU library.  The fixtures pin the oracle build
against itself over time (compiler, flags) and give the GPU tests a stored
reference that does not need the oracle to run.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2107_00555_amd import inputs  # noqa: E402

CASES = {
    "plain_16x12x10_dirichlet_T10": dict(shape=(16, 12, 10), bc=0, T=10, f="uniform"),
    "sinus_16x12x10_periodic_T10": dict(shape=(16, 12, 10), bc=1, T=10, f="sinusoids"),
}
SAMPLES = [(0, 0, 0), (15, 11, 9), (7, 5, 4), (3, 11, 0), (15, 0, 6), (8, 6, 9)]


def make(name, case, seed=0):
    nx, ny, nz = case["shape"]
    u0, f = inputs.make_fields(dict(f=case["f"]), seed=seed, shape=case["shape"])
    c = dict(inputs.BASE_COEFFS)
    uT, e, r = oracle.run(u0, f, c, case["T"], case["bc"])
    return {
        "name": name, "seed": seed, "shape_xyz": [nx, ny, nz], "bc": case["bc"], "T": case["T"],
        "f": case["f"], "coeffs": c,
        "energy": [repr(float(v)) for v in e],
        "resid": [repr(float(v)) for v in r],
        "samples": [[x, y, z, repr(float(uT[z, y, x]))] for x, y, z in SAMPLES],
        "checksum_sum": repr(float(np.sum(uT))),
    }


if __name__ == "__main__":
    for name, case in CASES.items():
        with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as fh:
            json.dump(make(name, case), fh, indent=1)
        print("wrote", name)
