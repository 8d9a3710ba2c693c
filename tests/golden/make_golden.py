"""Writes the stored expected values under tests/golden/ by calling the
oracle only (oracle/fem.py: explicit P1 assembly on the Kuhn simplices and a
sparse direct solve).  The paper prints no value for the periodic cell
problem, so these are not quotes of it: they freeze the oracle's results on
two small cells, which tests/test_oracle_golden.py recomputes (a change of the
oracle's arithmetic shows up there) and the GPU tests compare against.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fem  # noqa: E402
from paper_2004_05197_amd import microstructures as ms  # noqa: E402


def circle2d_case():
    """32 x 32 pixels, centred circle of radius 0.25 (E 10, nu 0.3) in a
    matrix (E 1, nu 0.3), plane strain: C* and the mean stress of the
    macro strain eps_xx = 1e-2."""
    E, nu = ms.circle2d(32)
    grid = fem.Grid((32, 32))
    C, _, _ = fem.effective_stiffness(grid, E, nu)
    eb = np.array([[1e-2, 0.0, 0.0]])
    u = fem.solve_direct(grid, E, nu, eb)
    s = fem.homogenize(grid, E, nu, u, eb)["mean_stress"][0]
    return {"case": "circle2d_32", "shape": [32, 32], "C_energy": C.tolist(), "eps_bar": eb[0].tolist(),
            "mean_stress": s.tolist()}


def random3d_case():
    """12 x 8 x 6 voxels, E ~ U[1, 30], nu ~ U[0.05, 0.45] (numpy default_rng
    seed 7, arrays of shape (6, 8, 12), x fastest), edge lengths 1.0, 1.4,
    0.8: C*."""
    rng = np.random.default_rng(7)
    nshape = (6, 8, 12)
    E = rng.uniform(1.0, 30.0, nshape)
    nu = rng.uniform(0.05, 0.45, nshape)
    grid = fem.Grid((12, 8, 6), lengths=(1.0, 1.4, 0.8))
    C, _, _ = fem.effective_stiffness(grid, E, nu)
    return {"case": "random3d_12x8x6", "shape": [12, 8, 6], "lengths": [1.0, 1.4, 0.8], "seed": 7,
            "E_range": [1.0, 30.0], "nu_range": [0.05, 0.45], "C_energy": C.tolist()}


CASES = {"circle2d_32": circle2d_case, "random3d_12x8x6": random3d_case}


def main():
    for name, fn in CASES.items():
        d = fn()
        d["source"] = ("oracle/fem.py direct solve (written by tests/golden/make_golden.py); "
                       "the paper prints no value for this problem")
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(d, fh, indent=1)
            fh.write("\n")
        print(name)


if __name__ == "__main__":
    main()
