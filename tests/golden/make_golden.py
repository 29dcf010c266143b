"""Writes the stored expected values under tests/golden/.

Every value here comes from the FP64 oracle (oracle/) or from the seeded
generators; nothing is taken from the HIP library.  Run from the repo root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2510_15649_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def c0():
    """The c0 problem (n=20, p=3, lambda=1; the paper's evaluation regime of
    Section 4: 10-30 rows, 1-5 features) solved by brute-force vertex
    enumeration (Section 3.2) at four lambdas, on the FP64 draw and on its
    FP32 cast."""
    w = W.config0()
    out = {"source": "tests/golden/make_golden.py (oracle brute force, Section 3.2)",
           "X64": w.X64.tolist(), "y64": w.y64.tolist(), "cases": []}
    for lam in [0.01, 0.1, 1.0, 5.0, 30.0]:
        for prec in ["f64", "f32"]:
            X = w.X64 if prec == "f64" else w.X64.astype(np.float32).astype(np.float64)
            y = w.y64 if prec == "f64" else w.y64.astype(np.float32).astype(np.float64)
            f, b, nv = O.brute_force(X, y, lam)
            out["cases"].append({"lambda": lam, "data": prec, "f": f, "b": b.tolist(), "vertices": nv})
    with open(os.path.join(HERE, "c0_bruteforce.json"), "w") as fh:
        json.dump(out, fh, indent=1)


def stuck2d():
    """A 2-D instance on which plain cyclical coordinate descent stops at an
    axis-wise minimum above the optimum (the situation of the paper's
    contour figure, Section 3.4).  Found by a seeded search over rounded
    6-row instances; the optimum is from brute force (Section 3.2)."""
    X = np.array([[0.0, 0.7], [-0.3, 1.1], [0.0, 0.6], [-1.3, 0.3], [-1.7, -2.0], [-0.3, -0.9]])
    y = np.array([0.3, 4.5, -1.7, -1.2, 0.4, 1.0])
    lam = 0.1
    f, b, _ = O.brute_force(X, y, lam)
    bc, fc, _ = O.ccd(X, y, lam)
    out = {"source": "tests/golden/make_golden.py (oracle brute force and CCD)", "X": X.tolist(),
           "y": y.tolist(), "lambda": lam, "f_opt": f, "b_opt": b.tolist(), "f_ccd": fc,
           "b_ccd": bc.tolist()}
    with open(os.path.join(HERE, "stuck2d.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    c0()
    stuck2d()
