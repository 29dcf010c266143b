"""Oracle: the chop's bracket cut in golden sections instead of thirds (the
same ternary search along the locus of axis-wise minima, Sections 3.5-3.6,
with interior points at the golden ratio so that one probe carries over to
the next step).  Pinned like the thirds form: by the exact minimum (vertex
enumeration, HiGHS) on problems where the chop alone must reach it, and by
the stuck instance of Section 3.4."""
import json
import os

import numpy as np

import oracle as O
from test_oracle import f_np, lp_highs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_p2_chop_exact_without_finisher():
    rng = np.random.default_rng(9)
    for i in range(100):
        n = int(rng.integers(3, 25))
        X = rng.standard_normal((n, 2))
        if i % 2:
            X[:, 1] = 0.9 * X[:, 0] + 0.3 * X[:, 1]
        y = rng.standard_normal(n) * 2
        lam = float(10 ** rng.uniform(-2, 1))
        fb, _, _ = O.brute_force(X, y, lam)
        b, info = O.solve(X, y, lam, use_finisher=0, max_rounds=1, golden=1)
        assert info["certified"] and info["stage"] in (O.STAGE_CCD, O.STAGE_TERNARY), i
        assert abs(f_np(X, y, lam, b) - fb) <= 1e-9 * max(1, fb), i


def test_golden_stuck_point_rescued():
    g = json.load(open(os.path.join(GOLD, "stuck2d.json")))
    X, y, lam = np.array(g["X"]), np.array(g["y"]), g["lambda"]
    fb, bb, _ = O.brute_force(X, y, lam)
    b, info = O.solve(X, y, lam, use_finisher=0, max_rounds=1, golden=1)
    assert info["stage"] == O.STAGE_TERNARY
    np.testing.assert_allclose(b, bb, rtol=1e-9)


def test_golden_fewer_probes_same_optimum():
    """Over the same bracket tolerance the golden split needs about
    log(1/tol)/log(1/0.618) probes against 2 log(1/tol)/log(1.5) for thirds,
    and the certified optimum is the same (HiGHS)."""
    rng = np.random.default_rng(12)
    pt, pg = 0, 0
    for it in range(30):
        n, p = int(rng.integers(20, 60)), int(rng.integers(2, 6))
        X = rng.standard_normal((n, p))
        y = X @ rng.uniform(-3, 3, p) + rng.laplace(0, 1, n)
        lam = float(10 ** rng.uniform(-2, 1))
        fh, _ = lp_highs(X, y, lam)
        bt, it_ = O.solve(X, y, lam, max_rounds=1)
        bg, ig = O.solve(X, y, lam, max_rounds=1, golden=1)
        assert abs(it_["f"] - fh) <= 1e-9 * max(1, fh) and abs(ig["f"] - fh) <= 1e-9 * max(1, fh)
        pt += it_["probes"]
        pg += ig["probes"]
    assert pg < 0.75 * pt, (pg, pt)
