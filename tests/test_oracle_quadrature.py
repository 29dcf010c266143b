"""Oracle: the quadrature variant of the coordinate descent (Sections 1, 3.5
and 5 name a quadrature search of the 1-D section as the second of the
paper's two algorithms; the search itself is a reading, written out in the
oracle's source).  What pins it, independently of the oracle's own code:

* the section minimum found by brute force over the section's kinks (a
  convex piecewise-linear function takes its minimum at a kink), evaluated
  here in numpy;
* closed forms for one-row sections;
* the exact LP optimum from scipy's HiGHS solver, and brute-force vertex
  enumeration, for whole solves;
* the stuck instance of Section 3.4, which the plain descent cannot leave.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from test_oracle import f_np, lp_highs

GOLD = os.path.join(os.path.dirname(__file__), "golden")
Q = dict(section=O.SECTION_QUADRATURE)


def section_minimum(X, y, lam, b, j):
    """Brute force: g at every kink of the section, in numpy.  Returns the
    minimum value and the interval of kinks that attain it (to 1e-12)."""
    r = y - X @ b
    x = X[:, j]
    nz = x != 0
    kinks = list(b[j] + r[nz] / x[nz]) + ([0.0] if lam > 0 else [])
    if not kinks:
        return None
    kinks = np.array(kinks)

    def g(t):
        return float(np.abs(r - x * (t - b[j])).sum() + lam * abs(t))

    vals = np.array([g(t) for t in kinks])
    gmin = vals.min()
    at = kinks[vals <= gmin + 1e-12 * (1 + gmin)]
    return gmin, at.min(), at.max(), kinks, g


def test_section_search_reaches_the_section_minimum():
    rng = np.random.default_rng(3)
    checked = 0
    for it in range(300):
        n = int(rng.integers(1, 60))
        p = int(rng.integers(1, 5))
        X = rng.standard_normal((n, p))
        if it % 5 == 0:
            X[rng.random((n, p)) < 0.3] = 0.0  # missing kinks
        if it % 7 == 0 and n > 2:
            X[1] = X[0]  # duplicated rows: tied kinks
        y = rng.standard_normal(n) * 3
        lam = 0.0 if it % 4 == 0 else float(10 ** rng.uniform(-2, 1.5))
        b = rng.standard_normal(p) * (it % 3)
        j = int(rng.integers(0, p))
        ref = section_minimum(X, y, lam, b, j)
        bq, ev = O.quadrature_update(X, y, lam, b, j)
        if ref is None:
            np.testing.assert_array_equal(bq, b)
            continue
        gmin, mlo, mhi, kinks, g = ref
        assert np.array_equal(np.delete(bq, j), np.delete(b, j))
        span = kinks.max() - kinks.min()
        tol = 1e-13 * (1 + 2 * np.abs(kinks).max())
        slope = np.abs(X[:, j]).sum() + lam
        # the value reached is the section minimum, up to the final bracket
        assert g(bq[j]) <= gmin + slope * 2 * tol + 1e-13 * (1 + gmin), (it, g(bq[j]), gmin)
        # and the point lies within the bracket of the minimisers
        assert mlo - 2 * tol <= bq[j] <= mhi + 2 * tol or g(b[j]) <= g(bq[j]), (it, bq[j], mlo, mhi)
        # the number of section values: one at the centre, two per halving,
        # one at the start point; halvings stop at the tolerance
        halvings = (ev - 2) // 2
        assert ev == 2 + 2 * halvings
        if span > 0:
            assert halvings <= math.ceil(math.log2(span / (1e-13 * (1 + 0)))) + 1
            # the final bracket is within the tolerance
            assert span / 2 ** halvings <= 1e-13 * (1 + 2 * np.abs(kinks).max()) * (1 + 1e-9)
        checked += 1
    assert checked >= 250


def test_section_search_closed_forms():
    # one row, no penalty: the only kink is y/x; the bracket is that point
    X = np.array([[2.5]])
    y = np.array([-3.0])
    b, ev = O.quadrature_update(X, y, 0.0, np.zeros(1), 0)
    assert b[0] == -3.0 / 2.5 and ev == 2
    # one row with a penalty below |x|: minimiser y/x
    b, _ = O.quadrature_update(X, y, 1.0, np.zeros(1), 0)
    assert abs(b[0] + 1.2) <= 1e-12
    # a penalty above |x|: the minimiser is 0, and the start point 0 is kept
    b, _ = O.quadrature_update(X, y, 4.0, np.zeros(1), 0)
    assert b[0] == 0.0
    b, _ = O.quadrature_update(X, y, 4.0, np.array([0.7]), 0)
    assert abs(b[0]) <= 1e-12
    # no kinks at all: b is kept
    b, ev = O.quadrature_update(np.zeros((3, 1)), np.ones(3), 0.0, np.array([0.3]), 0)
    assert b[0] == 0.3 and ev == 0


def test_section_search_never_raises_f():
    """From a point that already minimises the section, the search keeps it."""
    rng = np.random.default_rng(4)
    for _ in range(100):
        n = int(rng.integers(2, 40))
        X = rng.standard_normal((n, 3))
        y = rng.standard_normal(n)
        lam = float(10 ** rng.uniform(-2, 1))
        b = O.coord_update(X, y, lam, rng.standard_normal(3), 1)  # exact section minimum
        bq, _ = O.quadrature_update(X, y, lam, b, 1)
        assert f_np(X, y, lam, bq) <= f_np(X, y, lam, b) + 1e-12 * (1 + f_np(X, y, lam, b))


def test_quadrature_solve_matches_highs():
    rng = np.random.default_rng(5)
    for it in range(60):
        n = int(rng.integers(4, 80))
        p = int(rng.integers(1, 7))
        X = rng.standard_normal((n, p))
        bt = rng.uniform(-3, 3, p) * (rng.random(p) < 0.6)
        y = X @ bt + rng.laplace(0, 1, n)
        lam = float(10 ** rng.uniform(-2, 1.5))
        fh, bh = lp_highs(X, y, lam)
        b, info = O.solve(X, y, lam, **Q)
        assert info["certified"]
        assert abs(info["f"] - fh) <= 1e-9 * max(1, fh), (it, info["f"], fh)
        if info["unique"] and info["margin_uc"] > 1e-6:
            np.testing.assert_allclose(b, bh, atol=1e-7 * max(1, np.abs(bh).max()))
        # the same vertex as the median variant
        bm, im = O.solve(X, y, lam)
        if im["unique"]:
            assert info["S_mask"] == im["S_mask"] and list(info["Z"]) == list(im["Z"])


def test_quadrature_p2_chop_exact_without_finisher():
    """p = 2 with quadrature sections: the restricted sub-search is one 1-D
    search, so F(s) is convex to the search's tolerance, and the chop alone
    certifies the brute-force optimum."""
    rng = np.random.default_rng(9)
    for i in range(60):
        n = int(rng.integers(3, 25))
        X = rng.standard_normal((n, 2))
        y = rng.standard_normal(n) * 2
        lam = float(10 ** rng.uniform(-2, 1))
        fb, _, _ = O.brute_force(X, y, lam)
        b, info = O.solve(X, y, lam, use_finisher=0, max_rounds=1, **Q)
        assert info["certified"] and info["stage"] in (O.STAGE_CCD, O.STAGE_TERNARY), i
        assert abs(f_np(X, y, lam, b) - fb) <= 1e-9 * max(1, fb), i


def test_quadrature_stuck_point_rescued_by_chop():
    g = json.load(open(os.path.join(GOLD, "stuck2d.json")))
    X, y, lam = np.array(g["X"]), np.array(g["y"]), g["lambda"]
    fb, bb, _ = O.brute_force(X, y, lam)
    bc, fc, _ = O.ccd(X, y, lam, **Q)
    assert fc > fb + 0.5  # the quadrature descent is stuck too
    b, info = O.solve(X, y, lam, use_finisher=0, max_rounds=1, **Q)
    assert info["stage"] == O.STAGE_TERNARY
    np.testing.assert_allclose(b, bb, rtol=1e-9)


def test_quadrature_batch_reaches_the_same_optima():
    """The batch driver with quadrature sections (warm-started path) ends at
    the same certified optima as with exact weighted medians."""
    from paper_2510_15649_amd import workloads as W
    w = W.config1(num_problems=6, num_lambda=4, as_path=True)
    rq = O.solve_batch(w, **Q)
    rm = O.solve_batch(w)
    assert np.all(rq["cert"] > 0) and np.all(rm["cert"] > 0)
    np.testing.assert_allclose(rq["f"], rm["f"], rtol=1e-10)
    both = (rq["cert"] == 2) & (rm["cert"] == 2)
    assert np.array_equal(rq["smask"][both], rm["smask"][both])
    assert np.array_equal(rq["zrows"][both], rm["zrows"][both])


def test_ccd_ends_at_an_axiswise_minimum():
    """Both section searches: coordinate descent run to convergence stops at a
    point where every coordinate minimises its own section (Section 3.3's
    stopping point, an axis-wise minimum), checked by brute force over each
    section's kinks in numpy."""
    rng = np.random.default_rng(17)
    for it in range(40):
        n, p = int(rng.integers(5, 50)), int(rng.integers(2, 6))
        X = rng.standard_normal((n, p))
        y = X @ rng.uniform(-2, 2, p) + rng.laplace(0, 1, n)
        lam = float(10 ** rng.uniform(-2, 1))
        for opts in (dict(), Q):
            b, f, sweeps = O.ccd(X, y, lam, **opts)
            assert sweeps < 1000
            for j in range(p):
                gmin, mlo, mhi, kinks, g = section_minimum(X, y, lam, b, j)
                assert g(b[j]) <= gmin + 1e-9 * (1 + gmin), (it, opts, j, g(b[j]), gmin)
