"""Pins of the oracle's K-fold cross-validation (the paper's interactive
use: many regularisation settings solved while cross-validating, Section 5)
against brute force, a closed form and invariants.  None re-types the
oracle's own loop: the fold solutions come from vertex enumeration or from
a median written out here."""
import numpy as np

import oracle as O


def lowest_weighted_median(vals, wts):
    """Smallest v minimising sum_k w_k |v - vals_k| (independent of the
    oracle: sort and scan)."""
    order = np.argsort(vals, kind="stable")
    v, w = np.asarray(vals)[order], np.asarray(wts)[order]
    c = np.cumsum(w)
    return float(v[np.searchsorted(c, 0.5 * c[-1])])


def test_cv_folds_match_brute_force():
    """Every fold's training solve is an exact optimum (vertex enumeration of
    the training rows) and, where that optimum is unique, the held-out error
    equals the brute-force point's held-out absolute error."""
    rng = np.random.default_rng(11)
    checked = 0
    for trial in range(30):
        n, p, K = int(rng.integers(6, 11)), int(rng.integers(1, 4)), int(rng.integers(2, 5))
        X = rng.standard_normal((n, p))
        y = X @ rng.uniform(-2, 2, p) + rng.laplace(0, 0.5, n)
        lams = np.array([4.0, 1.0, 0.25])
        r = O.cv(X, y, lams, K, max_rounds=0)
        lab = np.arange(n) % K
        for f in range(K):
            tr, va = lab != f, lab == f
            for t, lam in enumerate(lams):
                fbf, bbf, _ = O.brute_force(X[tr], y[tr], lam)
                fo = np.abs(y[tr] - X[tr] @ r["b"][f, t]).sum() + lam * np.abs(r["b"][f, t]).sum()
                assert abs(fo - fbf) <= 1e-9 * max(1.0, fbf), (trial, f, t)
                if r["unique"][f, t]:
                    e = np.abs(y[va] - X[va] @ bbf).sum()
                    assert abs(r["err"][f, t] - e) <= 1e-9 * max(1.0, e), (trial, f, t)
                    checked += 1
        assert np.allclose(r["cv"], r["err"].sum(axis=0))
        assert r["best"] == int(np.argmin(r["cv"]))
    assert checked > 200, checked


def test_cv_intercept_only_closed_form():
    """x_i = 1 (p = 1): each fold's b is the lowest weighted median of the
    training y and 0 (weight lambda), so every held-out error has a closed
    form."""
    rng = np.random.default_rng(5)
    n, K = 23, 4
    y = rng.normal(1.5, 2.0, n)
    X = np.ones((n, 1))
    lams = np.array([30.0, 3.0, 0.3, 0.0])
    r = O.cv(X, y, lams, K, max_rounds=0)
    lab = np.arange(n) % K
    for f in range(K):
        tr, va = lab != f, lab == f
        for t, lam in enumerate(lams):
            vals = np.concatenate([y[tr], [0.0]])
            wts = np.concatenate([np.ones(tr.sum()), [lam]])
            b = lowest_weighted_median(vals, wts) if lam > 0 else lowest_weighted_median(y[tr], np.ones(tr.sum()))
            e = np.abs(y[va] - b).sum()
            # an even training set has a flat optimal segment: compare only
            # where the optimum is unique
            if r["unique"][f, t]:
                assert abs(r["err"][f, t] - e) <= 1e-10 * max(1.0, e), (f, t, r["b"][f, t], b)
            fo = np.abs(y[tr] - r["b"][f, t, 0]).sum() + lam * abs(r["b"][f, t, 0])
            fb = np.abs(y[tr] - b).sum() + lam * abs(b)
            assert abs(fo - fb) <= 1e-10 * max(1.0, fb)


def test_cv_large_lambda_gives_null_model():
    """lambda >= ||X_tr^T sign(y_tr)||_inf makes b = 0 the optimum of every
    fold, so the held-out error is sum |y| over the fold."""
    rng = np.random.default_rng(8)
    n, p, K = 40, 5, 5
    X = rng.standard_normal((n, p))
    y = rng.standard_normal(n)
    lam_big = 2.0 * float(np.abs(X).sum(axis=0).max())
    r = O.cv(X, y, [lam_big], K)
    lab = np.arange(n) % K
    for f in range(K):
        assert np.all(r["b"][f, 0] == 0.0)
        assert abs(r["err"][f, 0] - np.abs(y[lab == f]).sum()) <= 1e-12 * n


def test_cv_leave_one_out_and_row_permutation():
    """Leave-one-out (K = n) against brute force; and permuting the rows
    together with their fold labels leaves every unique fold error
    unchanged."""
    rng = np.random.default_rng(3)
    n, p = 8, 2
    X = rng.standard_normal((n, p))
    y = X @ np.array([1.0, -0.5]) + rng.laplace(0, 0.3, n)
    lams = np.array([1.0, 0.1])
    r = O.cv(X, y, lams, n, max_rounds=0)
    for f in range(n):
        tr = np.arange(n) != f
        for t, lam in enumerate(lams):
            if r["unique"][f, t]:
                _, bbf, _ = O.brute_force(X[tr], y[tr], lam)
                assert abs(r["err"][f, t] - abs(y[f] - X[f] @ bbf)) <= 1e-9
    K = 3
    lab = np.arange(n) % K
    perm = rng.permutation(n)
    r1 = O.cv(X, y, lams, K, fold_of_row=lab, max_rounds=0)
    r2 = O.cv(X[perm], y[perm], lams, K, fold_of_row=lab[perm], max_rounds=0)
    both = r1["unique"] & r2["unique"]
    assert both.sum() >= 3
    assert np.allclose(r1["err"][both], r2["err"][both], rtol=1e-9, atol=1e-12)
