"""GPU: K-fold cross-validation along a lambda path against the oracle's
cross-validation (same instances; training solves compared where the
oracle's optimum is unique, selections where the CV minimum is clear)."""
import numpy as np
import pytest

import oracle as O
import paper_2510_15649_amd as L
from paper_2510_15649_amd import workloads as W
from parity import to_numpy

pytestmark = pytest.mark.gpu

TOL_B = 1e-4   # the coefficient bar: |b - b*| <= TOL_B * max(1, |b*|)


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def held_out_tolerance(X, lab, f, b):
    """Largest change of sum_{i in fold f} |y_i - x_i b| that coefficients
    within the TOL_B bar can cause, plus fp32 rounding of the residuals."""
    va = lab == f
    Xa = np.abs(X[va])
    return TOL_B * float(Xa.sum(axis=0) @ np.maximum(1.0, np.abs(b))) + 1e-6 * float(Xa.sum() + 1.0)


def check_cv(w, K, gpu, fold_of_row=None, min_fold_checks=1, min_best_checks=0):
    Lp = w.path_len
    P = w.num_problems
    ferr = gpu["fold_error"].reshape(P, K, Lp)
    curve = gpu["cv_error"].reshape(P, Lp)
    st = gpu["fold_status"].reshape(P, K, Lp)
    fold_checks = best_checks = 0
    for k in range(P):
        Xk, yk = w.block(k)
        n = Xk.shape[0]
        lab = O.cv_folds(n, K, None if fold_of_row is None else fold_of_row[w.row_off[k]:w.row_off[k + 1]])
        lams = w.lam[k * Lp:(k + 1) * Lp]
        ref = O.cv(Xk, yk, lams, K, fold_of_row=lab, max_rounds=0)
        assert np.all((st[k] == L.CERTIFIED) | (st[k] == L.NONUNIQUE)), (k, st[k])
        tol = np.zeros((K, Lp))
        for f in range(K):
            for t in range(Lp):
                tol[f, t] = held_out_tolerance(Xk, lab, f, ref["b"][f, t])
                if ref["unique"][f, t]:
                    assert abs(ferr[k, f, t] - ref["err"][f, t]) <= tol[f, t], (k, f, t, ferr[k, f, t], ref["err"][f, t])
                    fold_checks += 1
        # the curve is the fp64 sum over folds of the reported fold errors
        assert np.allclose(curve[k], ferr[k].astype(np.float64).sum(axis=0), rtol=1e-6, atol=1e-6)
        ok_t = ref["unique"].all(axis=0)
        for t in np.flatnonzero(ok_t):
            assert abs(curve[k, t] - ref["cv"][t]) <= tol[:, t].sum(), (k, t)
        if ok_t.all():
            srt = np.sort(ref["cv"])
            if Lp == 1 or srt[1] - srt[0] > 2 * tol.sum(axis=0).max():
                assert gpu["best"][k] == ref["best"], (k, gpu["best"][k], ref["best"], ref["cv"])
                best_checks += 1
    assert fold_checks >= min_fold_checks, fold_checks
    assert best_checks >= min_best_checks, best_checks
    return fold_checks, best_checks


def test_cv_c1_path_5_folds(torch):
    """48 problems of n = 200, p = 8, 5 folds, the 16-lambda path
    (descending), default fold assignment.  A selection is compared where
    every fold solve along the path has a unique optimum and the CV minimum
    is clear of the runner-up."""
    w = W.config1(num_problems=48, as_path=True)
    K = 5
    print(f"[gpu] cv c1 P={w.num_problems} K={K} L={w.path_len}", flush=True)
    cv = L.CrossValidation.for_workload(w, K)
    d = L.to_device(w)
    out = to_numpy(cv.run(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    fc, bc = check_cv(w, K, out, min_fold_checks=2400, min_best_checks=3)
    print("fold checks", fc, "selection checks", bc, flush=True)


def test_cv_ragged_custom_folds(torch):
    """Ragged row subsets (n in [50, 1000], p = 16), one lambda, 3 folds
    given by an explicit random label per row."""
    w = W.config2(num_subsets=12)
    K = 3
    rng = np.random.default_rng(21)
    fold = rng.integers(0, K, size=int(w.row_off[-1])).astype(np.int32)
    print(f"[gpu] cv c2 P={w.num_problems} K={K} custom folds", flush=True)
    cv = L.CrossValidation.for_workload(w, K, fold_of_row=fold)
    d = L.to_device(w)
    out = to_numpy(cv.run(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    check_cv(w, K, out, fold_of_row=fold, min_fold_checks=20, min_best_checks=0)


def test_cv_validation_errors(torch):
    w = W.config1(num_problems=2, as_path=True)
    with pytest.raises(L.LadlError):
        L.CrossValidation.for_workload(w, 1)
    bad = np.zeros(int(w.row_off[-1]), dtype=np.int32)
    bad[3] = 7
    with pytest.raises(L.LadlError):
        L.CrossValidation.for_workload(w, 5, fold_of_row=bad)
    one = np.zeros(int(w.row_off[-1]), dtype=np.int32)   # fold 0 holds every row
    with pytest.raises(L.LadlError):
        L.CrossValidation.for_workload(w, 2, fold_of_row=one)
