"""GPU: the paper's ternary chop along the locus of axis-wise minima
(Sections 3.5-3.6) on its own, with the simplex finisher switched off.

For p = 2 the sub-search with the chop axis frozen is one exact 1-D
minimisation, so the chop's objective F(s) is the partial minimum of a
convex function, itself convex, and the chop alone reaches the global
minimum.  These tests run the HIP chop without the finisher and check that
it does: 256 random p = 2 problems (half of them with strongly correlated
columns, where plain coordinate descent stalls) against the exact minimum
by vertex enumeration or the dense simplex, and the stuck instance of the
golden file.  No finisher pivot may occur, and the iteration counters show
that the chop's probes ran."""
import json
import os

import numpy as np
import pytest

import oracle as O
import paper_2510_15649_amd as L
from paper_2510_15649_amd import workloads as W
from parity import to_numpy

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
OK = (L.CERTIFIED, L.NONUNIQUE)


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def p2_workload(num=256, seed=31):
    rng = np.random.default_rng(seed)
    blocks, lams = [], []
    for i in range(num):
        n = int(rng.integers(3, 120))
        X = rng.standard_normal((n, 2))
        if i % 2:
            X[:, 1] = 0.9 * X[:, 0] + 0.3 * X[:, 1]
        y = X @ rng.uniform(-3, 3, 2) + rng.laplace(0, 1, n)
        blocks.append((X, y))
        lams.append(float(10 ** rng.uniform(-2, 1)))
    return W._pack(f"{num} random p=2 problems", blocks, [2] * num, np.arange(num), lams, 1)


def exact_min(w):
    f = np.zeros(w.num_solves)
    for s in range(w.num_solves):
        Xk, yk = w.block(s)
        lam = float(w.lam[s])
        f[s] = O.brute_force(Xk, yk, lam)[0] if Xk.shape[0] <= 60 else O.lp_simplex(Xk, yk, lam)[0]
    return f


SPLITS = pytest.mark.parametrize("split", [0, L.FLAG_GOLDEN], ids=["thirds", "golden"])


@SPLITS
@pytest.mark.parametrize("kernel", ["wave", "plain"])
def test_p2_chop_alone_reaches_the_minimum(torch, kernel, split):
    w = p2_workload()
    print(f"[gpu] chop without finisher, {w.name}, {kernel}, split {split}", flush=True)
    fstar = exact_min(w)
    d = L.to_device(w)
    res = {}
    for rounds in (0, 1):
        plan = L.Plan.for_workload(w, flags=L.FLAG_NO_FINISHER | split, max_rounds=rounds)
        fn = plan.solve if kernel == "wave" else plan.solve_plain
        res[rounds] = to_numpy(fn(d["X"], d["y"], d["lam"]))
        torch.cuda.synchronize()
    f0, f1 = res[0]["obj"].astype(np.float64), res[1]["obj"].astype(np.float64)
    it1 = res[1]["iters"].reshape(-1, 4)
    rel0 = (f0 - fstar) / np.maximum(fstar, 1e-30)
    rel1 = np.abs(f1 - fstar) / np.maximum(fstar, 1e-30)
    # without the chop, coordinate descent and the snap stall on many of them
    stuck = np.flatnonzero(rel0 > 1e-5)
    assert len(stuck) >= 64, len(stuck)
    # with it, every one reaches the minimum, with no finisher pivot; the
    # vertex certificate (an addition to the paper's method) then holds on
    # nearly all (a rare near-tie of hyperplanes at the optimum can make the
    # nearest-vertex snap pick a neighbour)
    assert np.max(rel1) <= 1e-5, (np.argmax(rel1), np.max(rel1))
    assert np.all(it1[:, 3] == 0)
    cert = np.isin(res[1]["status"], OK)
    assert cert.mean() >= 0.98, np.bincount(res[1]["status"], minlength=6)
    assert np.all(np.isin(res[1]["status"][~cert], [L.NOTCERTIFIED]))
    # the rescued ones were certified after chop probes (stage: the chop)
    assert np.all(it1[stuck, 2] > 0)
    # each problem's b is the minimiser, checked in fp64
    for s in range(w.num_solves):
        Xk, yk = w.block(s)
        b = res[1]["b"][2 * s:2 * s + 2].astype(np.float64)
        fb = float(np.abs(yk - Xk @ b).sum() + w.lam[s] * np.abs(b).sum())
        assert abs(fb - fstar[s]) <= 1e-5 * max(fstar[s], 1e-30), s
    print(f"stuck without the chop: {len(stuck)} of {w.num_solves}; "
          f"max rel error with it {np.max(rel1):.2e}", flush=True)


@SPLITS
@pytest.mark.parametrize("kernel", ["wave", "plain"])
def test_stuck_instance_escaped_by_the_chop(torch, kernel, split):
    """The golden stuck instance: coordinate descent stops at an axis-wise
    minimum 0.55 above the optimum, and its nearest vertex does not certify;
    the chop reaches the optimum."""
    g = json.load(open(os.path.join(GOLD, "stuck2d.json")))
    X, y = np.array(g["X"]), np.array(g["y"])
    w = W._pack("stuck2d", [(X, y)], [2], [0], [g["lambda"]], 1)
    d = L.to_device(w)
    out = {}
    for rounds in (0, 1):
        plan = L.Plan.for_workload(w, flags=L.FLAG_NO_FINISHER | split, max_rounds=rounds)
        fn = plan.solve if kernel == "wave" else plan.solve_plain
        out[rounds] = to_numpy(fn(d["X"], d["y"], d["lam"]))
        torch.cuda.synchronize()
    assert out[0]["status"][0] == L.NOTCERTIFIED
    assert out[0]["obj"][0] >= g["f_opt"] + 0.5
    assert out[1]["status"][0] in OK
    assert abs(out[1]["obj"][0] - g["f_opt"]) <= 1e-5 * g["f_opt"]
    np.testing.assert_allclose(out[1]["b"], g["b_opt"], rtol=1e-4, atol=1e-4)
    it = out[1]["iters"].reshape(-1, 4)[0]
    assert it[2] > 0 and it[3] == 0, it
