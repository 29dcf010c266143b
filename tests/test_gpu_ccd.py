"""GPU: the coordinate descent on its own (Section 3.3), with the snap,
certificate, chop and finisher switched off.  Its iterates are not compared
with the oracle's (their order of floating-point operations differs), but
its end point has a property the paper fixes: run to convergence, every
coordinate minimises its own 1-D section (an axis-wise minimum).  That is
checked in fp64 by brute force over each section's kinks, for the exact
weighted-median update and for the quadrature search, on both kernels."""
import numpy as np
import pytest

import paper_2510_15649_amd as L
from paper_2510_15649_amd import workloads as W
from parity import to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def section_gap(X, y, lam, b, j):
    """g(b_j) - min g over the section's kinks, relative to 1 + min g."""
    r = y - X @ b
    x = X[:, j]
    nz = x != 0
    kinks = np.concatenate([b[j] + r[nz] / x[nz], [0.0] if lam > 0 else []])
    if kinks.size == 0:
        return 0.0

    def g(t):
        return float(np.abs(r - x * (t - b[j])).sum() + lam * abs(t))

    gmin = min(g(t) for t in kinks)
    return (g(b[j]) - gmin) / (1.0 + gmin)


@pytest.mark.parametrize("quad", [False, True], ids=["median", "quadrature"])
@pytest.mark.parametrize("kernel", ["wave", "plain"])
def test_descent_stops_at_an_axiswise_minimum(torch, kernel, quad):
    w = W.config1(num_problems=24, num_lambda=4)
    flags = L.FLAG_NO_SNAP | (L.FLAG_QUADRATURE if quad else 0)
    plan = L.Plan.for_workload(w, flags=flags, max_rounds=0, max_sweeps=500, tol_f=0.0)
    d = L.to_device(w)
    fn = plan.solve if kernel == "wave" else plan.solve_plain
    g = to_numpy(fn(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    assert np.all(g["status"] == L.MAXITER)
    it = g["iters"].reshape(-1, 4)
    assert np.all(it[:, 2] == 0) and np.all(it[:, 3] == 0)  # no probe, no pivot
    p = int(w.p[0])
    worst = 0.0
    for s in range(w.num_solves):
        Xk, yk = w.block(int(w.problem[s]))
        b = g["b"][s * p:(s + 1) * p].astype(np.float64)
        lam = float(w.lam[s])
        for j in range(p):
            worst = max(worst, section_gap(Xk, yk, lam, b, j))
    print(f"largest section gap {worst:.2e}", flush=True)
    assert worst <= (2e-5 if quad else 1e-5), worst
