"""GPU: single coordinate updates (Sections 3.3, 3.5), element by element
against the oracle.  A problem with p = 1, the snap and chop off and one
sweep is exactly one update from b_init: the new coefficient must be the
lower weighted median of the section's kinks.  Where the median is not
decided by a near-tie of the cumulative weight at half the total (within
fp32 resolution), the kernels must pick the same kink as the oracle's exact
fp64 median, and return its value to fp32 accuracy.  One full sweep over
p = 4 coordinates is compared the same way."""
import numpy as np
import pytest

import oracle as O
import paper_2510_15649_amd as L
from paper_2510_15649_amd import workloads as W
from parity import to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def one_sweep(torch, w, b0, kernel):
    plan = L.Plan.for_workload(w, flags=L.FLAG_NO_SNAP, max_rounds=0, max_sweeps=1)
    d = L.to_device(w)
    fn = plan.solve if kernel == "wave" else plan.solve_plain
    g = to_numpy(fn(d["X"], d["y"], d["lam"], b_init=torch.from_numpy(b0).cuda()))
    torch.cuda.synchronize()
    it = g["iters"].reshape(-1, 4)
    assert np.all(it[:, 0] == 1)  # exactly one sweep
    return g


def margin_of_median(X, y, lam, b, j):
    """The exact lower weighted median's kink value, and how far the
    cumulative weight on either side of it is from half the total
    (relative to the total): a small margin means a near-tie."""
    r = y - X @ b
    x = X[:, j]
    nz = x != 0
    t = list(b[j] + r[nz] / x[nz])
    wts = list(np.abs(x[nz]))
    if lam > 0:
        t.append(0.0)
        wts.append(lam)
    if not t:
        return None, np.inf
    t, wts = np.array(t), np.array(wts)
    k = O.weighted_median(t, wts)
    W = wts.sum()
    below = wts[t < t[k]].sum()
    upto = wts[t <= t[k]].sum()
    return t[k], min(abs(W / 2 - below), abs(upto - W / 2)) / W


@pytest.mark.parametrize("kernel", ["wave", "plain"])
def test_single_update_is_the_weighted_median(torch, kernel):
    rng = np.random.default_rng(23)
    blocks, lams, b0 = [], [], []
    for i in range(400):
        n = int(rng.integers(1, 300))
        x = rng.standard_normal(n)
        if i % 5 == 0:
            x[rng.random(n) < 0.2] = 0.0
        if i % 7 == 0 and n > 3:
            x[1], x[2] = x[0], x[0]
        y = rng.standard_normal(n) * 2 + (rng.standard_t(2, n) if i % 3 == 0 else 0)
        blocks.append((x[:, None], y))
        lams.append(0.0 if i % 6 == 0 else float(10 ** rng.uniform(-2, 2)))
        b0.append(np.float32(rng.standard_normal() * (i % 4)))
    w = W._pack("400 one-feature sections", blocks, [1] * 400, np.arange(400), lams, 1)
    b0 = np.array(b0, np.float32)
    g = one_sweep(torch, w, b0, kernel)
    exact, checked = 0, 0
    for s in range(w.num_solves):
        X, y = w.block(s)
        tk, margin = margin_of_median(X, y, float(w.lam[s]), np.array([float(b0[s])]), 0)
        bg = float(g["b"][s])
        if tk is None:
            assert bg == float(b0[s])
            continue
        if margin < 1e-5:
            continue  # a near-tie at half the weight: either neighbour is a median in fp32
        scale = 1.0 + abs(tk) + abs(float(b0[s]))
        assert abs(bg - tk) <= 4e-6 * scale, (s, bg, tk)
        exact += bg == 0.0 and tk == 0.0
        checked += 1
    assert checked >= 360, checked
    print(f"{checked} updates checked ({exact} at the penalty kink)", flush=True)


@pytest.mark.parametrize("kernel", ["wave", "plain"])
def test_one_sweep_matches_the_oracle(torch, kernel):
    w = W.config1(num_problems=32, num_lambda=4)
    p = int(w.p[0])
    rng = np.random.default_rng(24)
    b0 = (rng.standard_normal(w.num_solves * p) * 0.5).astype(np.float32)
    g = one_sweep(torch, w, b0, kernel)
    close = 0
    for s in range(w.num_solves):
        X, y = w.block(int(w.problem[s]))
        bo, _, _ = O.ccd(X, y, float(w.lam[s]), b0=b0[s * p:(s + 1) * p].astype(np.float64), max_sweeps=1)
        bg = g["b"][s * p:(s + 1) * p].astype(np.float64)
        close += np.max(np.abs(bg - bo) / (1 + np.abs(bo))) <= 1e-5
    assert close >= 0.95 * w.num_solves, close
