"""GPU: the quadrature variant (LADL_FLAG_QUADRATURE), the paper's second
coordinate-descent algorithm (Sections 1, 3.5 and 5), in which every 1-D
section is minimised by a quadrature search of its values instead of the
exact weighted median.  Its iterates are approximate by construction, so it
is pinned at its result: the same certified optimum as the oracle (whose own
quadrature variant is pinned against HiGHS and vertex enumeration on the
CPU), element by element, for the wavefront kernel (one wave and a team of
waves) and the one-thread-per-solve kernel; and on its own, without the
finisher, the chop with quadrature sections reaches the p = 2 minima."""
import json
import os

import numpy as np
import pytest

import oracle as O
import paper_2510_15649_amd as L
from paper_2510_15649_amd import workloads as W
from parity import compare, oracle_ref, to_numpy
from test_gpu_chop import exact_min, p2_workload

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
OK = (L.CERTIFIED, L.NONUNIQUE)
QF = L.FLAG_QUADRATURE


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.mark.parametrize("kernel", ["wave", "plain"])
def test_quadrature_parity_c1(torch, kernel):
    """64 problems of the 200 x 8 recipe at 16 lambdas (1024 solves)."""
    w = W.config1(num_problems=64 if kernel == "wave" else 16)
    print(f"[gpu] quadrature sections, {w.name}, {kernel}", flush=True)
    d = L.to_device(w)
    plan = L.Plan.for_workload(w, flags=QF)
    fn = plan.solve if kernel == "wave" else plan.solve_plain
    g = to_numpy(fn(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    fails, st = compare(w, g, oracle_ref(w))
    print(st, flush=True)
    assert not fails, fails[:5]
    assert st["strict"] >= 0.95 * st["unique"], st
    # the median variant on the same solves: the same objectives
    plan_m = L.Plan.for_workload(w)
    fm = plan_m.solve if kernel == "wave" else plan_m.solve_plain
    gm = to_numpy(fm(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    rel = np.abs(g["obj"].astype(np.float64) - gm["obj"]) / np.maximum(gm["obj"], 1e-30)
    assert np.max(rel) <= 2e-5, np.max(rel)


def test_quadrature_parity_ragged_with_teams(torch):
    """Ragged problems of the large recipe (n up to 2048, p up to 32, a
    4-step lambda path), including n > 1024 solved by a team of 2 waves."""
    ns = [int(W._rng(W.BASE_SEED + 4000, k).integers(32, 2049)) for k in range(400)]
    big = [k for k in range(400) if ns[k] > 1024][:6]
    small = [k for k in range(400) if ns[k] <= 1024][:18]
    w = W.config4(problems=sorted(big + small), path_len=4)
    print(f"[gpu] quadrature sections, {w.name}, team 2", flush=True)
    d = L.to_device(w)
    plan = L.Plan.for_workload(w, flags=QF, team=2)
    g = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    fails, st = compare(w, g, oracle_ref(w))
    print(st, flush=True)
    assert not fails, fails[:5]
    assert st["strict"] >= 0.9 * st["unique"], st


@pytest.mark.parametrize("kernel", ["wave", "plain"])
def test_quadrature_p2_chop_without_finisher(torch, kernel):
    """p = 2: with the chop axis frozen the sub-search is one quadrature
    search, so F(s) is convex up to the search's tolerance and the chop
    alone reaches the minimum; no finisher pivot runs."""
    w = p2_workload(num=128, seed=32)
    print(f"[gpu] quadrature chop without finisher, {w.name}, {kernel}", flush=True)
    fstar = exact_min(w)
    d = L.to_device(w)
    plan = L.Plan.for_workload(w, flags=QF | L.FLAG_NO_FINISHER, max_rounds=1)
    fn = plan.solve if kernel == "wave" else plan.solve_plain
    g = to_numpy(fn(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    it = g["iters"].reshape(-1, 4)
    assert np.all(it[:, 3] == 0)
    rel = np.abs(g["obj"].astype(np.float64) - fstar) / np.maximum(fstar, 1e-30)
    assert np.max(rel) <= 1e-5, (np.argmax(rel), np.max(rel))
    cert = np.isin(g["status"], OK)
    assert cert.mean() >= 0.97, np.bincount(g["status"], minlength=6)


def test_quadrature_stuck_instance(torch):
    g = json.load(open(os.path.join(GOLD, "stuck2d.json")))
    X, y = np.array(g["X"]), np.array(g["y"])
    w = W._pack("stuck2d", [(X, y)], [2], [0], [g["lambda"]], 1)
    d = L.to_device(w)
    out = {}
    for rounds in (0, 1):
        plan = L.Plan.for_workload(w, flags=QF | L.FLAG_NO_FINISHER, max_rounds=rounds)
        out[rounds] = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
        torch.cuda.synchronize()
    assert out[0]["obj"][0] >= g["f_opt"] + 0.5
    assert out[1]["status"][0] in OK
    assert abs(out[1]["obj"][0] - g["f_opt"]) <= 1e-5 * g["f_opt"]
    np.testing.assert_allclose(out[1]["b"], g["b_opt"], rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("kernel", ["wave", "plain"])
def test_quadrature_edge_shapes(torch, kernel):
    """Shapes across every register-slot count and ragged tail (n = 1 ..
    2048, p = 1 .. 32), with the quadrature sections."""
    from test_gpu_parity import _pack, assert_parity, gpu_solve
    rng = np.random.default_rng(13)
    blocks, lams = [], []
    for n in [1, 2, 5, 63, 64, 65, 129, 257, 513, 1025, 2048]:
        for p in [1, 2, 17, 32]:
            X = rng.standard_normal((n, p))
            y = X[:, : min(p, 3)] @ rng.uniform(-3, 3, min(p, 3)) + rng.laplace(0, 1, n)
            blocks.append((X, y))
            lams.append(float(10 ** rng.uniform(-2, 1)))
    w = _pack(blocks, lams)
    plan, g = gpu_solve(torch, w, plain=(kernel == "plain"), flags=QF)
    assert_parity(w, g, oracle_ref(w), min_strict=0.0)


@pytest.mark.parametrize("kernel", ["wave", "plain"])
def test_quadrature_degenerate_inputs(torch, kernel):
    """y = 0, a zero column (no kinks on that axis), duplicated rows (equal
    kinks), lambda above lambda_max and lambda = 0."""
    from test_gpu_parity import _pack, gpu_solve
    rng = np.random.default_rng(4)
    n, p = 100, 6
    X = rng.standard_normal((n, p))
    y = X @ np.array([1.0, 0, -2, 0, 0, 0.5]) + rng.laplace(0, 1, n)
    Xz = X.copy()
    Xz[:, 3] = 0.0
    Xd = np.repeat(X[:50], 2, axis=0)
    yd = np.repeat(y[:50], 2)
    blocks = [(X, np.zeros(n)), (Xz, y), (Xd, yd), (X, y), (X, y)]
    lmax = float(np.max(np.abs(X.astype(np.float32).astype(np.float64).T @ np.sign(y))))
    w = _pack(blocks, [1.0, 1.0, 0.5, 1.5 * lmax, 0.0])
    plan, g = gpu_solve(torch, w, plain=(kernel == "plain"), flags=QF)
    fails, st = compare(w, g, oracle_ref(w))
    assert not fails, fails
    assert g["obj"][0] == 0.0 and np.all(g["b"][:p] == 0)
    assert g["b"][p * 1 + 3] == 0.0
    assert np.all(g["b"][3 * p: 4 * p] == 0) and g["active"][3] == 0


def test_quadrature_full_c2_sampled(torch):
    """All 4096 ragged row subsets with quadrature sections in one plan: every
    output certified, 64 seeded solves against the oracle."""
    from test_gpu_full_sizes import check_every_output
    w = W.config2()
    print(f"[gpu] quadrature sections, full c2 solves={w.num_solves}", flush=True)
    plan = L.Plan.for_workload(w, flags=QF)
    d = L.to_device(w)
    g = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    check_every_output(w, g)
    sample = np.sort(np.random.default_rng(22).choice(w.num_solves, size=64, replace=False))
    fails, st = compare(w, g, oracle_ref(w, solves=sample), solves=sample)
    print(st, flush=True)
    assert not fails, fails[:5]


def test_quadrature_path_graph_and_backward(torch):
    """A 4-step lambda path of ragged problems with quadrature sections: the
    HIP graph path (one launch per step) equals the in-kernel path bit for
    bit, and the backward at the last step matches the oracle's vertex-form
    gradient where the optimum is strictly unique."""
    from test_gpu_backward_path import check_backward
    w = W.config4(problems=range(12), path_len=4)
    d = L.to_device(w)
    plan = L.Plan.for_workload(w, flags=QF)
    ref_out = plan.solve(d["X"], d["y"], d["lam"])
    ref = to_numpy(ref_out)
    out = plan.alloc_outputs()
    graph = plan.graph(d["X"], d["y"], d["lam"], out)
    graph.launch()
    torch.cuda.synchronize()
    got = to_numpy(out)
    for key in ("b", "obj", "active", "zero_rows", "status"):
        assert np.array_equal(got[key], ref[key]), key
    g = torch.from_numpy(w.grad_b).cuda()
    gy, gX = plan.backward(d["X"], ref_out, g, step=w.path_len - 1)
    torch.cuda.synchronize()
    oref = oracle_ref(w)
    checked = check_backward(w, ref, gy.cpu().numpy(), gX.cpu().numpy(), oref, w.grad_b, w.path_len - 1, 1)
    print(f"gradients checked against the oracle: {checked}", flush=True)
