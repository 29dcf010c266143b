"""GPU: backward kernel, autograd layer, lambda paths (in-kernel and HIP
graph), and the large ragged c4 workload on a sample."""
import numpy as np
import pytest

import oracle as O
import paper_2510_15649_amd as L
from paper_2510_15649_amd import workloads as W
from parity import compare, gradient_error, oracle_ref, strict_unique, to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def solve_and_backward(torch, w, grad, step=None, **opts):
    print(f"[gpu] {w.name} solves={w.num_solves} path={w.path_len} backward", flush=True)
    plan = L.Plan.for_workload(w, **opts)
    d = L.to_device(w)
    out = plan.solve(d["X"], d["y"], d["lam"])
    g = torch.from_numpy(grad).cuda()
    gy, gX = plan.backward(d["X"], out, g, step=-1 if step is None else step)
    torch.cuda.synchronize()
    return plan, to_numpy(out), gy.cpu().numpy(), gX.cpu().numpy()


def check_backward(w, gpu, gy, gX, ref, grad, step, min_checked):
    """Every output's gradient block: zero without a certificate; at an
    optimum the oracle certifies unique with fp32-resolvable margins, the
    oracle's vertex-form gradient (and the GPU must have certified it);
    elsewhere (certified, not strictly unique) the vertex-form gradient at
    the GPU's own vertex.  Returns the number checked against the oracle."""
    Lp = w.path_len
    checked = 0
    for s in range(w.num_solves):
        k = int(w.problem[s])
        n, p = w.n(k), int(w.p[k])
        o = s * Lp + step
        xo, ro = int(w.x_off[k]), int(w.row_off[k])
        gyk = gy[ro:ro + n]
        gXk = gX[xo:xo + n * p].reshape(n, p)
        st = int(gpu["status"][o])
        if st not in (L.CERTIFIED, L.NONUNIQUE):
            assert np.all(gyk == 0) and np.all(gXk == 0)
            continue
        Xk, yk = w.block(k)
        goff = int(ref["b_off"][s])
        gk = grad[goff:goff + p]
        if strict_unique(ref, o):
            assert st == L.CERTIFIED, (s, st)
            bo = Lp * int(ref["b_off"][s]) + step * p
            bref = ref["b"][bo:bo + p]
            Z = [z for z in ref["zrows"][o] if z >= 0]
            err = gradient_error(Xk, yk, w.lam[o], bref, Z, gk, gyk, gXk)
            assert err <= 1e-4, (s, err)
            checked += 1
        else:
            bo = Lp * goff + step * p
            bg = gpu["b"][bo:bo + p]
            zg = gpu["zero_rows"][32 * o:32 * o + 32]
            err = gradient_error(Xk, yk, w.lam[o], bg, zg[zg >= 0], gk, gyk, gXk)
            assert err <= 1e-4, (s, st, err)
    assert checked >= min_checked, checked
    return checked


def test_backward_c3_vs_closed_form(torch):
    w = W.config3(num_problems=128)
    plan, g, gy, gX = solve_and_backward(torch, w, w.grad_b)
    ref = oracle_ref(w)
    fails, st = compare(w, g, ref)
    assert not fails, fails[:3]
    n = check_backward(w, g, gy, gX, ref, w.grad_b, 0, min_checked=120)
    print("checked", n, flush=True)


def test_backward_vs_finite_differences(torch):
    """The GPU gradient against FP64 central differences (step 1e-6) of the
    oracle's solution map, at entries whose perturbation keeps the vertex
    (away from kinks)."""
    w = W.config3(num_problems=12)
    plan, g, gy, gX = solve_and_backward(torch, w, w.grad_b)
    rng = np.random.default_rng(7)
    h = 1e-6
    checked = 0
    for s in range(w.num_solves):
        if g["status"][s] not in (L.CERTIFIED, L.NONUNIQUE):
            continue
        k = s
        Xk, yk = w.block(k)
        n, p = Xk.shape
        lam = float(w.lam[s])
        gb = w.grad_b[s * p:(s + 1) * p].astype(np.float64)
        b0, i0 = O.solve(Xk, yk, lam, max_rounds=0)
        if not i0["unique"]:
            continue
        Z0, S0 = i0["Z"], set(np.flatnonzero(b0))
        ents = [("y", i, 0) for i in Z0] + [("X", i, j) for i in Z0 for j in sorted(S0)]
        ents += [("y", int(rng.integers(n)), 0), ("X", int(rng.integers(n)), int(rng.integers(p)))]
        for kind, i, j in ents:
            Xp, Xm, yp, ym = Xk.copy(), Xk.copy(), yk.copy(), yk.copy()
            if kind == "y":
                yp[i] += h
                ym[i] -= h
                an = gy[int(w.row_off[k]) + i]
            else:
                Xp[i, j] += h
                Xm[i, j] -= h
                an = gX[int(w.x_off[k]) + i * p + j]
            bp, ip = O.solve(Xp, yp, lam, b_init=b0, max_rounds=0)
            bm, im = O.solve(Xm, ym, lam, b_init=b0, max_rounds=0)
            if not (ip["Z"] == im["Z"] == Z0 and set(np.flatnonzero(bp)) == set(np.flatnonzero(bm)) == S0):
                continue
            fd = (gb @ bp - gb @ bm) / (2 * h)
            assert abs(fd - an) <= 1e-4 * (1 + abs(fd)), (s, kind, i, j, fd, an)
            checked += 1
    assert checked >= 60, checked


def test_autograd_function(torch):
    from paper_2510_15649_amd.autograd import LadLassoFunction
    w = W.config3(num_problems=8)
    plan = L.Plan.for_workload(w)
    d = L.to_device(w)
    X = d["X"].clone().requires_grad_(True)
    y = d["y"].clone().requires_grad_(True)
    b = LadLassoFunction.apply(X, y, d["lam"], plan)
    g = torch.from_numpy(w.grad_b).cuda()
    (b * g).sum().backward()
    out = plan.solve(d["X"], d["y"], d["lam"])
    gy, gX = plan.backward(d["X"], out, g)
    torch.cuda.synchronize()
    assert torch.equal(X.grad, gX) and torch.equal(y.grad, gy)
    assert torch.equal(b.detach(), out["b"])


def test_lambda_path_in_kernel(torch):
    w = W.config1(num_problems=24, as_path=True)   # 24 solves x 16 descending lambdas
    plan = L.Plan.for_workload(w)
    d = L.to_device(w)
    out = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    fails, st = compare(w, out, oracle_ref(w))
    print(st, flush=True)
    assert not fails, fails[:3]


def test_graph_path_matches_in_kernel_path(torch):
    w = W.config1(num_problems=24, as_path=True)
    plan = L.Plan.for_workload(w)
    d = L.to_device(w)
    ref = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
    out = plan.alloc_outputs()
    graph = plan.graph(d["X"], d["y"], d["lam"], out)
    for rep in range(3):
        for v in out.values():
            if v is not None:
                v.fill_(-7)                  # eager work between replays
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        got = to_numpy(out)
        for key in ("b", "obj", "active", "zero_rows", "status"):
            assert np.array_equal(got[key], ref[key]), (rep, key)


def test_c4_sample_path_and_backward(torch):
    """A seeded sample of the large ragged workload: n up to 2048, p up to
    32, a 32-value descending lambda path per problem, backward at the last
    lambda."""
    rng = np.random.default_rng(4)
    ids = np.sort(rng.choice(65536, size=48, replace=False))
    w = W.config4(problems=ids)
    plan, g, gy, gX = solve_and_backward(torch, w, w.grad_b)
    print(plan.describe(), flush=True)
    ref = oracle_ref(w)
    fails, st = compare(w, g, ref)
    print(st, flush=True)
    assert not fails, fails[:3]
    check_backward(w, g, gy, gX, ref, w.grad_b, w.path_len - 1, min_checked=20)
