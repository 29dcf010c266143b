"""GPU: exact solve by vertex enumeration (Section 3.2) against the oracle's
vertex enumeration (itself pinned against HiGHS and the c0 golden file),
and against the wave-kernel solver on the same problems."""
import json
import os

import numpy as np
import pytest

import oracle as O
import paper_2510_15649_amd as L
from paper_2510_15649_amd import workloads as W
from parity import compare, oracle_ref, to_numpy

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def run_brute(w):
    print(f"[gpu] vertex enumeration {w.name}", flush=True)
    plan = L.Plan.for_workload(w)
    d = L.to_device(w)
    out = to_numpy(plan.brute_force(d["X"], d["y"], d["lam"]))
    return plan, d, out


def test_brute_c0_golden(torch):
    """The c0 instance at the golden file's lambdas: the enumerated minimum
    equals the stored brute-force optimum."""
    gold = json.load(open(os.path.join(GOLD, "c0_bruteforce.json")))
    w0 = W.config0()
    X, y = w0.block(0)
    checked = 0
    for case in gold["cases"]:
        if case["data"] != "f32":   # the GPU solves the float32 instance
            continue
        lam = float(case["lambda"])
        w = W._pack("c0", [(X.astype(np.float64), y.astype(np.float64))], [3], [0], [lam], 1)
        plan, d, out = run_brute(w)
        f = float(out["obj"][0])
        assert abs(f - case["f"]) <= 1e-6 * max(1.0, abs(case["f"])), (lam, f, case["f"])
        assert abs(np.abs(y - X @ out["b"].astype(np.float64)).sum() + lam * np.abs(out["b"]).sum()
                   - case["f"]) <= 1e-5 * max(1.0, abs(case["f"]))
        assert int(out["vertices"][0]) == case["vertices"]
        checked += 1
    assert checked >= 3


def test_brute_paper_sizes_vs_oracle(torch):
    """Ragged problems n in [5, 20], p in [1, 4] at three lambdas: minimum
    f equal to the oracle's enumeration (fp64 on both sides; the output is
    fp32), b equal where the optimum is unique, vertex counts consistent."""
    w = W.paper_sizes(num_problems=160, n_range=(5, 20), p_range=(1, 4))
    plan, d, out = run_brute(w)
    Lp = w.path_len
    b_off = np.concatenate([[0], np.cumsum(w.p[w.problem])[:-1]])
    uniq_checked = 0
    for s in range(w.num_solves):
        k = int(w.problem[s])
        Xk, yk = w.block(k)
        n, p = Xk.shape
        lam = float(w.lam[s])
        fo, bo, cnt = O.brute_force(Xk, yk, lam)
        fg = float(out["obj"][s])
        assert abs(fg - fo) <= 1e-6 * max(1.0, fo), (s, fg, fo)
        bg = out["b"][b_off[s]:b_off[s] + p].astype(np.float64)
        fb = float(np.abs(yk - Xk @ bg).sum() + lam * np.abs(bg).sum())
        assert abs(fb - fo) <= 1e-5 * max(1.0, fo), (s, fb, fo)
        vg = int(out["vertices"][s])
        from math import comb
        assert vg <= comb(n + p, p) and abs(vg - cnt) <= max(2, cnt // 100), (s, vg, cnt)
        _, info = O.solve(Xk, yk, lam, max_rounds=0)
        if info["unique"] and info["margin_uc"] >= 1e-4 and info["margin_r"] >= 4e-6:
            assert np.max(np.abs(bg - bo)) <= 1e-4 * max(1.0, np.abs(bo).max()), (s, bg, bo)
            uniq_checked += 1
    assert uniq_checked >= 200, uniq_checked


def test_brute_agrees_with_wave_solver(torch):
    """The paper's largest evaluation size (n = 30, p = 5): enumeration and
    the wave-kernel solver (coordinate descent, chop, certificate) reach the
    same minimum on the GPU, and both match the oracle's solver."""
    w = W.paper_sizes(num_problems=64, n_range=(30, 30), p_range=(5, 5))
    plan, d, out = run_brute(w)
    sol = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
    f_brute = out["obj"].astype(np.float64)
    f_wave = sol["obj"].astype(np.float64)
    assert np.all(np.abs(f_brute - f_wave) <= 1e-5 * np.maximum(1.0, f_brute))
    fails, st = compare(w, sol, oracle_ref(w))
    assert not fails, fails[:3]


def test_brute_rejects_large_problems(torch):
    w = W.config1(num_problems=1)
    plan = L.Plan.for_workload(w)
    d = L.to_device(w)
    with pytest.raises(L.LadlError):
        plan.brute_force(d["X"], d["y"], d["lam"])


def test_brute_p5_to_p8_vs_oracle(torch):
    """The kernel instances for p = 5 .. 8 (n in [8, 14], three lambdas, 8
    problems per p) against the oracle's enumeration: the minimum, the
    minimiser where it is unique, and the count of vertices."""
    from math import comb
    blocks, ps = [], []
    for p in (5, 6, 7, 8):
        wp = W.paper_sizes(replica=p, num_problems=8, n_range=(8, 14), p_range=(p, p))
        for k in range(wp.num_problems):
            blocks.append(wp.block(k, np.float32))
            ps.append(p)
    lams = (0.1, 1.0, 10.0)
    P = len(blocks)
    w = W._pack("p = 5..8 enumeration", blocks, ps, np.repeat(np.arange(P), 3), np.tile(lams, P), 1)
    plan, d, out = run_brute(w)
    b_off = np.concatenate([[0], np.cumsum(w.p[w.problem])[:-1]])
    seen_p, uniq = set(), 0
    for s in range(w.num_solves):
        k = int(w.problem[s])
        Xk, yk = w.block(k)
        n, p = Xk.shape
        lam = float(w.lam[s])
        fo, bo, cnt = O.brute_force(Xk, yk, lam)
        fg = float(out["obj"][s])
        assert abs(fg - fo) <= 1e-6 * max(1.0, fo), (s, p, fg, fo)
        bg = out["b"][b_off[s]:b_off[s] + p].astype(np.float64)
        fb = float(np.abs(yk - Xk @ bg).sum() + lam * np.abs(bg).sum())
        assert abs(fb - fo) <= 1e-5 * max(1.0, fo), (s, p, fb, fo)
        vg = int(out["vertices"][s])
        assert vg <= comb(n + p, p) and abs(vg - cnt) <= max(2, cnt // 100), (s, vg, cnt)
        _, info = O.solve(Xk, yk, lam, max_rounds=0)
        if info["unique"] and info["margin_uc"] >= 1e-4 and info["margin_r"] >= 4e-6:
            assert np.max(np.abs(bg - bo)) <= 1e-4 * max(1.0, np.abs(bo).max()), (s, bg, bo)
            uniq += 1
        seen_p.add(p)
    assert seen_p == {5, 6, 7, 8}
    assert uniq >= 48, uniq
