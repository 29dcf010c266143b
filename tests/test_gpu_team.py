"""GPU: teams of 2 and 4 wavefronts per solve (the rows of a problem split
between the waves of one workgroup) for the n > 1024 bucket, against the
oracle and against the one-wavefront schedule on the same problems."""
import numpy as np
import pytest

import paper_2510_15649_amd as L
from paper_2510_15649_amd import workloads as W
from parity import compare, oracle_ref, to_numpy

pytestmark = pytest.mark.gpu
OK = (L.CERTIFIED, L.NONUNIQUE)


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def big_and_small(n_big=24, n_small=8, path_len=8, seed=41):
    """Problems of the large ragged recipe: n_big with n > 1024 (mixed p,
    including n = 2048 and p = 32 when drawn) and n_small smaller ones."""
    rng = np.random.default_rng(seed)
    ns, ps = [], []
    for k in range(4096):
        g = W._rng(W.BASE_SEED + 4000, k)
        ns.append(int(g.integers(32, 2049)))
        ps.append(int(g.integers(4, 33)))
    ns, ps = np.array(ns), np.array(ps)
    big = np.flatnonzero(ns > 1024)
    small = np.flatnonzero(ns <= 1024)
    ids = np.union1d(rng.choice(big, size=n_big, replace=False), rng.choice(small, size=n_small, replace=False))
    return W.config4(problems=ids, path_len=path_len)


@pytest.mark.parametrize("team", [2, 4])
def test_team_schedule_parity(torch, team):
    w = big_and_small()
    print(f"[gpu] team of {team} waves: {w.num_problems} problems, path {w.path_len}", flush=True)
    d = L.to_device(w)
    plan = L.Plan.for_workload(w, team=team)
    desc = plan.describe()
    print(desc, flush=True)
    tws = dict(zip([b[0] for b in plan.buckets()], plan.waves_per_solve()))
    assert tws[32] == team and all(v == 1 for R, v in tws.items() if R != 32)
    g = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    fails, st = compare(w, g, oracle_ref(w))
    print(st, flush=True)
    assert not fails, fails[:5]
    assert st["strict"] >= 0.9 * st["unique"], st
    # the same problems with one wave per solve: the same optimum
    plan1 = L.Plan.for_workload(w, team=1)
    g1 = to_numpy(plan1.solve(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    assert np.all(np.isin(g["status"], OK)) and np.all(np.isin(g1["status"], OK))
    rel = np.abs(g["obj"].astype(np.float64) - g1["obj"]) / np.maximum(g1["obj"], 1e-30)
    assert np.max(rel) <= 2e-5, np.max(rel)


def test_team_graph_path_matches_in_kernel(torch):
    w = big_and_small(n_big=8, n_small=4, path_len=4, seed=42)
    d = L.to_device(w)
    plan = L.Plan.for_workload(w, team=4)
    ref = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
    out = plan.alloc_outputs()
    graph = plan.graph(d["X"], d["y"], d["lam"], out)
    for rep in range(2):
        for v in out.values():
            if v is not None:
                v.fill_(-7)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        got = to_numpy(out)
        for key in ("b", "obj", "active", "zero_rows", "status"):
            assert np.array_equal(got[key], ref[key]), (rep, key)


def test_autotune_chooses_among_teams(torch, tmp_path, monkeypatch):
    """The autotuner times one wave and teams of 2 and 4 for the n > 1024
    bucket on the caller's data and keeps parity with its choice."""
    monkeypatch.setenv("LADL_TUNE_CACHE", str(tmp_path / "tune.txt"))
    w = big_and_small(n_big=16, n_small=0, path_len=2, seed=43)
    d = L.to_device(w)
    plan = L.Plan.for_workload(w)
    plan.autotune(d["X"], d["y"], d["lam"], plan.alloc_outputs())
    print(plan.describe(), flush=True)
    g = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    fails, st = compare(w, g, oracle_ref(w))
    assert not fails, fails[:5]
    lines = open(tmp_path / "tune.txt").read().split()
    assert len(lines) >= 4 and int(lines[3]) in (1, 3, 4)
