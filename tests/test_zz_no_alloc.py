"""GPU: the allocation-free entry point against the plan-based solve on the
same uniform batches, two calls in a row (the second on a smaller batch,
so it reuses the fixed scratch array left by the first)."""
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


def plan_solve(torch, w, d):
    plan = L.Plan.for_workload(w)
    out = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
    torch.cuda.synchronize()
    return out


def agree(w, ref, got):
    """Same statuses; objectives within 1e-5 relative; at certified outputs
    the same b (1e-4), support and zero rows."""
    Lp = w.path_len
    assert np.array_equal(got["status"], ref["status"])
    rel = np.abs(got["obj"].astype(np.float64) - ref["obj"]) / np.maximum(np.abs(ref["obj"]), 1e-30)
    assert np.max(rel) <= 1e-5, np.max(rel)
    cert = ref["status"] == L.CERTIFIED
    assert np.array_equal(got["active"][cert], ref["active"][cert])
    zr, zg = ref["zero_rows"].reshape(-1, 32), got["zero_rows"].reshape(-1, 32)
    assert np.array_equal(zg[cert], zr[cert])
    p = int(w.p[0])
    br, bg = ref["b"].reshape(-1, p), got["b"].reshape(-1, p)
    db = np.abs(bg[cert] - br[cert]) / np.maximum(1.0, np.abs(br[cert]))
    assert db.size == 0 or np.max(db) <= 1e-4, np.max(db)
    return int(cert.sum())


def test_noalloc_matches_plan_solve_twice(torch):
    big = W.config1(num_problems=256, num_lambda=4, as_path=True)    # n=200, p=8, 4-step paths
    small = W.config3(num_problems=48)                                # n=300, p=12, one lambda
    for w in (big, small):
        n, p = w.n(0), int(w.p[0])
        print(f"[gpu] no-alloc solve {w.name}: problems={w.num_problems} n={n} p={p} path={w.path_len}",
              flush=True)
        d = L.to_device(w)
        ref = plan_solve(torch, w, d)
        got = to_numpy(L.solve_uniform_noalloc(d["X"], d["y"], d["lam"], w.num_problems, n, p, w.path_len))
        torch.cuda.synchronize()
        ncert = agree(w, ref, got)
        assert ncert >= 0.9 * w.num_solves * w.path_len, ncert


def test_noalloc_quadrature_variant(torch):
    """The quadrature variant through the allocation-free entry point: the
    same outputs as the plan-based solve with the same flag."""
    w = W.config1(num_problems=64, num_lambda=2, as_path=True)
    n, p = w.n(0), int(w.p[0])
    d = L.to_device(w)
    plan = L.Plan.for_workload(w, flags=L.FLAG_QUADRATURE)
    ref = to_numpy(plan.solve(d["X"], d["y"], d["lam"]))
    got = to_numpy(L.solve_uniform_noalloc(d["X"], d["y"], d["lam"], w.num_problems, n, p, w.path_len,
                                           flags=L.FLAG_QUADRATURE))
    torch.cuda.synchronize()
    assert agree(w, ref, got) >= 0.9 * w.num_solves * w.path_len


def test_noalloc_rejects_out_of_limits(torch):
    dev = "cuda"
    X = torch.zeros(2 * 1100 * 4, dtype=torch.float32, device=dev)
    y = torch.zeros(2 * 1100, dtype=torch.float32, device=dev)
    lam = torch.ones(2, dtype=torch.float32, device=dev)
    with pytest.raises(L.LadlError) as e:
        L.solve_uniform_noalloc(X, y, lam, 2, 1100, 4)
    assert e.value.code == L.EUNSUPPORTED
    with pytest.raises(L.LadlError) as e:
        L.solve_uniform_noalloc(X, y, lam[:1], 1, 10, 33)
    assert e.value.code == L.EUNSUPPORTED
