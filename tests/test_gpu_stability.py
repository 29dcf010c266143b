"""GPU: subset-stability selection frequencies.  The counting kernel is
checked bit-exactly against the oracle's counting on seeded synthetic
masks; the whole pipeline (solve many row subsets, count) against the
oracle's pipeline within the bound that non-unique optima allow."""
import numpy as np
import pytest

import oracle as O
import paper_2510_15649_amd as L
from paper_2510_15649_amd import workloads as W
from parity import oracle_ref, strict_unique, to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def test_counting_exact_on_synthetic_masks(torch):
    """Seeded masks, statuses and groups (every status code, 4 groups, a
    3-step path): counts equal the oracle's exactly, frequencies to fp32
    rounding."""
    rng = np.random.default_rng(17)
    S, Lp, G = 3000, 3, 4
    active = rng.integers(0, 2 ** 32, size=S * Lp, dtype=np.uint64).astype(np.uint32)
    status = rng.integers(0, 6, size=S * Lp).astype(np.int32)
    group = rng.integers(0, G, size=S).astype(np.int32)
    plan = L.Plan(np.arange(S + 1), 1, x_len=S, y_len=S, path_len=Lp)
    out = {"active": torch.from_numpy(active.view(np.int32)).cuda(), "status": torch.from_numpy(status).cuda()}
    res = plan.selection_frequency(out, group=torch.from_numpy(group).cuda(), num_groups=G)
    torch.cuda.synchronize()
    freq, cnt = O.selection_frequency(active, status, group, G, Lp)
    counts = res["counts"].cpu().numpy()
    assert np.array_equal(counts[:, :, 32], cnt.astype(np.int64))
    bits = ((active.reshape(S, Lp)[:, :, None].astype(np.uint64) >> np.arange(32, dtype=np.uint64)) & 1)
    for g in range(G):
        ok = (group[:, None] == g) & ((status.reshape(S, Lp) == L.CERTIFIED) | (status.reshape(S, Lp) == L.NONUNIQUE))
        assert np.array_equal(counts[g, :, :32], (bits * ok[:, :, None]).sum(axis=0))
    assert np.allclose(res["freq"].cpu().numpy(), freq, rtol=1e-6, atol=1e-7)
    assert int(res["bad_group"].cpu()[0]) == 0
    bad = group.copy()
    bad[5] = G
    res2 = plan.selection_frequency(out, group=torch.from_numpy(bad).cuda(), num_groups=G)
    torch.cuda.synchronize()
    assert int(res2["bad_group"].cpu()[0]) == 1


def test_row_subset_stability_c2(torch):
    """512 row subsets of the correlated base dataset (p = 16, 5 informative
    features): frequencies from the GPU solves against those from the
    oracle's solves, within (subsets with a non-unique optimum)/(subsets)."""
    w = W.config2(num_subsets=512)
    print(f"[gpu] stability {w.name}", flush=True)
    plan = L.Plan.for_workload(w)
    d = L.to_device(w)
    out = plan.solve(d["X"], d["y"], d["lam"])
    res = plan.selection_frequency(out)
    torch.cuda.synchronize()
    g = to_numpy(out)
    ref = oracle_ref(w)
    ok = (ref["cert"] >= 1)
    assert ok.all()
    freq_o, cnt_o = O.selection_frequency(ref["smask"], np.where(ok, 0, 5), np.zeros(w.num_solves, int), 1, 1)
    uniq = np.array([strict_unique(ref, o) for o in range(w.num_solves)])
    assert uniq.mean() >= 0.95, uniq.mean()
    nonunique = int(np.sum(~uniq))
    fg = res["freq"].cpu().numpy()[0, 0]
    assert res["counts"].cpu().numpy()[0, 0, 32] == w.num_solves
    assert np.all(np.abs(fg - freq_o[0, 0]) <= nonunique / w.num_solves + 1e-6), (fg[:16], freq_o[0, 0, :16])
    # where a subset's optimum is unique (with margin) the active sets agree exactly
    assert np.array_equal(g["active"][uniq], ref["smask"][uniq].astype(np.uint32))
    print("selection frequencies", np.round(fg[:16], 3), flush=True)
