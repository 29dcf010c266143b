"""GPU parity of the wavefront-per-solve kernels against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
import paper_2510_15649_amd as L
from paper_2510_15649_amd import workloads as W
from parity import compare, oracle_ref, to_numpy

pytestmark = pytest.mark.gpu


KERNELS = pytest.mark.parametrize("kernel", ["wave", "plain"])


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def gpu_solve(torch, w, plain=False, **opts):
    print(f"[gpu] {w.name} solves={w.num_solves} path={w.path_len} opts={opts} plain={plain}", flush=True)
    plan = L.Plan.for_workload(w, **opts)
    d = L.to_device(w)
    fn = plan.solve_plain if plain else plan.solve
    out = fn(d["X"], d["y"], d["lam"])
    torch.cuda.synchronize()
    return plan, to_numpy(out)


def assert_parity(w, gpu, ref, solves=None, min_strict=0.5):
    fails, st = compare(w, gpu, ref, solves)
    print(st, flush=True)
    assert not fails, f"{len(fails)} mismatches, first: {fails[:5]}"
    assert st["strict"] >= min_strict * st["outputs"], st


@KERNELS
def test_c0_fp32(torch, kernel):
    w = W.config0()
    plan, g = gpu_solve(torch, w, plain=(kernel == "plain"))
    ref = oracle_ref(w)
    assert_parity(w, g, ref, min_strict=1.0)
    # brute force on the same fp32 instance (Section 3.2)
    Xk, yk = w.block(0)
    fb, bb, _ = O.brute_force(Xk, yk, 1.0)
    assert abs(g["obj"][0] - fb) <= 1e-5 * fb


@KERNELS
def test_c1_subset(torch, kernel):
    w = W.config1(num_problems=48)
    plan, g = gpu_solve(torch, w, plain=(kernel == "plain"))
    assert_parity(w, g, oracle_ref(w))


@KERNELS
def test_c3_subset(torch, kernel):
    w = W.config3(num_problems=96)
    plan, g = gpu_solve(torch, w, plain=(kernel == "plain"))
    assert_parity(w, g, oracle_ref(w))


@KERNELS
def test_c2_subset(torch, kernel):
    w = W.config2(num_subsets=160)
    plan, g = gpu_solve(torch, w, plain=(kernel == "plain"))
    assert_parity(w, g, oracle_ref(w))


@pytest.mark.parametrize("opts", [dict(max_rounds=0), dict(max_rounds=1, flags=L.FLAG_GOLDEN),
                                  dict(max_rounds=1, flags=0),
                                  dict(max_rounds=2, tol_s=1e-3), dict(chop_range=1.0, max_sweeps=64),
                                  dict(chop_range=1e-3, max_sweeps=1), dict(max_rounds=-1, schedule=0),
                                  dict(schedule=1)])
def test_schedules(torch, opts):
    w = W.config1(num_problems=16)
    plan, g = gpu_solve(torch, w, **opts)
    assert_parity(w, g, oracle_ref(w))


def test_dense_variant_ragged(torch):
    """Ragged row subsets with every bucket in the HBM workspace and the
    4-waves-per-SIMD kernel variant for n <= 256."""
    w = W.config2(num_subsets=160)
    plan, g = gpu_solve(torch, w, schedule=1)
    desc = plan.describe()
    print(desc, flush=True)
    assert "(dense)" in desc
    assert_parity(w, g, oracle_ref(w))


def _pack(blocks, lams):
    """blocks: list of (X, y) float64 -> workload with one solve per block"""
    from paper_2510_15649_amd.workloads import _pack as pack
    return pack("edge", blocks, [b[0].shape[1] for b in blocks], np.arange(len(blocks)), lams, 1)


@KERNELS
def test_edge_shapes(torch, kernel):
    rng = np.random.default_rng(3)
    blocks, lams = [], []
    for n in [1, 2, 3, 5, 63, 64, 65, 127, 128, 129, 255, 257, 511, 513, 1000, 1024, 1025, 1500, 2048]:
        for p in [1, 2, 5, 17, 32]:
            X = rng.standard_normal((n, p))
            y = X[:, : min(p, 3)] @ rng.uniform(-3, 3, min(p, 3)) + rng.laplace(0, 1, n)
            blocks.append((X, y))
            lams.append(float(10 ** rng.uniform(-2, 1)))
    w = _pack(blocks, lams)
    plan, g = gpu_solve(torch, w, plain=(kernel == "plain"))
    assert_parity(w, g, oracle_ref(w), min_strict=0.0)


@KERNELS
def test_degenerate_inputs(torch, kernel):
    rng = np.random.default_rng(4)
    n, p = 100, 6
    X = rng.standard_normal((n, p))
    y = X @ np.array([1.0, 0, -2, 0, 0, 0.5]) + rng.laplace(0, 1, n)
    Xz = X.copy()
    Xz[:, 3] = 0.0                       # zero column
    Xd = np.repeat(X[:50], 2, axis=0)    # duplicated rows (equal kinks)
    yd = np.repeat(y[:50], 2)
    blocks = [(X, np.zeros(n)),          # y = 0 -> b = 0, f = 0
              (Xz, y),
              (Xd, yd),
              (X, y),                    # lambda above lambda_max -> b = 0
              (X, y)]                    # lambda = 0: plain LAD
    lmax = float(np.max(np.abs(X.astype(np.float32).astype(np.float64).T @ np.sign(y))))
    w = _pack(blocks, [1.0, 1.0, 0.5, 1.5 * lmax, 0.0])
    plan, g = gpu_solve(torch, w, plain=(kernel == "plain"))
    fails, st = compare(w, g, oracle_ref(w))
    assert not fails, fails
    assert g["obj"][0] == 0.0 and np.all(g["b"][:p] == 0)
    assert g["b"][p * 1 + 3] == 0.0
    assert np.all(g["b"][3 * p: 4 * p] == 0) and g["active"][3] == 0


@KERNELS
def test_status_codes(torch, kernel):
    rng = np.random.default_rng(5)
    n, p = 80, 4
    blocks = [(rng.standard_normal((n, p)), rng.standard_normal(n)) for _ in range(4)]
    blocks[1][0][7, 2] = np.nan
    blocks[2][1][3] = np.inf
    w = _pack(blocks, [1.0, 1.0, 1.0, -1.0])
    plan, g = gpu_solve(torch, w, plain=(kernel == "plain"))
    assert list(g["status"]) [1:] == [L.NONFINITE, L.NONFINITE, L.BADLAMBDA]
    assert g["status"][0] in (L.CERTIFIED, L.NONUNIQUE)
    fails, _ = compare(w, g, oracle_ref(w, solves=[0]), solves=[0])
    assert not fails


def test_validation_errors(torch):
    ro = np.array([0, 10, 20], dtype=np.int64)
    with pytest.raises(L.LadlError) as e:
        L.Plan(ro, 33, x_len=20 * 33, y_len=20)
    assert e.value.code == L.EUNSUPPORTED
    with pytest.raises(L.LadlError) as e:
        L.Plan(np.array([1, 10, 20]), 3, x_len=60, y_len=20)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LadlError) as e:
        L.Plan(np.array([0, 10, 10]), 3, x_len=60, y_len=20)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LadlError) as e:
        L.Plan(ro, 3, x_len=59, y_len=20)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LadlError) as e:
        L.Plan(ro, 3, x_len=60, y_len=20, problem=[0, 2])
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LadlError) as e:
        L.Plan(ro, 3, x_len=60, y_len=20, max_sweeps=0)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LadlError) as e:
        L.Plan(ro, 3, x_len=60, y_len=20, chop_range=0.0)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LadlError) as e:
        L.Plan(ro, 3, x_len=60, y_len=20, schedule=2)
    assert e.value.code == L.EINVAL


def test_c1_full_size_sampled(torch):
    """The full c1 workload (512 problems x 16 lambdas, 8192 solves, one
    launch per bucket as timed by the benchmark); parity on a seeded sample
    of 512 solves."""
    w = W.config1()
    plan, g = gpu_solve(torch, w)
    print(plan.describe(), flush=True)
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(w.num_solves, size=512, replace=False))
    fails, st = compare(w, g, oracle_ref(w, solves=sample), solves=sample)
    print(st, flush=True)
    assert not fails, fails[:5]
    assert np.all(np.isin(g["status"], [L.CERTIFIED, L.NONUNIQUE]))


def test_autotune_then_solve(torch, tmp_path, monkeypatch):
    """The autotuner times both X placements per bucket on the caller's data,
    caches its choice, and the tuned plan keeps parity."""
    monkeypatch.setenv("LADL_TUNE_CACHE", str(tmp_path / "tune.txt"))
    w = W.config2(num_subsets=96)
    plan = L.Plan.for_workload(w)
    d = L.to_device(w)
    out = plan.alloc_outputs()
    plan.autotune(d["X"], d["y"], d["lam"], out)
    print(plan.describe(), flush=True)
    out = plan.solve(d["X"], d["y"], d["lam"])
    torch.cuda.synchronize()
    assert_parity(w, to_numpy(out), oracle_ref(w))
    assert (tmp_path / "tune.txt").exists()
    plan2 = L.Plan.for_workload(w)          # second plan reads the cache
    plan2.autotune(d["X"], d["y"], d["lam"], plan2.alloc_outputs())
    assert plan2.describe() == plan.describe()
