"""Benchmark: batched LAD-LASSO solves/s on one MI355X.

One step = one forward pass of the whole solve path (CCD with exact
weighted-median coordinate updates, ternary chop, vertex snap and
certificate, finisher) over one batch; the default workload is 512
problems (n=200, p=8) x 16 lambdas = 8192 solves.  Inputs are resident in
HBM before timing starts.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# fp32 VALU lane-ops/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (an FMA counted once)
PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
# algorithmic lane-ops per row of one exact coordinate update: sign test of
# r_i x_ij, |x_ij|, two weight accumulations (below / at the current value),
# one residual FMA
OPS_PER_ROW_UPDATE = 5


def make_workload(cfg: str):
    from paper_2510_15649_amd import workloads as W
    if cfg == "c1":
        return W.config1()
    if cfg == "c1path":
        return W.config1(as_path=True)
    if cfg == "c2":
        return W.config2()
    if cfg == "c3":
        return W.config3()
    raise SystemExit(f"unknown config {cfg}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c1")
    ap.add_argument("--max-rounds", type=int, default=1)
    ap.add_argument("--golden", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--parity-sample", type=int, default=256)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): problems are independent, so a "
              f"multi-GPU run is the same kernel on each GPU's share of the queue", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_15649_amd as L

    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    w = make_workload(args.config)
    flags = L.FLAG_GOLDEN if args.golden else 0
    plan = L.Plan.for_workload(w, max_rounds=args.max_rounds, flags=flags)
    d = L.to_device(w, dev)
    out = plan.alloc_outputs(dev, iters=True)
    stream = torch.cuda.current_stream()
    n_out = w.num_solves * w.path_len

    def step():
        plan.solve(d["X"], d["y"], d["lam"], out=out, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    solves_per_s = n_out / (ms_per_step / 1e3)

    g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    it = g["iters"].reshape(-1, 4)
    ns = np.diff(w.row_off)[w.problem]
    ns_out = np.repeat(ns, w.path_len)
    row_updates = float(np.sum(it[:, 1].astype(np.float64) * ns_out))
    lane_ops = OPS_PER_ROW_UPDATE * row_updates
    achieved_ops = lane_ops / (ms_per_step / 1e3)
    alg_bytes = w.algorithmic_bytes()
    hbm_gbs = alg_bytes / (ms_per_step / 1e3) / 1e9
    status_counts = {L.STATUS_NAMES[s]: int(c) for s, c in zip(*np.unique(g["status"], return_counts=True))}

    # parity sample against the FP64 oracle (the metric counts only if it passes)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import compare, oracle_ref
    rng = np.random.default_rng(2024)
    sample = np.sort(rng.choice(w.num_solves, size=min(args.parity_sample, w.num_solves), replace=False))
    fails, pst = compare(w, g, oracle_ref(w, solves=sample), solves=sample)
    parity_ok = not fails

    plain = None
    if not args.no_plain:
        try:
            out_p = plan.alloc_outputs(dev, iters=False)
            plan.solve_plain(d["X"], d["y"], d["lam"], out=out_p, stream=stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            plan.solve_plain(d["X"], d["y"], d["lam"], out=out_p, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            pms = e0.elapsed_time(e1)
            gp = {k: v.cpu().numpy() for k, v in out_p.items() if v is not None}
            pf, _ = compare(w, gp, oracle_ref(w, solves=sample), solves=sample)
            plain = {"value": n_out / (pms / 1e3), "ms_per_step": pms, "parity_ok": not pf}
        except L.LadlError as e:
            plain = {"error": str(e)}

    cpu = None
    if not args.no_cpu:
        import oracle as O
        threads = min(os.cpu_count() or 1, 16)
        k = max(1, min(w.num_solves, 64))
        solves = np.sort(rng.choice(w.num_solves, size=k, replace=False))
        opts = dict(max_rounds=args.max_rounds, tol_f=1e-6, tol_s=2.0 ** -20, max_sweeps=64, max_ternary=48)
        r = O.solve_batch(w, nthreads=threads, solves=solves, **opts)
        # grow the sample until the CPU work is ~10 s
        while r["seconds"] < 5.0 and k < w.num_solves:
            k = min(w.num_solves, k * 4)
            solves = np.sort(rng.choice(w.num_solves, size=k, replace=False))
            r = O.solve_batch(w, nthreads=threads, solves=solves, **opts)
        cpu = {"value": k * w.path_len / r["seconds"], "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"{k} of {w.num_solves} solves (uniform, seeded), FP64 C oracle, same schedule "
                         f"(max_rounds={args.max_rounds}), {r['seconds']:.1f} s"}

    line = {
        "metric": "LAD-LASSO solves/sec at 1e-5 rel objective vs plain kernel; achieved HBM GB/s",
        "value": solves_per_s if parity_ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded generator, no dataset)",
        "config": {"workload": w.name, "solves_per_step": n_out, "max_rounds": args.max_rounds,
                   "golden": bool(args.golden), "parallelism": "1 GPU, wave per solve"},
        "roofline": {"bound": "alu", "achieved": achieved_ops / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved_ops / PEAK_VALU_LANE_OPS, "traffic": None,
                     "work_per_launch": lane_ops, "row_updates": row_updates},
        "hbm": {"achieved_GBs": hbm_gbs, "peak_GBs": PEAK_HBM_GBS, "frac": hbm_gbs / PEAK_HBM_GBS,
                "algorithmic_bytes": alg_bytes},
        "cpu_baseline": cpu,
        "plain_kernel": plain,
        "vs_plain": (solves_per_s / plain["value"]) if plain and "value" in plain else None,
        "parity": {"ok": parity_ok, "sample": int(len(sample)), **pst, "first_failures": [str(f) for f in fails[:3]]},
        "status": status_counts,
        "iters_mean": {"sweeps": float(it[:, 0].mean()), "updates": float(it[:, 1].mean()),
                       "probes": float(it[:, 2].mean()), "pivots": float(it[:, 3].mean())},
        "wall_s_timed": wall,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
