"""Benchmark: batched LAD-LASSO solves/s on one MI355X.

One step = one forward pass of the whole solve path (cyclical coordinate
descent with exact weighted-median coordinate updates, ternary chop along
the locus of axis-wise minima, vertex snap and optimality certificate,
edge-descent finisher) over one batch.  The headline workload is 512
problems (n=200, p=8) x 16 lambdas = 8192 solves with the paper's schedule
(one ternary-chop round).  Inputs are resident in HBM before timing starts.
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

PEAK_HBM_GBS = 8000.0
# fp32 VALU lane-ops/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (an FMA counted once)
PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
# algorithmic lane-ops per row of one exact coordinate update: sign test of
# r_i x_ij, |x_ij|, two weight accumulations (below / at the current value),
# one residual FMA
OPS_PER_ROW_UPDATE = 5
METRIC = "LAD-LASSO solves/sec at 1e-5 rel objective vs plain kernel; achieved HBM GB/s"


def make_workload(cfg: str):
    from paper_2510_15649_amd import workloads as W
    return {"c1": lambda: W.config1(), "c1path": lambda: W.config1(as_path=True), "c2": lambda: W.config2(),
            "c3": lambda: W.config3(), "c4": lambda: W.config4(),
            "c4s": lambda: W.config4(problems=range(C4_SAMPLE))}[cfg]()


# problems of the 65536-problem ragged path workload timed by default (the
# generator draws each problem independently, so the first 4096 are a
# uniform sample of the full draw)
C4_SAMPLE = 4096


# device sources whose hash the committed byte-counter summaries record
KERNEL_SOURCES = ["ladl_solve_wave.hip", "ladl_wave.hpp", "ladl_common.hpp", "ladl_kernels.hpp"]


def kernel_source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_15649_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(summary, key):
    """HBM bytes per launch that a committed rocprofv3 summary under
    profiles/ records for `key` (FETCH_SIZE + WRITE_SIZE, scaled by a copy
    of known size), or None when the kernel sources changed since."""
    vals = {}
    try:
        with open(os.path.join(ROOT, "profiles", summary)) as fh:
            for line in fh:
                m = re.match(r"^\s*-\s*(\w+):\s*(\S+)\s*$", line)
                if m:
                    vals[m.group(1)] = m.group(2)
    except OSError:
        return None
    if vals.get("source_sha256") != kernel_source_sha() or key not in vals:
        return None
    return int(vals[key])


def log(msg):
    """Progress to stderr (the JSON line is the only stdout output)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def backward_bytes(w, out_np, step):
    """Algorithmic bytes of one backward launch: dL/dy and dL/dX written in
    full (n + n p floats per problem); read per certified solve: g, b, the
    zero-row list, status and the |S| x |S| vertex matrix."""
    wr = 4 * (w.X.size + w.y.size)
    L = w.path_len
    act = out_np["active"].reshape(-1, L)[:, step]
    ns = np.array([bin(int(a)).count("1") for a in act], dtype=np.int64)
    ps = w.p[w.problem].astype(np.int64)
    rd = int(np.sum(4 * (2 * ps + 32 + 1 + ns * ns)))
    return int(wr + rd)


def measure(L, torch, w, steps, warmup, parity_sample, autotune=False, **opts):
    """Times `steps` solves of workload w (after `warmup`), checks a seeded
    parity sample against the oracle.  Returns a dict."""
    from parity import compare, oracle_ref
    log(f"{w.name}: {w.num_solves * w.path_len} solves, options {opts}")
    dev = torch.device("cuda:0")
    plan = L.Plan.for_workload(w, **opts)
    d = L.to_device(w, dev)
    out = plan.alloc_outputs(dev, iters=True)
    stream = torch.cuda.current_stream()
    if autotune:
        plan.autotune(d["X"], d["y"], d["lam"], out, stream=stream)
    for _ in range(warmup):
        plan.solve(d["X"], d["y"], d["lam"], out=out, stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        plan.solve(d["X"], d["y"], d["lam"], out=out, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    log(f"{w.name}: {ms:.3f} ms per step; checking {min(parity_sample, w.num_solves)} solves against the oracle")
    n_out = w.num_solves * w.path_len
    g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    it = g["iters"].reshape(-1, 4)
    ns_out = np.repeat(np.diff(w.row_off)[w.problem], w.path_len)
    row_updates = float(np.sum(it[:, 1].astype(np.float64) * ns_out))
    rng = np.random.default_rng(2024)
    sample = np.sort(rng.choice(w.num_solves, size=min(parity_sample, w.num_solves), replace=False))
    fails, pst = compare(w, g, oracle_ref(w, solves=sample), solves=sample)
    status = {L.STATUS_NAMES[s]: int(c) for s, c in zip(*np.unique(g["status"], return_counts=True))}
    return dict(plan=plan, d=d, ms=ms, solves_per_s=n_out / (ms / 1e3), n_out=n_out, row_updates=row_updates,
                parity_ok=not fails, parity=pst, fails=fails, status=status,
                iters_mean={"sweeps": float(it[:, 0].mean()), "updates": float(it[:, 1].mean()),
                            "probes": float(it[:, 2].mean()), "pivots": float(it[:, 3].mean())},
                describe=plan.describe())


def path_graph_and_backward(L, torch, w, s, reps=5):
    """For a path workload already measured by `measure`: the same path as a
    replayed HIP graph (one launch per lambda step), and the backward kernel
    at the last lambda timed against the HBM roofline."""
    plan, d = s["plan"], s["d"]
    stream = torch.cuda.current_stream()
    out = plan.alloc_outputs(d["X"].device, iters=False)
    graph = plan.graph(d["X"], d["y"], d["lam"], out)
    graph.launch(stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    graph.launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1)
    log(f"{w.name}: path as a HIP graph {graph_ms:.3f} ms")
    step = w.path_len - 1
    g = d["grad_b"]
    gy = torch.empty(d["y"].numel(), dtype=torch.float32, device=d["X"].device)
    gX = torch.empty_like(d["X"])
    plan.backward(d["X"], out, g, step=step, grad_y=gy, grad_X=gX, stream=stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        plan.backward(d["X"], out, g, step=step, grad_y=gy, grad_X=gX, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    bms = e0.elapsed_time(e1) / reps
    log(f"{w.name}: backward {bms:.3f} ms per launch")
    onp = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    nbytes = backward_bytes(w, onp, step)
    gbs = nbytes / (bms / 1e3) / 1e9
    return graph_ms, {"workload": w.name, "kernel": "k_backward", "ms_per_launch": bms, "bound": "hbm",
                      "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                      "traffic": None, "algorithmic_bytes": nbytes}


def measure_cv(L, torch, folds=5, steps=3, sample=4):
    """K-fold cross-validation of the 512 c1 problems along their 16-lambda
    path (the training solves run on the wave kernels); parity of the fold
    errors on a few problems against the oracle's cross-validation."""
    import oracle as O
    from paper_2510_15649_amd import workloads as W
    w = W.config1(as_path=True)
    log(f"cross-validation: {w.num_problems} problems x {folds} folds x {w.path_len} lambdas")
    cv = L.CrossValidation.for_workload(w, folds)
    d = L.to_device(w)
    stream = torch.cuda.current_stream()
    out = cv.run(d["X"], d["y"], d["lam"], stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        out = cv.run(d["X"], d["y"], d["lam"], stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    g = {k: v.cpu().numpy() for k, v in out.items()}
    Lp, P = w.path_len, w.num_problems
    ferr = g["fold_error"].reshape(P, folds, Lp)
    worst = 0.0
    for k in range(sample):
        Xk, yk = w.block(k)
        ref = O.cv(Xk, yk, w.lam[k * Lp:(k + 1) * Lp], folds, max_rounds=0)
        u = ref["unique"]
        rel = np.abs(ferr[k][u] - ref["err"][u]) / np.maximum(1.0, ref["err"][u])
        worst = max(worst, float(rel.max()) if rel.size else 0.0)
    st = g["fold_status"]
    return {"workload": f"cross-validation of {w.name} (as a path), {folds} folds", "ms_per_step": ms,
            "selections_per_s": P / (ms / 1e3), "training_solves_per_s": P * folds * Lp / (ms / 1e3),
            "parity_sample_problems": sample, "max_rel_fold_error": worst, "parity_ok": worst <= 1e-5,
            "certified_or_nonunique": int(np.sum((st == L.CERTIFIED) | (st == L.NONUNIQUE))),
            "training_solves": int(st.size)}


def measure_brute(L, torch, steps=3, sample=16):
    """Vertex enumeration (Section 3.2) of 4096 problems of the paper's
    evaluation sizes at 3 lambdas; fp64 ALU roofline; parity of the minimum
    on a sample against the oracle's enumeration; the oracle's enumeration
    on one host thread for the same sample."""
    import oracle as O
    from math import comb
    from paper_2510_15649_amd import workloads as W
    w = W.paper_sizes()
    log(f"vertex enumeration: {w.name}")
    plan = L.Plan.for_workload(w)
    d = L.to_device(w)
    stream = torch.cuda.current_stream()
    out = plan.brute_force(d["X"], d["y"], d["lam"], stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        out = plan.brute_force(d["X"], d["y"], d["lam"], stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ns = np.diff(w.row_off)[w.problem]
    ps = w.p[w.problem]
    cand = np.array([comb(int(n) + int(p), int(p)) for n, p in zip(ns, ps)], dtype=np.float64)
    # per candidate: LU 2p^3/3, two triangular solves 2p^2, residuals 2np, |r| sums n
    flops = float(np.sum(cand * (2.0 * ps ** 3 / 3 + 2.0 * ps ** 2 + 2.0 * ns * ps + ns)))
    achieved = flops / (ms / 1e3) / 1e12
    obj = out["obj"].cpu().numpy()
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(w.num_solves, size=sample, replace=False))
    worst, t_cpu = 0.0, 0.0
    for s_ in pick:
        Xk, yk = w.block(int(w.problem[s_]))
        t0 = time.perf_counter()
        fo, _, _ = O.brute_force(Xk, yk, float(w.lam[s_]))
        t_cpu += time.perf_counter() - t0
        worst = max(worst, abs(float(obj[s_]) - fo) / max(1.0, fo))
    cpu_rate = sample / t_cpu * (cand.mean() / cand[pick].mean())
    return {"workload": f"vertex enumeration, {w.name}", "ms_per_step": ms,
            "solves_per_s": w.num_solves / (ms / 1e3), "candidate_vertices_per_step": float(cand.sum()),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s (fp64)",
                         "frac": achieved / 78.6},
            "parity_sample": sample, "max_rel_f": worst, "parity_ok": worst <= 1e-6,
            "oracle_1_thread_solves_per_s": cpu_rate}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c1")
    ap.add_argument("--max-rounds", type=int, default=1)
    ap.add_argument("--golden", action="store_true")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--parity-sample", type=int, default=256)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (a known-size reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solves are independent, so a "
              f"multi-GPU run is this kernel on each GPU's share of the queue", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_15649_amd as L

    assert torch.cuda.is_available()
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return
    log(f"generating workload {args.config}")
    w = make_workload(args.config)
    flags = L.FLAG_GOLDEN if args.golden else 0
    m = measure(L, torch, w, args.steps, args.warmup, args.parity_sample, args.autotune,
                max_rounds=args.max_rounds, flags=flags)
    ms = m["ms"]
    main_graph_ms, main_backward = None, None
    if w.path_len > 1 and w.grad_b is not None:
        main_graph_ms, main_backward = path_graph_and_backward(L, torch, w, m)
    lane_ops = OPS_PER_ROW_UPDATE * m["row_updates"]
    achieved_ops = lane_ops / (ms / 1e3)
    alg_bytes = w.algorithmic_bytes()
    hbm_gbs = alg_bytes / (ms / 1e3) / 1e9
    default_c1 = args.config == "c1" and args.max_rounds == 1 and not args.golden and not args.autotune
    traffic = recorded_traffic("k_wave_c1_hbm_bytes.md", "traffic_bytes_per_launch") if default_c1 else None

    plain = None
    if not args.no_plain:
        log("plain one-thread-per-solve kernel")
        from parity import compare, oracle_ref
        plan, d = m["plan"], m["d"]
        stream = torch.cuda.current_stream()
        out_p = plan.alloc_outputs(d["X"].device, iters=False)
        plan.solve_plain(d["X"], d["y"], d["lam"], out=out_p, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.solve_plain(d["X"], d["y"], d["lam"], out=out_p, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1)
        gp = {k: v.cpu().numpy() for k, v in out_p.items() if v is not None}
        rng = np.random.default_rng(2024)
        sample = np.sort(rng.choice(w.num_solves, size=min(args.parity_sample, w.num_solves), replace=False))
        pf, _ = compare(w, gp, oracle_ref(w, solves=sample), solves=sample)
        plain = {"value": m["n_out"] / (pms / 1e3), "ms_per_step": pms, "parity_ok": not pf}

    cpu = None
    if not args.no_cpu:
        log("oracle on the host cores")
        import oracle as O
        threads = min(os.cpu_count() or 1, 16)
        rng = np.random.default_rng(99)
        d_opt = L.default_options()
        opts = dict(max_rounds=args.max_rounds, tol_f=float(d_opt.tol_f), tol_s=float(d_opt.tol_s),
                    max_sweeps=int(d_opt.max_sweeps), max_ternary=int(d_opt.max_ternary),
                    chop_range=float(d_opt.chop_range))
        k = min(w.num_solves, 64)
        while True:
            solves = np.sort(rng.choice(w.num_solves, size=k, replace=False))
            r = O.solve_batch(w, nthreads=threads, solves=solves, **opts)
            if r["seconds"] >= 5.0 or k == w.num_solves:
                break
            k = min(w.num_solves, k * 4)
        cpu = {"value": k * w.path_len / r["seconds"], "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"{k} of {w.num_solves} solves (uniform, seeded); FP64 C oracle with the same schedule "
                         f"(max_rounds={args.max_rounds}); {r['seconds']:.1f} s on {threads} threads"}
        # the same oracle on one host thread, on the first quarter of that sample
        k1 = max(1, k // 4)
        r1 = O.solve_batch(w, nthreads=1, solves=solves[:k1], **opts)
        cpu["one_thread"] = {"value": k1 * w.path_len / r1["seconds"], "unit": "solves/s",
                             "sample": f"{k1} of the sampled solves; {r1['seconds']:.1f} s on 1 thread"}

    secondary = []
    backward = main_backward
    if not args.no_secondary:
        for cfg, mr, fl in [("c1", 0, 0), ("c1", 1, L.FLAG_GOLDEN), ("c2", 1, 0), ("c2", 0, 0), ("c3", 1, 0),
                            ("c4s", 1, 0)]:
            if cfg == args.config and mr == args.max_rounds and fl == flags:
                continue
            log(f"generating workload {cfg}")
            ws = make_workload(cfg)
            big = cfg == "c4s"
            s = measure(L, torch, ws, 2 if big else 3, 1, 8 if big else 128, args.autotune, max_rounds=mr, flags=fl)
            entry = {"workload": ws.name, "max_rounds": mr, "golden": bool(fl), "solves_per_s": s["solves_per_s"],
                     "ms_per_step": s["ms"], "parity_ok": s["parity_ok"], "max_rel_f": s["parity"]["max_rel_f"],
                     "iters_mean": s["iters_mean"], "status": s["status"]}
            if big:
                entry["graph_ms_per_step"], bw = path_graph_and_backward(L, torch, ws, s)
                bw["traffic"] = recorded_traffic("c4_sample_kernel_stats.md", "backward_traffic_bytes_per_launch")
                backward = backward or bw
            elif cfg == "c3":
                # the differentiation workload: its backward (dL/dy, dL/dX of all 1024 problems)
                _, entry["backward"] = path_graph_and_backward(L, torch, ws, s)
            secondary.append(entry)
        secondary.append(measure_cv(L, torch))
        secondary.append(measure_brute(L, torch))

    line = {
        "metric": METRIC,
        "value": m["solves_per_s"] if m["parity_ok"] else 0.0,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded generator, no dataset)",
        "config": {"workload": w.name, "solves_per_step": m["n_out"], "max_rounds": args.max_rounds,
                   "golden": bool(args.golden), "autotune": bool(args.autotune),
                   "parallelism": "1 GPU, one wavefront per solve", "path_len": w.path_len,
                   "graph_ms_per_step": main_graph_ms},
        "roofline": {"bound": "alu", "achieved": achieved_ops / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved_ops / PEAK_VALU_LANE_OPS, "traffic": traffic,
                     "work_per_launch_lane_ops": lane_ops, "row_updates": m["row_updates"]},
        "hbm": {"achieved_GBs": hbm_gbs, "peak_GBs": PEAK_HBM_GBS, "frac": hbm_gbs / PEAK_HBM_GBS,
                "algorithmic_bytes": alg_bytes},
        "cpu_baseline": cpu,
        "plain_kernel": plain,
        "vs_plain": (m["solves_per_s"] / plain["value"]) if plain else None,
        "parity": {"ok": m["parity_ok"], "sample": m["parity"]["outputs"], **m["parity"],
                   "first_failures": [str(f) for f in m["fails"][:3]]},
        "status": m["status"],
        "iters_mean": m["iters_mean"],
        "secondary": secondary,
        "roofline_backward": backward,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
