"""Benchmark: batched LAD-LASSO solves/s on one MI355X.

One step = one forward pass of the whole solve path (cyclical coordinate
descent with exact weighted-median coordinate updates, or with the quadrature
search of each section under --quadrature, ternary chop along
the locus of axis-wise minima, vertex snap and optimality certificate,
edge-descent finisher) over one batch.  The headline workload is the large
ragged batch: 65536 problems, n ~ U[32, 2048], p ~ U[4, 32], each solved
along a warm-started 32-value lambda path in one persistent launch per
bucket (2,097,152 solves per step).  Inputs are resident in HBM before
timing starts.  Prints one JSON line.

Secondary lines: 512 problems x 16 lambdas with the plain one-thread-per-
solve kernel beside the wave kernel (the speed-up claim), the same
problems without the chop, with the bracket cut in thirds and with the quadrature
variant (on both kernels), the 4096 row
subsets of one correlated dataset (achieved HBM GB/s against the peak), the
differentiation workload with its backward, the ragged batch's lambda path
as a HIP graph and its backward against the HBM roofline, K-fold
cross-validation and vertex enumeration.
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
# fp32 VALU lane-ops/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, every lane
# operation counted once (157.3 TFLOP/s counts an FMA as 2 and packed pairs)
PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
# algorithmic lane-ops per row of one exact coordinate update (the low end
# of 12-30): classification pass |x|, sign test, zero test, two weight
# selects and sums; moving pass |r|, reciprocal, product, side test, running
# minimum; residual FMA
OPS_PER_ROW_UPDATE = 12
METRIC = "LAD-LASSO solves/sec at 1e-5 rel objective vs plain kernel; achieved HBM GB/s"

# device sources whose hash the committed byte-counter summaries record
KERNEL_SOURCES = ["ladl_solve_wave.hip", "ladl_wave.hpp", "ladl_team.hpp", "ladl_common.hpp", "ladl_kernels.hpp"]


def make_workload(cfg: str, **kw):
    from paper_2510_15649_amd import workloads as W
    return {"c1": lambda: W.config1(**kw), "c1path": lambda: W.config1(as_path=True), "c2": lambda: W.config2(),
            "c3": lambda: W.config3(), "c4": lambda: W.config4(),
            "c4s": lambda: W.config4(problems=range(4096)), "paper": lambda: W.paper_sizes(**kw)}[cfg]()


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


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": usable}


def log(msg):
    """Progress to stderr (the JSON line is the only stdout output)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rows_per_lane(n):
    r, R = (n + 63) // 64, 1
    while R < r:
        R <<= 1
    return R


def median_ms(torch, fn, reps, stream):
    """Median of `reps` launches, each bracketed by HIP events on `stream`."""
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), ts


def backward_bytes(w, out_np, step):
    """Algorithmic bytes of one backward launch: dL/dy and dL/dX written in
    full (n + n p floats per problem); read per certified solve: g, b, the
    zero-row list, status and the |S| x |S| vertex matrix."""
    wr = 4 * (w.X.size + w.y.size)
    L = w.path_len
    act = out_np["active"].reshape(-1, L)[:, step]
    ns = np.array([bin(int(a) & 0xFFFFFFFF).count("1") for a in act], dtype=np.int64)
    ps = w.p[w.problem].astype(np.int64)
    rd = int(np.sum(4 * (2 * ps + 32 + 1 + ns * ns)))
    return int(wr + rd)


def measure(L, torch, w, steps, warmup, parity_solves, autotune=False, **opts):
    """Times `steps` solves of workload w (after `warmup`) with HIP events on
    the caller's stream, and each bucket's kernel with HIP events on its own
    stream; checks the listed solves against the oracle.  Returns a dict."""
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
    plan.profile(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        plan.solve(d["X"], d["y"], d["lam"], out=out, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    prof = plan.profile_read()
    plan.profile(False)
    buckets = plan.buckets()
    n_out = w.num_solves * w.path_len
    g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    it = g["iters"].reshape(-1, 4)
    n_solve = np.diff(w.row_off)[w.problem]
    ns_out = np.repeat(n_solve, w.path_len)
    upd_rows = it[:, 1].astype(np.float64) * ns_out
    R_out = np.repeat(np.array([rows_per_lane(int(n)) for n in n_solve]), w.path_len)
    per_bucket = []
    for (R, nmax, pmax, count), (bms, launches) in zip(buckets, prof):
        per_bucket.append({"R": R, "n_max": nmax, "p_max": pmax, "solves": count, "launches": launches,
                           "ms_per_launch": bms / max(launches, 1),
                           "row_updates": float(np.sum(upd_rows[R_out == R]))})
    log(f"{w.name}: {ms:.3f} ms per step; buckets " +
        ", ".join(f"R={b['R']}: {b['ms_per_launch']:.2f} ms" for b in per_bucket))
    sample = np.asarray(parity_solves)
    log(f"{w.name}: checking {len(sample)} solves ({len(sample) * w.path_len} outputs) against the oracle")
    fails, pst = compare(w, g, oracle_ref(w, solves=sample), solves=sample)
    log(f"{w.name}: parity {'ok' if not fails else 'FAILED'} {pst}")
    status = {L.STATUS_NAMES[s]: int(c) for s, c in zip(*np.unique(g["status"], return_counts=True))}
    # which stage certified each output: no probe and no pivot = the first
    # descent and its vertex; probes but no pivot = the chop; pivots = the
    # finisher (the counters are per output)
    cert = np.isin(g["status"], [L.CERTIFIED, L.NONUNIQUE])
    stages = {"descent_and_snap": int(np.sum(cert & (it[:, 2] == 0) & (it[:, 3] == 0))),
              "chop": int(np.sum(cert & (it[:, 2] > 0) & (it[:, 3] == 0))),
              "finisher": int(np.sum(cert & (it[:, 3] > 0))), "uncertified": int(np.sum(~cert))}
    every_ok = bool(np.all(np.isfinite(g["obj"])) and np.all(g["obj"] >= 0))
    return dict(plan=plan, d=d, out=out, g=g, ms=ms, solves_per_s=n_out / (ms / 1e3), n_out=n_out,
                row_updates=float(upd_rows.sum()), buckets=per_bucket, parity_ok=not fails and every_ok,
                parity=pst, fails=fails, status=status, stages=stages,
                iters_mean={"sweeps": float(it[:, 0].mean()), "updates": float(it[:, 1].mean()),
                            "probes": float(it[:, 2].mean()), "pivots": float(it[:, 3].mean())},
                describe=plan.describe())


def alu_roofline(m, profile_summary=None):
    """ALU roofline of the dominant bucket kernel, the one that runs the most
    row-updates (the buckets run side by side, so which one ends last varies
    from run to run): algorithmic lane-ops (OPS_PER_ROW_UPDATE per row of
    each coordinate update it ran) over its launch time from HIP events on
    its own stream.  The HBM traffic of that kernel comes from the committed
    byte-counter summary (key traffic_bytes_per_launch_R<rows per lane>)."""
    dom = max(m["buckets"], key=lambda b: b["row_updates"])
    ops = OPS_PER_ROW_UPDATE * dom["row_updates"]
    achieved = ops / (dom["ms_per_launch"] / 1e3)
    traffic = recorded_traffic(profile_summary, f"traffic_bytes_per_launch_R{dom['R']}") if profile_summary else None
    return {"bound": "alu", "kernel": f"k_wave bucket R={dom['R']} (n<={dom['n_max']}, p<={dom['p_max']})",
            "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12, "unit": "Tlane-op/s",
            "frac": achieved / PEAK_VALU_LANE_OPS, "traffic": traffic, "ms_per_launch": dom["ms_per_launch"],
            "work_per_launch_lane_ops": ops, "row_updates": dom["row_updates"],
            "ops_per_row_update": OPS_PER_ROW_UPDATE}


def c4_parity_solves(w, n_uniform=48, n_big=16, seed=2024):
    """Problems of the ragged batch checked against the oracle along their
    whole path: a uniform draw plus a draw from those with n > 1024 and
    p > 24 (the largest bucket)."""
    rng = np.random.default_rng(seed)
    ns = np.diff(w.row_off)
    big = np.flatnonzero((ns > 1024) & (w.p > 24))
    ids = np.union1d(rng.choice(w.num_solves, size=min(n_uniform, w.num_solves), replace=False),
                     rng.choice(big, size=min(n_big, len(big)), replace=False) if len(big) else [])
    return ids.astype(np.int64)


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
    same = all(torch.equal(out[k], s["out"][k]) for k in ("b", "obj", "status", "zero_rows"))
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
    return graph_ms, same, {"workload": w.name, "kernel": "k_bw_vertex + k_bw_scatter", "ms_per_launch": bms,
                            "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                            "frac": gbs / PEAK_HBM_GBS, "traffic": None, "algorithmic_bytes": nbytes}


def cpu_baseline(L, w, seed=99, target_s=8.0):
    """The FP64 oracle, with the library's default schedule and tolerances,
    timed on the host cores on a uniform sample of solves (grown until the
    run takes target_s), and on one thread on a quarter of that sample."""
    import oracle as O
    info = cpu_info()
    threads = max(1, min(info["usable_cpus"], 16))
    d_opt = L.default_options()
    opts = dict(max_rounds=int(d_opt.max_rounds), tol_f=float(d_opt.tol_f), tol_s=float(d_opt.tol_s),
                max_sweeps=int(d_opt.max_sweeps), max_ternary=int(d_opt.max_ternary),
                chop_range=float(d_opt.chop_range), golden=int(bool(d_opt.flags & L.FLAG_GOLDEN)))
    rng = np.random.default_rng(seed)
    perm = rng.permutation(w.num_solves)
    k = min(w.num_solves, max(threads, 8))
    while True:
        solves = np.sort(perm[:k])
        r = O.solve_batch(w, nthreads=threads, solves=solves, **opts)
        if r["seconds"] >= target_s or k == w.num_solves:
            break
        k = min(w.num_solves, k * 2)
    res = {"value": k * w.path_len / r["seconds"], "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"{k} of {w.num_solves} solves x {w.path_len} path steps (uniform, seeded) of {w.name}; "
                     f"FP64 C oracle with the library's default schedule; {r['seconds']:.1f} s on {threads} "
                     f"threads", "host": info}
    k1 = max(1, k // 4)
    r1 = O.solve_batch(w, nthreads=1, solves=solves[:k1], **opts)
    res["one_thread"] = {"value": k1 * w.path_len / r1["seconds"], "unit": "solves/s",
                         "sample": f"{k1} of the sampled solves; {r1['seconds']:.1f} s on 1 thread"}
    return res


def plain_comparison(L, torch, m, w, reps=10, parity=128):
    """The plain one-thread-per-solve kernel on the workload `m` measured:
    median of `reps` launches, parity on a sample."""
    from parity import compare, oracle_ref
    plan, d = m["plan"], m["d"]
    stream = torch.cuda.current_stream()
    out_p = plan.alloc_outputs(d["X"].device, iters=False)
    fn = lambda: plan.solve_plain(d["X"], d["y"], d["lam"], out=out_p, stream=stream)
    fn()
    torch.cuda.synchronize()
    pms, ts = median_ms(torch, fn, reps, stream)
    gp = {k: v.cpu().numpy() for k, v in out_p.items() if v is not None}
    rng = np.random.default_rng(2024)
    sample = np.sort(rng.choice(w.num_solves, size=min(parity, w.num_solves), replace=False))
    pf, _ = compare(w, gp, oracle_ref(w, solves=sample), solves=sample)
    return {"value": m["n_out"] / (pms / 1e3), "unit": "solves/s", "ms_per_step": pms, "launches": reps,
            "ms_min_max": [float(min(ts)), float(max(ts))], "parity_ok": not pf}


def measure_cv(L, torch, folds=5, steps=3, sample=4):
    """K-fold cross-validation of the 512 problems of n=200, p=8 along their
    16-lambda path (the training solves run on the wave kernels); parity of
    the fold errors on a few problems against the oracle's cross-validation."""
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
    # the paper's comparison at these sizes (Section 4): its coordinate
    # descent against vertex enumeration, here both on the GPU, and the
    # coordinate descent on one thread per problem
    out_s = plan.solve(d["X"], d["y"], d["lam"], stream=stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        out_s = plan.solve(d["X"], d["y"], d["lam"], out=out_s, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_cd = e0.elapsed_time(e1) / steps
    f_cd = out_s["obj"].cpu().numpy().astype(np.float64)
    cd_vs_brute = float(np.max(np.abs(f_cd - obj) / np.maximum(1.0, np.abs(obj))))
    st_cd = out_s["status"].cpu().numpy()
    pms, _ = median_ms(torch, lambda: plan.solve_plain(d["X"], d["y"], d["lam"], stream=stream), 3, stream)
    # the tile schedule (4 problems per wavefront for the descent and chop)
    plan_t = L.Plan.for_workload(w, tile=2)
    out_t = plan_t.solve(d["X"], d["y"], d["lam"], stream=stream)
    tms, _ = median_ms(torch, lambda: plan_t.solve(d["X"], d["y"], d["lam"], out=out_t, stream=stream), steps, stream)
    f_t = out_t["obj"].cpu().numpy().astype(np.float64)
    st_t = out_t["status"].cpu().numpy()
    return {"workload": f"vertex enumeration, {w.name}", "ms_per_step": ms,
            "solves_per_s": w.num_solves / (ms / 1e3), "candidate_vertices_per_step": float(cand.sum()),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s (fp64)",
                         "frac": achieved / 78.6},
            "parity_sample": sample, "max_rel_f": worst, "parity_ok": worst <= 1e-6,
            "oracle_1_thread_solves_per_s": cpu_rate,
            "coordinate_descent": {"ms_per_step": ms_cd, "solves_per_s": w.num_solves / (ms_cd / 1e3),
                                   "max_rel_f_vs_enumeration": cd_vs_brute,
                                   "certified": int(np.sum(np.isin(st_cd, [L.CERTIFIED, L.NONUNIQUE])))},
            "coordinate_descent_plain_kernel": {"ms_per_step": pms, "solves_per_s": w.num_solves / (pms / 1e3),
                                                "launches": 3},
            "coordinate_descent_tile_schedule": {
                "ms_per_step": tms, "solves_per_s": w.num_solves / (tms / 1e3), "tile": plan_t.tiles()[0],
                "max_rel_f_vs_enumeration": float(np.max(np.abs(f_t - obj) / np.maximum(1.0, np.abs(obj)))),
                "certified": int(np.sum(np.isin(st_t, [L.CERTIFIED, L.NONUNIQUE])))}}


def secondary_entry(w, s, mr, fl):
    return {"workload": w.name, "max_rounds": mr, "golden": bool(fl & 1), "quadrature": bool(fl & 8),
            "solves_per_s": s["solves_per_s"],
            "ms_per_step": s["ms"], "parity_ok": s["parity_ok"], "max_rel_f": s["parity"]["max_rel_f"],
            "strict_of_unique": [s["parity"]["strict"], s["parity"]["unique"]],
            "iters_mean": s["iters_mean"], "status": s["status"], "certified_by_stage": s["stages"],
            "buckets": s["buckets"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c4")
    ap.add_argument("--max-rounds", type=int, default=1)
    ap.add_argument("--thirds", action="store_true",
                    help="cut the chop's bracket in thirds instead of golden sections (the library default)")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--quadrature", action="store_true",
                    help="the quadrature variant: 1-D sections minimised by a quadrature search of their values")
    ap.add_argument("--team", type=int, default=0,
                    help="waves per solve for n > 1024 (0: the library's choice; 1, 2 or 4)")
    ap.add_argument("--tile", type=int, default=0,
                    help="tile schedule for n <= 64 (0: the library's choice; 1 off; 2 on)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the HIP-graph replay of the path and the backward (profiling the forward alone)")
    ap.add_argument("--parity-sample", type=int, default=48,
                    help="solves of the headline workload checked against the oracle (plus 16 of the largest "
                         "problems on the ragged batch)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (a known-size reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): every solve is independent, so a "
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
    default_flags = int(L.default_options().flags)
    flags = (default_flags & ~L.FLAG_GOLDEN if args.thirds else default_flags) | \
        (L.FLAG_QUADRATURE if args.quadrature else 0)
    if args.config in ("c4", "c4s"):
        psolves = c4_parity_solves(w, n_uniform=args.parity_sample)
    else:
        rng = np.random.default_rng(2024)
        psolves = np.sort(rng.choice(w.num_solves, size=min(args.parity_sample, w.num_solves), replace=False))
    m = measure(L, torch, w, args.steps, args.warmup, psolves, args.autotune, max_rounds=args.max_rounds,
                flags=flags, team=args.team, tile=args.tile)
    ms = m["ms"]
    default_run = (args.max_rounds == 1 and flags == default_flags and not args.autotune and args.team == 0 and
                   args.tile == 0)
    summary = {"c4": "k_wave_c4_full_hbm_bytes.md", "c2": "k_wave_c2_kernel_stats.md",
               "c1": "k_wave_c1_hbm_bytes.md"}.get(args.config) if default_run else None
    roof = alu_roofline(m, summary)
    alg_bytes = w.algorithmic_bytes()
    hbm_gbs = alg_bytes / (ms / 1e3) / 1e9
    graph_ms = graph_same = backward = None
    if w.path_len > 1 and w.grad_b is not None and not args.no_graph:
        graph_ms, graph_same, backward = path_graph_and_backward(L, torch, w, m)
        if args.config == "c4" and default_run:
            backward["traffic"] = recorded_traffic("k_bw_c4_full_hbm_bytes.md", "backward_traffic_bytes_per_launch")

    cpu = None
    if not args.no_cpu:
        log("oracle on the host cores")
        cpu = cpu_baseline(L, w)
        log(f"oracle: {cpu['value']:.1f} solves/s on {cpu['cores']} threads")

    secondary = []
    plain = None
    if not args.no_secondary:
        G, Q = L.FLAG_GOLDEN, L.FLAG_QUADRATURE
        for cfg, mr, fl in [("c1", 1, G), ("c1", 0, G), ("c1", 1, 0), ("c1", 1, G | Q),
                            ("c2", 1, G), ("c2", 0, G), ("c3", 1, G)]:
            if cfg == args.config and mr == args.max_rounds and fl == flags:
                continue
            log(f"generating workload {cfg}")
            ws = make_workload(cfg)
            rng = np.random.default_rng(2024)
            samp = np.sort(rng.choice(ws.num_solves, size=min(128, ws.num_solves), replace=False))
            s = measure(L, torch, ws, 3, 1, samp, args.autotune, max_rounds=mr, flags=fl)
            entry = secondary_entry(ws, s, mr, fl)
            if cfg == "c1" and mr == 1 and fl == G:
                log("plain one-thread-per-solve kernel, median of 10 launches")
                plain = plain_comparison(L, torch, s, ws)
                entry["plain_kernel"] = plain
                entry["vs_plain"] = s["solves_per_s"] / plain["value"]
                entry["roofline"] = alu_roofline(s, "k_wave_c1_hbm_bytes.md")
            if cfg == "c1" and fl & Q:
                # the paper's one-thread-per-problem design with quadrature
                # sections, on the first 64 of the 512 problems (1024 solves)
                log("plain kernel with quadrature sections, 1024 solves, median of 3 launches")
                wq = make_workload("c1", num_problems=64)
                mq = dict(plan=L.Plan.for_workload(wq, max_rounds=mr, flags=fl), d=L.to_device(wq),
                          n_out=wq.num_solves * wq.path_len)
                entry["plain_kernel_1024"] = plain_comparison(L, torch, mq, wq, reps=3, parity=64)
                mm = dict(plan=L.Plan.for_workload(wq, max_rounds=mr), d=mq["d"], n_out=mq["n_out"])
                entry["plain_kernel_1024_median_sections"] = plain_comparison(L, torch, mm, wq, reps=3, parity=64)
            if cfg == "c2" and mr == 1:
                gbs = ws.algorithmic_bytes() / (s["ms"] / 1e3) / 1e9
                entry["hbm"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                "frac": gbs / PEAK_HBM_GBS, "algorithmic_bytes": ws.algorithmic_bytes(),
                                "traffic": recorded_traffic("k_wave_c2_kernel_stats.md", "traffic_bytes_per_step")}
                entry["roofline"] = alu_roofline(s, "k_wave_c2_kernel_stats.md")
            if cfg == "c3":
                entry["backward"] = backward_c3(L, torch, ws, s)
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
                   "golden": bool(flags & L.FLAG_GOLDEN), "quadrature": bool(args.quadrature),
                   "autotune": bool(args.autotune), "team": args.team, "tile": args.tile,
                   "parallelism": "1 GPU, one wavefront per solve, buckets side by side",
                   "path_len": w.path_len, "graph_ms_per_step": graph_ms, "graph_equals_in_kernel": graph_same},
        "roofline": roof,
        "hbm": {"achieved_GBs": hbm_gbs, "peak_GBs": PEAK_HBM_GBS, "frac": hbm_gbs / PEAK_HBM_GBS,
                "algorithmic_bytes": alg_bytes},
        "cpu_baseline": cpu,
        "plain_kernel": plain,
        "vs_plain": None,
        "parity": {"ok": m["parity_ok"], "sample_solves": int(len(psolves)), **m["parity"],
                   "first_failures": [str(f) for f in m["fails"][:3]]},
        "status": m["status"],
        "certified_by_stage": m["stages"],
        "iters_mean": m["iters_mean"],
        "buckets": m["buckets"],
        "secondary": secondary,
        "roofline_backward": backward,
    }
    print(json.dumps(line), flush=True)


def backward_c3(L, torch, w, s, reps=5):
    """Backward of a single-step workload (the differentiation workload)."""
    plan, d = s["plan"], s["d"]
    stream = torch.cuda.current_stream()
    g = d["grad_b"]
    gy = torch.empty(d["y"].numel(), dtype=torch.float32, device=d["X"].device)
    gX = torch.empty_like(d["X"])
    plan.backward(d["X"], s["out"], g, grad_y=gy, grad_X=gX, stream=stream)
    torch.cuda.synchronize()
    bms, _ = median_ms(torch, lambda: plan.backward(d["X"], s["out"], g, grad_y=gy, grad_X=gX, stream=stream),
                       reps, stream)
    nbytes = backward_bytes(w, s["g"], 0)
    gbs = nbytes / (bms / 1e3) / 1e9
    zero = int(np.sum(~np.isin(s["g"]["status"], [L.CERTIFIED, L.NONUNIQUE])))
    return {"workload": w.name, "kernel": "k_bw_vertex + k_bw_scatter", "ms_per_launch": bms, "bound": "hbm",
            "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "algorithmic_bytes": nbytes, "solves_without_gradient": zero}


if __name__ == "__main__":
    main()
