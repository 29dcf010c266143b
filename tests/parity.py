"""Element-by-element comparison of the HIP solve with the FP64 oracle.

Both sides solve the identical instance: the oracle upcasts the float32
inputs exactly.  The oracle's answer is certified optimal (LP duality), so
objective parity is checked on every solve; coefficients, the active set S
and the zero-residual rows Z are compared exactly only where the optimum is
unique with a comfortable margin, because elsewhere several answers are
correct (a flat optimal face).  stats["strict"] / stats["unique"] is the
share of the oracle's unique optima that were compared strictly.
"""
import numpy as np

import oracle as O
import paper_2510_15649_amd as L

TOL_F = 1e-5       # relative objective (both the reported fp32 value and the fp64 re-evaluation)
TOL_B = 1e-4       # |b - b*| <= TOL_B * max(1, |b*|) at a unique optimum
# An optimum the oracle certifies unique is compared strictly (b, S, Z, and
# the GPU must label it CERTIFIED) when its margins are ones an fp32 solve
# resolves: dual margin 1 - |u_i| and (lam - |c_j|) / (lam + sum_{i in Z}
# |x_ij|) at least MARGIN_UC, row margin |r_i| / (|y_i| + sum_j |x_ij b_j|)
# at least MARGIN_R.  The kernels label an output unique from 2e-5 and 1e-6
# on, so these gates sit a factor 4-5 above that, and they admit about 98%
# or more of the oracle's unique optima on the ragged workloads.
MARGIN_UC = 1e-4
MARGIN_R = 4e-6


def strict_unique(ref, ro) -> bool:
    """The oracle's optimum at output ro is unique with fp32-resolvable margins."""
    mu, mr = ref["margin"][ro]
    return bool(ref["cert"][ro] == 2 and mu >= MARGIN_UC and mr >= MARGIN_R)


def gradient_error(Xk, yk, lam, b, Z, g, gyk, gXk):
    """Largest scaled difference between a gradient block (dL/dy_k, dL/dX_k)
    and the oracle's vertex-form gradient at (b, Z)."""
    dy, dX = O.backward(Xk, yk, float(lam), np.asarray(b, np.float64), [int(z) for z in Z],
                        np.asarray(g, np.float64))
    ey = np.max(np.abs(gyk - dy)) / (1 + np.max(np.abs(dy))) if dy.size else 0.0
    eX = np.max(np.abs(gXk - dX)) / (1 + np.max(np.abs(dX))) if dX.size else 0.0
    return max(float(ey), float(eX))


def to_numpy(out):
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def oracle_ref(w, solves=None, nthreads=None, **opts):
    opts.setdefault("max_rounds", 0)   # exact optimum; the schedule does not change the answer
    return O.solve_batch(w, nthreads=nthreads, solves=solves, **opts)


def f64(w, k, lam, b):
    Xk, yk = w.block(int(k))
    return float(np.abs(yk - Xk @ b.astype(np.float64)).sum() + float(lam) * np.abs(b.astype(np.float64)).sum())


def compare(w, gpu, ref, solves=None, check_status=True):
    """Returns (failures, stats).  gpu: numpy outputs of the whole workload;
    ref: oracle_ref on `solves` (all if None)."""
    Lp = w.path_len
    ps = w.p[w.problem].astype(np.int64)
    b_off = np.zeros(w.num_solves, dtype=np.int64)
    b_off[1:] = np.cumsum(ps)[:-1]
    ids = np.arange(w.num_solves) if solves is None else np.asarray(solves)
    fails = []
    st = dict(outputs=0, unique=0, strict=0, max_rel_f=0.0, max_rel_f64=0.0, max_b=0.0)
    for idx, s in enumerate(ids):
        k = int(w.problem[s])
        p = int(w.p[k])
        for t in range(Lp):
            o = int(s) * Lp + t
            ro = idx * Lp + t
            lam = float(w.lam[o])
            fr = float(ref["f"][ro])
            fg = float(gpu["obj"][o])
            bg = gpu["b"][Lp * b_off[s] + t * p: Lp * b_off[s] + t * p + p]
            fg64 = f64(w, k, lam, bg)
            st["outputs"] += 1
            scale = max(fr, 1e-30)
            rel, rel64 = abs(fg - fr) / scale, abs(fg64 - fr) / scale
            st["max_rel_f"] = max(st["max_rel_f"], rel)
            st["max_rel_f64"] = max(st["max_rel_f64"], rel64)
            status = int(gpu["status"][o])
            tag = (int(s), t, k)
            if ref["cert"][ro] == 0:
                fails.append((tag, "oracle did not certify its answer"))
                continue
            if check_status and status not in (L.CERTIFIED, L.NONUNIQUE):
                fails.append((tag, f"status {L.STATUS_NAMES[status] if 0 <= status < 6 else status}"))
                continue
            if fr == 0.0:
                if fg != 0.0 or fg64 != 0.0:
                    fails.append((tag, f"f* = 0 but gpu f = {fg} / {fg64}"))
                continue
            if rel > TOL_F or rel64 > TOL_F:
                fails.append((tag, f"objective gpu {fg:.9g} (fp64 {fg64:.9g}) vs oracle {fr:.9g}"))
                continue
            st["unique"] += int(ref["cert"][ro] == 2)
            if strict_unique(ref, ro):
                st["strict"] += 1
                if check_status and status != L.CERTIFIED:
                    it = gpu.get("iters")
                    fails.append((tag, f"unique optimum (margins {ref['margin'][ro]}) labelled "
                                       f"{L.STATUS_NAMES[status]}; iters "
                                       f"{None if it is None else it[4 * o:4 * o + 4].tolist()}"))
                    continue
                bref = ref["b"][Lp * int(ref["b_off"][idx]) + t * p: Lp * int(ref["b_off"][idx]) + t * p + p]
                db = np.max(np.abs(bg - bref) / np.maximum(1.0, np.abs(bref)))
                st["max_b"] = max(st["max_b"], float(db))
                if db > TOL_B:
                    fails.append((tag, f"b differs by {db:.3g}: {bg} vs {bref}"))
                    continue
                sm = int(gpu["active"][o]) & 0xFFFFFFFF
                if sm != int(ref["smask"][ro]):
                    fails.append((tag, f"S mask {sm:#x} vs {int(ref['smask'][ro]):#x}"))
                    continue
                zg = gpu["zero_rows"][32 * o: 32 * o + 32]
                zr = ref["zrows"][ro]
                if not np.array_equal(zg, zr):
                    fails.append((tag, f"Z {zg[zg >= 0]} vs {zr[zr >= 0]}"))
    return fails, st
