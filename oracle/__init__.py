"""ctypes binding of the FP64 CPU oracle (``ladl_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg, never by the product package.  It shares
no code with the HIP library; only the seeded workload generators are
common to both sides.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ladl_oracle.c")
_LIB = os.path.join(_HERE, "libladl_oracle.so")

MAX_P = 64
STAGE_CCD, STAGE_TERNARY, STAGE_FINISHER, STAGE_NONE = 0, 1, 100, -1
SECTION_MEDIAN, SECTION_QUADRATURE = 0, 1


class Opts(C.Structure):
    _fields_ = [("tol_f", C.c_double), ("tol_s", C.c_double), ("lambda_min", C.c_double),
                ("max_sweeps", C.c_int), ("max_ternary", C.c_int), ("max_rounds", C.c_int),
                ("max_pivots", C.c_int), ("use_finisher", C.c_int), ("chop_range", C.c_double),
                ("section", C.c_int), ("tol_q", C.c_double), ("golden", C.c_int)]


class Prob(C.Structure):
    _fields_ = [("n", C.c_int), ("p", C.c_int), ("X", C.POINTER(C.c_double)),
                ("y", C.POINTER(C.c_double)), ("lambda_", C.c_double)]


class Info(C.Structure):
    _fields_ = [("f", C.c_double), ("stage", C.c_int), ("certified", C.c_int), ("unique", C.c_int),
                ("nS", C.c_int), ("S_mask", C.c_uint64), ("Z", C.c_int * MAX_P), ("umax", C.c_double),
                ("cmax", C.c_double), ("gap", C.c_double), ("margin_uc", C.c_double),
                ("margin_r", C.c_double), ("sweeps", C.c_long), ("updates", C.c_long),
                ("probes", C.c_long), ("pivots", C.c_long), ("f_ccd", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "Z"}
        d["Z"] = [z for z in self.Z if z >= 0]
        return d


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O3, portable code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lpthread", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_default_opts.argtypes = [C.POINTER(Opts)]
        L.orc_objective.argtypes = [C.POINTER(Prob), dp]
        L.orc_objective.restype = C.c_double
        L.orc_weighted_median.argtypes = [C.c_int, dp, dp]
        L.orc_weighted_median.restype = C.c_int
        L.orc_coord_update.argtypes = [C.POINTER(Prob), C.c_double, dp, dp, C.c_int]
        L.orc_coord_update.restype = C.c_double
        L.orc_quadrature_update.argtypes = [C.POINTER(Prob), C.c_double, C.c_double, dp, dp, C.c_int,
                                            C.POINTER(C.c_long)]
        L.orc_quadrature_update.restype = C.c_double
        L.orc_ccd.argtypes = [C.POINTER(Prob), C.POINTER(Opts), C.c_double, dp, dp, C.c_int, dp,
                              C.POINTER(C.c_long)]
        L.orc_ccd.restype = C.c_int
        L.orc_certify.argtypes = [C.POINTER(Prob), C.c_double, dp, dp, C.POINTER(Info)]
        L.orc_certify.restype = C.c_int
        L.orc_solve.argtypes = [C.POINTER(Prob), C.POINTER(Opts), dp, dp, C.POINTER(Info)]
        L.orc_solve.restype = C.c_int
        L.orc_brute_force.argtypes = [C.POINTER(Prob), C.c_double, dp, C.POINTER(C.c_long)]
        L.orc_brute_force.restype = C.c_double
        L.orc_lp_simplex.argtypes = [C.POINTER(Prob), C.c_double, dp, dp, C.POINTER(C.c_long)]
        L.orc_lp_simplex.restype = C.c_double
        L.orc_backward.argtypes = [C.POINTER(Prob), dp, C.POINTER(C.c_int), dp, dp, dp]
        L.orc_backward.restype = C.c_int
        i32p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.orc_solve_batch.argtypes = [C.c_int, i32p, i64p, i64p, i32p, dp, dp, dp, C.c_int, i64p,
                                      C.POINTER(Opts), C.c_int, dp, dp, i32p, C.POINTER(C.c_uint32), i32p,
                                      i32p, i64p, dp]
        L.orc_solve_batch.restype = C.c_double
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().orc_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Problem:
    """Keeps float64 contiguous copies alive for the C side."""

    def __init__(self, X, y, lam: float):
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.y = np.ascontiguousarray(y, dtype=np.float64)
        n, p = self.X.shape
        assert self.y.shape == (n,)
        self.n, self.p, self.lam = n, p, float(lam)
        self.c = Prob(n, p, _d(self.X), _d(self.y), float(lam))


def objective(X, y, lam, b) -> float:
    P = Problem(X, y, lam)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return lib().orc_objective(C.byref(P.c), _d(b))


def weighted_median(t, w) -> int:
    t = np.ascontiguousarray(t, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    return lib().orc_weighted_median(t.shape[0], _d(t), _d(w))


def coord_update(X, y, lam, b, j):
    """One exact coordinate minimisation from b; returns the new b."""
    P = Problem(X, y, lam)
    b = np.array(b, dtype=np.float64)
    r = P.y - P.X @ b
    lib().orc_coord_update(C.byref(P.c), float(lam), _d(b), _d(r), int(j))
    return b


def quadrature_update(X, y, lam, b, j, tol_q=1e-13):
    """One coordinate minimisation by the quadrature search of the section's
    values; returns (new b, number of section values computed)."""
    P = Problem(X, y, lam)
    b = np.array(b, dtype=np.float64)
    r = P.y - P.X @ b
    ev = C.c_long(0)
    lib().orc_quadrature_update(C.byref(P.c), float(lam), float(tol_q), _d(b), _d(r), int(j), C.byref(ev))
    return b, ev.value


def ccd(X, y, lam, b0=None, frozen=-1, **opts):
    P = Problem(X, y, lam)
    b = np.zeros(P.p) if b0 is None else np.array(b0, dtype=np.float64)
    r = P.y - P.X @ b
    f = C.c_double()
    upd = C.c_long(0)
    o = default_opts(**opts)
    sweeps = lib().orc_ccd(C.byref(P.c), C.byref(o), float(lam), _d(b), _d(r), int(frozen), C.byref(f),
                           C.byref(upd))
    return b, f.value, sweeps


def certify(X, y, lam, b):
    """Snap b to its vertex and evaluate the KKT certificate.
    Returns (certified, b_vertex, u, info)."""
    P = Problem(X, y, lam)
    b = np.array(b, dtype=np.float64)
    u = np.zeros(P.n)
    info = Info()
    ok = lib().orc_certify(C.byref(P.c), float(lam), _d(b), _d(u), C.byref(info))
    return bool(ok > 0), b, u, info.as_dict()


def solve(X, y, lam, b_init=None, **opts):
    """The paper's method (+ finisher) in FP64.  Returns (b, info)."""
    P = Problem(X, y, lam)
    b = np.zeros(P.p)
    bi = None if b_init is None else np.ascontiguousarray(b_init, dtype=np.float64)
    info = Info()
    o = default_opts(**opts)
    rc = lib().orc_solve(C.byref(P.c), C.byref(o), None if bi is None else _d(bi), _d(b), C.byref(info))
    if rc < 0:
        raise ValueError("orc_solve rejected the problem")
    return b, info.as_dict()


def brute_force(X, y, lam):
    P = Problem(X, y, lam)
    b = np.zeros(P.p)
    cnt = C.c_long(0)
    f = lib().orc_brute_force(C.byref(P.c), float(lam), _d(b), C.byref(cnt))
    return f, b, cnt.value


def lp_simplex(X, y, lam):
    P = Problem(X, y, lam)
    b = np.zeros(P.p)
    u = np.zeros(P.n)
    piv = C.c_long(0)
    f = lib().orc_lp_simplex(C.byref(P.c), float(lam), _d(b), _d(u), C.byref(piv))
    return f, b, u, piv.value


def backward(X, y, lam, b, Z, g):
    P = Problem(X, y, lam)
    b = np.ascontiguousarray(b, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    Zc = (C.c_int * MAX_P)(*([int(z) for z in Z] + [-1] * (MAX_P - len(Z))))
    dy = np.zeros(P.n)
    dX = np.zeros((P.n, P.p))
    rc = lib().orc_backward(C.byref(P.c), _d(b), Zc, _d(g), _d(dy), _d(dX))
    if rc != 0:
        raise ValueError("singular vertex matrix")
    return dy, dX


def solve_batch(w, nthreads: Optional[int] = None, solves=None, b_init=None, **opts):
    """Solve every (or the listed) solve of a Workload in FP64 on host
    threads.  Returns a dict of outputs laid out like the HIP library's plus
    the wall time of the solve loop."""
    nthreads = nthreads or os.cpu_count() or 1
    if solves is None:
        problem = w.problem
        lam = w.lam
    else:
        solves = np.asarray(solves, dtype=np.int64)
        problem = w.problem[solves]
        L = w.path_len
        lam = w.lam.reshape(-1, L)[solves].ravel()
    problem = np.ascontiguousarray(problem, dtype=np.int32)
    ps = w.p[problem].astype(np.int64)
    b_off = np.zeros(problem.shape[0], dtype=np.int64)
    if problem.shape[0] > 1:
        b_off[1:] = np.cumsum(ps)[:-1]
    S, L = problem.shape[0], w.path_len
    X64 = np.ascontiguousarray(w.X, dtype=np.float64)
    y64 = np.ascontiguousarray(w.y, dtype=np.float64)
    lam64 = np.ascontiguousarray(lam, dtype=np.float64)
    out = dict(b=np.zeros(int(ps.sum()) * L), f=np.zeros(S * L), stage=np.zeros(S * L, np.int32),
               smask=np.zeros(S * L, np.uint32), zrows=np.zeros(S * L * 32, np.int32),
               cert=np.zeros(S * L, np.int32), counters=np.zeros(S * L * 4, np.int64),
               margin=np.zeros(S * L * 2))
    o = default_opts(**opts)
    i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    i64 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
    row_off = np.ascontiguousarray(w.row_off, np.int64)
    x_off = np.ascontiguousarray(w.x_off, np.int64)
    p_arr = np.ascontiguousarray(w.p, np.int32)
    secs = lib().orc_solve_batch(S, i32(problem), i64(row_off), i64(x_off), i32(p_arr), _d(X64), _d(y64),
                                 _d(lam64), L, i64(b_off), C.byref(o), int(nthreads), _d(out["b"]),
                                 _d(out["f"]), i32(out["stage"]),
                                 out["smask"].ctypes.data_as(C.POINTER(C.c_uint32)), i32(out["zrows"]),
                                 i32(out["cert"]), i64(out["counters"]), _d(out["margin"]))
    out["zrows"] = out["zrows"].reshape(S * L, 32)
    out["counters"] = out["counters"].reshape(S * L, 4)
    out["margin"] = out["margin"].reshape(S * L, 2)
    out["seconds"] = secs
    out["threads"] = nthreads
    out["b_off"] = b_off
    out["problem"] = problem
    return out


def cv_folds(n: int, folds: int, fold_of_row=None) -> np.ndarray:
    """Fold label of each of the n rows: row i -> i mod K unless given."""
    if fold_of_row is None:
        return np.arange(n) % folds
    return np.asarray(fold_of_row, dtype=np.int64)


def cv(X, y, lams, folds: int, fold_of_row=None, **opts):
    """K-fold cross-validation of one problem along a lambda path, in FP64.

    The paper motivates solving many regularisation settings together while
    cross-validating (Section 5); this is the plain definition: for each
    fold f, solve the lambda path in the given order on the rows outside f
    (each step started from the previous step's b), and score each b by the
    held-out absolute error sum_{i in f} |y_i - x_i b|.  The CV curve is the
    sum over folds; the selected index is the first minimiser.

    Returns dict(err [K, L], unique [K, L] (the fold solve's optimum is
    certified unique with clear margins), cv [L], best, b [K, L, p]).
    """
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    lams = np.asarray(lams, dtype=np.float64)
    n, p = X.shape
    lab = cv_folds(n, folds, fold_of_row)
    L = lams.shape[0]
    err = np.zeros((folds, L))
    uniq = np.zeros((folds, L), dtype=bool)
    bs = np.zeros((folds, L, p))
    for f in range(folds):
        tr, va = lab != f, lab == f
        b = None
        for t in range(L):
            b, info = solve(X[tr], y[tr], lams[t], b_init=b, **opts)
            bs[f, t] = b
            err[f, t] = float(np.sum(np.abs(y[va] - X[va] @ b)))
            uniq[f, t] = bool(info["unique"]) and info["margin_uc"] >= 1e-4 and info["margin_r"] >= 4e-6
    curve = err.sum(axis=0)
    return dict(err=err, unique=uniq, cv=curve, best=int(np.argmin(curve)), b=bs)


def selection_frequency(active, status, group, num_groups: int, path_len: int, ok_status=(0, 1)):
    """Subset-stability statistics (the paper's aim of telling informative
    from non-informative variables by fitting many row subsets, Section 1
    and Section 5), by plain counting: for group g, path step t and feature
    j, the fraction of the solves s in g (with an accepted status) whose
    coefficient j is non-zero, read from bit j of active[s*path_len + t].
    Returns (freq [G, L, 32], counts [G, L])."""
    active = np.asarray(active, dtype=np.uint64).reshape(-1, path_len)
    status = np.asarray(status).reshape(-1, path_len)
    group = np.asarray(group)
    hits = np.zeros((num_groups, path_len, 32))
    cnt = np.zeros((num_groups, path_len))
    for s in range(active.shape[0]):
        for t in range(path_len):
            if int(status[s, t]) not in ok_status:
                continue
            g = int(group[s])
            cnt[g, t] += 1
            for j in range(32):
                if (int(active[s, t]) >> j) & 1:
                    hits[g, t, j] += 1
    freq = np.divide(hits, cnt[:, :, None], out=np.zeros_like(hits), where=cnt[:, :, None] > 0)
    return freq, cnt
