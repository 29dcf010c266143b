"""Batched LAD-LASSO on AMD MI355X: Python binding of libladlasso.so.

Argument marshalling only: every step of the solve runs in the HIP kernels
of the library.  PyTorch provides device memory and streams.  When the
library has not been built, every entry point raises; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libladlasso.so")

# status codes
CERTIFIED, NONUNIQUE, MAXITER, NONFINITE, BADLAMBDA, NOTCERTIFIED = range(6)
STATUS_NAMES = ["CERTIFIED", "NONUNIQUE", "MAXITER", "NONFINITE", "BADLAMBDA", "NOTCERTIFIED"]
# option flags
FLAG_GOLDEN, FLAG_NO_FINISHER, FLAG_NO_SNAP, FLAG_QUADRATURE = 1, 2, 4, 8
# return codes
OK, EINVAL, EUNSUPPORTED, EHIP, ENOMEM = 0, -1, -2, -3, -4
ZPAD = 32

EXPORTED = ["ladl_create", "ladl_destroy", "ladl_default_options", "ladl_plan_create", "ladl_plan_destroy",
            "ladl_plan_b_len", "ladl_solve_f32", "ladl_solve_plain_f32", "ladl_backward_f32",
            "ladl_graph_create", "ladl_graph_launch", "ladl_graph_destroy", "ladl_autotune",
            "ladl_plan_describe", "ladl_error_string", "ladl_last_error_detail", "ladl_cv_create",
            "ladl_cv_destroy", "ladl_cv_run", "ladl_brute_force_f32", "ladl_selection_frequency",
            "ladl_solve_uniform_noalloc_f32", "ladl_plan_profile", "ladl_plan_profile_read"]


class Options(C.Structure):
    _fields_ = [("tol_f", C.c_float), ("tol_s", C.c_float), ("lambda_min", C.c_float),
                ("max_sweeps", C.c_int32), ("max_ternary", C.c_int32), ("max_rounds", C.c_int32),
                ("max_pivots", C.c_int32), ("flags", C.c_int32), ("schedule", C.c_int32),
                ("chop_range", C.c_float), ("team", C.c_int32), ("tile", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Layout(C.Structure):
    _fields_ = [("num_problems", C.c_int32), ("row_off", C.POINTER(C.c_int64)),
                ("x_off", C.POINTER(C.c_int64)), ("p", C.POINTER(C.c_int32)), ("p_uniform", C.c_int32),
                ("x_len", C.c_int64), ("y_len", C.c_int64), ("num_solves", C.c_int32),
                ("problem", C.POINTER(C.c_int32)), ("path_len", C.c_int32),
                ("lambda_hint", C.POINTER(C.c_float))]


class CVLayout(C.Structure):
    _fields_ = [("num_problems", C.c_int32), ("row_off", C.POINTER(C.c_int64)),
                ("x_off", C.POINTER(C.c_int64)), ("p", C.POINTER(C.c_int32)), ("p_uniform", C.c_int32),
                ("x_len", C.c_int64), ("y_len", C.c_int64), ("folds", C.c_int32),
                ("fold_of_row", C.POINTER(C.c_int32)), ("path_len", C.c_int32)]


class LadlError(RuntimeError):
    def __init__(self, code: int, detail: str):
        super().__init__(f"{detail} (code {code})")
        self.code = code


_lib = None


def lib() -> C.CDLL:
    """Load libladlasso.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                           f"g.build()'` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.ladl_create.argtypes = [C.POINTER(vp)]
    L.ladl_destroy.argtypes = [vp]
    L.ladl_default_options.argtypes = [C.POINTER(Options)]
    L.ladl_default_options.restype = None
    L.ladl_plan_create.argtypes = [vp, C.POINTER(Layout), C.POINTER(Options), C.POINTER(vp)]
    L.ladl_plan_destroy.argtypes = [vp]
    L.ladl_plan_b_len.argtypes = [vp]
    L.ladl_plan_b_len.restype = i64
    solve_args = [vp] + [vp] * 10 + [vp]
    L.ladl_solve_f32.argtypes = solve_args
    L.ladl_solve_plain_f32.argtypes = solve_args
    L.ladl_backward_f32.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp]
    L.ladl_graph_create.argtypes = [vp] + [vp] * 10 + [C.POINTER(vp)]
    L.ladl_graph_launch.argtypes = [vp, vp]
    L.ladl_graph_destroy.argtypes = [vp]
    L.ladl_autotune.argtypes = [vp] + [vp] * 9
    L.ladl_plan_describe.argtypes = [vp, C.c_char_p, i64]
    L.ladl_brute_force_f32.argtypes = [vp] * 8
    L.ladl_selection_frequency.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp]
    L.ladl_cv_create.argtypes = [vp, C.POINTER(CVLayout), C.POINTER(Options), C.POINTER(vp)]
    L.ladl_cv_destroy.argtypes = [vp]
    L.ladl_cv_run.argtypes = [vp] + [vp] * 7 + [vp]
    L.ladl_solve_uniform_noalloc_f32.argtypes = [i32, i32, i32, i32, C.POINTER(Options)] + [vp] * 11
    L.ladl_plan_profile.argtypes = [vp, i32]
    L.ladl_plan_profile_read.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(i32), i32, C.POINTER(i32)]
    L.ladl_error_string.argtypes = [C.c_int]
    L.ladl_error_string.restype = C.c_char_p
    L.ladl_last_error_detail.argtypes = []
    L.ladl_last_error_detail.restype = C.c_char_p
    for name in ["ladl_create", "ladl_destroy", "ladl_plan_create", "ladl_plan_destroy", "ladl_solve_f32",
                 "ladl_solve_plain_f32", "ladl_backward_f32", "ladl_graph_create", "ladl_graph_launch",
                 "ladl_graph_destroy", "ladl_autotune", "ladl_plan_describe", "ladl_cv_create", "ladl_cv_destroy",
                 "ladl_cv_run", "ladl_brute_force_f32", "ladl_selection_frequency",
                 "ladl_solve_uniform_noalloc_f32", "ladl_plan_profile", "ladl_plan_profile_read"]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc: int):
    if rc != OK:
        L = lib()
        raise LadlError(rc, f"{L.ladl_error_string(rc).decode()}: {L.ladl_last_error_detail().decode()}")


def default_options(**kw) -> Options:
    o = Options()
    lib().ladl_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Handle:
    """A library handle bound to the current HIP device."""

    def __init__(self):
        h = C.c_void_p()
        check(lib().ladl_create(C.byref(h)))
        self._h = h

    @property
    def ptr(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ladl_destroy(self._h)
            self._h = None


_default_handle = None


def default_handle() -> Handle:
    global _default_handle
    if _default_handle is None:
        _default_handle = Handle()
    return _default_handle


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


_DTYPES = {"f32": "torch.float32", "i32": "torch.int32", "i64": "torch.int64"}


def _check(t, name: str, kind: str, min_numel: int, optional: bool = False):
    """The C ABI cannot see device buffer sizes or element types: a tensor
    handed to it must be a contiguous device tensor of the expected dtype
    holding at least `min_numel` elements, else ValueError."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if str(t.dtype) != _DTYPES[kind]:
        raise ValueError(f"{name} must be {_DTYPES[kind]} (got {t.dtype})")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < min_numel:
        raise ValueError(f"{name} holds {t.numel()} elements, the plan needs {min_numel}")


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """A validated batch layout (host arrays are copied at creation).

    row_off   int64 [P+1]   rows of problem k: row_off[k]:row_off[k+1]
    p         int or int32 [P]   features per problem
    x_off     int64 [P] or None  (None: row_off[k] * p for uniform p)
    problem   int32 [S] or None  problem of each solve (None: identity)
    path_len  lambdas per solve (warm-started path)
    """

    def __init__(self, row_off, p, *, x_len: int, y_len: int, problem=None, path_len: int = 1, x_off=None,
                 lambda_hint=None, options: Optional[Options] = None, handle: Optional[Handle] = None, **opt_kw):
        self.handle = handle or default_handle()
        self.options = options if options is not None else default_options(**opt_kw)
        self._row_off = np.ascontiguousarray(row_off, dtype=np.int64)
        P = self._row_off.shape[0] - 1
        if np.isscalar(p):
            self._p = None
            p_uniform = int(p)
            self.p_per_problem = np.full(P, p_uniform, dtype=np.int32)
        else:
            self._p = np.ascontiguousarray(p, dtype=np.int32)
            p_uniform = int(self._p[0]) if P > 0 else 0
            self.p_per_problem = self._p
        self._x_off = None if x_off is None else np.ascontiguousarray(x_off, dtype=np.int64)
        self._problem = None if problem is None else np.ascontiguousarray(problem, dtype=np.int32)
        S = P if problem is None else int(self._problem.shape[0])
        lay = Layout()
        lay.num_problems = P
        lay.row_off = self._row_off.ctypes.data_as(C.POINTER(C.c_int64))
        lay.x_off = None if self._x_off is None else self._x_off.ctypes.data_as(C.POINTER(C.c_int64))
        lay.p = None if self._p is None else self._p.ctypes.data_as(C.POINTER(C.c_int32))
        lay.p_uniform = p_uniform
        lay.x_len = int(x_len)
        lay.y_len = int(y_len)
        lay.num_solves = S
        lay.problem = None if self._problem is None else self._problem.ctypes.data_as(C.POINTER(C.c_int32))
        lay.path_len = int(path_len)
        self._lambda_hint = None
        if lambda_hint is not None:
            self._lambda_hint = np.ascontiguousarray(lambda_hint, dtype=np.float32)
            if self._lambda_hint.size != S * int(path_len):
                raise ValueError(f"lambda_hint has {self._lambda_hint.size} values, expected {S * int(path_len)}")
            lay.lambda_hint = self._lambda_hint.ctypes.data_as(C.POINTER(C.c_float))
        h = C.c_void_p()
        check(lib().ladl_plan_create(self.handle.ptr, C.byref(lay), C.byref(self.options), C.byref(h)))
        self._plan = h
        self.num_problems, self.num_solves, self.path_len = P, S, int(path_len)
        self.x_len, self.y_len = int(x_len), int(y_len)
        self.b_len = int(lib().ladl_plan_b_len(h))
        prob = np.arange(S, dtype=np.int32) if self._problem is None else self._problem
        self.p_per_solve = self.p_per_problem[prob]
        self.b_off = np.zeros(S, dtype=np.int64)
        if S > 1:
            self.b_off[1:] = np.cumsum(self.p_per_solve.astype(np.int64))[:-1]

    @classmethod
    def for_workload(cls, w, **kw) -> "Plan":
        return cls(w.row_off, w.p, x_off=w.x_off, problem=w.problem, path_len=w.path_len,
                   x_len=w.X.size, y_len=w.y.size, lambda_hint=w.lam, **kw)

    def __del__(self):
        if getattr(self, "_plan", None) and _lib is not None:
            _lib.ladl_plan_destroy(self._plan)
            self._plan = None

    def describe(self) -> str:
        buf = C.create_string_buffer(8192)
        check(lib().ladl_plan_describe(self._plan, buf, 8192))
        return buf.value.decode()

    def alloc_outputs(self, device="cuda", iters=True):
        import torch
        n_out = self.num_solves * self.path_len
        return dict(b=torch.empty(self.b_len, dtype=torch.float32, device=device),
                    obj=torch.empty(n_out, dtype=torch.float32, device=device),
                    active=torch.empty(n_out, dtype=torch.int32, device=device),
                    zero_rows=torch.empty(n_out * ZPAD, dtype=torch.int32, device=device),
                    status=torch.empty(n_out, dtype=torch.int32, device=device),
                    iters=torch.empty(n_out * 4, dtype=torch.int32, device=device) if iters else None)

    def _check_inputs(self, X, y, lam, b_init=None):
        n_out = self.num_solves * self.path_len
        _check(X, "X", "f32", self.x_len)
        _check(y, "y", "f32", self.y_len)
        _check(lam, "lam", "f32", n_out)
        _check(b_init, "b_init", "f32", self.b_len // self.path_len, optional=True)

    def _check_outputs(self, out):
        n_out = self.num_solves * self.path_len
        _check(out.get("b"), "b", "f32", self.b_len)
        _check(out.get("obj"), "obj", "f32", n_out)
        _check(out.get("active"), "active", "i32", n_out)
        _check(out.get("zero_rows"), "zero_rows", "i32", ZPAD * n_out)
        _check(out.get("status"), "status", "i32", n_out)
        _check(out.get("iters"), "iters", "i32", 4 * n_out, optional=True)

    def _call(self, fn, X, y, lam, b_init, out, stream):
        self._check_inputs(X, y, lam, b_init)
        self._check_outputs(out)
        check(fn(self._plan, _ptr(X), _ptr(y), _ptr(lam), _ptr(b_init), _ptr(out["b"]), _ptr(out["obj"]),
                 _ptr(out["active"]), _ptr(out["zero_rows"]), _ptr(out["status"]), _ptr(out.get("iters")),
                 _stream(stream)))
        return out

    def solve(self, X, y, lam, b_init=None, out=None, stream=None, iters=True):
        """Forward solve with the wavefront-per-solve kernels (float32 device
        tensors).  Returns a dict of output tensors (enqueued on `stream`)."""
        out = out or self.alloc_outputs(X.device, iters)
        return self._call(lib().ladl_solve_f32, X, y, lam, b_init, out, stream)

    def solve_plain(self, X, y, lam, b_init=None, out=None, stream=None, iters=True):
        """The same solve with one GPU thread per solve (baseline kernel)."""
        out = out or self.alloc_outputs(X.device, iters)
        return self._call(lib().ladl_solve_plain_f32, X, y, lam, b_init, out, stream)

    def selection_frequency(self, out, group=None, num_groups: int = 1, stream=None):
        """Per group, path step and feature: the fraction of accepted solves
        with b_j != 0 (subset stability).  `out` holds a solve's outputs;
        group: device int32 [num_solves] or None.  Returns device tensors
        freq [G, L, 32], counts [G, L, 33] and bad_group [1]."""
        import torch
        n_out = self.num_solves * self.path_len
        _check(out.get("active"), "active", "i32", n_out)
        _check(out.get("status"), "status", "i32", n_out)
        _check(group, "group", "i32", self.num_solves, optional=True)
        dev = out["active"].device
        G, Lp = int(num_groups), self.path_len
        res = dict(freq=torch.empty(G * Lp * 32, dtype=torch.float32, device=dev),
                   counts=torch.empty(G * Lp * 33, dtype=torch.int32, device=dev),
                   bad_group=torch.empty(1, dtype=torch.int32, device=dev))
        check(lib().ladl_selection_frequency(self._plan, _ptr(out["active"]), _ptr(out["status"]), _ptr(group), G,
                                             _ptr(res["counts"]), _ptr(res["freq"]), _ptr(res["bad_group"]),
                                             _stream(stream)))
        res["freq"] = res["freq"].view(G, Lp, 32)
        res["counts"] = res["counts"].view(G, Lp, 33)
        return res

    def brute_force(self, X, y, lam, stream=None):
        """Exact solve by vertex enumeration on the device (small problems:
        p <= 8, n + p <= 64).  Returns device tensors b, obj, vertices."""
        import torch
        self._check_inputs(X, y, lam)
        n_out = self.num_solves * self.path_len
        out = dict(b=torch.empty(self.b_len, dtype=torch.float32, device=X.device),
                   obj=torch.empty(n_out, dtype=torch.float32, device=X.device),
                   vertices=torch.empty(n_out, dtype=torch.int64, device=X.device))
        check(lib().ladl_brute_force_f32(self._plan, _ptr(X), _ptr(y), _ptr(lam), _ptr(out["b"]), _ptr(out["obj"]),
                                         _ptr(out["vertices"]), _stream(stream)))
        return out

    def backward(self, X, out, grad_b, step: int = -1, grad_y=None, grad_X=None, stream=None):
        import torch
        step = self.path_len - 1 if step < 0 else step
        grad_y = grad_y if grad_y is not None else torch.empty(int(self._row_off[-1]), dtype=torch.float32,
                                                                 device=X.device)
        grad_X = grad_X if grad_X is not None else torch.empty_like(X)
        n_out = self.num_solves * self.path_len
        _check(X, "X", "f32", self.x_len)
        _check(out.get("b"), "b", "f32", self.b_len)
        _check(out.get("zero_rows"), "zero_rows", "i32", ZPAD * n_out)
        _check(out.get("status"), "status", "i32", n_out)
        _check(grad_b, "grad_b", "f32", self.b_len // self.path_len)
        _check(grad_y, "grad_y", "f32", self.y_len)
        _check(grad_X, "grad_X", "f32", self.x_len)
        check(lib().ladl_backward_f32(self._plan, _ptr(X), _ptr(out["b"]), _ptr(out["zero_rows"]),
                                      _ptr(out["status"]), int(step), _ptr(grad_b), _ptr(grad_y),
                                      _ptr(grad_X), _stream(stream)))
        return grad_y, grad_X

    def profile(self, enable: bool = True):
        """Start (or stop) recording each bucket's kernel time with HIP events
        on the bucket's own stream."""
        check(lib().ladl_plan_profile(self._plan, 1 if enable else 0))

    def profile_read(self):
        """Per bucket (in describe() order): (summed kernel ms, launches)
        since profiling started; waits for the recorded events."""
        nb = C.c_int32(0)
        ms = (C.c_float * 16)()
        cnt = (C.c_int32 * 16)()
        check(lib().ladl_plan_profile_read(self._plan, ms, cnt, 16, C.byref(nb)))
        return [(float(ms[i]), int(cnt[i])) for i in range(nb.value)]

    def buckets(self):
        """(R, n_max, pmax, solves) of each bucket, in describe() order."""
        import re
        return [tuple(int(v) for v in m.groups()) for m in
                re.finditer(r"bucket R=(\d+) \(n<=(\d+)\) pmax=(\d+) solves=(\d+)", self.describe())]

    def tiles(self):
        """Tile schedule of each bucket, in describe() order: "SxR" (segments
        of S lanes, R rows per lane), "off" (allowed, not taken) or "none"."""
        import re
        return re.findall(r" tile=(\w+)", self.describe())

    def waves_per_solve(self):
        """Waves per solve (team size) of each bucket, in describe() order."""
        import re
        return [int(v) for v in re.findall(r"waves/solve=(\d+)", self.describe())]

    def graph(self, X, y, lam, out, b_init=None) -> "PathGraph":
        return PathGraph(self, X, y, lam, out, b_init)

    def autotune(self, X, y, lam, out, stream=None):
        self._check_inputs(X, y, lam)
        self._check_outputs(out)
        check(lib().ladl_autotune(self._plan, _ptr(X), _ptr(y), _ptr(lam), _ptr(out["b"]), _ptr(out["obj"]),
                                  _ptr(out["active"]), _ptr(out["zero_rows"]), _ptr(out["status"]),
                                  _stream(stream)))

    def b_view(self, b, s: int, t: int = 0):
        """Coefficients of solve s at path step t inside a flat b array."""
        p = int(self.p_per_solve[s])
        o = self.path_len * int(self.b_off[s]) + t * p
        return b[o:o + p]


class PathGraph:
    """The lambda path captured as a HIP graph of path_len launches."""

    def __init__(self, plan: Plan, X, y, lam, out, b_init=None):
        plan._check_inputs(X, y, lam, b_init)
        plan._check_outputs(out)
        self.plan = plan
        self._keep = (X, y, lam, out, b_init)
        g = C.c_void_p()
        check(lib().ladl_graph_create(plan._plan, _ptr(X), _ptr(y), _ptr(lam), _ptr(b_init), _ptr(out["b"]),
                                      _ptr(out["obj"]), _ptr(out["active"]), _ptr(out["zero_rows"]),
                                      _ptr(out["status"]), _ptr(out.get("iters")), C.byref(g)))
        self._g = g

    def launch(self, stream=None):
        check(lib().ladl_graph_launch(self._g, _stream(stream)))

    def __del__(self):
        if getattr(self, "_g", None) and _lib is not None:
            _lib.ladl_graph_destroy(self._g)
            self._g = None


class CrossValidation:
    """K-fold cross-validation of every problem along its lambda path, on the
    device (gather of the training problems, wave-kernel solves, held-out
    scoring, selection).  Host layout arrays are copied at creation.

    row_off, p, x_off, x_len, y_len   the base problems, as for Plan
    folds         K
    path_len      lambdas per problem
    fold_of_row   int32 [total rows] or None (local row i -> fold i mod K)
    """

    def __init__(self, row_off, p, *, x_len: int, y_len: int, folds: int, path_len: int, x_off=None,
                 fold_of_row=None, options: Optional[Options] = None, handle: Optional[Handle] = None, **opt_kw):
        self.handle = handle or default_handle()
        self.options = options if options is not None else default_options(**opt_kw)
        self._row_off = np.ascontiguousarray(row_off, dtype=np.int64)
        P = self._row_off.shape[0] - 1
        self._p = None if np.isscalar(p) else np.ascontiguousarray(p, dtype=np.int32)
        self._x_off = None if x_off is None else np.ascontiguousarray(x_off, dtype=np.int64)
        self._fold = None if fold_of_row is None else np.ascontiguousarray(fold_of_row, dtype=np.int32)
        lay = CVLayout()
        lay.num_problems = P
        lay.row_off = self._row_off.ctypes.data_as(C.POINTER(C.c_int64))
        lay.x_off = None if self._x_off is None else self._x_off.ctypes.data_as(C.POINTER(C.c_int64))
        lay.p = None if self._p is None else self._p.ctypes.data_as(C.POINTER(C.c_int32))
        lay.p_uniform = int(p) if np.isscalar(p) else int(self._p[0])
        lay.x_len, lay.y_len = int(x_len), int(y_len)
        lay.folds = int(folds)
        lay.fold_of_row = None if self._fold is None else self._fold.ctypes.data_as(C.POINTER(C.c_int32))
        lay.path_len = int(path_len)
        h = C.c_void_p()
        check(lib().ladl_cv_create(self.handle.ptr, C.byref(lay), C.byref(self.options), C.byref(h)))
        self._cv = h
        self.num_problems, self.folds, self.path_len = P, int(folds), int(path_len)
        self.x_len, self.y_len = int(x_len), int(y_len)

    @classmethod
    def for_workload(cls, w, folds: int, **kw) -> "CrossValidation":
        """Base problems of a Workload whose solves walk each problem's path."""
        return cls(w.row_off, w.p, x_off=w.x_off, x_len=w.X.size, y_len=w.y.size, folds=folds,
                   path_len=w.path_len, **kw)

    def run(self, X, y, lam, stream=None):
        """Returns device tensors fold_error [P*K*L], cv_error [P*L], best [P],
        fold_status [P*K*L] (enqueued on `stream`)."""
        import torch
        P, K, L = self.num_problems, self.folds, self.path_len
        _check(X, "X", "f32", self.x_len)
        _check(y, "y", "f32", self.y_len)
        _check(lam, "lam", "f32", P * L)
        out = dict(fold_error=torch.empty(P * K * L, dtype=torch.float32, device=X.device),
                   cv_error=torch.empty(P * L, dtype=torch.float32, device=X.device),
                   best=torch.empty(P, dtype=torch.int32, device=X.device),
                   fold_status=torch.empty(P * K * L, dtype=torch.int32, device=X.device))
        check(lib().ladl_cv_run(self._cv, _ptr(X), _ptr(y), _ptr(lam), _ptr(out["fold_error"]),
                                _ptr(out["cv_error"]), _ptr(out["best"]), _ptr(out["fold_status"]),
                                _stream(stream)))
        return out

    def __del__(self):
        if getattr(self, "_cv", None) and _lib is not None:
            _lib.ladl_cv_destroy(self._cv)
            self._cv = None


def solve_uniform_noalloc(X, y, lam, num_problems: int, n: int, p: int, path_len: int = 1, b_init=None,
                          out=None, stream=None, iters=True, options: Optional[Options] = None, **opt_kw):
    """The allocation-free entry point: num_problems problems of n x p packed
    back to back, each solved along its path of path_len lambdas.  `out`
    (or freshly allocated tensors) receives the outputs, laid out as for
    Plan.solve.  The library allocates nothing during the call."""
    import torch
    P, Lp = int(num_problems), int(path_len)
    n_out = P * Lp
    opts = options if options is not None else default_options(**opt_kw)
    _check(X, "X", "f32", P * n * p)
    _check(y, "y", "f32", P * n)
    _check(lam, "lam", "f32", n_out)
    _check(b_init, "b_init", "f32", P * p, optional=True)
    if out is None:
        dev = X.device
        out = dict(b=torch.empty(n_out * p, dtype=torch.float32, device=dev),
                   obj=torch.empty(n_out, dtype=torch.float32, device=dev),
                   active=torch.empty(n_out, dtype=torch.int32, device=dev),
                   zero_rows=torch.empty(n_out * ZPAD, dtype=torch.int32, device=dev),
                   status=torch.empty(n_out, dtype=torch.int32, device=dev),
                   iters=torch.empty(n_out * 4, dtype=torch.int32, device=dev) if iters else None)
    _check(out.get("b"), "b", "f32", n_out * p)
    _check(out.get("obj"), "obj", "f32", n_out)
    _check(out.get("active"), "active", "i32", n_out)
    _check(out.get("zero_rows"), "zero_rows", "i32", ZPAD * n_out)
    _check(out.get("status"), "status", "i32", n_out)
    _check(out.get("iters"), "iters", "i32", 4 * n_out, optional=True)
    check(lib().ladl_solve_uniform_noalloc_f32(P, int(n), int(p), Lp, C.byref(opts), _ptr(X), _ptr(y), _ptr(lam),
                                              _ptr(b_init), _ptr(out["b"]), _ptr(out["obj"]), _ptr(out["active"]),
                                              _ptr(out["zero_rows"]), _ptr(out["status"]), _ptr(out.get("iters")),
                                              _stream(stream)))
    return out


def to_device(w, device="cuda"):
    """Copy a Workload's arrays to device tensors."""
    import torch
    d = dict(X=torch.from_numpy(w.X).to(device), y=torch.from_numpy(w.y).to(device),
             lam=torch.from_numpy(w.lam).to(device))
    if w.grad_b is not None:
        d["grad_b"] = torch.from_numpy(w.grad_b).to(device)
    return d
