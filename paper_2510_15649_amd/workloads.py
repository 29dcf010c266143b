"""Seeded synthetic LAD-LASSO workloads.

This module only draws random inputs: it holds none of the solver's
arithmetic, so both the FP64 oracle and the HIP path can consume it.

Every problem k of a workload is drawn from its own PCG64 stream seeded by
``SeedSequence([seed, k])`` with ``seed = 15649 + 1000*c + replica``, so any
subset of problems can be regenerated bit-identically without drawing the
rest.  Values are drawn in float64 and cast to float32 (the GPU solves the
float32 instance; the oracle upcasts the same float32 values exactly).

The five workload recipes (the paper's evaluation used scikit-learn's
regression generator at 10-30 rows and 1-5 features, Section 4; these
synthetic recipes stand in for it):

* c0 - one problem, n=20, p=3, X~N(0,1), b_true=[1.5,0,-2], Laplace(0,0.5)
  noise, two uniformly chosen rows get N(0,10^2) noise instead, lambda=1.
* c1 - 512 problems, n=200, p=8, X~N(0,1), b_true with 3 non-zeros at
  uniform positions ~U[-3,3], Student-t(3) noise, 20 rows (10%) get
  N(0,20^2) noise; each problem solved at 16 lambdas logspace(-2,2,16).
* c2 - one base dataset n=1000, p=16 with equicorrelated columns
  (sqrt(.5) z0 + sqrt(.5) zj), 5-sparse b_true ~U[-3,3], Laplace(0,1)
  noise, 5% rows N(0,20^2); 4096 row subsets of size U{50..1000} drawn
  without replacement (sorted), packed into ragged blocks; lambda=0.5.
* c3 - 1024 problems n=300, p=12, 4-sparse b_true, Laplace(0,1) noise,
  lambda=2; upstream gradient dL/db ~ N(0,1).
* c4 - 65536 problems, n~U{32..2048}, p~U{4..32}, max(1,round(.2p))
  non-zeros ~U[-3,3], noise Laplace(0,1) or Student-t(2) with prob 1/2,
  10% rows N(0,20^2); 32-value lambda path logspace(2,-2,32) (descending,
  warm-started); backward at the last lambda.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

BASE_SEED = 15649


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, *key])))


@dataclass
class Workload:
    """A packed batch of LAD-LASSO problems and the solves run on them.

    X        float32, problem k's row-major n_k x p_k block at x_off[k]
    y        float32, problem k's rows at row_off[k]:row_off[k+1]
    row_off  int64 [P+1]
    x_off    int64 [P]
    p        int32 [P]
    problem  int32 [S]   problem index of each solve
    lam      float32 [S*L]  lambda path of solve s at lam[s*L:(s+1)*L]
    b_off    int64 [S]   offset (in units of L*p) of solve s's coefficients:
                         outputs of path step t live at L*b_off[s] + t*p_s
    grad_b   float32 or None, upstream dL/db packed like one path step's b
    """
    name: str
    X: np.ndarray
    y: np.ndarray
    row_off: np.ndarray
    x_off: np.ndarray
    p: np.ndarray
    problem: np.ndarray
    lam: np.ndarray
    path_len: int
    b_off: np.ndarray
    grad_b: Optional[np.ndarray] = None
    X64: Optional[np.ndarray] = None   # c0 only: the original float64 draw
    y64: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def num_problems(self) -> int:
        return int(self.p.shape[0])

    @property
    def num_solves(self) -> int:
        return int(self.problem.shape[0])

    def n(self, k: int) -> int:
        return int(self.row_off[k + 1] - self.row_off[k])

    def block(self, k: int, dtype=np.float64):
        """(X_k, y_k) of problem k as dense arrays of the given dtype."""
        n, p = self.n(k), int(self.p[k])
        o = int(self.x_off[k])
        Xk = self.X[o:o + n * p].reshape(n, p).astype(dtype)
        yk = self.y[self.row_off[k]:self.row_off[k + 1]].astype(dtype)
        return Xk, yk

    def b_len(self) -> int:
        """Total length of one output b array (all solves, all path steps)."""
        ps = self.p[self.problem].astype(np.int64)
        return int(ps.sum()) * self.path_len

    def algorithmic_bytes(self) -> int:
        """Bytes a solve pass must move at least once: X, y, offsets, lambdas
        read; b, objective, active mask, zero rows and status written."""
        rd = 4 * (self.X.size + self.y.size + self.lam.size) + 8 * (self.row_off.size + self.x_off.size) \
            + 4 * (self.p.size + self.problem.size)
        L = self.path_len
        wr = 4 * self.b_len() + self.num_solves * L * 4 * (1 + 1 + 32 + 1)
        return int(rd + wr)


def _pack(name, blocks, p_list, problem, lam, path_len, grad=None, meta=None):
    P = len(blocks)
    ns = np.array([b[0].shape[0] for b in blocks], dtype=np.int64)
    ps = np.asarray(p_list, dtype=np.int32)
    row_off = np.zeros(P + 1, dtype=np.int64)
    row_off[1:] = np.cumsum(ns)
    sizes = ns * ps.astype(np.int64)
    x_off = np.zeros(P, dtype=np.int64)
    x_off[1:] = np.cumsum(sizes)[:-1]
    X = np.empty(int(sizes.sum()), dtype=np.float32)
    y = np.empty(int(ns.sum()), dtype=np.float32)
    for k, (Xk, yk) in enumerate(blocks):
        X[x_off[k]:x_off[k] + sizes[k]] = Xk.astype(np.float32).ravel()
        y[row_off[k]:row_off[k + 1]] = yk.astype(np.float32)
    problem = np.asarray(problem, dtype=np.int32)
    sp = ps[problem].astype(np.int64)
    b_off = np.zeros(problem.shape[0], dtype=np.int64)
    if problem.shape[0] > 1:
        b_off[1:] = np.cumsum(sp)[:-1]
    return Workload(name=name, X=X, y=y, row_off=row_off, x_off=x_off, p=ps, problem=problem,
                    lam=np.asarray(lam, dtype=np.float32).ravel(), path_len=int(path_len), b_off=b_off,
                    grad_b=grad, meta=meta or {})


def _sparse_beta(g: np.random.Generator, p: int, nnz: int) -> np.ndarray:
    b = np.zeros(p)
    pos = g.choice(p, size=nnz, replace=False)
    b[pos] = g.uniform(-3.0, 3.0, size=nnz)
    return b


def _outliers(g: np.random.Generator, e: np.ndarray, frac_or_count, scale: float) -> np.ndarray:
    n = e.shape[0]
    m = frac_or_count if isinstance(frac_or_count, (int, np.integer)) else int(round(frac_or_count * n))
    if m > 0:
        idx = g.choice(n, size=m, replace=False)
        e[idx] = g.normal(0.0, scale, size=m)
    return e


def config0(replica: int = 0) -> Workload:
    seed = BASE_SEED + replica
    g = _rng(seed, 0)
    n, p = 20, 3
    X = g.standard_normal((n, p))
    bt = np.array([1.5, 0.0, -2.0])
    e = g.laplace(0.0, 0.5, size=n)
    e = _outliers(g, e, 2, 10.0)
    y = X @ bt + e
    w = _pack("c0: n=20 p=3 lambda=1", [(X, y)], [p], [0], [1.0], 1)
    w.X64, w.y64 = X, y
    w.meta.update(b_true=bt)
    return w


def config1(replica: int = 0, num_problems: int = 512, num_lambda: int = 16,
            as_path: bool = False) -> Workload:
    """512 problems x 16 lambdas.  as_path=False: 8192 independent solves
    (solve s uses problem s // 16 and lambda index s % 16); as_path=True:
    512 solves each walking the 16 lambdas in descending order."""
    seed = BASE_SEED + 1000 + replica
    n, p = 200, 8
    blocks = []
    for k in range(num_problems):
        g = _rng(seed, k)
        X = g.standard_normal((n, p))
        bt = _sparse_beta(g, p, 3)
        e = g.standard_t(3, size=n)
        e = _outliers(g, e, 20, 20.0)
        blocks.append((X, X @ bt + e))
    lams = np.logspace(-2, 2, num_lambda)
    if as_path:
        problem = np.arange(num_problems)
        lam = np.tile(lams[::-1], num_problems)
        L = num_lambda
    else:
        problem = np.repeat(np.arange(num_problems), num_lambda)
        lam = np.tile(lams, num_problems)
        L = 1
    return _pack(f"c1: {num_problems} problems n=200 p=8 x {num_lambda} lambdas", blocks,
                 [p] * num_problems, problem, lam, L)


def config2(replica: int = 0, num_subsets: int = 4096, n_base: int = 1000, m_lo: int = 50) -> Workload:
    seed = BASE_SEED + 2000 + replica
    p = 16
    g = _rng(seed, 0)
    z0 = g.standard_normal((n_base, 1))
    Xb = np.sqrt(0.5) * z0 + np.sqrt(0.5) * g.standard_normal((n_base, p))
    bt = _sparse_beta(g, p, 5)
    e = g.laplace(0.0, 1.0, size=n_base)
    e = _outliers(g, e, 0.05, 20.0)
    yb = Xb @ bt + e
    blocks = []
    for k in range(num_subsets):
        gs = _rng(seed, 1, k)
        m = int(gs.integers(m_lo, n_base + 1))
        rows = np.sort(gs.choice(n_base, size=m, replace=False))
        blocks.append((Xb[rows], yb[rows]))
    w = _pack(f"c2: {num_subsets} row subsets of n=1000 p=16 lambda=0.5", blocks, [p] * num_subsets,
              np.arange(num_subsets), np.full(num_subsets, 0.5), 1)
    w.meta.update(b_true=bt)
    return w


def config3(replica: int = 0, num_problems: int = 1024) -> Workload:
    seed = BASE_SEED + 3000 + replica
    n, p = 300, 12
    blocks = []
    for k in range(num_problems):
        g = _rng(seed, k)
        X = g.standard_normal((n, p))
        bt = _sparse_beta(g, p, 4)
        e = g.laplace(0.0, 1.0, size=n)
        blocks.append((X, X @ bt + e))
    gg = _rng(seed, 1 << 30)
    grad = gg.standard_normal(num_problems * p).astype(np.float32)
    return _pack(f"c3: {num_problems} problems n=300 p=12 lambda=2", blocks, [p] * num_problems,
                 np.arange(num_problems), np.full(num_problems, 2.0), 1, grad=grad)


def config4(replica: int = 0, problems: Optional[Sequence[int]] = None, num_problems: int = 65536,
            path_len: int = 32) -> Workload:
    """65536 ragged problems with a descending 32-lambda path each.  With
    ``problems`` given, only those problem indices are drawn (bit-identical
    to the same problems of the full draw)."""
    seed = BASE_SEED + 4000 + replica
    idx = np.arange(num_problems) if problems is None else np.asarray(problems, dtype=np.int64)
    blocks, ps = [], []
    for k in idx:
        g = _rng(seed, int(k))
        n = int(g.integers(32, 2049))
        p = int(g.integers(4, 33))
        X = g.standard_normal((n, p))
        bt = _sparse_beta(g, p, max(1, int(round(0.2 * p))))
        if g.random() < 0.5:
            e = g.laplace(0.0, 1.0, size=n)
        else:
            e = g.standard_t(2, size=n)
        e = _outliers(g, e, 0.1, 20.0)
        blocks.append((X, X @ bt + e))
        ps.append(p)
    lams = np.logspace(2, -2, path_len)
    P = len(blocks)
    gg = _rng(seed, 1 << 30)
    w = _pack(f"c4: {P} ragged problems n~U[32,2048] p~U[4,32] x {path_len}-lambda path", blocks, ps,
              np.arange(P), np.tile(lams, P), path_len)
    w.grad_b = gg.standard_normal(int(np.sum(ps))).astype(np.float32)
    w.meta.update(problem_ids=idx)
    return w


def paper_sizes(replica: int = 0, num_problems: int = 4096, n_range=(10, 30), p_range=(1, 5),
                lams=(0.1, 1.0, 10.0)) -> Workload:
    """Problems of the sizes the paper evaluates (Section 4: 10 to 30 data
    points, one to five explanatory variables), each solved at every lambda
    in `lams` as independent solves: X ~ N(0,1), about half the
    coefficients non-zero ~U[-3,3], Laplace(0,1) noise with 10% outliers
    N(0, 10^2).  Stands in for the paper's scikit-learn generated data."""
    seed = BASE_SEED + 5000 + replica
    blocks, ps = [], []
    for k in range(num_problems):
        g = _rng(seed, k)
        n = int(g.integers(n_range[0], n_range[1] + 1))
        p = int(g.integers(p_range[0], p_range[1] + 1))
        X = g.standard_normal((n, p))
        bt = _sparse_beta(g, p, max(1, (p + 1) // 2))
        e = _outliers(g, g.laplace(0.0, 1.0, size=n), 0.1, 10.0)
        blocks.append((X, X @ bt + e))
        ps.append(p)
    L = len(lams)
    problem = np.repeat(np.arange(num_problems), L)
    lam = np.tile(np.asarray(lams, dtype=np.float64), num_problems)
    return _pack(f"paper sizes: {num_problems} problems n~U[{n_range[0]},{n_range[1]}] "
                 f"p~U[{p_range[0]},{p_range[1]}] x {L} lambdas", blocks, ps, problem, lam, 1)


def make(c: int, **kw) -> Workload:
    return [config0, config1, config2, config3, config4][c](**kw)
