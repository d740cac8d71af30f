"""Oracle for spectrum-preserving coarsening (Brissette, Huang, Slota,
arXiv 2204.11757): plain, serial, CPU-only.

TEST INFRASTRUCTURE ONLY.  The product path (the HIP library and its
binding) never imports this package; only ``tests/``, the package smoke
check and the benchmark's CPU-baseline leg use it.  It shares no code with
the GPU library: the coarsening arithmetic lives in ``spc_oracle.c`` (plain
C, serial) and the spectral quantities in ``spectral.py`` (numpy, FP64).

Functions follow the paper's steps:
  degrees / scores  -- the fitness of every edge (Theorem 1, Algorithm 1)
  order             -- the sort of the fitness list (Algorithm 1)
  merge             -- the merge loop (Algorithm 1)
  contract          -- the coarsened graph (Definition 1)
  coarsen_level     -- one application of Algorithm 1
  coarsen_to        -- repeated levels with re-scoring (conclusion)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from meshgen import Graph

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, EUNREACHABLE, EOVERFLOW, ENOMEM = 0, -1, -2, -3, -5


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (serial, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB_PATH)
        i64, p = C.c_int64, C.c_void_p
        for name, args in [
            ("or_exact_sum", [i64, p, p]),
            ("or_degrees_i", [i64, p, p, p, p, p]),
            ("or_degrees_f", [i64, p, p, p, p, p]),
            ("or_scores_i", [i64, p, p, p, p, p, p, p, p, p]),
            ("or_scores_f", [i64, p, p, p, p, p, p, p, p, p]),
            ("or_order_i", [i64, p, p, p, p, p]),
            ("or_order_f", [i64, p, p, p, p]),
            ("or_merge", [i64, i64, p, p, p, i64, p, p, p]),
            ("or_contract_i", [i64, p, p, p, p, p, p, i64, p, p, p, p, p, p]),
            ("or_contract_f", [i64, p, p, p, p, p, p, i64, p, p, p, p, p, p]),
            ("or_coarsen_level_i", [i64, p, p, p, p, p, i64, p, p, p, p, p, p, p, p, p]),
            ("or_coarsen_level_f", [i64, p, p, p, p, p, i64, p, p, p, p, p, p, p, p, p]),
            ("or_validate", [i64, p, p, p, p, p, p, p, C.c_int]),
        ]:
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = C.c_int
        _lib.or_count_edges.argtypes = [i64, p, p]
        _lib.or_count_edges.restype = i64
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def _host(g: Graph):
    """Contiguous host arrays of a graph in the oracle's types."""
    fp = not g.is_int
    rp = _c(g.row_ptr, np.int64)
    col = _c(g.col, np.int32)
    w = _c(g.w, np.float64 if fp else np.int32)
    sw = _c(g.self_w, np.float64 if fp else np.int64)
    sz = _c(g.size, np.int32)
    return fp, rp, col, w, sw, sz


# --------------------------------------------------------------------------
# exact summation (the definition of every floating-point sum in the method)
# --------------------------------------------------------------------------

def exact_sum(x) -> float:
    """Correctly rounded sum of non-negative doubles."""
    x = _c(np.asarray(x, dtype=np.float64).ravel(), np.float64)
    out = C.c_double()
    _check(_L().or_exact_sum(x.shape[0], _p(x), C.byref(out)), "exact_sum")
    return out.value


def validate(g: Graph) -> int:
    fp, rp, col, w, sw, sz = _host(g)
    return _L().or_validate(g.n, _p(rp), _p(col), None if fp else _p(w), _p(w) if fp else None,
                            None if fp else _p(sw), _p(sw) if fp else None, _p(sz), int(fp))


# --------------------------------------------------------------------------
# steps of Algorithm 1
# --------------------------------------------------------------------------

def degrees(g: Graph) -> np.ndarray:
    fp, rp, col, w, sw, sz = _host(g)
    out = np.zeros(g.n, dtype=np.float64 if fp else np.int64)
    fn = _L().or_degrees_f if fp else _L().or_degrees_i
    _check(fn(g.n, _p(rp), _p(col), _p(w), _p(sw), _p(out)), "degrees")
    return out


def scores(g: Graph):
    """Fitness of every edge u < v in lexicographic order.

    Integer graphs: (eu, ev, N, D) with score = N / D exactly.
    Floating-point graphs: (eu, ev, score, score_literal)."""
    fp, rp, col, w, sw, sz = _host(g)
    m = int(_L().or_count_edges(g.n, _p(rp), _p(col)))
    deg = degrees(g)
    eu = np.zeros(m, np.int64)
    ev = np.zeros(m, np.int64)
    if fp:
        s = np.zeros(m, np.float64)
        sl = np.zeros(m, np.float64)
        _check(_L().or_scores_f(g.n, _p(rp), _p(col), _p(w), _p(sw), _p(deg), _p(eu), _p(ev),
                                _p(s), _p(sl)), "scores")
        return eu, ev, s, sl
    N = np.zeros(m, np.uint64)
    D = np.zeros(m, np.uint64)
    _check(_L().or_scores_i(g.n, _p(rp), _p(col), _p(w), _p(sw), _p(deg), _p(eu), _p(ev),
                            _p(N), _p(D)), "scores")
    return eu, ev, N, D


def order(eu, ev, a, b=None) -> np.ndarray:
    """Sorted fitness list as edge indices: order[r] = edge at position r.
    Pass (N, D) for integer scores or a single float score array."""
    eu = _c(eu, np.int64)
    ev = _c(ev, np.int64)
    m = eu.shape[0]
    out = np.zeros(m, np.int64)
    if b is None:
        s = _c(a, np.float64)
        _check(_L().or_order_f(m, _p(eu), _p(ev), _p(s), _p(out)), "order")
    else:
        N = _c(a, np.uint64)
        D = _c(b, np.uint64)
        _check(_L().or_order_i(m, _p(eu), _p(ev), _p(N), _p(D), _p(out)), "order")
    return out


def merge(n: int, eu, ev, order_, t: int):
    """Merge loop of Algorithm 1.  Returns (cluster_of, accepted edge ids)."""
    eu = _c(eu, np.int64)
    ev = _c(ev, np.int64)
    order_ = _c(order_, np.int64)
    c = np.zeros(n, np.int32)
    acc = np.zeros(max(n, 1), np.int64)
    na = C.c_int64()
    _check(_L().or_merge(n, eu.shape[0], _p(eu), _p(ev), _p(order_), t, _p(c), _p(acc),
                         C.byref(na)), "merge")
    return c, acc[: na.value].copy()


def contract(g: Graph, cluster_of, n_c: int) -> Graph:
    """Coarsened graph of Definition 1, self-loops kept."""
    fp, rp, col, w, sw, sz = _host(g)
    c = _c(cluster_of, np.int32)
    rp_c = np.zeros(n_c + 1, np.int64)
    col_c = np.zeros(max(g.nnz, 1), np.int32)
    w_c = np.zeros(max(g.nnz, 1), np.float64 if fp else np.int32)
    self_c = np.zeros(n_c, np.float64 if fp else np.int64)
    size_c = np.zeros(n_c, np.int32)
    nnz = C.c_int64()
    fn = _L().or_contract_f if fp else _L().or_contract_i
    _check(fn(g.n, _p(rp), _p(col), _p(w), _p(sw), _p(sz), _p(c), n_c, _p(rp_c), _p(col_c),
              _p(w_c), _p(self_c), _p(size_c), C.byref(nnz)), "contract")
    k = nnz.value
    return Graph(n=n_c, row_ptr=rp_c, col=col_c[:k].copy(), w=w_c[:k].copy(), self_w=self_c,
                 size=size_c)


def relabel(g: Graph, perm) -> Graph:
    """The graph with node u renamed perm[u]: Definition 1's contraction with
    one member per super-node (perm must be a permutation of [0, n))."""
    perm = np.asarray(perm, dtype=np.int64)
    if perm.shape[0] != g.n or not np.array_equal(np.sort(perm), np.arange(g.n)):
        raise OracleError(EINVAL, "relabel")
    return contract(g, perm, g.n)


def coarsen_level(g: Graph, t: int):
    """One level of Algorithm 1 to t super-nodes.
    Returns (cluster_of, coarse Graph, eps_max)."""
    fp, rp, col, w, sw, sz = _host(g)
    n = g.n
    c = np.zeros(n, np.int32)
    n_c = C.c_int64()
    rp_c = np.zeros(n + 1, np.int64)
    col_c = np.zeros(max(g.nnz, 1), np.int32)
    w_c = np.zeros(max(g.nnz, 1), np.float64 if fp else np.int32)
    self_c = np.zeros(n, np.float64 if fp else np.int64)
    size_c = np.zeros(n, np.int32)
    nnz = C.c_int64()
    eps = C.c_double()
    fn = _L().or_coarsen_level_f if fp else _L().or_coarsen_level_i
    _check(fn(n, _p(rp), _p(col), _p(w), _p(sw), _p(sz), int(t), _p(c), C.byref(n_c), _p(rp_c),
              _p(col_c), _p(w_c), _p(self_c), _p(size_c), C.byref(nnz), C.byref(eps)),
           "coarsen_level")
    k, nc = nnz.value, n_c.value
    gc = Graph(n=nc, row_ptr=rp_c[: nc + 1].copy(), col=col_c[:k].copy(), w=w_c[:k].copy(),
               self_w=self_c[:nc].copy(), size=size_c[:nc].copy())
    return c, gc, eps.value


def level_targets(n: int, n_c: int, schedule: int = 0):
    """Targets of successive levels.  schedule 0: halve the node count per
    level, t = max(n_c, ceil(n_l / 2)); schedule 1: one pass straight to n_c
    (Algorithm 1 as printed); schedule -j: j merges per level, t = max(n_c,
    n_l - j), so the fitness is recomputed after every j merges (the
    re-scoring the conclusion proposes; j = 1 is the explicit greedy
    algorithm described before Theorem 2)."""
    ts = []
    cur = n
    if n_c >= n:
        return [n]
    if schedule == 1:
        return [n_c]
    if schedule > 1:
        raise ValueError(f"unknown schedule {schedule}")
    while cur > n_c:
        cur = max(n_c, cur + schedule) if schedule < 0 else max(n_c, (cur + 1) // 2)
        ts.append(cur)
    return ts


def coarsen_to(g: Graph, n_c: int, schedule: int = 0):
    """Coarsen level by level (re-scoring at every level).  Returns a list of
    (cluster_of, coarse Graph, eps_max), one entry per level."""
    out = []
    cur = g
    for t in level_targets(g.n, n_c, schedule):
        c, gc, eps = coarsen_level(cur, t)
        out.append((c, gc, eps))
        cur = gc
    return out


def compose(levels, upto: int | None = None) -> np.ndarray:
    """Map from level-0 nodes to super-nodes after `upto` levels (all if None)."""
    lv = levels if upto is None else levels[:upto]
    c = np.arange(lv[0][0].shape[0], dtype=np.int64)
    for cl, _, _ in lv:
        c = cl.astype(np.int64)[c]
    return c
