"""Seeded mesh and random-graph generators producing symmetric CSR graphs.

Conventions (shared by every generator):

* Node ids are row-major with x fastest: id = x + s*y (+ s*s*z in 3-D).
* The CSR is symmetric, each row's columns are strictly ascending, and there
  are no diagonal entries (self-loop weight lives in ``self_w``).
* Undirected edges are enumerated lexicographically by (u, v) with u < v,
  which is exactly the order of the upper-triangular CSR entries taken row
  by row.  Edge weights are drawn from a seeded ``numpy.random.Generator``
  in that order and mirrored onto the lower entries.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Graph:
    """A weighted undirected graph in symmetric CSR form (host arrays)."""

    n: int
    row_ptr: np.ndarray          # int64[n+1]
    col: np.ndarray              # int32[nnz], ascending per row, no self entries
    w: np.ndarray                # int32 / float32 / float64 [nnz]
    self_w: Optional[np.ndarray] = None   # int64 / float64 [n] or None (all zero)
    size: Optional[np.ndarray] = None     # int32 [n] or None (all one)
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Number of undirected edges (half the directed CSR entries)."""
        return self.nnz // 2

    @property
    def is_int(self) -> bool:
        return self.w.dtype.kind in "iu"

    def self_w_or_zero(self) -> np.ndarray:
        if self.self_w is not None:
            return self.self_w
        return np.zeros(self.n, dtype=np.int64 if self.is_int else np.float64)

    def size_or_one(self) -> np.ndarray:
        if self.size is not None:
            return self.size
        return np.ones(self.n, dtype=np.int32)

    def upper_edges(self):
        """(u, v, w) of the undirected edges u < v in lexicographic order."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        mask = self.col > rows
        return rows[mask], self.col[mask].astype(np.int64), self.w[mask]


# --------------------------------------------------------------------------
# weights
# --------------------------------------------------------------------------

def _draw_weights(rng: np.random.Generator, m: int, spec) -> np.ndarray:
    """Draw m edge weights.  spec is one of
    'unit'                 -> int32 ones
    ('uniform', lo, hi)    -> int32 uniform on {lo..hi}
    'lognormal'            -> float32(exp(N(0,1)))
    """
    if spec == "unit" or spec is None:
        return np.ones(m, dtype=np.int32)
    if spec == "lognormal":
        return np.exp(rng.standard_normal(m)).astype(np.float32)
    if isinstance(spec, tuple) and spec[0] == "uniform":
        lo, hi = int(spec[1]), int(spec[2])
        return rng.integers(lo, hi + 1, size=m, dtype=np.int64).astype(np.int32)
    raise ValueError(f"unknown weight spec {spec!r}")


def _assemble(n: int, offs: np.ndarray, exists: np.ndarray, wspec, wrng) -> Graph:
    """Build a symmetric CSR from a fixed stencil of ascending offsets.

    exists[i, k] says whether node i has neighbour i + offs[k].  The stencil
    must be symmetric (for every offset o, -o is present).
    """
    K = offs.shape[0]
    ids = np.arange(n, dtype=np.int64)
    upper = exists & (offs[None, :] > 0)
    m = int(upper.sum())
    w_up = _draw_weights(wrng, m, wspec)
    wd = np.zeros((n, K), dtype=w_up.dtype)
    wd[upper] = w_up                      # row-major True order == lexicographic (u, v)
    for k in range(K):
        o = int(offs[k])
        if o >= 0:
            continue
        kk = int(np.nonzero(offs == -o)[0][0])
        rows = np.nonzero(exists[:, k])[0]
        wd[rows, k] = wd[rows + o, kk]
    deg = exists.sum(axis=1).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    col = (ids[:, None] + offs[None, :].astype(np.int64))[exists].astype(np.int32)
    w = wd[exists]
    return Graph(n=n, row_ptr=row_ptr, col=col, w=w)


# --------------------------------------------------------------------------
# structured meshes
# --------------------------------------------------------------------------

def grid2d(s: int, weights="unit", seed: int = 0) -> Graph:
    """s x s 5-point grid mesh."""
    n = s * s
    ids = np.arange(n, dtype=np.int64)
    x, y = ids % s, ids // s
    offs = np.array([-s, -1, 1, s], dtype=np.int64)
    exists = np.stack([y > 0, x > 0, x < s - 1, y < s - 1], axis=1)
    g = _assemble(n, offs, exists, weights, np.random.Generator(np.random.PCG64(seed)))
    g.meta = {"kind": "grid2d", "s": s, "seed": seed, "weights": str(weights)}
    return g


def grid3d(s: int, weights="unit", seed: int = 0) -> Graph:
    """s x s x s 7-point grid mesh."""
    n = s * s * s
    ids = np.arange(n, dtype=np.int64)
    x, y, z = ids % s, (ids // s) % s, ids // (s * s)
    offs = np.array([-s * s, -s, -1, 1, s, s * s], dtype=np.int64)
    exists = np.stack([z > 0, y > 0, x > 0, x < s - 1, y < s - 1, z < s - 1], axis=1)
    g = _assemble(n, offs, exists, weights, np.random.Generator(np.random.PCG64(seed)))
    g.meta = {"kind": "grid3d", "s": s, "seed": seed, "weights": str(weights)}
    return g


def trimesh(s: int, weights="unit", seed=0, coords: bool = False) -> Graph:
    """s x s vertex grid, every cell split by one seeded random diagonal.

    Cell (x, y) has corners i = x + s*y, i+1, i+s, i+s+1.  With probability
    1/2 it receives the main diagonal (i, i+s+1), otherwise the anti
    diagonal (i+1, i+s).  Independent child streams of ``SeedSequence(seed)``
    draw, in this order of spawning: the diagonals (cells row-major), the
    vertex jitter (uniform in [-0.3, 0.3] per coordinate; only materialised
    when ``coords`` is set, it does not enter the graph), and the weights.
    """
    ss = np.random.SeedSequence(seed)
    s_diag, s_xy, s_w = ss.spawn(3)
    rd = np.random.Generator(np.random.PCG64(s_diag))
    diag = rd.integers(0, 2, size=(s - 1) * (s - 1), dtype=np.int8).reshape(s - 1, s - 1)  # [y, x]
    main = diag == 0
    n = s * s
    ids = np.arange(n, dtype=np.int64)
    x, y = ids % s, ids // s
    offs = np.array([-s - 1, -s, -s + 1, -1, 1, s - 1, s, s + 1], dtype=np.int64)

    def cell_main(cx, cy, valid):
        out = np.zeros(n, dtype=bool)
        out[valid] = main[cy[valid], cx[valid]]
        return out

    v_mm = (x > 0) & (y > 0)
    v_pa = (x < s - 1) & (y > 0)
    v_ma = (x > 0) & (y < s - 1)
    v_pp = (x < s - 1) & (y < s - 1)
    exists = np.stack([
        cell_main(x - 1, y - 1, v_mm),                 # -s-1 : main diag of cell (x-1, y-1)
        y > 0,                                         # -s
        v_pa & ~cell_main(x, y - 1, v_pa),             # -s+1 : anti diag of cell (x, y-1)
        x > 0,                                         # -1
        x < s - 1,                                     # +1
        v_ma & ~cell_main(x - 1, y, v_ma),             # s-1  : anti diag of cell (x-1, y)
        y < s - 1,                                     # +s
        cell_main(x, y, v_pp),                         # s+1  : main diag of cell (x, y)
    ], axis=1)
    g = _assemble(n, offs, exists, weights, np.random.Generator(np.random.PCG64(s_w)))
    g.meta = {"kind": "trimesh", "s": s, "seed": str(seed), "weights": str(weights)}
    if coords:
        rj = np.random.Generator(np.random.PCG64(s_xy))
        jit = rj.uniform(-0.3, 0.3, size=(n, 2))
        g.meta["xy"] = np.stack([x, y], axis=1).astype(np.float64) + jit
    return g


def batch_sides(count: int = 4096, seed: int = 4, lo: int = 16, hi: int = 256) -> np.ndarray:
    """Side lengths of a batch of triangulated meshes, uniform on {lo..hi}."""
    r = np.random.Generator(np.random.PCG64(seed))
    return r.integers(lo, hi + 1, size=count, dtype=np.int64)


def batch_trimeshes(count: int = 4096, seed: int = 4, lo: int = 16, hi: int = 256,
                    weights="unit"):
    """Independent jittered triangulations; graph g uses SeedSequence([seed, g])."""
    sides = batch_sides(count, seed, lo, hi)
    return [trimesh(int(s), weights=weights, seed=[seed, g]) for g, s in enumerate(sides)]


# --------------------------------------------------------------------------
# general graphs (tests, irregular workloads)
# --------------------------------------------------------------------------

def from_edges(n: int, u, v, w, self_w=None, size=None) -> Graph:
    """Symmetric CSR from an undirected edge list (u != v, no duplicates)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w)
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    if np.any(a == b):
        raise ValueError("self edges belong in self_w")
    key = a * n + b
    order = np.argsort(key, kind="stable")
    a, b, w = a[order], b[order], w[order]
    if np.any(np.diff(a * n + b) == 0):
        raise ValueError("duplicate edge")
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    ww = np.concatenate([w, w])
    order = np.lexsort((cols, rows))
    rows, cols, ww = rows[order], cols[order], ww[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    np.cumsum(row_ptr, out=row_ptr)
    return Graph(n=n, row_ptr=row_ptr, col=cols.astype(np.int32), w=ww,
                 self_w=None if self_w is None else np.asarray(self_w),
                 size=None if size is None else np.asarray(size, dtype=np.int32))


def random_graph(n: int, p: float = 0.3, seed: int = 0, wmax: int = 5,
                 float_weights: bool = False, self_loops: bool = False,
                 self_max: int = 4, connected: bool = True, sizes: bool = False) -> Graph:
    """Seeded random graph: a random spanning tree (if connected) plus
    Erdos-Renyi edges with probability p; integer weights uniform on
    {1..wmax} or float32 lognormal weights."""
    r = np.random.Generator(np.random.PCG64(seed))
    edges = set()
    if connected and n > 1:
        perm = r.permutation(n)
        for i in range(1, n):
            j = int(r.integers(0, i))
            a, b = int(perm[i]), int(perm[j])
            edges.add((min(a, b), max(a, b)))
    for a in range(n):
        for b in range(a + 1, n):
            if r.random() < p:
                edges.add((a, b))
    edges = sorted(edges)
    u = np.array([e[0] for e in edges], dtype=np.int64)
    v = np.array([e[1] for e in edges], dtype=np.int64)
    if float_weights:
        w = np.exp(r.standard_normal(len(edges))).astype(np.float32)
    else:
        w = r.integers(1, wmax + 1, size=len(edges), dtype=np.int64).astype(np.int32)
    self_w = None
    if self_loops:
        if float_weights:
            sw = np.exp(r.standard_normal(n))
            sw[r.random(n) < 0.4] = 0.0
            self_w = sw.astype(np.float64)
        else:
            self_w = r.integers(0, self_max + 1, size=n, dtype=np.int64)
    size = r.integers(1, 4, size=n).astype(np.int32) if sizes else None
    g = from_edges(n, u, v, w, self_w=self_w, size=size)
    g.meta = {"kind": "random", "n": n, "p": p, "seed": seed}
    return g


def powerlaw_graph(n: int, avg_deg: float = 8.0, gamma: float = 2.5, seed: int = 0,
                   wmax: int = 8) -> Graph:
    """Chung-Lu style graph with a power-law expected degree sequence plus a
    path through all nodes (keeps it connected); integer weights on {1..wmax}."""
    r = np.random.Generator(np.random.PCG64(seed))
    i = np.arange(1, n + 1, dtype=np.float64)
    wts = i ** (-1.0 / (gamma - 1.0))
    wts *= avg_deg * n / wts.sum()
    m_target = int(avg_deg * n / 2)
    pr = wts / wts.sum()
    a = r.choice(n, size=m_target, p=pr)
    b = r.choice(n, size=m_target, p=pr)
    perm = r.permutation(n)
    a = np.concatenate([a, perm[:-1]])
    b = np.concatenate([b, perm[1:]])
    keep = a != b
    a, b = a[keep], b[keep]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = np.unique(lo.astype(np.int64) * n + hi)
    u, v = key // n, key % n
    w = r.integers(1, wmax + 1, size=key.shape[0], dtype=np.int64).astype(np.int32)
    g = from_edges(n, u, v, w)
    g.meta = {"kind": "powerlaw", "n": n, "avg_deg": avg_deg, "gamma": gamma, "seed": seed}
    return g


def tie_permutation(n: int, seed: int) -> np.ndarray:
    """A seeded random permutation of [0, n) (int32), for relabeling a graph
    so that equal merge scores fall in a seeded pseudo-random order instead
    of by the lowest node ids."""
    r = np.random.Generator(np.random.PCG64([0x7e, seed]))
    return r.permutation(n).astype(np.int32)
