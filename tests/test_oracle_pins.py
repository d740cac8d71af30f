"""Pins for the oracle: checks against what the paper and the mathematics fix,
never against the oracle itself.

* scores: closed forms (bipartite graphs score exactly 2, K_n scores
  2/(n-1)), a hand-derived fixture, and a literal dense Fraction evaluation
  of || w_u/d_u - w_v/d_v ||_1 (Theorem 1's quantity);
* order + merge loop: a brute-force greedy that rescans every edge at each
  step, a Prim minimum spanning tree prefix, and the closed-form giant
  cluster on row-major bipartite grids;
* contraction: the matrix form B^T W B of Definition 1;
* lift / spectral: spec(L_hat) = spec(L_c) plus (n - n_c) ones, Theorems 1
  and 2 on tiny graphs, an independent dense evaluation of the loss and
  finite differences of its gradient;
* exact sums: Python's math.fsum (correctly rounded).
"""
import heapq
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import spectral as S
from meshgen import Graph, from_edges, grid2d, grid3d, random_graph, tie_permutation, trimesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# brute-force helpers written straight from the definitions
# ----------------------------------------------------------------------------

def dense_rows(g: Graph):
    """Full weighted adjacency rows as dicts x -> a_ux (diagonal included)."""
    rows = [dict() for _ in range(g.n)]
    for u in range(g.n):
        for j in range(g.row_ptr[u], g.row_ptr[u + 1]):
            rows[u][int(g.col[j])] = g.w[j].item()
    if g.self_w is not None:
        for u in range(g.n):
            if g.self_w[u] != 0:
                rows[u][u] = g.self_w[u].item()
    return rows


def literal_score(rows, u, v):
    """|| w_u/d_u - w_v/d_v ||_1 over all coordinates, in exact rationals."""
    du = sum(Fraction(a) for a in rows[u].values())
    dv = sum(Fraction(a) for a in rows[v].values())
    xs = set(rows[u]) | set(rows[v])
    return sum(abs(Fraction(rows[u].get(x, 0)) / du - Fraction(rows[v].get(x, 0)) / dv) for x in xs)


def edges_of(g: Graph):
    out = []
    for u in range(g.n):
        for j in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = int(g.col[j])
            if v > u:
                out.append((u, v))
    return out


def canonical(labels):
    """Renumber a node partition by ascending smallest member."""
    labels = list(labels)
    first = {}
    for x, l in enumerate(labels):
        first.setdefault(l, x)
    order = sorted(first, key=lambda l: first[l])
    rank = {l: i for i, l in enumerate(order)}
    return np.array([rank[l] for l in labels], dtype=np.int64)


def components(n, edges):
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    lab = [-1] * n
    k = 0
    for s in range(n):
        if lab[s] >= 0:
            continue
        stack = [s]
        lab[s] = k
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if lab[y] < 0:
                    lab[y] = k
                    stack.append(y)
        k += 1
    return lab


def greedy_bruteforce(g: Graph, t: int):
    """Algorithm 1 with literal Fraction fitness: at every step rescan all
    edges for the smallest (score, u, v) whose ends are in different
    super-nodes, merge it.  Returns canonical labels."""
    rows = dense_rows(g)
    E = edges_of(g)
    key = {e: (literal_score(rows, *e), e[0], e[1]) for e in E}
    lab = list(range(g.n))
    s = g.n
    while s > t:
        best = None
        for e in E:
            if lab[e[0]] != lab[e[1]] and (best is None or key[e] < key[best]):
                best = e
        assert best is not None
        a, b = lab[best[0]], lab[best[1]]
        lab = [a if l == b else l for l in lab]
        s -= 1
    return canonical(lab)


def prim_prefix(g: Graph, t: int):
    """Components of the n - t smallest edges of a Prim minimum spanning tree
    under the key (literal score, u, v).  Requires a connected graph."""
    rows = dense_rows(g)
    adj = [[] for _ in range(g.n)]
    for (u, v) in edges_of(g):
        k = (literal_score(rows, u, v), u, v)
        adj[u].append((k, u, v))
        adj[v].append((k, u, v))
    seen = [False] * g.n
    seen[0] = True
    heap = list(adj[0])
    heapq.heapify(heap)
    tree = []
    while heap:
        k, u, v = heapq.heappop(heap)
        x = v if seen[u] else u
        if seen[u] and seen[v]:
            continue
        seen[x] = True
        tree.append((k, u, v))
        for it in adj[x]:
            heapq.heappush(heap, it)
    tree.sort()
    return canonical(components(g.n, [(u, v) for _, u, v in tree[: g.n - t]]))


def explicit_greedy_bruteforce(g: Graph, t: int):
    """The explicit greedy algorithm, straight from its description: merge
    the adjacent pair of current super-nodes with the smallest literal
    score (ties by the smaller, then the larger current id, ids numbered by
    smallest member), rebuild the coarse graph (B^T W B, self-loops kept),
    recompute every score, repeat until t super-nodes.  Returns the input
    nodes' final labels, canonical."""
    n = g.n
    W = [[Fraction(0)] * n for _ in range(n)]
    for u, row in enumerate(dense_rows(g)):
        for x, a in row.items():
            W[u][x] = Fraction(a)
    members = [[u] for u in range(n)]
    while len(members) > t:
        k = len(members)
        d = [sum(W[a]) for a in range(k)]
        best = None
        for a in range(k):
            for b in range(a + 1, k):
                if W[a][b] == 0:
                    continue
                sc = sum(abs(W[a][x] / d[a] - W[b][x] / d[b]) for x in range(k))
                if best is None or (sc, a, b) < best:
                    best = (sc, a, b)
        assert best is not None
        _, a, b = best
        merged = members[a] + members[b]
        groups = [m for i, m in enumerate(members) if i not in (a, b)] + [merged]
        groups.sort(key=min)
        lab = {}
        for i, m in enumerate(groups):
            for u in m:
                lab[u] = i
        old_of = {}
        for i, m in enumerate(members):
            old_of[i] = lab[m[0]]
        Wn = [[Fraction(0)] * len(groups) for _ in range(len(groups))]
        for i in range(k):
            for j in range(k):
                if W[i][j]:
                    Wn[old_of[i]][old_of[j]] += W[i][j]
        W, members = Wn, groups
    out = np.zeros(n, dtype=np.int64)
    for i, m in enumerate(members):
        for u in m:
            out[u] = i
    return out


def small_graphs():
    out = []
    for seed in range(6):
        out.append(random_graph(7 + seed % 3, p=0.35, seed=seed, wmax=4))
    for seed in range(4):
        out.append(random_graph(8, p=0.4, seed=100 + seed, wmax=3, self_loops=True, sizes=True))
    out.append(random_graph(9, p=0.5, seed=7, wmax=1))   # unit weights: many ties
    return out


# ----------------------------------------------------------------------------
# exact summation
# ----------------------------------------------------------------------------

def test_exact_sum_is_correctly_rounded():
    r = np.random.default_rng(0)
    for trial in range(200):
        k = int(r.integers(1, 60))
        x = np.exp(r.normal(0, 12, size=k)) * r.random(k)
        if trial % 5 == 0:
            x = np.concatenate([x, [1e300, 1e-300, 3.0]])
        assert oracle.exact_sum(x) == math.fsum(x.tolist())
    # a case where naive left-to-right summation is wrong
    x = [1.0, 2.0 ** -53, 2.0 ** -53]
    assert oracle.exact_sum(x) == 1.0 + 2.0 ** -52 == math.fsum(x)


# ----------------------------------------------------------------------------
# scores (Theorem 1's quantity, Algorithm 1's fitness)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("g", [grid2d(7, ("uniform", 1, 9), seed=1),
                               grid3d(4, ("uniform", 1, 16), seed=2),
                               grid2d(5, "lognormal", seed=3)])
def test_bipartite_scores_are_exactly_two(g):
    # neighbours of u and of v lie on opposite sides, so the supports of the
    # two normalised rows are disjoint and the 1-norm is 1 + 1.
    if g.is_int:
        eu, ev, N, D = oracle.scores(g)
        assert np.all(N == 2 * D)
    else:
        eu, ev, s, sl = oracle.scores(g)
        assert np.all(s == 2.0)


@pytest.mark.parametrize("n", [3, 4, 5, 8])
def test_complete_graph_scores(n):
    u, v = np.triu_indices(n, 1)
    g = from_edges(n, u, v, np.ones(u.shape[0], np.int32))
    eu, ev, N, D = oracle.scores(g)
    for a, b in zip(N, D):
        assert Fraction(int(a), int(b)) == Fraction(2, n - 1)


def load_golden():
    path = os.path.join(GOLDEN, "scores_small.txt")
    G = {"edges": [], "scores": {}, "coarse_edges": []}
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        f = line.split()
        if f[0] == "graph":
            G["n"] = int(f[1])
        elif f[0] == "edge":
            G["edges"].append((int(f[1]), int(f[2]), int(f[3])))
        elif f[0] == "score":
            G["scores"][(int(f[1]), int(f[2]))] = Fraction(f[3])
        elif f[0] == "target":
            G["t"] = int(f[1])
        elif f[0] == "cluster":
            G["cluster"] = [int(x) for x in f[1:]]
        elif f[0] == "coarse_self":
            G["self"] = [int(x) for x in f[1:]]
        elif f[0] == "coarse_edge":
            G["coarse_edges"].append((int(f[1]), int(f[2]), int(f[3])))
        elif f[0] == "coarse_size":
            G["size"] = [int(x) for x in f[1:]]
        elif f[0] == "coarse_score":
            G["coarse_score"] = Fraction(f[3])
    return G


def test_golden_hand_example():
    G = load_golden()
    u, v, w = zip(*G["edges"])
    g = from_edges(G["n"], u, v, np.array(w, np.int32))
    eu, ev, N, D = oracle.scores(g)
    got = {(int(a), int(b)): Fraction(int(x), int(y)) for a, b, x, y in zip(eu, ev, N, D)}
    assert got == G["scores"]
    c, gc, eps = oracle.coarsen_level(g, G["t"])
    assert c.tolist() == G["cluster"]
    assert gc.self_w.tolist() == G["self"]
    assert gc.size.tolist() == G["size"]
    cu, cv, cN, cD = oracle.scores(gc)
    assert [(int(a), int(b)) for a, b in zip(cu, cv)] == [e[:2] for e in G["coarse_edges"]]
    assert Fraction(int(cN[0]), int(cD[0])) == G["coarse_score"]
    assert eps == pytest.approx(4 / 3)


@pytest.mark.parametrize("g", small_graphs())
def test_scores_match_literal_fraction(g):
    rows = dense_rows(g)
    eu, ev, N, D = oracle.scores(g)
    assert list(zip(eu.tolist(), ev.tolist())) == edges_of(g)
    for a, b, x, y in zip(eu, ev, N, D):
        assert Fraction(int(x), int(y)) == literal_score(rows, int(a), int(b))


@pytest.mark.parametrize("seed", range(4))
def test_fp_scores_close_to_exact(seed):
    g = random_graph(9, p=0.4, seed=seed, float_weights=True, self_loops=(seed % 2 == 1))
    rows = dense_rows(g)
    eu, ev, s, sl = oracle.scores(g)
    for a, b, x, xl in zip(eu, ev, s, sl):
        exact = literal_score(rows, int(a), int(b))
        assert abs(Fraction(float(x)) - exact) < Fraction(1, 2 ** 48)
        assert abs(Fraction(float(xl)) - exact) < Fraction(1, 2 ** 48)


# ----------------------------------------------------------------------------
# sort + merge loop (Algorithm 1)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("g", small_graphs())
def test_merge_loop_matches_bruteforce_greedy_and_prim(g):
    for t in range(1, g.n + 1):
        c, gc, eps = oracle.coarsen_level(g, t)
        want = greedy_bruteforce(g, t)
        assert np.array_equal(c.astype(np.int64), want), t
        assert np.array_equal(c.astype(np.int64), prim_prefix(g, t)), t
        assert gc.n == t


@pytest.mark.parametrize("seed", range(6))
def test_rescoring_every_merge_is_the_explicit_greedy(seed):
    """Schedule -1 (one merge per level, scores recomputed each time) equals
    the explicit greedy algorithm written from its description."""
    g = random_graph(8 + seed % 3, p=0.4, seed=200 + seed, wmax=4, self_loops=seed % 2 == 1,
                     sizes=seed % 3 == 0)
    for t in (g.n - 1, g.n // 2, 2):
        lv = oracle.coarsen_to(g, t, -1)
        assert len(lv) == g.n - t
        got = oracle.compose(lv)
        np.testing.assert_array_equal(got, explicit_greedy_bruteforce(g, t))


def test_rescoring_cadence_extremes():
    """j = n - n_c merges per level is the single pass; every cadence reaches
    n_c with levels of exactly j merges (the last one fewer)."""
    g = trimesh(9, ("uniform", 1, 5), seed=3)
    n_c = g.n // 4
    single = oracle.coarsen_to(g, n_c, 1)
    whole = oracle.coarsen_to(g, n_c, -(g.n - n_c))
    assert len(single) == len(whole) == 1
    np.testing.assert_array_equal(single[0][0], whole[0][0])
    for j in (1, 5, 17):
        lv = oracle.coarsen_to(g, n_c, -j)
        sizes = [gc.n for _, gc, _ in lv]
        steps = [a - b for a, b in zip([g.n] + sizes[:-1], sizes)]
        assert sizes[-1] == n_c and all(x == j for x in steps[:-1]) and 0 < steps[-1] <= j


# ----------------------------------------------------------------------------
# the seeded-hash tie-break variant (relabeling by a seeded permutation)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_relabel_is_the_permuted_adjacency(seed):
    g = random_graph(11, p=0.4, seed=300 + seed, wmax=5, self_loops=True, sizes=True,
                     float_weights=seed % 2 == 1)
    perm = tie_permutation(g.n, seed)
    r = oracle.relabel(g, perm)
    W, Wr = S.dense_w(g), S.dense_w(r)
    P = np.zeros((g.n, g.n))
    P[perm, np.arange(g.n)] = 1.0           # P e_u = e_perm[u]
    np.testing.assert_array_equal(Wr, P @ W @ P.T)
    np.testing.assert_array_equal(r.size[perm], g.size)
    inv = np.argsort(perm)
    back = oracle.relabel(r, inv)
    for name in ("row_ptr", "col", "w", "self_w", "size"):
        np.testing.assert_array_equal(getattr(back, name), getattr(oracle.contract(g, np.arange(g.n), g.n), name))


def test_relabel_rejects_non_permutations():
    g = random_graph(6, p=0.5, seed=1)
    with pytest.raises(oracle.OracleError):
        oracle.relabel(g, [0, 1, 2, 3, 4, 4])


@pytest.mark.parametrize("seed", range(4))
def test_hash_tie_break_is_greedy_under_the_permuted_order(seed):
    """Coarsening the relabeled graph is Algorithm 1 on the original graph
    with ties between equal scores broken by (perm[u], perm[v]): scores are
    unchanged, only the order of equal ones moves."""
    g = random_graph(9, p=0.45, seed=400 + seed, wmax=2)      # small weights: many ties
    perm = tie_permutation(g.n, seed)
    rows = dense_rows(g)
    E = edges_of(g)
    key = {e: (literal_score(rows, *e), min(perm[e[0]], perm[e[1]]), max(perm[e[0]], perm[e[1]])) for e in E}
    r = oracle.relabel(g, perm)
    eu, ev, N, D = oracle.scores(r)
    got = sorted(Fraction(int(a), int(b)) for a, b in zip(N, D))
    assert got == sorted(k[0] for k in key.values())
    for t in (g.n - 1, g.n // 2, 2):
        lab = list(range(g.n))
        s_ = g.n
        while s_ > t:
            best = min((e for e in E if lab[e[0]] != lab[e[1]]), key=lambda e: key[e])
            a, b = lab[best[0]], lab[best[1]]
            lab = [a if l == b else l for l in lab]
            s_ -= 1
        c, _, _ = oracle.coarsen_level(r, t)
        np.testing.assert_array_equal(canonical(c[perm]), canonical(lab))


def test_hash_tie_break_avoids_the_giant_cluster():
    """On a bipartite grid every score ties: the lowest-id rule grows one
    super-node {0..k}, a seeded order does not."""
    g = grid2d(24)
    t = g.n // 2
    k = g.n - t
    c0, _, _ = oracle.coarsen_level(g, t)
    assert np.bincount(c0).max() == k + 1
    perm = tie_permutation(g.n, 1)
    c1, _, _ = oracle.coarsen_level(oracle.relabel(g, perm), t)
    assert np.bincount(c1).max() < (k + 1) // 4


def test_merge_loop_accepts_only_cross_edges_in_order():
    g = random_graph(10, p=0.4, seed=11, wmax=3)
    eu, ev, N, D = oracle.scores(g)
    order = oracle.order(eu, ev, N, D)
    keys = [(Fraction(int(N[e]), int(D[e])), int(eu[e]), int(ev[e])) for e in order]
    assert keys == sorted(keys)
    c, acc = oracle.merge(g.n, eu, ev, order, 3)
    assert len(acc) == g.n - 3
    pos = {int(e): r for r, e in enumerate(order)}
    assert [pos[int(e)] for e in acc] == sorted(pos[int(e)] for e in acc)


def giant_closed_form(n, k):
    """Row-major bipartite grid with all scores equal: the merge loop takes
    edges in (u, v) order, which grows one cluster {0, ..., k}."""
    return np.array([0 if x <= k else x - k for x in range(n)], dtype=np.int64)


@pytest.mark.parametrize("s,dim", [(9, 2), (12, 2), (5, 3), (6, 3)])
def test_bipartite_grid_giant_cluster(s, dim):
    g = grid2d(s, ("uniform", 1, 9), seed=s) if dim == 2 else grid3d(s, ("uniform", 1, 9), seed=s)
    n = g.n
    kmin = 2 * s - 1 if dim == 2 else 2 * s * s - 1
    for k in sorted({kmin, kmin + 3, n // 2, n - 2}):
        if k < kmin or k > n - 1:
            continue
        c, gc, eps = oracle.coarsen_level(g, n - k)
        assert np.array_equal(c.astype(np.int64), giant_closed_form(n, k))
        assert eps == 2.0


def test_first_config_level0_giant():
    # 64 x 64 unit 5-point grid: halving gives {0..2048}; a single pass to
    # 1024 super-nodes gives {0..3072}
    g = grid2d(64)
    c, gc, _ = oracle.coarsen_level(g, 2048)
    assert np.array_equal(c.astype(np.int64), giant_closed_form(g.n, 2048))
    c, gc, _ = oracle.coarsen_level(g, 1024)
    assert np.array_equal(c.astype(np.int64), giant_closed_form(g.n, 3072))


def test_unreachable_and_identity():
    g = from_edges(6, [0, 1, 3, 4], [1, 2, 4, 5], np.array([1, 2, 1, 1], np.int32))
    with pytest.raises(oracle.OracleError) as ei:
        oracle.coarsen_level(g, 1)
    assert ei.value.code == oracle.EUNREACHABLE
    c, gc, _ = oracle.coarsen_level(g, 2)
    assert c.tolist() == [0, 0, 0, 1, 1, 1]
    c, gc, eps = oracle.coarsen_level(g, 6)
    assert c.tolist() == list(range(6)) and gc.nnz == g.nnz and eps == 0.0


def test_validation_rejects_bad_csr():
    g = random_graph(6, p=0.5, seed=3)
    assert oracle.validate(g) == 0
    bad = Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy())
    bad.w[0] += 1                       # asymmetric weight
    assert oracle.validate(bad) == oracle.EINVAL
    bad = Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy())
    bad.w[1] = 0                        # non-positive weight
    assert oracle.validate(bad) == oracle.EINVAL
    bad = Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy())
    r0 = slice(bad.row_ptr[0], bad.row_ptr[1])
    bad.col[r0] = bad.col[r0][::-1].copy()   # unsorted row
    if bad.row_ptr[1] - bad.row_ptr[0] > 1:
        assert oracle.validate(bad) == oracle.EINVAL
    big = from_edges(3, [0, 1], [1, 2], np.array([2 ** 30, 1], np.int32))
    assert oracle.validate(big) == oracle.EOVERFLOW


# ----------------------------------------------------------------------------
# contraction (Definition 1) and the lift (Definition 2)
# ----------------------------------------------------------------------------

def random_partition(n, k, seed):
    r = np.random.default_rng(seed)
    lab = np.concatenate([np.arange(k), r.integers(0, k, size=n - k)])
    r.shuffle(lab)
    return canonical(lab)


@pytest.mark.parametrize("seed", range(6))
def test_contract_equals_BtWB(seed):
    fp = seed % 3 == 2
    g = random_graph(11, p=0.35, seed=seed, wmax=5, float_weights=fp, self_loops=seed % 2 == 1,
                     sizes=True)
    k = 4 + seed % 4
    c = random_partition(g.n, k, seed)
    gc = oracle.contract(g, c, k)
    B = np.zeros((g.n, k))
    B[np.arange(g.n), c] = 1.0
    want = B.T @ S.dense_w(g) @ B
    np.testing.assert_allclose(S.dense_w(gc), want, rtol=1e-15, atol=0)
    assert gc.size.tolist() == np.bincount(c, weights=g.size_or_one(), minlength=k).astype(int).tolist()
    # structure: ascending rows, no diagonal, symmetric
    for a in range(k):
        cols = gc.col[gc.row_ptr[a]:gc.row_ptr[a + 1]]
        assert np.all(np.diff(cols) > 0) and a not in cols


def test_contract_fp_sums_are_correctly_rounded():
    # many float weights summed into one super-node: the coarse weight must be
    # the correctly rounded exact sum whatever the order
    g = grid2d(8, "lognormal", seed=9)
    c = np.zeros(g.n, np.int64)
    c[g.n // 2:] = 1
    gc = oracle.contract(g, c, 2)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    intra0 = [float(x) for x, a, b in zip(g.w, c[rows], c[g.col]) if a == b == 0]
    cross = [float(x) for x, a, b in zip(g.w, c[rows], c[g.col]) if a == 0 and b == 1]
    assert gc.self_w[0] == math.fsum(intra0)
    assert gc.w[0] == math.fsum(cross)


@pytest.mark.parametrize("seed", range(5))
def test_lift_spectrum_identity(seed):
    g = random_graph(10, p=0.4, seed=seed, wmax=4, self_loops=seed % 2 == 0)
    for t in (3, 6, 9):
        c, gc, _ = oracle.coarsen_level(g, t)
        Wh = S.lift_dense(S.dense_w(gc), c, gc.size_or_one())
        lh = S.spectrum(Wh)
        lc = S.spectrum(S.dense_w(gc))
        want = np.sort(np.concatenate([lc, np.ones(g.n - t)]))
        np.testing.assert_allclose(lh, want, atol=1e-12)


def test_lift_vectors_orthonormal():
    g = random_graph(12, p=0.3, seed=4)
    c, gc, _ = oracle.coarsen_level(g, 5)
    Q = S.lift_vectors(np.eye(5), c, gc.size, mode=1)
    np.testing.assert_allclose(Q.T @ Q, np.eye(5), atol=1e-14)
    one = S.lift_vectors(np.ones(5), c, gc.size, mode=0)
    assert np.all(one == 1.0)
    U = np.random.default_rng(0).normal(size=(12, 3))
    np.testing.assert_allclose(S.restrict(U, c, gc.size), Q.T @ U, atol=1e-14)


@pytest.mark.parametrize("seed", range(3))
def test_lift_between_levels(seed):
    """Lift between intermediate levels: orthonormal columns, composition
    with the lift from the input equals the input's orthonormal lift
    B S^-1/2 (built here from a dense membership matrix), and piecewise
    constant vectors stay constant."""
    g = random_graph(24, p=0.2, seed=seed, wmax=4)
    levels = oracle.coarsen_to(g, 4, 0)
    maps = [c for c, _, _ in levels]
    sizes = [np.ones(g.n, np.int32)] + [gc.size for _, gc, _ in levels]
    L = len(levels)
    assert L >= 3
    for a, b in [(1, L), (1, 2), (2, L), (0, L), (L - 1, L)]:
        nb = sizes[b].shape[0]
        P = S.lift_between(maps, sizes, a, b, np.eye(nb), mode=1)
        np.testing.assert_allclose(P.T @ P, np.eye(nb), atol=1e-14)
        one = S.lift_between(maps, sizes, a, b, np.ones(nb), mode=0)
        assert np.all(one == 1.0)
        # Q_a P = Q_b with Q_l = B_l S_l^-1/2 from the composed membership
        def Q(lvl):
            c = oracle.compose(levels, lvl) if lvl else np.arange(g.n)
            k = sizes[lvl].shape[0]
            B = np.zeros((g.n, k))
            B[np.arange(g.n), c] = 1.0
            return B / np.sqrt(B.sum(axis=0))[None, :]
        np.testing.assert_allclose(Q(a) @ P, Q(b), atol=1e-14)
    # identity when from == to
    x = np.random.default_rng(seed).normal(size=(sizes[2].shape[0], 2))
    assert np.array_equal(S.lift_between(maps, sizes, 2, 2, x, mode=1), x)


# ----------------------------------------------------------------------------
# Theorems 1 and 2 (brute force on tiny graphs)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_theorem1_single_merge(seed):
    g = random_graph(8, p=0.4, seed=seed, wmax=4, self_loops=seed >= 4)
    lam = S.spectrum(S.dense_w(g))
    eu, ev, N, D = oracle.scores(g)
    for a, b, x, y in zip(eu, ev, N, D):
        eps = int(x) / int(y)
        lab = np.arange(g.n)
        lab[b] = a
        c = canonical(lab)
        gc = oracle.contract(g, c, g.n - 1)
        lh = S.spectrum(S.lift_dense(S.dense_w(gc), c, gc.size_or_one()))
        assert np.max(np.abs(lam - lh)) <= eps + 1e-12


@pytest.mark.parametrize("seed", range(8))
def test_theorem2_merge_prefixes(seed):
    g = random_graph(9, p=0.4, seed=seed, wmax=4)
    lam = S.spectrum(S.dense_w(g))
    eu, ev, N, D = oracle.scores(g)
    order = oracle.order(eu, ev, N, D)
    c, acc = oracle.merge(g.n, eu, ev, order, 1)
    for s in range(1, len(acc) + 1):
        pre = acc[:s]
        eps = max(int(N[e]) / int(D[e]) for e in pre)
        lab = components(g.n, [(int(eu[e]), int(ev[e])) for e in pre])
        cc = canonical(lab)
        k = int(cc.max()) + 1
        gc = oracle.contract(g, cc, k)
        lh = S.spectrum(S.lift_dense(S.dense_w(gc), cc, gc.size_or_one()))
        assert np.max(np.abs(lam - lh)) <= s * (s + 1) / 2 * eps + 1e-12


# ----------------------------------------------------------------------------
# contraction invariants across a multilevel run
# ----------------------------------------------------------------------------

def test_multilevel_invariants():
    g = trimesh(20, ("uniform", 1, 8), seed=3)
    levels = oracle.coarsen_to(g, 40)
    assert [gc.n for _, gc, _ in levels] == oracle.level_targets(g.n, 40)
    total = int(g.w.sum())
    prev = g
    for c, gc, _ in levels:
        assert int(gc.w.sum()) + int(gc.self_w.sum()) == total
        assert int(gc.size.sum()) == g.n
        # degree of a super-node = sum of its members' degrees
        dprev = oracle.degrees(prev)
        assert np.array_equal(oracle.degrees(gc), np.bincount(c, weights=dprev).astype(np.int64))
        # connectivity kept
        lab = components(gc.n, [(u, int(v)) for u in range(gc.n)
                                for v in gc.col[gc.row_ptr[u]:gc.row_ptr[u + 1]]])
        assert max(lab) == 0
        prev = gc
    comp = oracle.compose(levels)
    assert np.array_equal(np.bincount(comp), levels[-1][1].size)


# ----------------------------------------------------------------------------
# spectral error and its gradient
# ----------------------------------------------------------------------------

def _eig_setup(g, k):
    lam, U = S.eigenpairs(S.dense_w(g))
    return lam[1:k + 1], U[:, 1:k + 1]


def test_spectral_error_identity_is_zero():
    g = random_graph(10, p=0.4, seed=2, wmax=4)
    lam, U = _eig_setup(g, 4)
    c, gc, _ = oracle.coarsen_level(g, g.n)
    loss, R = S.spectral_error(gc, c, U, lam)
    np.testing.assert_allclose(R, lam, atol=1e-13)
    assert loss < 1e-24


@pytest.mark.parametrize("seed", range(4))
def test_spectral_error_matches_dense_lift(seed):
    g = random_graph(12, p=0.35, seed=seed, wmax=5, self_loops=seed % 2 == 1)
    lam, U = _eig_setup(g, 5)
    for t in (4, 8):
        c, gc, _ = oracle.coarsen_level(g, t)
        l1, R1 = S.spectral_error(gc, c, U, lam)
        l2, R2 = S.spectral_error_dense(gc, c, U, lam)
        np.testing.assert_allclose(R1, R2, atol=1e-13)
        assert abs(l1 - l2) <= 1e-12 * max(1.0, l2)


def test_spectral_error_gradient_fd():
    g = random_graph(12, p=0.4, seed=5, wmax=5)
    lam, U = _eig_setup(g, 4)
    c, gc, _ = oracle.coarsen_level(g, 6)
    gf = Graph(gc.n, gc.row_ptr, gc.col, gc.w.astype(np.float64), gc.self_w.astype(np.float64),
               gc.size)
    g_w, g_s = S.spectral_error_grad(gf, c, U, lam)
    rows = np.repeat(np.arange(gf.n), np.diff(gf.row_ptr))
    for j in range(gf.nnz):
        a, b = rows[j], gf.col[j]
        if a > b:
            continue
        jm = gf.row_ptr[b] + np.searchsorted(gf.col[gf.row_ptr[b]:gf.row_ptr[b + 1]], a)
        h = 1e-6 * gf.w[j]
        vals = []
        for sgn in (1, -1):
            w2 = gf.w.copy()
            w2[j] += sgn * h
            w2[jm] += sgn * h
            vals.append(S.spectral_error(Graph(gf.n, gf.row_ptr, gf.col, w2, gf.self_w, gf.size),
                                         c, U, lam)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert g_w[j] == pytest.approx(fd, rel=1e-5, abs=1e-9)
        assert g_w[jm] == pytest.approx(g_w[j], rel=1e-13)
    for a in range(gf.n):
        if gf.self_w[a] == 0:
            continue
        h = 1e-6 * gf.self_w[a]
        vals = []
        for sgn in (1, -1):
            s2 = gf.self_w.copy()
            s2[a] += sgn * h
            vals.append(S.spectral_error(Graph(gf.n, gf.row_ptr, gf.col, gf.w, s2, gf.size),
                                         c, U, lam)[0])
        assert g_s[a] == pytest.approx((vals[0] - vals[1]) / (2 * h), rel=1e-5, abs=1e-9)
