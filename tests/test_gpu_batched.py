"""GPU parity of batched coarsening: many graphs packed block-diagonally and
coarsened in shared launches must give, graph by graph, exactly what a
separate coarsening of each graph gives (and what the oracle gives).

Every case prints its name and shape before the GPU call."""
import numpy as np
import pytest

import oracle
from meshgen import Graph, batch_trimeshes, grid2d, random_graph, trimesh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_2204_11757_amd import spc
    spc.lib()
    torch.cuda.init()
    yield spc
    spc.set_option("rank_order", 0)
    spc.set_option("redo_rank", 0)


def say(*a):
    print("[case]", *a, flush=True)


def host(x):
    return None if x is None else x.cpu().numpy()


def split(g_union, cl_union, offs_in, offs_out):
    """Per-graph (cluster_of, Graph) views of a packed level."""
    rp = host(g_union.row_ptr)
    col, w = host(g_union.col), host(g_union.w)
    sw, sz = host(g_union.self_w), host(g_union.size)
    cl = host(cl_union)
    out = []
    for i in range(len(offs_out) - 1):
        a, b = offs_out[i], offs_out[i + 1]
        e0, e1 = rp[a], rp[b]
        gi = Graph(n=int(b - a), row_ptr=rp[a: b + 1] - e0, col=col[e0:e1] - a, w=w[e0:e1],
                   self_w=sw[a:b], size=sz[a:b])
        ci = cl[offs_in[i]: offs_in[i + 1]] - a
        out.append((ci, gi))
    return out


def check_batch(P, graphs, n_c, schedule=0, what=""):
    union, offs = P.pack_graphs(graphs)
    say(what, f"G={len(graphs)} n={union.n} m={union.m}")
    dg = P.DeviceGraph.from_host(union)
    h = P.coarsen_batched(dg, offs, n_c, schedule)
    want = [oracle.coarsen_to(g, int(c), schedule) for g, c in zip(graphs, n_c)]
    assert h.num_levels == max(len(wv) for wv in want)
    for lvl in range(1, h.num_levels + 1):
        cl, gc, st = h.level(lvl)
        parts = split(gc, cl, h.offsets(lvl - 1), h.offsets(lvl))
        for i, (ci, gi) in enumerate(parts):
            wv = want[i]
            if lvl <= len(wv):
                c_or, g_or, _ = wv[lvl - 1]
            else:   # the graph reached its target earlier: carried over unchanged
                c_or, g_or = np.arange(gi.n, dtype=np.int32), wv[-1][1] if wv else graphs[i]
            tag = f"{what} level {lvl} graph {i}"
            np.testing.assert_array_equal(ci, c_or, err_msg=tag + " cluster_of")
            for name in ("row_ptr", "col", "w"):
                np.testing.assert_array_equal(getattr(gi, name), getattr(g_or, name), err_msg=tag + " " + name)
            np.testing.assert_array_equal(gi.self_w, g_or.self_w_or_zero(), err_msg=tag + " self_w")
            np.testing.assert_array_equal(gi.size, g_or.size_or_one(), err_msg=tag + " size")
    return h


def test_batch_of_uneven_triangle_meshes(P):
    graphs = batch_trimeshes(24, seed=4, lo=8, hi=40)
    n_c = [max(1, g.n // 10) for g in graphs]
    check_batch(P, graphs, n_c, 0, "trimesh batch")


def test_batch_single_pass_and_mixed_graphs(P):
    graphs = [grid2d(16), random_graph(50, p=0.1, seed=3, wmax=4),
              trimesh(20, ("uniform", 1, 8), seed=5), random_graph(2, p=1.0, seed=1), grid2d(3)]
    n_c = [16, 7, 50, 1, 9]
    check_batch(P, graphs, n_c, 1, "mixed single pass")
    check_batch(P, graphs, n_c, 0, "mixed halving")


def test_batch_rank_order_path(P):
    graphs = batch_trimeshes(10, seed=9, lo=10, hi=30)
    n_c = [max(1, g.n // 10) for g in graphs]
    try:
        P.set_option("rank_order", 1)
        check_batch(P, graphs, n_c, 0, "rank-order batch")
    finally:
        P.set_option("rank_order", 0)


def test_batch_inexact_key_fallback(P):
    # a batch level flagged inexact is redone with rank keys before its
    # contraction
    graphs = batch_trimeshes(8, seed=13, lo=10, hi=30)
    n_c = [max(1, g.n // 8) for g in graphs]
    try:
        P.set_option("redo_rank", 1)
        check_batch(P, graphs, n_c, 0, "batch redo with rank keys")
    finally:
        P.set_option("redo_rank", 0)


def test_batch_matches_separate_gpu_calls(P):
    graphs = batch_trimeshes(16, seed=4, lo=16, hi=64)
    n_c = [max(1, g.n // 10) for g in graphs]
    union, offs = P.pack_graphs(graphs)
    say("batch vs separate", f"G={len(graphs)} n={union.n}")
    h = P.coarsen_batched(P.DeviceGraph.from_host(union), offs, n_c, 0)
    L = h.num_levels
    cl, gc, _ = h.level(L)
    parts = split(gc, cl, h.offsets(L - 1), h.offsets(L))
    for i, g in enumerate(graphs):
        hi = P.coarsen_to(P.DeviceGraph.from_host(g), n_c[i], 0)
        _, gi_sep, _ = hi.level(hi.num_levels)
        gi = parts[i][1]
        np.testing.assert_array_equal(gi.col, host(gi_sep.col))
        np.testing.assert_array_equal(gi.w, host(gi_sep.w))
        np.testing.assert_array_equal(gi.self_w, host(gi_sep.self_w))


def test_batch_unreachable_target(P):
    from meshgen import from_edges
    g0 = from_edges(4, np.array([0, 2]), np.array([1, 3]), np.array([1, 1], np.int32))   # 2 components
    graphs = [trimesh(10, "unit", seed=1), g0]
    union, offs = P.pack_graphs(graphs)
    say("batch unreachable")
    with pytest.raises(P.SpcError) as ei:
        P.coarsen_batched(P.DeviceGraph.from_host(union), offs, [10, 1], 0)
    assert ei.value.code == -2


def test_batch_band_short_redo(P):
    # bands aimed at a quarter of each graph's merges fall short: the level
    # is redone over every edge, with the same result
    graphs = batch_trimeshes(12, seed=21, lo=12, hi=40, weights=("uniform", 1, 9))
    n_c = [max(1, g.n // 10) for g in graphs]
    try:
        P.set_option("timing", 1)
        P.timing_report()
        P.set_option("batch_band_short", 1)
        h = check_batch(P, graphs, n_c, 0, "batch bands fall short")
        rep = P.timing_report()
    finally:
        P.set_option("batch_band_short", 0)
        P.set_option("timing", 0)
    assert rep["batch_bands"][0] >= 1
    assert rep["rowpass"][0] > h.num_levels   # some level was redone


def test_batch_bands_hold(P):
    # per-graph bands that hold: one forest pass per level
    graphs = batch_trimeshes(12, seed=22, lo=12, hi=40, weights=("uniform", 1, 9))
    n_c = [max(1, g.n // 10) for g in graphs]
    try:
        P.set_option("timing", 1)
        P.timing_report()
        h = check_batch(P, graphs, n_c, 0, "batch bands")
        rep = P.timing_report()
    finally:
        P.set_option("timing", 0)
    assert rep["batch_bands"][0] >= 1
    assert rep["rowpass"][0] == h.num_levels
