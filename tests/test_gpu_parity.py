"""GPU parity: the HIP path through the C ABI against the CPU oracle,
bit-exact (cluster maps, coarse CSR, self-loops, sizes) on seeded inputs.

Every case prints its name and shape before the GPU call."""
import numpy as np
import pytest

import oracle
from meshgen import from_edges, grid2d, grid3d, random_graph, trimesh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_2204_11757_amd import spc
    spc.lib()
    torch.cuda.init()
    yield spc
    spc.set_option("rank_order", 0)
    spc.set_option("full_forest", 0)
    spc.set_option("huge_sort", 0)
    spc.set_option("redo_rank", 0)
    spc.set_option("bad_select_guess", 0)
    spc.set_option("contract_wait", 0)
    spc.set_option("speculate", 0)


def say(*a):
    print("[case]", *a, flush=True)


def host(x):
    return None if x is None else x.cpu().numpy()


def assert_same_graph(dg, hg, what=""):
    assert dg.n == hg.n, what
    np.testing.assert_array_equal(host(dg.row_ptr), hg.row_ptr, err_msg=what + " row_ptr")
    np.testing.assert_array_equal(host(dg.col), hg.col, err_msg=what + " col")
    np.testing.assert_array_equal(host(dg.w), hg.w, err_msg=what + " w")
    np.testing.assert_array_equal(host(dg.self_w), hg.self_w, err_msg=what + " self_w")
    np.testing.assert_array_equal(host(dg.size), hg.size, err_msg=what + " size")


def check_level(P, g, t, what=""):
    say(what, f"n={g.n} m={g.m} t={t}")
    dg = P.DeviceGraph.from_host(g)
    cl, gc, st = P.coarsen_level(dg, t)
    c_or, gc_or, eps = oracle.coarsen_level(g, t)
    np.testing.assert_array_equal(host(cl), c_or, err_msg=what + " cluster_of")
    assert_same_graph(gc, gc_or, what)
    assert st.n_out == gc_or.n
    if g.n > t and g.m > 0:
        assert st.eps_max == eps
    return st


def check_hierarchy(P, g, n_c, schedule=0, what=""):
    say(what, f"hierarchy n={g.n} m={g.m} n_c={n_c} schedule={schedule}")
    dg = P.DeviceGraph.from_host(g)
    h = P.coarsen_to(dg, n_c, schedule)
    want = oracle.coarsen_to(g, n_c, schedule)
    assert h.num_levels == len(want)
    stats = []
    for l, (c_or, gc_or, _) in enumerate(want, start=1):
        cl, gc, st = h.level(l)
        np.testing.assert_array_equal(host(cl), c_or, err_msg=f"{what} level {l} cluster_of")
        assert_same_graph(gc, gc_or, f"{what} level {l}")
        stats.append(st)
    return h, want, stats


# ----------------------------------------------------------------------------

RANDOM_CASES = [(n, p, s, sl, fw) for (n, p, s, sl, fw) in [
    (2, 1.0, 0, False, 1), (3, 0.5, 1, False, 3), (5, 0.6, 2, True, 2), (9, 0.3, 3, False, 5),
    (17, 0.25, 4, True, 4), (33, 0.2, 5, False, 9), (40, 0.5, 6, True, 1), (64, 0.1, 7, False, 3),
    (65, 0.08, 8, True, 6), (127, 0.05, 9, False, 2), (300, 0.02, 10, True, 7),
    (513, 0.01, 11, False, 1), (700, 0.015, 12, True, 3)]]


@pytest.mark.parametrize("n,p,seed,self_loops,wmax", RANDOM_CASES)
def test_random_graphs_every_target(P, n, p, seed, self_loops, wmax):
    g = random_graph(n, p=p, seed=seed, wmax=wmax, self_loops=self_loops, sizes=self_loops)
    targets = sorted({1, max(1, n // 3), max(1, n // 2), max(1, n - 1), n})
    for t in targets:
        check_level(P, g, t, f"random(n={n},seed={seed})")


def test_first_config_halving_and_single_pass(P):
    g = grid2d(64)
    check_hierarchy(P, g, 1024, 0, "grid2d-64 halving")
    check_hierarchy(P, g, 1024, 1, "grid2d-64 single pass")


@pytest.mark.parametrize("j", [1, 7, 64, 1000])
def test_rescoring_cadence(P, j):
    # j merges per level (the scores recomputed after every j merges); j = 1
    # is the explicit greedy algorithm, j large enough is the single pass
    g = trimesh(24, ("uniform", 1, 8), seed=40 + j)
    check_hierarchy(P, g, g.n // 4, -j, f"trimesh-24 cadence {j}")
    if j == 1:
        f = grid2d(12, ("uniform", 1, 6), seed=9)   # self-loops from the second level on
        check_hierarchy(P, f, f.n // 3, -1, "grid2d-12 cadence 1")


@pytest.mark.parametrize("s,seed", [(96, 3), (131, 5)])
def test_trimesh_multilevel(P, s, seed):
    g = trimesh(s, ("uniform", 1, 8), seed=seed)
    check_hierarchy(P, g, g.n // 100, 0, f"trimesh-{s}")


def test_trimesh_unit_weights_ties(P):
    g = trimesh(80, "unit", seed=[4, 17])
    check_hierarchy(P, g, g.n // 10, 0, "trimesh-80 unit")


@pytest.mark.parametrize("s", [12, 20])
def test_grid3d_multilevel(P, s):
    g = grid3d(s, ("uniform", 1, 16), seed=2)
    check_hierarchy(P, g, max(1, g.n // 64), 0, f"grid3d-{s}")


def test_alternate_order_and_forest_paths_agree(P):
    g = trimesh(70, ("uniform", 1, 8), seed=9)
    base = check_level(P, g, g.n // 2, "trimesh-70 packed")
    assert base.key_mode == 0
    try:
        P.set_option("rank_order", 1)
        st = check_level(P, g, g.n // 2, "trimesh-70 rank order")
        assert st.key_mode == 1
        P.set_option("full_forest", 1)
        check_level(P, g, g.n // 2, "trimesh-70 rank order + full forest")
        P.set_option("rank_order", 0)
        check_level(P, g, g.n // 3, "trimesh-70 packed + full forest")
        g3 = grid3d(10, ("uniform", 1, 16), seed=4)
        check_hierarchy(P, g3, 20, 0, "grid3d-10 full forest")
    finally:
        P.set_option("rank_order", 0)
        P.set_option("full_forest", 0)


def test_inexact_key_fallback_redoes_the_level(P):
    # a level whose packed keys took an inexact decision is redone with rank
    # keys; the integer path notices this only after its contraction ran, so
    # the labels and the coarse graph are built twice and must still match
    try:
        P.set_option("redo_rank", 1)
        g = trimesh(60, ("uniform", 1, 8), seed=21)
        st = check_level(P, g, g.n // 2, "trimesh-60 redo with rank keys")
        assert st.key_mode == 1
        _, _, stats = check_hierarchy(P, grid3d(12, ("uniform", 1, 16), seed=6), 30, 0, "grid3d-12 redo")
        assert all(s.key_mode == 1 for s in stats)
    finally:
        P.set_option("redo_rank", 0)
    st = check_level(P, g, g.n // 2, "trimesh-60 packed again")
    assert st.key_mode == 0


def test_cutoff_selection_start_over(P):
    # the merge cutoff's selection starts from bounds guessed from the key
    # samples (the selected sample's K bucket, or the smallest sample up to
    # the band threshold); a cutoff outside them makes it start over, which
    # must not change anything (forests of more than 16,384 edges take the
    # multi-block path; the tied-bucket guess itself runs on the bench
    # workload's levels 2-5 in the full-size test)
    try:
        P.set_option("bad_select_guess", 1)
        g = trimesh(160, ("uniform", 1, 8), seed=23)
        check_hierarchy(P, g, g.n // 16, 0, "trimesh-160 bad cutoff guess")
        check_level(P, grid3d(32, ("uniform", 1, 16), seed=8), 8192, "grid3d-32 bad cutoff guess")
    finally:
        P.set_option("bad_select_guess", 0)


def interleaved_grids(copies, side):
    """copies disjoint side x side grids with node x of copy i numbered
    copies * x + i, so that tied merges in edge order reach every copy."""
    g = grid2d(side)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    up = g.col > rows
    u, v, w = rows[up], g.col[up], g.w[up]
    U = np.concatenate([u * copies + i for i in range(copies)])
    V = np.concatenate([v * copies + i for i in range(copies)])
    return from_edges(g.n * copies, U, V, np.concatenate([w] * copies).astype(np.int32))


def test_contraction_class_counts_on_device_and_host(P):
    # the contraction's row classes run on counts the device holds, with up
    # to four huge rows; six giant super-nodes (one per grid) exceed that and
    # take the fallback that reads the counts first; the option that always
    # reads them first, and the adaptive default, must agree as well
    g = interleaved_grids(6, 64)
    try:
        for flag in (2, 3, 1, 0):
            P.set_option("contract_wait", flag)
            check_hierarchy(P, g, g.n // 16, 0, f"6 interleaved grid2d-64, contract_wait={flag}")
            check_hierarchy(P, trimesh(90, ("uniform", 1, 8), seed=31), 800, 0,
                            f"trimesh-90, contract_wait={flag}")
    finally:
        P.set_option("contract_wait", 0)


def test_forest_without_waiting_and_its_redo(P):
    # the host need not wait for the first batch of forest rounds; a forest
    # that needs more rounds than that batch (or a band short of forest
    # edges) makes the level start over with the wait, which must change
    # nothing; never and always-with-one-round must agree with the oracle
    try:
        for mode in (2, 1):
            P.set_option("speculate", mode)
            check_hierarchy(P, trimesh(90, ("uniform", 1, 8), seed=41), 500, 0, f"trimesh-90 speculate={mode}")
            check_hierarchy(P, grid3d(16, ("uniform", 1, 16), seed=3), 64, 0, f"grid3d-16 speculate={mode}")
            check_level(P, random_graph(700, 0.015, seed=12, self_loops=True), 200, f"random-700 speculate={mode}")
    finally:
        P.set_option("speculate", 0)


def test_huge_rows_sort_and_dense_paths(P):
    # a giant super-node (bipartite grids tie every score) and power-law hubs
    # give coarse rows above the block capacity; both contraction strategies
    # for such rows must agree with the oracle
    from meshgen import powerlaw_graph
    cases = [(grid2d(64), 1024, "grid2d-64"),
             (grid3d(20, ("uniform", 1, 16), seed=2), 125, "grid3d-20")]
    gp = powerlaw_graph(20000, avg_deg=8.0, gamma=2.05, seed=5)
    cases.append((gp, gp.n // 8, "powerlaw-20000"))
    try:
        for flag in (0, 1):
            P.set_option("huge_sort", flag)
            for g, n_c, name in cases:
                check_hierarchy(P, g, n_c, 0, f"{name} huge_sort={flag}")
    finally:
        P.set_option("huge_sort", 0)


def test_edge_cases(P):
    import torch
    # single edge
    g = from_edges(2, [0], [1], np.array([3], np.int32))
    check_level(P, g, 1, "single edge")
    check_level(P, g, 2, "single edge identity")
    # target above n is the identity
    g = random_graph(20, p=0.3, seed=1)
    check_level(P, g, 50, "target above n")
    # disconnected graph: reachable and unreachable targets
    g = from_edges(6, [0, 1, 3, 4], [1, 2, 4, 5], np.array([1, 2, 1, 1], np.int32))
    check_level(P, g, 2, "two components")
    say("two components, unreachable target")
    with pytest.raises(P.SpcError) as ei:
        P.coarsen_level(P.DeviceGraph.from_host(g), 1)
    assert ei.value.code == P.SPC_EUNREACHABLE
    # isolated nodes (a graph with no edges can only keep every node)
    g = from_edges(3, [0], [1], np.array([1], np.int32))
    check_level(P, g, 2, "isolated node")
    # integer overflow guard
    g = from_edges(3, [0, 1], [1, 2], np.array([2 ** 30, 5], np.int32))
    say("overflow")
    with pytest.raises(P.SpcError) as ei:
        P.coarsen_level(P.DeviceGraph.from_host(g), 2)
    assert ei.value.code == P.SPC_EOVERFLOW
    # bad target
    with pytest.raises(P.SpcError) as ei:
        P.coarsen_level(P.DeviceGraph.from_host(random_graph(5, 0.5, 2)), 0)
    assert ei.value.code == P.SPC_EINVAL
    torch.cuda.synchronize()


def _tile_boundary_graph(seed=21):
    # a row of 900 upper entries (it spans a boundary of the score's
    # 768-edge tiles), a run of isolated nodes, then a sparse random part in
    # which every seventh node is isolated: many tiles start inside long
    # rows or after rows without upper entries
    rng = np.random.default_rng(seed)
    n = 6000
    us = [np.zeros(900, np.int64)]
    vs = [np.arange(1, 901)]
    pool = np.array([x for x in range(2000, n) if x % 7])
    a = rng.choice(pool, 20000)
    b = rng.choice(pool, 20000)
    keep = a != b
    us.append(a[keep])
    vs.append(b[keep])
    u = np.concatenate(us)
    v = np.concatenate(vs)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    pairs = np.unique(lo * n + hi)
    w = rng.integers(1, 9, len(pairs)).astype(np.int32)
    return from_edges(n, (pairs // n).astype(np.int64), (pairs % n).astype(np.int64), w)


def test_tiles_across_long_and_empty_rows(P):
    g = _tile_boundary_graph()
    # every node of the connected part but one merges away at most; isolated
    # nodes stay, so aim well above the number of components
    check_level(P, g, g.n - 1500, "tile boundaries in long and empty rows")
    h, want, _ = check_hierarchy(P, g, g.n - 2500, 0, "tile boundaries, halving")


def _star_gap_graph(seed=5):
    # a star of 1024 leaves fills the first 2048 CSR entries exactly, then 76
    # isolated nodes start at entry 2048, ahead of the row that holds it: the
    # contraction's record scatter tiles (2048 entries) start right there
    n = 3000
    rng = np.random.default_rng(seed)
    a = rng.integers(1101, n, 6000)
    b = rng.integers(1101, n, 6000)
    keep = a != b
    u = np.concatenate([np.zeros(1024, np.int64), a[keep]])
    v = np.concatenate([np.arange(1, 1025), b[keep]])
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    pairs = np.unique(lo * n + hi)
    w = rng.integers(1, 9, len(pairs)).astype(np.int32)
    g = from_edges(n, (pairs // n).astype(np.int64), (pairs % n).astype(np.int64), w)
    assert g.row_ptr[1025] == 2048 and g.row_ptr[1101] == 2048
    return g


def test_empty_rows_at_a_tile_start(P):
    g = _star_gap_graph()
    check_level(P, g, g.n - 800, "empty rows at a scatter tile's start")
    check_hierarchy(P, g, g.n - 1600, 0, "empty rows at a scatter tile's start, halving")


def _heavy_edge_graph():
    # a 30x30 triangle mesh whose edges at three nodes weigh 2^23: degrees
    # reach 2^26 (the score's products then take 64-bit multiplies) while
    # the total weight stays far below 2^31
    g = trimesh(30, ("uniform", 1, 8), seed=11)
    rp = np.asarray(g.row_ptr)
    col = np.asarray(g.col, np.int64)
    w = np.asarray(g.w, np.int64)
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    up = col > rows
    u, v, ww = rows[up], col[up], w[up].copy()
    ww[np.isin(u, [100, 437, 781]) | np.isin(v, [100, 437, 781])] = 1 << 23
    return from_edges(g.n, u, v, ww.astype(np.int32))


def test_degrees_above_2_24(P):
    g = _heavy_edge_graph()
    rp = np.asarray(g.row_ptr)
    assert np.add.reduceat(np.asarray(g.w, np.int64), rp[:-1]).max() >= 1 << 24
    assert g.m > 1 << 11   # (keys from the corrected double-precision quotient)
    check_level(P, g, g.n // 2, "degrees above 2^24")
    check_hierarchy(P, g, g.n // 16, 0, "degrees above 2^24, halving")


def test_deterministic_reruns(P):
    g = trimesh(100, ("uniform", 1, 8), seed=12)
    dg = P.DeviceGraph.from_host(g)
    say("determinism trimesh-100")
    ref = None
    for _ in range(4):
        cl, gc, st = P.coarsen_level(dg, g.n // 2)
        cur = [host(cl), host(gc.row_ptr), host(gc.col), host(gc.w), host(gc.self_w), host(gc.size)]
        if ref is None:
            ref = cur
        else:
            for a, b in zip(ref, cur):
                assert np.array_equal(a, b)


def test_lift_and_spectral_error(P):
    import torch
    from oracle import spectral as S
    g = trimesh(24, ("uniform", 1, 8), seed=21)
    say("lift/spectral trimesh-24")
    dg = P.DeviceGraph.from_host(g)
    h = P.coarsen_to(dg, g.n // 8, 0)
    want = oracle.coarsen_to(g, g.n // 8, 0)
    lam, U = S.eigenpairs(S.dense_w(g))
    k = 6
    lam, U = lam[1:k + 1], U[:, 1:k + 1]
    Ud = torch.from_numpy(U).cuda()
    ld = torch.from_numpy(lam).cuda()
    for lvl in range(1, len(want) + 1):
        comp = oracle.compose(want, lvl)
        gc = want[lvl - 1][1]
        loss_o, R_o = S.spectral_error(gc, comp, U, lam)
        loss_g, R_g = P.spectral_error(h, lvl, Ud, ld)
        np.testing.assert_allclose(host(R_g), R_o, rtol=1e-12, atol=1e-13)
        assert abs(loss_g - loss_o) <= 1e-10 * max(loss_o, 1e-300)
        xc = np.random.default_rng(lvl).normal(size=(gc.n, 3))
        for mode in (0, 1):
            xf = P.lift(h, 0, lvl, mode, torch.from_numpy(xc).cuda())
            np.testing.assert_array_equal(host(xf), S.lift_vectors(xc, comp, gc.size, mode))
    # between intermediate levels: the lift of the oracle's hierarchy
    maps = [c for c, _, _ in want]
    sizes = [np.ones(g.n, np.int32)] + [gc.size for _, gc, _ in want]
    L = len(want)
    for a, b in [(1, L), (1, 2), (2, L), (L - 1, L), (2, 2)]:
        xc = np.random.default_rng(10 * a + b).normal(size=(sizes[b].shape[0], 3))
        for mode in (0, 1):
            xf = P.lift(h, a, b, mode, torch.from_numpy(xc).cuda())
            np.testing.assert_array_equal(host(xf), S.lift_between(maps, sizes, a, b, xc, mode),
                                          err_msg=f"lift {b} -> {a} mode {mode}")


def test_calls_queued_back_to_back_and_freed_without_waiting(P):
    # a call returns once its last level is queued and freeing a hierarchy
    # does not wait: hierarchies freed while later calls run, and blocks
    # handed out again in stream order, must leave every result intact
    ga = grid3d(24, ("uniform", 1, 16), seed=31)
    gb = trimesh(90, ("uniform", 1, 8), seed=32)
    da, db = P.DeviceGraph.from_host(ga), P.DeviceGraph.from_host(gb)
    say("back-to-back calls", f"grid3d-24 n={ga.n}, trimesh-90 n={gb.n}")
    ha = P.coarsen_to(da, ga.n // 16, 0)
    hb = P.coarsen_to(db, gb.n // 8, 0)
    ha.free()                                   # hb's work may still be queued
    ha2 = P.coarsen_to(da, ga.n // 16, 0)       # takes ha's blocks again
    hb.free()
    hb2 = P.coarsen_to(db, gb.n // 8, 0)
    for h, g, n_c, what in ((ha2, ga, ga.n // 16, "grid3d-24"), (hb2, gb, gb.n // 8, "trimesh-90")):
        want = oracle.coarsen_to(g, n_c, 0)
        assert h.num_levels == len(want)
        for l, (c_or, gc_or, _) in enumerate(want, start=1):
            cl, gc, st = h.level(l)
            np.testing.assert_array_equal(host(cl), c_or, err_msg=f"{what} level {l} cluster_of")
            assert_same_graph(gc, gc_or, f"{what} level {l}")
            assert st.ms_total > 0
        h.free()


def test_scan_flag_raised_once_does_not_fail_later_calls(P):
    # one level that finds the scan chain's error flag raised fails; the
    # next call on the same context starts with the flag clear
    g = trimesh(40, ("uniform", 1, 8), seed=41)
    dg = P.DeviceGraph.from_host(g)
    say("scan flag", f"trimesh-40 n={g.n}")
    P.coarsen_to(dg, g.n // 4, 0).free()        # the context's scan chain exists
    P.set_option("scan_flag", 1)
    with pytest.raises(P.SpcError) as e:
        P.coarsen_to(dg, g.n // 4, 0)
    assert e.value.code == P.SPC_EINVAL and "look-back" in str(e.value)
    h = P.coarsen_to(dg, g.n // 4, 0)
    want = oracle.coarsen_to(g, g.n // 4, 0)
    for l, (c_or, gc_or, _) in enumerate(want, start=1):
        cl, gc, _ = h.level(l)
        np.testing.assert_array_equal(host(cl), c_or, err_msg=f"level {l} cluster_of")
        assert_same_graph(gc, gc_or, f"level {l}")
    h.free()


def test_calls_on_two_streams(P):
    # a call on one torch stream, then at once a call and the level exports
    # on another: the context orders the new stream after the old one
    import torch
    ga = grid3d(28, ("uniform", 1, 16), seed=51)
    gb = trimesh(120, ("uniform", 1, 8), seed=52)
    da, db = P.DeviceGraph.from_host(ga), P.DeviceGraph.from_host(gb)
    torch.cuda.synchronize()
    say("two streams", f"grid3d-28 n={ga.n}, trimesh-120 n={gb.n}")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        ha = P.coarsen_to(da, ga.n // 32, 0)
    with torch.cuda.stream(s2):
        hb = P.coarsen_to(db, gb.n // 16, 0)
        out_a = [ha.level(l) for l in range(1, ha.num_levels + 1)]
        out_b = [hb.level(l) for l in range(1, hb.num_levels + 1)]
    s2.synchronize()
    for outs, g, n_c, what in ((out_a, ga, ga.n // 32, "grid3d-28"), (out_b, gb, gb.n // 16, "trimesh-120")):
        want = oracle.coarsen_to(g, n_c, 0)
        assert len(outs) == len(want)
        for l, ((c_or, gc_or, _), (cl, gc, _)) in enumerate(zip(want, outs), start=1):
            np.testing.assert_array_equal(host(cl), c_or, err_msg=f"{what} level {l} cluster_of")
            assert_same_graph(gc, gc_or, f"{what} level {l}")
    torch.cuda.synchronize()
    ha.free()
    hb.free()


@pytest.mark.parametrize("fp", [False, True])
def test_relabel_and_hash_tie_break(P, fp):
    # the graph relabeled by a seeded permutation (equal scores then fall in
    # a seeded order), and its hierarchy, against the oracle
    from meshgen import tie_permutation
    g = grid3d(10, "lognormal", seed=5) if fp else trimesh(40, ("uniform", 1, 4), seed=[9, 1])
    perm = tie_permutation(g.n, 3)
    say("relabel", f"n={g.n} m={g.m} fp={fp}")
    dg = P.DeviceGraph.from_host(g)
    r = P.relabel(dg, perm)
    want = oracle.relabel(g, perm)
    assert_same_graph(r, want, "relabel")
    check_hierarchy(P, want, g.n // 8, 0, "hash tie-break hierarchy")
    with pytest.raises(P.SpcError) as e:
        bad = perm.copy()
        bad[0] = bad[1]
        P.relabel(dg, bad)
    assert e.value.code == P.SPC_EINVAL


def test_hash_tie_break_on_a_bipartite_grid(P):
    # every score ties: the lowest-id rule grows one giant super-node, the
    # seeded order does not; both bit-exact against the oracle
    from meshgen import tie_permutation
    g = grid3d(16, ("uniform", 1, 16), seed=2)
    say("hash tie-break grid3d-16", f"n={g.n}")
    t = g.n // 2
    st0 = check_level(P, g, t, "lowest id")
    perm = tie_permutation(g.n, 7)
    r = P.relabel(P.DeviceGraph.from_host(g), perm)
    st1 = check_level(P, r.to_host(), t, "seeded order")
    assert st0.largest_cluster == g.n - t + 1
    assert st1.largest_cluster < st0.largest_cluster // 2


@pytest.mark.parametrize("opt,val", [("lane_max", 16), ("wave_max", 64), ("wave_max", 200), ("small_rpt", 1),
                                     ("small_rpt", 2), ("small_rpt", 4), ("huge_tile", 1024), ("huge_tile", 4096),
                                     ("sel_blocks", 2), ("sel_blocks", 32), ("bv_short", 1),
                                     ("bv_short", 1 << 40)])
def test_launch_settings_do_not_change_results(P, opt, val):
    # every launch setting the autotuner may pick gives the same result
    P.set_option(opt, val)
    try:
        g = trimesh(96, ("uniform", 1, 8), seed=61)
        check_hierarchy(P, g, g.n // 50, 0, f"trimesh-96 {opt}={val}")
        f = grid3d(16, ("uniform", 1, 16), seed=62)   # a giant super-node: huge rows
        check_hierarchy(P, f, f.n // 32, 0, f"grid3d-16 {opt}={val}")
    finally:
        P.set_option(opt, 0)


def test_autotune_plain_and_batched(P):
    g = trimesh(120, ("uniform", 1, 8), seed=63)
    dg = P.DeviceGraph.from_host(g)
    say("autotune trimesh-120", f"n={g.n}")
    rep = P.autotune(dg, g.n // 100, 0)
    assert "best" in rep and "start" in rep
    check_hierarchy(P, g, g.n // 100, 0, "trimesh-120 tuned")
    from meshgen import batch_trimeshes
    graphs = batch_trimeshes(24, seed=64, lo=16, hi=48)
    union, offs = P.pack_graphs(graphs)
    n_c = [max(1, x.n // 10) for x in graphs]
    say("autotune batch-24", f"n={union.n}")
    du = P.DeviceGraph.from_host(union)
    rep = P.autotune(du, None, 0, offs, n_c)
    assert "best" in rep
    h = P.coarsen_batched(du, offs, n_c, 0)
    cl, gc, _ = h.level(h.num_levels)
    o = h.offsets(h.num_levels)
    for i, x in enumerate(graphs):
        want = oracle.coarsen_to(x, n_c[i], 0)[-1][1]
        a, b = o[i], o[i + 1]
        e0, e1 = int(host(gc.row_ptr)[a]), int(host(gc.row_ptr)[b])
        np.testing.assert_array_equal(host(gc.col)[e0:e1] - a, want.col, err_msg=f"graph {i}")
        np.testing.assert_array_equal(host(gc.w)[e0:e1], want.w, err_msg=f"graph {i}")
    h.free()
