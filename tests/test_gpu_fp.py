"""GPU parity of the floating-point path (FP32 / FP64 weights, FP64 scores,
correctly rounded exact sums) and of the differentiable pieces (spectral
error forward and backward, entry map, contraction adjoint), through the
C ABI, against the CPU oracle.

Every case prints its name and shape before the GPU call."""
import numpy as np
import pytest

import oracle
from oracle import spectral as osp
from meshgen import Graph, grid3d, random_graph, trimesh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_2204_11757_amd import spc
    spc.lib()
    torch.cuda.init()
    yield spc


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
    say(what, f"n={g.n} m={g.m} t={t} w={g.w.dtype}")
    dg = P.DeviceGraph.from_host(g)
    cl, gc, st = P.coarsen_level(dg, t)
    c_or, gc_or, eps = oracle.coarsen_level(g, t)
    np.testing.assert_array_equal(host(cl), c_or, err_msg=what + " cluster_of")
    assert_same_graph(gc, gc_or, what)
    if g.n > t and g.m > 0:
        assert st.key_mode == 3
        assert st.eps_max == eps
    return st


def check_hierarchy(P, g, n_c, schedule=0, what=""):
    say(what, f"hierarchy n={g.n} m={g.m} n_c={n_c} w={g.w.dtype}")
    dg = P.DeviceGraph.from_host(g)
    h = P.coarsen_to(dg, n_c, schedule)
    want = oracle.coarsen_to(g, n_c, schedule)
    assert h.num_levels == len(want)
    for l, (c_or, gc_or, _) in enumerate(want, start=1):
        cl, gc, st = h.level(l)
        np.testing.assert_array_equal(host(cl), c_or, err_msg=f"{what} level {l} cluster_of")
        assert_same_graph(gc, gc_or, f"{what} level {l}")
    return h, want


FP_RANDOM = [(2, 1.0, 0, False), (5, 0.6, 1, True), (17, 0.25, 2, True), (40, 0.3, 3, False),
             (65, 0.1, 4, True), (300, 0.02, 5, True), (700, 0.01, 6, False)]


@pytest.mark.parametrize("n,p,seed,self_loops", FP_RANDOM)
def test_fp32_random_graphs_every_target(P, n, p, seed, self_loops):
    g = random_graph(n, p=p, seed=seed, float_weights=True, self_loops=self_loops, sizes=self_loops)
    for t in sorted({1, max(1, n // 3), max(1, n // 2), max(1, n - 1), n}):
        check_level(P, g, t, f"fp32 random(n={n},seed={seed})")


def test_fp64_wide_exponent_range(P):
    # weights spread over ~80 binades: the sums are still exact and rounded once
    g = random_graph(200, p=0.05, seed=11, float_weights=True, self_loops=True)
    r = np.random.Generator(np.random.PCG64(12))
    u, v, w = g.upper_edges()
    scale = np.ldexp(1.0, r.integers(-40, 40, size=w.shape[0]))
    from meshgen import from_edges
    g64 = from_edges(g.n, u, v, w.astype(np.float64) * scale, self_w=g.self_w)
    for t in (150, 100, 37, 1):
        check_level(P, g64, t, "fp64 wide range")


def test_fp_meshes_multilevel(P):
    check_hierarchy(P, grid3d(12, "lognormal", seed=5), 12 ** 3 // 8, 0, "grid3d-12 lognormal")
    check_hierarchy(P, grid3d(16, "lognormal", seed=5), 16 ** 3 // 8, 1, "grid3d-16 lognormal single")
    check_hierarchy(P, trimesh(64, "lognormal", seed=7), 64 * 64 // 20, 0, "trimesh-64 lognormal")


def test_fp_errors(P):
    from meshgen import from_edges
    u = np.array([0, 1, 2], np.int64)
    v = np.array([1, 2, 3], np.int64)
    say("fp errors")
    wide = from_edges(4, u, v, np.array([1e-30, 1.0, 1e30], np.float64))
    dg = P.DeviceGraph.from_host(wide)
    with pytest.raises(P.SpcError) as ei:
        P.coarsen_level(dg, 2)
    assert ei.value.code == -7
    bad = from_edges(4, u, v, np.array([1.0, -2.0, 1.0], np.float64))
    with pytest.raises(P.SpcError) as ei:
        P.coarsen_level(P.DeviceGraph.from_host(bad), 2)
    assert ei.value.code == -1
    nan = from_edges(4, u, v, np.array([1.0, np.nan, 1.0], np.float64))
    with pytest.raises(P.SpcError) as ei:
        P.coarsen_level(P.DeviceGraph.from_host(nan), 2)
    assert ei.value.code == -1


# ----------------------------------------------------------------------------
# differentiable pieces
# ----------------------------------------------------------------------------

def _spectral_case(P, s=8, levels_to=None, k=6, seed=5):
    import torch
    g = grid3d(s, "lognormal", seed=seed)
    W = osp.dense_w(g)
    lam, U = osp.eigenpairs(W)
    lam, U = lam[1:k + 1], U[:, 1:k + 1]        # nontrivial pairs
    n_c = levels_to or g.n // 8
    dg = P.DeviceGraph.from_host(g)
    h = P.coarsen_to(dg, n_c, 0)
    want = oracle.coarsen_to(g, n_c, 0)
    L = h.num_levels
    cl, gc, st = h.level(L)
    cmap = P.cluster_map(h, L)
    cmap_or = oracle.compose(want)
    np.testing.assert_array_equal(host(cmap), cmap_or)
    Ut = torch.from_numpy(U).cuda()
    lt = torch.from_numpy(lam).cuda()
    return g, h, gc, want[-1][1], cmap, cmap_or, Ut, lt, U, lam


def test_spectral_error_forward_and_backward(P):
    say("spectral error grid3d-8 lognormal")
    g, h, gc, gc_or, cmap, cmap_or, Ut, lt, U, lam = _spectral_case(P)
    loss, R = P.spectral_error_graph(gc, cmap, Ut, lt)
    loss_or, R_or = osp.spectral_error(gc_or, cmap_or, U, lam)
    assert loss == pytest.approx(loss_or, rel=1e-10, abs=1e-14)
    np.testing.assert_allclose(host(R), R_or, rtol=1e-12, atol=1e-13)
    loss_h, _ = P.spectral_error(h, h.num_levels, Ut, lt)
    assert loss_h == pytest.approx(loss_or, rel=1e-10, abs=1e-14)
    dw, ds = P.spectral_error_backward(gc, cmap, Ut, lt)
    gw_or, gs_or = osp.spectral_error_grad(gc_or, cmap_or, U, lam)
    scale = max(np.abs(gw_or).max(), np.abs(gs_or).max())
    np.testing.assert_allclose(host(dw), gw_or, rtol=1e-10, atol=1e-12 * scale)
    np.testing.assert_allclose(host(ds), gs_or, rtol=1e-10, atol=1e-12 * scale)


def test_fp32_spectral_error_and_gradients(P):
    # the FP32 form against the FP64 oracle: loss and R to 1e-5 relative,
    # gradients to 1e-5 relative in the max norm
    say("spectral error FP32 grid3d-16")
    g, h, gc, gc_or, cmap, cmap_or, Ut, lt, U, lam = _spectral_case(P, s=16, k=12)
    U32 = Ut.float()
    loss, R = P.spectral_error_graph(gc, cmap, U32, lt)
    loss_or, R_or = osp.spectral_error(gc_or, cmap_or, U, lam)
    assert R.dtype.is_floating_point and R.element_size() == 4
    assert loss == pytest.approx(loss_or, rel=1e-5)
    np.testing.assert_allclose(host(R), R_or, rtol=1e-5, atol=1e-6)
    dw, ds = P.spectral_error_backward(gc, cmap, U32, lt)
    assert dw.element_size() == 4 and ds.element_size() == 4
    gw_or, gs_or = osp.spectral_error_grad(gc_or, cmap_or, U, lam)
    scale = max(np.abs(gw_or).max(), np.abs(gs_or).max())
    assert np.abs(host(dw).astype(np.float64) - gw_or).max() <= 1e-5 * scale
    assert np.abs(host(ds).astype(np.float64) - gs_or).max() <= 1e-5 * scale
    # through autograd: FP64 parameters, FP32 spectral kernels
    w = gc.w.clone().requires_grad_(True)
    sw = gc.self_w.clone().requires_grad_(True)
    P.spectral_error_loss(w, sw, gc, cmap, U32, lt).backward()
    assert w.grad.dtype == w.dtype
    np.testing.assert_allclose(host(w.grad), 0.5 * host(dw).astype(np.float64), rtol=1e-6, atol=0)


def test_spectral_gradient_central_differences(P):
    import torch
    say("spectral gradient FD grid3d-8")
    g, h, gc, gc_or, cmap, cmap_or, Ut, lt, U, lam = _spectral_case(P)
    dw, ds = P.spectral_error_backward(gc, cmap, Ut, lt)
    dw, ds = host(dw), host(ds)
    rp, col = host(gc.row_ptr), host(gc.col)
    rows = np.repeat(np.arange(gc.n), np.diff(rp))
    r = np.random.Generator(np.random.PCG64(3))
    upper = np.nonzero(col > rows)[0]
    picks = r.choice(upper, size=min(8, upper.shape[0]), replace=False)
    w0 = gc.w.clone()
    for j in picks:
        a, b = rows[j], col[j]
        jm = rp[b] + np.searchsorted(col[rp[b]:rp[b + 1]], a)
        hstep = 1e-6 * float(w0[j])
        vals = []
        for sgn in (1.0, -1.0):
            w = w0.clone()
            w[j] += sgn * hstep
            w[jm] += sgn * hstep
            gg = P.DeviceGraph(n=gc.n, row_ptr=gc.row_ptr, col=gc.col, w=w, self_w=gc.self_w, size=gc.size)
            vals.append(P.spectral_error_graph(gg, cmap, Ut, lt)[0])
        fd = (vals[0] - vals[1]) / (2 * hstep)
        assert fd == pytest.approx(dw[j], rel=1e-5, abs=1e-9 * max(1.0, abs(dw).max()))
    for a in r.choice(gc.n, size=4, replace=False):
        hstep = 1e-6 * max(1.0, float(gc.self_w[a]))
        vals = []
        for sgn in (1.0, -1.0):
            s = gc.self_w.clone()
            s[a] += sgn * hstep
            gg = P.DeviceGraph(n=gc.n, row_ptr=gc.row_ptr, col=gc.col, w=gc.w, self_w=s, size=gc.size)
            vals.append(P.spectral_error_graph(gg, cmap, Ut, lt)[0])
        fd = (vals[0] - vals[1]) / (2 * hstep)
        assert fd == pytest.approx(ds[a], rel=1e-5, abs=1e-9 * max(1.0, abs(ds).max()))


def test_autograd_function_matches_backward(P):
    import torch
    say("autograd grid3d-8")
    g, h, gc, gc_or, cmap, cmap_or, Ut, lt, U, lam = _spectral_case(P)
    w = gc.w.clone().requires_grad_(True)
    s = gc.self_w.clone().requires_grad_(True)
    loss = P.spectral_error_loss(w, s, gc, cmap, Ut, lt)
    (3.0 * loss).backward()
    dw, ds = P.spectral_error_backward(gc, cmap, Ut, lt)
    np.testing.assert_allclose(host(w.grad), 1.5 * host(dw), rtol=1e-14, atol=0)
    np.testing.assert_allclose(host(s.grad), 3.0 * host(ds), rtol=1e-14, atol=0)


def test_entry_map_and_contraction_adjoint(P):
    import torch
    for g, t, name in [(grid3d(10, "lognormal", seed=5), 500, "grid3d-10 fp32"),
                       (random_graph(120, p=0.05, seed=9, float_weights=True, self_loops=True), 50,
                        "random-120 fp32 self"),
                       (trimesh(30, ("uniform", 1, 8), seed=3), 450, "trimesh-30 int")]:
        say("entry map", name)
        dg = P.DeviceGraph.from_host(g)
        cl, gc, st = P.coarsen_level(dg, t)
        emap = host(P.entry_map(dg, cl, gc))
        c = host(cl)
        rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        rpc, colc = host(gc.row_ptr), host(gc.col)
        for j in range(g.nnz):
            a, b = c[rows[j]], c[g.col[j]]
            if a == b:
                assert emap[j] == -1 - a
            else:
                p = emap[j]
                assert rpc[a] <= p < rpc[a + 1] and colc[p] == b
        # adjoint identity <C^T y, x> = <y, C x> with C the (linear) contraction
        r = np.random.Generator(np.random.PCG64(7))
        u, v, _ = g.upper_edges()
        from meshgen import from_edges
        dx = r.random(u.shape[0]) + 0.5
        dself = r.random(g.n) + 0.5
        gx = from_edges(g.n, u, v, dx, self_w=dself)
        Cx = oracle.contract(gx, c, gc.n)
        yw = r.standard_normal(gc.nnz)
        ys = r.standard_normal(gc.n)
        dwf, dsf = P.contract_backward(torch.from_numpy(emap).cuda(), cl, torch.from_numpy(yw).cuda(),
                                       torch.from_numpy(ys).cuda(), g.n)
        lhs = float(np.dot(host(dwf), gx.w) + np.dot(host(dsf), dself))
        rhs = float(np.dot(yw, Cx.w) + np.dot(ys, Cx.self_w))
        assert lhs == pytest.approx(rhs, rel=1e-12)


def test_reweight_lowers_the_spectral_error(P):
    import torch
    from paper_2204_11757_amd.reweight import reweight
    say("reweight grid3d-8")
    g, h, gc, gc_or, cmap, cmap_or, Ut, lt, U, lam = _spectral_case(P)
    out, hist = reweight(gc, cmap, Ut, lt, steps=40, lr=1e-2)
    # Adam on log-weights with a small step: the loss goes down step by step
    assert hist[-1] < 0.99 * hist[0], hist
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist[:10], hist[1:11])), hist
    # the refined weights stay symmetric and positive
    w = host(out.w)
    rp, col = host(out.row_ptr), host(out.col)
    rows = np.repeat(np.arange(out.n), np.diff(rp))
    for j in range(0, out.nnz, 7):
        a, b = rows[j], col[j]
        jm = rp[b] + np.searchsorted(col[rp[b]:rp[b + 1]], a)
        assert w[j] == w[jm] and w[j] > 0
    # the oracle agrees with the library on the refined graph's loss
    gh = Graph(n=out.n, row_ptr=rp, col=col, w=w, self_w=host(out.self_w), size=host(out.size))
    loss_or, _ = osp.spectral_error(gh, cmap_or, U, lam)
    assert hist[-1] == pytest.approx(loss_or, rel=1e-10)


def test_spectral_error_long_member_lists_and_rows(P):
    # a power-law hub gives a coarse row longer than one thread walks; the
    # first level of a bipartite grid gives a super-node with thousands of
    # members: both take the block-reduction kernels
    import torch
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    from meshgen import powerlaw_graph
    for g, t, name in [(powerlaw_graph(20000, avg_deg=8.0, gamma=2.05, seed=5), 10000, "powerlaw-20000"),
                       (grid3d(24, "lognormal", seed=5), 24 ** 3 // 2, "grid3d-24 lognormal")]:
        say("spectral long lists", name)
        Wd = osp.sparse_w(g)
        d = np.asarray(Wd.sum(axis=1)).ravel()
        s = 1.0 / np.sqrt(d)
        L = (sp.identity(g.n) - sp.diags(s) @ Wd @ sp.diags(s)).tocsr()
        lam, U = sla.eigsh(L, k=5, which="SA", tol=1e-12)
        o = np.argsort(lam)
        lam, U = lam[o][1:], np.ascontiguousarray(U[:, o][:, 1:])
        dg = P.DeviceGraph.from_host(g)
        cl, gc, st = P.coarsen_level(dg, t)
        c_or, gc_or, _ = oracle.coarsen_level(g, t)
        Ut, lt = torch.from_numpy(U).cuda(), torch.from_numpy(lam).cuda()
        loss, R = P.spectral_error_graph(gc, cl, Ut, lt)
        loss_or, R_or = osp.spectral_error(gc_or, c_or, U, lam)
        assert loss == pytest.approx(loss_or, rel=1e-10)
        np.testing.assert_allclose(host(R), R_or, rtol=1e-11, atol=1e-12)
        dw, ds = P.spectral_error_backward(gc, cl, Ut, lt)
        gw_or, gs_or = osp.spectral_error_grad(gc_or, c_or, U, lam)
        scale = max(np.abs(gw_or).max(), np.abs(gs_or).max())
        np.testing.assert_allclose(host(dw), gw_or, rtol=1e-9, atol=1e-11 * scale)
        np.testing.assert_allclose(host(ds), gs_or, rtol=1e-9, atol=1e-11 * scale)
        rp = host(gc.row_ptr)
        members = np.bincount(c_or)
        assert members.max() > 2048 or np.diff(rp).max() > 2048
