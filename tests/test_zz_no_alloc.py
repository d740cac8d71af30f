"""The entry point that allocates nothing (spc_coarsen_level_noalloc),
through the C ABI, against spc_coarsen_level on the same inputs, bit for
bit: two calls in a row, the second on a smaller input, then a
floating-point graph, then a graph too large for the scratch array (a clear
SPC_ECAPACITY before any work).  Each result is also compared with the
oracle.  Prints each case before its GPU call."""
import numpy as np
import pytest

import oracle
from meshgen import grid3d, trimesh

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
    return x.cpu().numpy()


def run_both(P, g, t, what):
    import torch
    say(what, f"n={g.n} m={g.m} t={t}")
    dg = P.DeviceGraph.from_host(g, "cuda:0")
    cl_ref, gc_ref, st_ref = P.coarsen_level(dg, t)
    fp = dg.wtype != P.SPC_W_I32
    cl = torch.full((g.n,), -7, dtype=torch.int32, device="cuda:0")
    out = P._empty_out(t, g.nnz, torch.device("cuda:0"), fp=fp)
    for x in (out.row_ptr, out.col, out.w, out.self_w, out.size):
        x.fill_(-3)                      # stale values must not survive
    k, st = P.coarsen_level_noalloc(dg, t, cl, out)
    torch.cuda.synchronize()
    assert k == gc_ref.nnz and st.n_out == st_ref.n_out == t
    assert st.eps_max == st_ref.eps_max and st.ms_total == 0.0
    np.testing.assert_array_equal(host(cl), host(cl_ref), err_msg=what + " cluster_of")
    np.testing.assert_array_equal(host(out.row_ptr[: t + 1]), host(gc_ref.row_ptr), err_msg=what + " row_ptr")
    for name in ("col", "w"):
        np.testing.assert_array_equal(host(getattr(out, name)[:k]), host(getattr(gc_ref, name)),
                                      err_msg=what + " " + name)
    for name in ("self_w", "size"):
        np.testing.assert_array_equal(host(getattr(out, name)[:t]), host(getattr(gc_ref, name)),
                                      err_msg=what + " " + name)
    c_or, gc_or, eps = oracle.coarsen_level(g, t)
    np.testing.assert_array_equal(host(cl), c_or, err_msg=what + " oracle cluster_of")
    np.testing.assert_array_equal(host(out.col[:k]), gc_or.col, err_msg=what + " oracle col")
    np.testing.assert_array_equal(host(out.w[:k]), gc_or.w, err_msg=what + " oracle w")
    assert st.eps_max == eps


def test_noalloc_matches_coarsen_level(P):
    big = trimesh(300, ("uniform", 1, 8), seed=61)          # 90,000 nodes
    run_both(P, big, big.n // 2, "trimesh-300 first call")
    small = trimesh(70, ("uniform", 1, 8), seed=62)         # the array keeps the last call's contents
    run_both(P, small, small.n // 3, "trimesh-70 second call")
    fpg = grid3d(20, "lognormal", seed=63)
    run_both(P, fpg, fpg.n // 2, "grid3d-20 lognormal")
    again = trimesh(300, ("uniform", 1, 8), seed=61)
    run_both(P, again, again.n // 4, "trimesh-300 again, other target")


def test_noalloc_rejects_a_graph_beyond_the_scratch(P):
    import torch
    g = trimesh(700, ("uniform", 1, 8), seed=64)            # about 2.9 M CSR entries
    say("trimesh-700 beyond the scratch", f"n={g.n} nnz={g.nnz}")
    dg = P.DeviceGraph.from_host(g, "cuda:0")
    t = g.n // 2
    cl = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    out = P._empty_out(t, g.nnz, torch.device("cuda:0"))
    with pytest.raises(P.SpcError) as e:
        P.coarsen_level_noalloc(dg, t, cl, out)
    assert e.value.code == P.SPC_ECAPACITY and "scratch" in str(e.value)
    # the regular entry point is unaffected
    small = trimesh(64, ("uniform", 1, 8), seed=65)
    run_both(P, small, small.n // 2, "trimesh-64 after the rejection")
