"""The spectral-quality report (paper Section 4, Figure 2) from the GPU
hierarchy equals the one from the oracle's hierarchy (the hierarchies are
bit-exact, so every measure is identical), for every schedule the report
uses.  Prints each case before its GPU call."""
import numpy as np
import pytest

import oracle
from meshgen import grid2d, trimesh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_2204_11757_amd import spc
    spc.lib()
    torch.cuda.init()
    yield spc


@pytest.mark.parametrize("mesh", ["trimesh", "grid"])
def test_quality_report_gpu_equals_oracle(P, mesh):
    from paper_2204_11757_amd import quality as Qm
    g = trimesh(20, ("uniform", 1, 8), seed=3) if mesh == "trimesh" else grid2d(20)
    lam, U = Qm.input_spectrum(g)
    dg = P.DeviceGraph.from_host(g, "cuda:0")
    for ratio in (2, 8):
        for _, sched in Qm.SCHEDULES:
            print("[case] quality", mesh, ratio, sched, flush=True)
            h = P.coarsen_to(dg, g.n // ratio, sched)
            got = Qm.hierarchy_levels(h, g.n)
            h.free()
            lv = oracle.coarsen_to(g, g.n // ratio, sched)
            want = []
            prev = g.n
            for c, gc, eps in lv:
                want.append((c, gc, eps, prev - gc.n))
                prev = gc.n
            qg, _, ag = Qm.evaluate_levels(lam, U, got, g.n, k=20)
            qo, _, ao = Qm.evaluate_levels(lam, U, want, g.n, k=20)
            assert qg == qo
            assert np.array_equal(ag, ao)


def test_quality_cli_runs(P, tmp_path):
    from paper_2204_11757_amd import quality as Qm
    print("[case] quality cli side 16", flush=True)
    rep = Qm.main(["--side", "16", "--k", "8", "--out", str(tmp_path / "q.json")])
    assert len(rep["meshes"]) == 2 and all(len(m["runs"]) == 21 for m in rep["meshes"])
    for m in rep["meshes"]:
        for r in m["runs"]:
            assert r["spectral_error_inf"] <= r["thm2_bound"] + 1e-9
