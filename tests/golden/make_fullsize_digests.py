"""Write tests/golden/fullsize_digests.json: per-level digests of the oracle's
results on the full-size workloads, which the GPU tests compare against.

Runs on the CPU only and calls nothing but the oracle (``oracle``), the
input generators (``meshgen``) and the hashing helpers (``digest``):

* trimesh-4096: 4096^2 triangle mesh, weights U{1..8}, seed 3, halving
  levels to n/100 = 167,772 super-nodes (7 levels);
* batch-4096: 4,096 triangle meshes, sides U{16..256} (seed 4), unit
  weights, each halved level by level to n/10 (4 levels per graph); the
  digests of every level's block-diagonal union plus one digest per graph
  over all its levels;
* grid3d-64-lognormal: 64^3 7-point grid, float32 lognormal(0, 1) weights,
  seed 5, halving levels to 32,768 super-nodes (3 levels).

Usage: python tests/golden/make_fullsize_digests.py [name ...]
(about four minutes for trimesh-4096 and six for batch-4096 on this
container's cores; the batch uses a thread per core, each oracle call is
serial).
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import digest as D  # noqa: E402
import oracle  # noqa: E402
from meshgen import batch_sides, batch_trimeshes, grid3d, trimesh  # noqa: E402

OUT = os.path.join(HERE, "fullsize_digests.json")

RECIPES = {
    "trimesh-4096": "trimesh(4096, ('uniform', 1, 8), seed=3); coarsen_to(n // 100, schedule 0)",
    "batch-4096": "batch_trimeshes(4096, seed=4); graph g to max(1, n_g // 10), schedule 0",
    "grid3d-64-lognormal": "grid3d(64, 'lognormal', seed=5); coarsen_to(32768, schedule 0)",
}


def single(g, n_c):
    t0 = time.time()
    levels = oracle.coarsen_to(g, n_c, 0)
    dt = time.time() - t0
    fp = not g.is_int
    out = []
    for c, gc, eps in levels:
        d = D.level_digest(c, gc, fp)
        d["eps_max"] = float(eps).hex()
        out.append(d)
    return {"n": g.n, "m": g.m, "n_c": n_c, "levels": out, "oracle_s": round(dt, 1)}


def batch():
    graphs = batch_trimeshes(4096, seed=4)
    n_c = [max(1, x.n // 10) for x in graphs]
    t0 = time.time()

    def run(i):
        return oracle.coarsen_to(graphs[i], n_c[i], 0)

    with ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
        res = list(ex.map(run, range(len(graphs))))
    dt = time.time() - t0
    L = len(res[0])
    assert all(len(r) == L for r in res)
    per_graph = [D.graph_levels_digest([(c, gc) for c, gc, _ in r], False) for r in res]
    levels = []
    for lvl in range(L):
        h = D.GraphHasher(False)
        for r in res:
            c, gc, _ = r[lvl]
            h.add(c, gc)
        levels.append({"n": h.node_out, "nnz": h.entries, "sha": h.digest()})
    return {"graphs": len(graphs), "n": int(sum(x.n for x in graphs)),
            "m": int(sum(x.m for x in graphs)), "sides_sha": D.sha(np.ascontiguousarray(
                batch_sides(4096, 4), dtype="<i8"))[:16],
            "levels": levels, "graph_sha": per_graph, "oracle_s": round(dt, 1)}


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        t0 = time.time()
        if name == "trimesh-4096":
            g = trimesh(4096, ("uniform", 1, 8), seed=3)
            rec = single(g, g.n // 100)
        elif name == "grid3d-64-lognormal":
            rec = single(grid3d(64, "lognormal", seed=5), 32768)
        elif name == "batch-4096":
            rec = batch()
        else:
            raise SystemExit(f"unknown workload {name}")
        rec["recipe"] = RECIPES[name]
        data[name] = rec
        print(f"{name}: {len(rec['levels'])} levels in {time.time() - t0:.1f} s", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or list(RECIPES))
