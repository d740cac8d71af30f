#!/usr/bin/env python3
"""Throughput of the coarsening hot path on one MI355X.

One step = one full multilevel coarsen_to call (every level: degrees,
scores, order, merge selection, contraction) over a synthetic mesh that is
already resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME]
                  [--no-cpu-baseline]

value = sum over levels of the level's input edge count, divided by the
time of one step (fine edges coarsened per second, edge-weighted over the
levels).  The per-level breakdown is in "levels".
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fine edges coarsened/sec per level + % HBM peak; batched vs per-graph graphs/s"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak


def make_config(name):
    from meshgen import grid2d, grid3d, trimesh
    if name == "grid3d-128":
        g = grid3d(128, ("uniform", 1, 16), seed=2)
        return g, g.n // 64, ("3D 7-point structured mesh 128^3 (2,097,152 nodes, 6,242,304 edges), "
                              "int32 weights uniform in [1,16] (seed 2), halving levels to n/64 = 32,768")
    if name == "trimesh-4096":
        g = trimesh(4096, ("uniform", 1, 8), seed=3)
        return g, g.n // 100, ("jittered triangle mesh 4096x4096 (16,777,216 nodes, 50,315,265 edges), "
                               "int32 weights uniform in [1,8] (seed 3), halving levels to n/100 = 167,772")
    if name == "trimesh-1024":
        g = trimesh(1024, ("uniform", 1, 8), seed=3)
        return g, g.n // 100, "jittered triangle mesh 1024x1024, int32 weights uniform in [1,8], to n/100"
    if name == "grid2d-64":
        g = grid2d(64)
        return g, 1024, "2D 5-point grid 64x64, unit weights, halving to 1,024"
    raise SystemExit(f"unknown config {name}")


# Algorithmic HBM bytes of one launch, from the level's sizes: the data the
# kernel must move at least once (inputs read once, outputs written once).
def algo_bytes(kernel, L):
    n, m, nnz, n_c, nnz_c, selfb = L["n"], L["m"], 2 * L["m"], L["n_c"], L["nnz_c"], L["self"]
    if kernel == "score":            # CSR rows once, per-node prefix/degree/bests, key written
        return 24 * m + 44 * n + 8 * n * selfb
    if kernel == "degree":           # row_ptr, col + w once, per-node outputs
        return 8 * nnz + 56 * n + 8 * n * selfb
    if kernel == "filter":           # keys and per-node prefixes read
        return 8 * m + 20 * n
    if kernel == "contract_small":   # member rows, their neighbours' labels, coarse rows written
        return 12 * nnz + 28 * n + 32 * n_c + 8 * nnz_c + 12 * n * selfb
    if kernel == "contract_pack":
        return 16 * nnz_c + 16 * n_c
    if kernel == "contract_members":
        return 20 * n + 24 * n_c
    if kernel == "components":
        return 16 * n
    if kernel == "relabel":
        return 16 * n
    return None


def method_floor_bytes(L):
    """Compulsory traffic of a level plus one 8-byte key written and read per edge."""
    n, m, n_c, nnz_c = L["n"], L["m"], L["n_c"], L["nnz_c"]
    comp = 8 * (n + 1) + 16 * m + (8 * n if L["self"] else 0) + 4 * n
    comp += 8 * (n_c + 1) + 8 * nnz_c + 8 * n_c + 4 * n_c
    return comp + 16 * m


def cpu_baseline(g):
    import oracle
    t = (g.n + 1) // 2
    t0 = time.perf_counter()
    oracle.coarsen_level(g, t)
    dt = time.perf_counter() - t0
    return {"value": g.m / dt, "unit": "fine edges/s", "cores": 1, "kind": "oracle",
            "seconds": round(dt, 3),
            "sample": f"one level (the first) of the same mesh: {g.n} nodes, {g.m} edges, "
                      f"halving to {t}; serial C oracle on one host core"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="grid3d-128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device tensor copy (reference kernel for "
                         "scaling hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    print(f"[bench] building input {args.config}", file=sys.stderr, flush=True)
    g, n_c, desc = make_config(args.config)
    import torch
    from paper_2204_11757_amd import spc
    dg = spc.DeviceGraph.from_host(g, "cuda:0")
    torch.cuda.synchronize()
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        h = spc.coarsen_to(dg, n_c, 0)
        return h

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    h = None
    for _ in range(args.warmup):
        h = step()
        h.free()
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    last = None
    for _ in range(args.steps):
        hh = step()
        if last is not None:
            last.free()      # returns the level buffers to the caching allocator
        last = hh
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    levels = []
    prev_n = g.n
    for l in range(1, last.num_levels + 1):
        st = last.stats(l)
        L = {"level": l, "n": st.n_in, "m": st.m_in, "n_c": st.n_out, "nnz_c": st.nnz_out,
             "self": 1 if l > 1 else 0, "ms": round(st.ms_total, 4),
             "key_mode": {0: "exact-packed", 1: "rank", 2: "guarded-packed"}.get(st.key_mode, "?"),
             "forest_rounds": st.boruvka_rounds, "candidate_edges": st.candidate_edges,
             "largest_cluster": st.largest_cluster}
        L["fine_edges_per_s"] = st.m_in / (st.ms_total * 1e-3) if st.ms_total > 0 else None
        L["hbm_floor_frac"] = (method_floor_bytes(L) / (st.ms_total * 1e-3) / (HBM_PEAK_GBS * 1e9)
                               if st.ms_total > 0 else None)
        levels.append(L)
        prev_n = st.n_out
    last.free()
    total_edges = sum(L["m"] for L in levels)
    value = total_edges / (ms * 1e-3)

    roofline = None
    kernels = None
    if not args.no_roofline:
        print("[bench] per-kernel timing pass", file=sys.stderr, flush=True)
        spc.set_option("timing", 1)
        spc.timing_report()   # clear
        for _ in range(args.steps):
            hh = step()
            hh.free()
        rep = spc.timing_report()
        spc.set_option("timing", 0)
        kernels = {k: {"launches": c, "ms_total": round(t, 4), "ms_avg": round(t / c, 5)}
                   for k, (c, t, u) in sorted(rep.items(), key=lambda kv: -kv[1][1])}
        dom = None
        for k, (c, t, u) in sorted(rep.items(), key=lambda kv: -kv[1][1]):
            dom = k
            break
        per_step_bytes = None
        if dom is not None:
            b = [algo_bytes(dom, L) for L in levels]
            if all(x is not None for x in b):
                per_step_bytes = sum(b)
        if dom is not None:
            c, t, u = rep[dom]
            avg_ms = t / c
            if per_step_bytes is not None:
                launches_per_step = c / args.steps
                bytes_per_launch = per_step_bytes / launches_per_step
                achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
                roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                            "avg_launch_ms": round(avg_ms, 5),
                            "algo_bytes_per_launch": int(bytes_per_launch)}
            else:
                roofline = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": None, "traffic": None,
                            "avg_launch_ms": round(avg_ms, 5),
                            "note": "no algorithmic byte model for this kernel"}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, one level)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(g)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "fine edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.config, "nodes": g.n, "edges": g.m,
                   "n_c": n_c, "levels": len(levels), "schedule": "halving"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "levels": levels,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
