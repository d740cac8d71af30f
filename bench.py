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
    if name == "powerlaw-131k":
        from meshgen import powerlaw_graph
        g = powerlaw_graph(1 << 17, avg_deg=8.0, gamma=2.5, seed=7)
        return g, g.n // 100, (f"Chung-Lu power-law graph (irregular degrees): 131,072 nodes, {g.m:,} edges, "
                               "expected degrees ~ i^(-1/1.5), mean 8, plus a path through all nodes, int32 "
                               "weights uniform in [1,8] (seed 7), halving levels to n/100 = 1,310")
    if name == "grid2d-64":
        g = grid2d(64)
        return g, 1024, "2D 5-point grid 64x64, unit weights, halving to 1,024"
    if name.startswith("batch-"):
        from meshgen import batch_trimeshes
        from paper_2204_11757_amd.spc import pack_graphs
        count = int(name.split("-")[1])
        graphs = batch_trimeshes(count, seed=4)
        union, offs = pack_graphs(graphs)
        union.meta = {"graphs": graphs, "offsets": offs, "n_c": [max(1, x.n // 10) for x in graphs]}
        return union, None, (f"{count} jittered triangle meshes, sides uniform in [16,256] (seed 4), unit "
                             f"weights, {union.n:,} nodes and {union.m:,} edges in total, each graph "
                             f"halving to n/10")
    raise SystemExit(f"unknown config {name}")


# Algorithmic HBM bytes over one level, from the level's sizes: what the
# method must move at least once (inputs read once, outputs written once).
# Units: n nodes and m undirected edges in, n_c nodes and nnz_c entries out;
# `self` is 1 on coarse levels, which carry per-node self-loops.
def csr_read_bytes(L):
    """The level's CSR read once: row pointers, columns and weights of both
    directions (4 + 4 bytes per entry), self-loops on coarse levels."""
    return 8 * (L["n"] + 1) + 16 * L["m"] + 8 * L["n"] * L["self"]


def coarse_write_bytes(L):
    """Labels (4 B per fine node) and the coarse CSR written once: row
    pointers, columns and weights, self-loops and sizes."""
    return 4 * L["n"] + 8 * (L["n_c"] + 1) + 8 * L["nnz_c"] + 8 * L["n_c"] + 4 * L["n_c"]


def algo_bytes(kernel, L):
    """Per-level algorithmic bytes of a kernel (or a phase) as the method
    defines its work; None where no unit applies."""
    m = L["m"]
    if kernel == "score":
        # degrees and scores: the CSR read once, one 8-byte score per edge written
        return csr_read_bytes(L) + 8 * m
    if kernel == "degree":
        return csr_read_bytes(L) + 8 * L["n"]
    if kernel == "rowpass":
        # the order: each edge's score read once
        return 8 * m
    if kernel == "phase:contract":
        # Definition 1: the fine CSR and each node's label and size read once,
        # the coarse CSR written once
        return csr_read_bytes(L) + 8 * L["n"] + coarse_write_bytes(L) - 4 * L["n"]
    return None


# timing scopes per phase of a level
PHASES = {
    "score": ["degree", "degree_total", "scan_upper", "score", "score_rank", "rank_sort", "rank_scatter"],
    "select": ["select_threshold", "rowpass", "forest_candidates", "forest_merge", "forest_shortcut",
               "select_cutoff", "components", "relabel"],
    "contract": ["contract_members", "contract_small", "contract_reg32", "contract_wave_rows",
                 "contract_block_rows", "contract_huge", "contract_rowptr", "contract_pack"],
}


# kernels timed one launch per scope (the candidates for the roofline line)
SINGLE_KERNEL_SCOPES = ["score", "rowpass", "degree", "forest_candidates", "forest_merge",
                        "contract_small", "contract_reg32", "contract_wave_rows",
                        "contract_block_rows", "contract_pack"]
KERNEL_SYMBOL = {"score": "k_score<0>", "rowpass": "k_rowpass", "degree": "k_degree",
                 "forest_candidates": "k_bv_candidates", "forest_merge": "k_bv_merge",
                 "contract_small": "k_contract_small", "contract_reg32": "k_contract_reg32",
                 "contract_wave_rows": "k_contract_row<64, 512>",
                 "contract_block_rows": "k_contract_row<256, 4096>", "contract_pack": "k_pack"}
# source file of each kernel: a stored counter reading is used only while
# this file is unchanged
KERNEL_SOURCE = {"score": "score.hip", "rowpass": "select.hip", "degree": "select.hip",
                 "forest_candidates": "select.hip", "forest_merge": "select.hip",
                 "contract_small": "contract.hip", "contract_reg32": "contract.hip",
                 "contract_wave_rows": "contract.hip", "contract_block_rows": "contract.hip",
                 "contract_pack": "contract.hip"}


def stored_traffic(kernel, config_name):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current source of the kernel and this workload."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(f"{kernel}@{config_name}")
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2204_11757_amd", "csrc", KERNEL_SOURCE[kernel])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    return rec["bytes_per_launch"]


def method_floor_bytes(L):
    """Compulsory traffic of a level (the CSR read once, labels and the
    coarse CSR written once) plus one 8-byte score written and read per edge."""
    return csr_read_bytes(L) + coarse_write_bytes(L) + 16 * L["m"]


def cpu_sample(name, g, n_c):
    """A bounded sample of the workload for the oracle's timing (about 10-30 s
    of one host core): the whole step when it is that short, else the same
    generator at a smaller size, every level to the same relative target."""
    if name == "trimesh-4096":
        from meshgen import trimesh
        x = trimesh(1024, ("uniform", 1, 8), seed=3)
        return x, x.n // 100, ("the whole step on a 1024x1024 triangle mesh of the same generator and "
                               "weights (1/16 of the nodes; 1,048,576 nodes, 3,141,633 edges), halving "
                               "levels to n/100")
    return g, n_c, f"the whole step ({name}, every level to n_c={n_c})"


def cpu_baseline(g, n_c, what):
    """The oracle on one step of `g`, repeated until about 10 s of host time
    have passed (at least once), on one host core."""
    import oracle
    runs, total_edges, t_all = 0, 0, 0.0
    while runs == 0 or t_all < 10.0:
        t0 = time.perf_counter()
        lv = oracle.coarsen_to(g, n_c, 0)
        t_all += time.perf_counter() - t0
        prev = g
        for _, gc, _ in lv:
            total_edges += prev.m
            prev = gc
        runs += 1
    return {"value": total_edges / t_all, "unit": "fine edges/s", "cores": 1, "kind": "oracle",
            "seconds": round(t_all, 3),
            "sample": f"{what}, run {runs} time(s) by the serial C oracle on one host core"}


def cpu_baseline_batch(graphs, n_c, seconds=10.0):
    """The oracle on the batch's graphs in order, one coarsening each, until
    about `seconds` of host time have passed, on one host core."""
    import oracle
    done, t_all = 0, 0.0
    for x, c in zip(graphs, n_c):
        t0 = time.perf_counter()
        oracle.coarsen_to(x, c, 0)
        t_all += time.perf_counter() - t0
        done += 1
        if t_all >= seconds:
            break
    return {"value": done / t_all, "unit": "graphs/s", "cores": 1, "kind": "oracle",
            "seconds": round(t_all, 3),
            "sample": f"the first {done} graphs of the batch, each coarsened to n/10 by the serial C "
                      f"oracle on one host core"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="trimesh-4096")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-graph", action="store_true",
                    help="batch configs: skip the one-call-per-graph comparison (for profiling)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the library's autotuner (run before the warmup, outside the timed steps)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device tensor copy (reference kernel for "
                         "scaling hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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

    batch = g.meta.get("graphs") is not None if isinstance(g.meta, dict) else False

    def step():
        if batch:
            return spc.coarsen_batched(dg, g.meta["offsets"], g.meta["n_c"], 0)
        return spc.coarsen_to(dg, n_c, 0)

    tuned = None
    if not args.no_autotune:
        print("[bench] autotune", file=sys.stderr, flush=True)
        if batch:
            rep = spc.autotune(dg, None, 0, g.meta["offsets"], g.meta["n_c"])
        else:
            rep = spc.autotune(dg, n_c, 0)
        tuned = rep.strip().splitlines()[-1]
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
             "keys_written": int(st.keys_written), "bands": int(st.bands),
             "forest_rounds": st.boruvka_rounds, "candidate_edges": st.candidate_edges,
             "forest_in": st.forest_in, "forest_kept": st.forest_kept, "merge_in": st.merge_in,
             "forest_edges": st.forest_edges, "largest_cluster": st.largest_cluster}
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
    phases = None
    if not args.no_roofline:
        # per-kernel times: the same K steps again with a HIP event pair
        # recorded on the context stream around every launch
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
        single = [(k, rep[k]) for k in SINGLE_KERNEL_SCOPES if k in rep]
        single.sort(key=lambda kv: -kv[1][1])
        if single:
            dom, (c, t, u) = single[0]
            avg_ms = t / c
            per_level = [algo_bytes(dom, L) for L in levels]
            roofline = {"bound": "hbm", "kernel": KERNEL_SYMBOL[dom], "scope": dom,
                        "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                        "traffic": None, "avg_launch_ms": round(avg_ms, 5),
                        "launches_per_step": c / args.steps}
            if all(x is not None for x in per_level):
                bytes_per_launch = sum(per_level) / (c / args.steps)
                achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
                roofline.update(achieved=round(achieved, 2), frac=round(achieved / HBM_PEAK_GBS, 4),
                                algo_bytes_per_launch=int(bytes_per_launch))
            tr = stored_traffic(dom, args.config)
            if tr is not None:
                roofline["traffic"] = int(tr)
        # per phase of the step: time (sum of its scopes) and the fraction of
        # peak its algorithmic bytes reach
        phases = {}
        for ph, scopes in PHASES.items():
            t_ph = sum(rep[k][1] for k in scopes if k in rep) / args.steps
            b = [algo_bytes("phase:contract", L) if ph == "contract" else
                 algo_bytes("score", L) if ph == "score" else algo_bytes("rowpass", L) for L in levels]
            phases[ph] = {"ms_per_step": round(t_ph, 4), "algo_bytes_per_step": int(sum(b)),
                          "frac_of_peak": (round(sum(b) / (t_ph * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
                                           if t_ph > 0 else None)}

    per_graph = None
    if batch and not args.no_per_graph:
        # the same graphs coarsened by one coarsen_to call each (inputs resident)
        G = len(g.meta["graphs"])
        print(f"[bench] per-graph calls ({G} graphs)", file=sys.stderr, flush=True)
        dgs = [spc.DeviceGraph.from_host(x, "cuda:0") for x in g.meta["graphs"]]
        for x, c in zip(dgs[:8], g.meta["n_c"][:8]):
            spc.coarsen_to(x, c, 0).free()
        torch.cuda.synchronize()
        t0.record()
        for x, c in zip(dgs, g.meta["n_c"]):
            spc.coarsen_to(x, c, 0).free()
        t1.record()
        torch.cuda.synchronize()
        ms_pg = t0.elapsed_time(t1)
        per_graph = {"graphs_per_s": G / (ms_pg * 1e-3), "ms_all_graphs": round(ms_pg, 3),
                     "batched_speedup": (G / (ms * 1e-3)) / (G / (ms_pg * 1e-3))}
        del dgs

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        if batch:
            cpu = cpu_baseline_batch(g.meta["graphs"], g.meta["n_c"])
        else:
            cpu = cpu_baseline(*cpu_sample(args.config, g, n_c))

    if batch:
        value = len(g.meta["graphs"]) / (ms * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "graphs/s" if batch else "fine edges/s",
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
                   "n_c": n_c if not batch else "n/10 per graph", "levels": len(levels),
                   "schedule": "halving"},
        "fine_edges_per_s": total_edges / (ms * 1e-3),
        "autotune": tuned,
        "per_graph": per_graph,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_floor_frac": (sum(method_floor_bytes(L) for L in levels) / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
                            if levels else None),
        "phases": phases,
        "levels": levels,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
