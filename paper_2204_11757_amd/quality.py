"""Spectral quality of a coarsening: the measures of the paper's
experiments (Section 4, Figure 2) and the bounds of Theorems 1 and 2.

For an input graph G with normalised Laplacian L (eigenvalues lambda_0 = 0
<= lambda_1 <= ..., eigenvectors U) and a coarsening G_c with super-node map
c and sizes s, the lift of Definition 2 has the normalised Laplacian

    L_hat = I - Q M Q^T,   Q = B S^-1/2,   M = D_c^-1/2 W_c D_c^-1/2,

(B the membership matrix, W_c with its self-loops on the diagonal), so its
spectrum is spec(L_c) together with n - n_c ones, and the lift of an
eigenvector z of L_c is Q z.  This gives the paper's two measures without
forming the n x n lift:

* the first k nontrivial eigenvalues of the lift against the input's
  (their largest and mean absolute difference, and over the whole
  spectrum ||Lambda - Lambda_hat||_inf);
* the alignment |<u_i, Q z_i>| of the i-th nontrivial eigenvectors (the
  diagonal of |U_k^T U_hat_k|), and the share of the input's k-dimensional
  eigenspace that the lifted one spans, ||U_k^T U_hat_k||_F^2 / k (robust
  to reordered close eigenvalues).

Theorem 2 bounds the change of a level of s merges whose scores are at most
epsilon by s (s + 1) / 2 epsilon (Theorem 1 is s = 1); over a hierarchy the
level bounds add up (both spectra gain the same ones at every level).

Everything here runs on the host in numpy FP64 (dense eigendecompositions,
for graphs of a few thousand nodes); the coarsening itself comes from the
GPU library (run with --help for the report this module writes).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _dense_w(n, row_ptr, col, w, self_w=None):
    W = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    W[rows, np.asarray(col, dtype=np.int64)] = np.asarray(w, dtype=np.float64)
    if self_w is not None:
        W[np.arange(n), np.arange(n)] += np.asarray(self_w, dtype=np.float64)
    return W


def _laplacian_eig(W):
    d = W.sum(axis=1)
    r = 1.0 / np.sqrt(d)
    L = np.eye(W.shape[0]) - (r[:, None] * W) * r[None, :]
    return np.linalg.eigh(L)


def input_spectrum(g):
    """(eigenvalues ascending, eigenvectors) of the input's normalised
    Laplacian (g: host graph with n, row_ptr, col, w, self_w)."""
    return _laplacian_eig(_dense_w(g.n, g.row_ptr, g.col, g.w, g.self_w))


def evaluate(lam, U, gc, cmap, k=50, level_bounds=None):
    """Quality of one coarsening: gc the coarse host graph (its size[] in
    input nodes), cmap the input node -> super-node map; (lam, U) from
    input_spectrum.  level_bounds: (merges, epsilon) of every level."""
    n, nc = U.shape[0], gc.n
    mu, Z = _laplacian_eig(_dense_w(nc, gc.row_ptr, gc.col, gc.w, gc.self_w))
    lam_hat = np.sort(np.concatenate([mu, np.ones(n - nc)]))
    kk = min(k, nc - 1, n - 1)
    size = np.asarray(gc.size, dtype=np.float64)
    c = np.asarray(cmap, dtype=np.int64)
    # Q^T u_i for the k nontrivial input eigenvectors, then <u_i, Q z_i>
    QtU = np.zeros((nc, kk))
    np.add.at(QtU, c, U[:, 1:kk + 1])
    QtU /= np.sqrt(size)[:, None]
    cross = QtU.T @ Z[:, 1:kk + 1]            # U_k^T U_hat_k
    align = np.abs(np.diag(cross))
    err = np.abs(lam[1:kk + 1] - lam_hat[1:kk + 1])
    out = {
        "n": int(n), "n_c": int(nc), "k": int(kk),
        "spectral_error_inf": float(np.max(np.abs(lam - lam_hat))),
        "eig_err_k_max": float(err.max()) if kk else 0.0,
        "eig_err_k_mean": float(err.mean()) if kk else 0.0,
        "align_k_mean": float(align.mean()) if kk else 1.0,
        "align_k_min": float(align.min()) if kk else 1.0,
        "align_k_above_0.9": int((align > 0.9).sum()),
        # share of the input's k-dimensional eigenspace the lifted one spans
        # (||U_k^T U_hat_k||_F^2 / k; 1 when the subspaces agree)
        "subspace_k": float((cross ** 2).sum() / kk) if kk else 1.0,
        "coarse_ones_in_k": int((mu[1:kk + 1] >= 1.0).sum()),
    }
    if level_bounds is not None:
        out["levels"] = len(level_bounds)
        out["thm2_bound"] = float(sum(s * (s + 1) / 2.0 * e for s, e in level_bounds))
        out["eps_max"] = float(max((e for _, e in level_bounds), default=0.0))
        out["bound_over_error"] = (out["thm2_bound"] / out["spectral_error_inf"]
                                   if out["spectral_error_inf"] > 0 else None)
    return out, lam_hat, align


def hierarchy_levels(h, n0):
    """Host copies of a GPU hierarchy: [(cluster_of, coarse graph, eps,
    merges)] per level."""
    out = []
    prev = n0
    for lvl in range(1, h.num_levels + 1):
        cl, gc, st = h.level(lvl)
        out.append((cl.cpu().numpy(), gc.to_host(), float(st.eps_max), int(prev - gc.n)))
        prev = gc.n
    return out


def compose_levels(levels, n0):
    c = np.arange(n0, dtype=np.int64)
    for cl, _, _, _ in levels:
        c = np.asarray(cl, dtype=np.int64)[c]
    return c


def evaluate_levels(lam, U, levels, n0, k=50, perm=None):
    """Quality of a hierarchy's last level.  perm: the relabeling the
    hierarchy was computed on (input node u was node perm[u]), if any."""
    gc = levels[-1][1]
    cmap = compose_levels(levels, n0)
    if perm is not None:
        cmap = cmap[np.asarray(perm, dtype=np.int64)]
    return evaluate(lam, U, gc, cmap, k, [(m, e) for _, _, e, m in levels])


SCHEDULES = [("halving", 0), ("single pass", 1), ("every merge (explicit greedy)", -1),
             ("every 16 merges", -16), ("every 256 merges", -256)]
# the seeded-hash tie-break (the graph relabeled by a seeded permutation)
HASHED = [("halving, hash tie-break", 0), ("single pass, hash tie-break", 1)]


def main(argv=None):
    ap = argparse.ArgumentParser(description="spectral quality of the GPU coarsening on 64x64 meshes "
                                             "(the measures of the paper's Figure 2)")
    ap.add_argument("--out", default=None, help="write the report as JSON here")
    ap.add_argument("--k", type=int, default=50)
    ap.add_argument("--side", type=int, default=64)
    args = ap.parse_args(argv)
    import torch
    from meshgen import grid2d, tie_permutation, trimesh
    from paper_2204_11757_amd import spc

    s = args.side
    meshes = [
        (f"triangle mesh {s}x{s}, weights U{{1..8}} (seed 3)", trimesh(s, ("uniform", 1, 8), seed=3)),
        (f"5-point grid {s}x{s}, unit weights", grid2d(s)),
    ]
    report = {"k": args.k, "meshes": []}
    for name, g in meshes:
        t0 = time.time()
        lam, U = input_spectrum(g)
        dg = spc.DeviceGraph.from_host(g, "cuda:0")
        perm = tie_permutation(g.n, 1)
        dr = spc.relabel(dg, perm)
        entry = {"mesh": name, "n": g.n, "m": g.m, "runs": []}
        for ratio in (2, 4, 8):
            n_c = g.n // ratio
            for sname, sched in SCHEDULES + HASHED:
                hashed = (sname, sched) in HASHED
                h = spc.coarsen_to(dr if hashed else dg, n_c, sched)
                levels = hierarchy_levels(h, g.n)
                h.free()
                q, _, _ = evaluate_levels(lam, U, levels, g.n, args.k, perm if hashed else None)
                q.update({"ratio": f"1/{ratio}", "schedule": sname})
                entry["runs"].append(q)
                print(f"[quality] {name} 1/{ratio} {sname}: eig err k max {q['eig_err_k_max']:.4f} "
                      f"mean {q['eig_err_k_mean']:.4f}, ||dLambda||inf {q['spectral_error_inf']:.4f}, "
                      f"align mean {q['align_k_mean']:.3f} subspace {q['subspace_k']:.3f}, Thm 2 bound {q['thm2_bound']:.3g}", flush=True)
        entry["seconds"] = round(time.time() - t0, 1)
        report["meshes"].append(entry)
        torch.cuda.synchronize()
    if args.out:
        with open(args.out, "w") as f:
            json.dump(report, f, indent=1)
            f.write("\n")
    return report


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
