"""Refining a coarse graph's weights after coarsening.

The coarse graph keeps its structure; its undirected edge weights and
self-loop weights are refined so that the lift (Definition 2) better keeps
the input graph's leading spectrum: gradient steps (Adam) on the logarithms
of the weights (which keeps them positive) minimise
loss = sum_i (R_i - lambda_i)^2, R_i the lift's Rayleigh quotient at the
input's eigenvector u_i.  Loss and gradient run in the library's kernels
(spectral_error_graph / spectral_error_backward); torch only holds the
parameters and runs the optimiser.
"""
from __future__ import annotations

import torch

from . import spc


def edge_parameters(g: spc.DeviceGraph):
    """(upper entry positions, entry -> undirected edge index)."""
    n = g.n
    rows = torch.repeat_interleave(torch.arange(n, device=g.row_ptr.device),
                                   g.row_ptr[1:] - g.row_ptr[:-1])
    col = g.col.to(torch.int64)
    upper = torch.nonzero(col > rows).flatten()
    # undirected edge id of every entry: rank of (min, max) among upper entries
    lo = torch.minimum(rows, col)
    hi = torch.maximum(rows, col)
    key = lo * n + hi
    ukey = key[upper]
    edge_of = torch.searchsorted(ukey, key)
    return upper, edge_of


def reweight(g: spc.DeviceGraph, cmap: torch.Tensor, U: torch.Tensor, lam: torch.Tensor,
             steps: int = 200, lr: float = 1e-2):
    """Returns (refined graph, [loss before step 0, ..., loss after the last step])."""
    if g.w.dtype != torch.float64:
        raise ValueError("reweighting needs FP64 coarse weights")
    upper, edge_of = edge_parameters(g)
    theta = torch.log(g.w[upper]).clone().requires_grad_(True)
    self0 = g.self_w.to(torch.float64)
    has_self = self0 > 0
    phi = torch.log(torch.where(has_self, self0, torch.ones_like(self0))).clone().requires_grad_(True)
    opt = torch.optim.Adam([theta, phi], lr=lr)
    hist = []

    def weights():
        w = torch.exp(theta)[edge_of]
        s = torch.where(has_self, torch.exp(phi), torch.zeros_like(phi))
        return w, s

    for _ in range(steps):
        opt.zero_grad()
        w, s = weights()
        loss = spc.spectral_error_loss(w, s, g, cmap, U, lam)
        loss.backward()
        hist.append(float(loss.detach()))
        opt.step()
    with torch.no_grad():
        w, s = weights()
        out = spc.DeviceGraph(n=g.n, row_ptr=g.row_ptr, col=g.col, w=w.contiguous(),
                              self_w=s.contiguous(), size=g.size)
    hist.append(spc.spectral_error_graph(out, cmap, U, lam)[0])
    return out, hist


def _leading_eigenpairs(g, k):
    """k smallest nontrivial eigenpairs of the normalised Laplacian of a host
    graph (FP64 Lanczos on the host)."""
    import numpy as np
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    W = sp.csr_matrix((np.asarray(g.w, dtype=np.float64), (rows, g.col)), shape=(g.n, g.n))
    if g.self_w is not None:
        W = W + sp.diags(np.asarray(g.self_w, dtype=np.float64))
    d = np.asarray(W.sum(axis=1)).ravel()
    s = 1.0 / np.sqrt(d)
    L = (sp.identity(g.n) - sp.diags(s) @ W @ sp.diags(s)).tocsr()
    vals, vecs = sla.eigsh(L, k=k + 1, which="SA", tol=1e-10, ncv=max(4 * (k + 1), 60))
    order = np.argsort(vals)
    vals, vecs = vals[order], vecs[:, order]
    return vals[1:], vecs[:, 1:]


def _coarse_eigenvalues(g: spc.DeviceGraph, k):
    """The k smallest nontrivial eigenvalues of a coarse graph's normalised
    Laplacian (self-loops on the diagonal), FP64 Lanczos on the host."""
    return _leading_eigenpairs(g.to_host(), k)[0]


def main():
    """Coarsen the 64^3 lognormal-weighted mesh to 32,768 super-nodes, then
    refine the coarse weights against the 16 leading nontrivial eigenpairs
    with 200 Adam steps; prints one JSON line."""
    import argparse
    import json
    import time
    import numpy as np
    from meshgen import grid3d
    ap = argparse.ArgumentParser()
    ap.add_argument("--side", type=int, default=64)
    ap.add_argument("--n-c", type=int, default=32768)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--prec", choices=["f64", "f32"], default="f64",
                    help="precision of the spectral loss and gradient kernels")
    ap.add_argument("--hash-seed", type=int, default=None,
                    help="coarsen with the seeded-hash tie-break (the graph relabeled first)")
    a = ap.parse_args()
    g = grid3d(a.side, "lognormal", seed=5)
    t0 = time.perf_counter()
    lam, U = _leading_eigenpairs(g, a.k)
    t_eig = time.perf_counter() - t0
    dg = spc.DeviceGraph.from_host(g, "cuda:0")
    perm = None
    if a.hash_seed is not None:
        from meshgen import tie_permutation
        perm = torch.from_numpy(tie_permutation(g.n, a.hash_seed).astype(np.int64)).cuda()
        dg = spc.relabel(dg, perm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = spc.coarsen_to(dg, a.n_c, 0)
    torch.cuda.synchronize()
    t_coarsen = time.perf_counter() - t0
    L = h.num_levels
    _, gc, _ = h.level(L)
    cmap = spc.cluster_map(h, L)
    if perm is not None:
        cmap = cmap[perm].contiguous()   # input node u was node perm[u]
    Ut = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    if a.prec == "f32":
        Ut = Ut.float()
    lt = torch.from_numpy(lam).cuda()
    ev0 = _coarse_eigenvalues(gc, a.k)
    _, R0 = spc.spectral_error_graph(gc, cmap, Ut, lt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, hist = reweight(gc, cmap, Ut, lt, steps=a.steps, lr=a.lr)
    torch.cuda.synchronize()
    t_opt = time.perf_counter() - t0
    _, R1 = spc.spectral_error_graph(out, cmap, Ut, lt)
    err0 = float((R0.double() - lt).abs().max())
    err1 = float((R1.double() - lt).abs().max())
    ev1 = _coarse_eigenvalues(out, a.k)
    print(json.dumps({
        "workload": f"3D 7-point mesh {a.side}^3, FP32 lognormal(0,1) weights (seed 5), halving to {a.n_c}",
        "tie_break": "lowest id" if a.hash_seed is None else f"seeded hash (seed {a.hash_seed})",
        "spectral_precision": a.prec,
        "levels": L, "coarse_nodes": gc.n, "coarse_edges": gc.nnz // 2, "k": a.k,
        "coarsen_s": round(t_coarsen, 4), "eigensolve_host_s": round(t_eig, 2),
        "adam_steps": a.steps, "lr": a.lr, "ms_per_step": round(1e3 * t_opt / a.steps, 3),
        "loss_before": hist[0], "loss_after": hist[-1],
        "max_abs_R_minus_lambda_before": err0, "max_abs_R_minus_lambda_after": err1,
        # the coarse graph's own k smallest nontrivial eigenvalues against the input's
        "max_abs_eig_coarse_minus_input_before": float(np.max(np.abs(ev0 - lam))),
        "max_abs_eig_coarse_minus_input_after": float(np.max(np.abs(ev1 - lam)))}), flush=True)


if __name__ == "__main__":
    main()
