"""Spectral side of the oracle, in numpy FP64 (dense for tiny graphs, sparse
matrix-vector products for large ones).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
benchmark's CPU baseline, never by the product path.

Definitions followed:
  * normalised Laplacian L = I - D^{-1/2} W D^{-1/2}, with W the weighted
    adjacency including the diagonal (self-loops) and D its row sums
    (the notation after Theorem 1);
  * the lift of a coarsened graph (Definition 2): an n-node graph with
    w_hat(u, v) = W_c(c(u), c(v)) / (|c(u)| |c(v)|), the pair u = v
    included, where W_c(a, a) is super-node a's self-loop weight;
  * the spectral error compares the original graph's eigenpairs with the
    lift.  R_i = u_i^T L_hat u_i is the lift's Rayleigh quotient at the
    original eigenvector u_i, and loss = sum_i (R_i - lambda_i)^2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from meshgen import Graph


def dense_w(g: Graph) -> np.ndarray:
    """Dense weighted adjacency with the self-loop weights on the diagonal."""
    W = np.zeros((g.n, g.n), dtype=np.float64)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    W[rows, g.col.astype(np.int64)] = g.w.astype(np.float64)
    if g.self_w is not None:
        W[np.arange(g.n), np.arange(g.n)] += np.asarray(g.self_w, dtype=np.float64)
    return W


def sparse_w(g: Graph) -> sp.csr_matrix:
    W = sp.csr_matrix((g.w.astype(np.float64), g.col.astype(np.int64), g.row_ptr),
                      shape=(g.n, g.n))
    if g.self_w is not None:
        W = W + sp.diags(np.asarray(g.self_w, dtype=np.float64))
    return W.tocsr()


def normalized_laplacian_dense(W: np.ndarray) -> np.ndarray:
    d = W.sum(axis=1)
    s = 1.0 / np.sqrt(d)
    return np.eye(W.shape[0]) - (s[:, None] * W) * s[None, :]


def spectrum(W: np.ndarray) -> np.ndarray:
    """Ascending eigenvalues of the normalised Laplacian of a dense W."""
    return np.linalg.eigvalsh(normalized_laplacian_dense(W))


def eigenpairs(W: np.ndarray):
    return np.linalg.eigh(normalized_laplacian_dense(W))


def lift_dense(Wc: np.ndarray, cluster_of: np.ndarray, size_c: np.ndarray) -> np.ndarray:
    """Definition 2 on dense matrices: W_hat[u, v] = Wc[a, b] / (|a| |b|)."""
    c = np.asarray(cluster_of, dtype=np.int64)
    s = np.asarray(size_c, dtype=np.float64)
    return Wc[np.ix_(c, c)] / (s[c][:, None] * s[c][None, :])


def lift_vectors(x_c: np.ndarray, cluster_of: np.ndarray, size_c: np.ndarray,
                 mode: int = 0) -> np.ndarray:
    """Lift coarse vectors (n_c x k) to the fine nodes.
    mode 0: piecewise constant, x_f[u] = x_c[c(u)];
    mode 1: orthonormal, x_f[u] = x_c[c(u)] / sqrt(|c(u)|)."""
    c = np.asarray(cluster_of, dtype=np.int64)
    x = np.asarray(x_c, dtype=np.float64)
    out = x[c]
    if mode == 1:
        sc = np.sqrt(np.asarray(size_c, dtype=np.float64))[c]
        out = out / (sc[:, None] if out.ndim == 2 else sc)
    return out


def lift_between(maps, sizes, from_lvl: int, to_lvl: int, x_c: np.ndarray, mode: int = 0) -> np.ndarray:
    """Lift coarse vectors from level to_lvl to level from_lvl <= to_lvl of a
    hierarchy (Definition 2 applied between levels).

    maps[l] is the cluster map from level l to level l + 1 (level 0 is the
    input); sizes[l] the node sizes of level l (input nodes per node; level
    0 all ones).  c(u) composes the maps from from_lvl to to_lvl.
    mode 0: x_f[u] = x_c[c(u)];
    mode 1: x_f[u] = x_c[c(u)] / sqrt(s(c(u)) / s(u)), the coordinates of the
    orthonormal lift B S^-1/2 in level from_lvl's orthonormal basis."""
    n_from = np.asarray(sizes[from_lvl]).shape[0]
    c = np.arange(n_from, dtype=np.int64)
    for lvl in range(from_lvl, to_lvl):
        c = np.asarray(maps[lvl], dtype=np.int64)[c]
    x = np.asarray(x_c, dtype=np.float64)
    out = x[c]
    if mode == 1:
        ratio = np.asarray(sizes[to_lvl], dtype=np.float64)[c] / np.asarray(sizes[from_lvl], dtype=np.float64)
        s = np.sqrt(ratio)
        out = out / (s[:, None] if out.ndim == 2 else s)
    return out


def restrict(U: np.ndarray, cluster_of: np.ndarray, size_c: np.ndarray) -> np.ndarray:
    """Transpose of the orthonormal lift: y[a] = sum_{x in a} U[x] / sqrt(|a|)."""
    c = np.asarray(cluster_of, dtype=np.int64)
    U = np.asarray(U, dtype=np.float64)
    k = U.shape[1] if U.ndim == 2 else 1
    U2 = U.reshape(U.shape[0], k)
    n_c = np.asarray(size_c).shape[0]
    y = np.zeros((n_c, k))
    np.add.at(y, c, U2)
    y /= np.sqrt(np.asarray(size_c, dtype=np.float64))[:, None]
    return y if U.ndim == 2 else y[:, 0]


def spectral_error(gc: Graph, cluster_of: np.ndarray, U: np.ndarray, lam: np.ndarray):
    """loss = sum_i (R_i - lambda_i)^2 with R_i = 1 - t_i^T W_c t_i,
    t_i = D_c^{-1/2} Q^T u_i (Q the orthonormal lift).  Returns (loss, R)."""
    Wc = sparse_w(gc)
    dc = np.asarray(Wc.sum(axis=1)).ravel()
    y = restrict(U, cluster_of, gc.size_or_one())
    t = y / np.sqrt(dc)[:, None]
    z = Wc @ t
    R = 1.0 - np.einsum("ik,ik->k", t, z)
    lam = np.asarray(lam, dtype=np.float64)
    loss = float(np.sum((R - lam) ** 2))
    return loss, R


def spectral_error_dense(gc: Graph, cluster_of: np.ndarray, U: np.ndarray, lam: np.ndarray):
    """The same quantity evaluated literally: build the lift of Definition 2
    densely and take Rayleigh quotients of its normalised Laplacian."""
    Wh = lift_dense(dense_w(gc), cluster_of, gc.size_or_one())
    Lh = normalized_laplacian_dense(Wh)
    U = np.asarray(U, dtype=np.float64)
    R = np.einsum("ik,ij,jk->k", U, Lh, U)
    return float(np.sum((R - lam) ** 2)), R


def spectral_error_grad(gc: Graph, cluster_of: np.ndarray, U: np.ndarray, lam: np.ndarray):
    """Gradient of the loss with respect to the coarse weights.

    Each undirected coarse edge {a, b} is one parameter w_ab stored in both
    mirror CSR entries; the returned per-entry value is d loss / d w_ab (the
    same number in both mirrors).  The self-loop parameter is self_w[a].
    With f_i = t^T W t, z = W t and d_a the coarse degree:
      d f / d w_ab    = 2 t_a t_b - t_a z_a / d_a - t_b z_b / d_b
      d f / d self_a  = t_a^2 - t_a z_a / d_a
    and d loss / d f_i = -2 (R_i - lambda_i)."""
    Wc = sparse_w(gc)
    dc = np.asarray(Wc.sum(axis=1)).ravel()
    y = restrict(U, cluster_of, gc.size_or_one())
    t = y / np.sqrt(dc)[:, None]
    z = Wc @ t
    R = 1.0 - np.einsum("ik,ik->k", t, z)
    coef = -2.0 * (R - np.asarray(lam, dtype=np.float64))      # d loss / d f_i
    h = t * z / dc[:, None]                                     # t_a z_a / d_a
    rows = np.repeat(np.arange(gc.n), np.diff(gc.row_ptr))
    cols = gc.col.astype(np.int64)
    g_w = (2.0 * t[rows] * t[cols] - h[rows] - h[cols]) @ coef
    g_self = (t * t - h) @ coef
    return g_w, g_self
