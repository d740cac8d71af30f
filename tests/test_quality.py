"""The spectral-quality measures (paper Section 4, Figure 2) checked on the
CPU against a brute force: the n x n lift of Definition 2 formed densely and
diagonalised.  The coarsenings come from the oracle."""
import numpy as np
import pytest

import oracle
from oracle import spectral as S
from meshgen import random_graph, trimesh
from paper_2204_11757_amd import quality as Qm


@pytest.mark.parametrize("sched", [0, 1, -1, -7])
def test_lift_spectrum_and_alignment_match_dense_lift(sched):
    g = trimesh(9, ("uniform", 1, 8), seed=11)          # random weights: simple spectra
    lam, U = Qm.input_spectrum(g)
    n_c = g.n // 3
    lv = oracle.coarsen_to(g, n_c, sched)
    levels = []
    prev = g.n
    for c, gc, eps in lv:
        levels.append((c, gc, eps, prev - gc.n))
        prev = gc.n
    q, lam_hat, align = Qm.evaluate_levels(lam, U, levels, g.n, k=12)
    # brute force: the lift formed densely
    cmap = oracle.compose(lv)
    gc = lv[-1][1]
    Wh = S.lift_dense(S.dense_w(gc), cmap, gc.size_or_one())
    mu_h, V = S.eigenpairs(Wh)
    np.testing.assert_allclose(lam_hat, mu_h, atol=1e-11)
    assert q["spectral_error_inf"] == pytest.approx(np.max(np.abs(lam - mu_h)), abs=1e-11)
    # eigenvectors of simple eigenvalues: the lift's own vectors
    k = q["k"]
    gaps = np.minimum(np.diff(mu_h)[1:k + 1], np.diff(mu_h)[:k])
    for i in range(1, k + 1):
        if gaps[i - 1] > 1e-6 and mu_h[i] < 1 - 1e-6:
            assert align[i - 1] == pytest.approx(abs(U[:, i] @ V[:, i]), abs=1e-8)
    # the subspace share from the dense lift's eigenvectors of the k
    # smallest nontrivial eigenvalues (when they are the coarse graph's)
    if q["coarse_ones_in_k"] == 0 and mu_h[k] < 1 - 1e-6 and mu_h[k + 1] - mu_h[k] > 1e-6:
        M = U[:, 1:k + 1].T @ V[:, 1:k + 1]
        assert q["subspace_k"] == pytest.approx((M ** 2).sum() / k, abs=1e-9)
    # Theorem 2 per level, added up over the levels, bounds the change
    assert q["spectral_error_inf"] <= q["thm2_bound"] + 1e-12


def test_identity_coarsening_is_exact():
    g = random_graph(12, p=0.4, seed=5, wmax=3)
    lam, U = Qm.input_spectrum(g)
    ident = np.arange(g.n)
    gid = oracle.contract(g, ident, g.n)
    q, lam_hat, align = Qm.evaluate(lam, U, gid, ident, k=6, level_bounds=[])
    assert q["spectral_error_inf"] < 1e-12 and q["eig_err_k_max"] < 1e-12
    np.testing.assert_allclose(align, 1.0, atol=1e-9)
