"""Pins of the FP64 CPU reference of the learned-preconditioner network.

The reference's gradients (autograd) are checked against central finite differences of its
own loss in exact FP64 mode, and its neighbour lists against an independent brute-force
ranking; its curvature feature against the sphere's 2/R.
"""
import numpy as np
import pytest

from oracle import nn_ref


def _shell(n, R=3.0, seed=0):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = R + rng.uniform(-0.3, 0.3, size=n)
    x = u * R
    phi = r - R
    return np.column_stack([x, u, phi, np.ones(n)])


def test_knn_matches_bruteforce_ranking():
    nodes = _shell(300, seed=1)
    nbr = nn_ref.knn(nodes[:, :3])
    for i in (0, 17, 123, 299):
        d = np.linalg.norm(nodes[:, :3] - nodes[i, :3], axis=1)
        ranked = sorted(range(len(d)), key=lambda j: (d[j], j))[:16]
        assert set(ranked) == set(nbr[i])
        assert nbr[i][0] == i


def test_curvature_feature_on_sphere():
    R = 3.0
    rng = np.random.default_rng(2)
    u = rng.normal(size=(4000, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    nodes = np.column_stack([u * R, u, np.zeros(4000), np.ones(4000)])
    nbr = nn_ref.knn(nodes[:, :3])
    eps = 0.5
    f = nn_ref.features(nodes, nbr, eps)
    assert np.median(f[:, 4]) == pytest.approx(2.0 / R * eps, rel=0.02)


def test_reference_gradients_match_finite_differences():
    nodes = _shell(60, seed=3)
    nbr = nn_ref.knn(nodes[:, :3])
    eps = 0.5
    feat = nn_ref.features(nodes, nbr, eps).astype(np.float32)
    rng = np.random.default_rng(4)
    npar = sum(K * C + C for K, C in nn_ref.layer_shapes())
    params = rng.normal(size=npar) * 0.05
    n = len(nodes)
    v = rng.normal(size=2 * n)
    u = rng.normal(size=2 * n)
    lam = (40.5, 0.50625)
    L, g = nn_ref.loss_and_grads(nodes, nbr, feat, v, u, params, lam, eps, rounding=False)
    idx = rng.choice(npar, 12, replace=False)
    h = 1e-6
    for k in idx:
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        Lp, _ = nn_ref.loss_and_grads(nodes, nbr, feat, v, u, pp, lam, eps, rounding=False)
        Lm, _ = nn_ref.loss_and_grads(nodes, nbr, feat, v, u, pm, lam, eps, rounding=False)
        fd = (Lp - Lm) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_zero_network_is_the_diagonal_solve():
    nodes = _shell(50, seed=5)
    nbr = nn_ref.knn(nodes[:, :3])
    feat = nn_ref.features(nodes, nbr, 0.5).astype(np.float32)
    npar = sum(K * C + C for K, C in nn_ref.layer_shapes())
    v = np.random.default_rng(6).normal(size=100)
    p = nn_ref.apply(nodes, nbr, feat, v, np.zeros(npar), (40.5, 0.50625), 0.5)
    np.testing.assert_allclose(p, np.concatenate([v[:50] / 40.5, v[50:] / 0.50625]), rtol=1e-15)
