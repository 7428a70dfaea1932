"""Pins for the FP64 diffusion oracle (Eq. 8) and the kNN-graph input builder."""
import numpy as np
import scipy.sparse as sp

from oracle import diffuse as od
from synth import graph


def random_graph(n, k, seed, feats_dim=4):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (n, 3))
    f = rng.normal(size=(n, feats_dim))
    rp, c, v = graph.knn_graph(x, f, k)
    return x, f, od.csr_matrix(n, rp, c, v)


def test_constant_signal_is_preserved():
    """Row-stochastic A fixes the constant vector: g_T = 1/sqrt(n) for T >= 1."""
    n = 300
    _, _, A = random_graph(n, 8, 1)
    g = od.diffuse(A, np.full(n, 3.0), 7)
    assert np.allclose(g, 1.0 / np.sqrt(n), rtol=1e-12)


def test_scale_invariance_and_channel_independence():
    n = 200
    _, _, A = random_graph(n, 8, 2)
    rng = np.random.default_rng(3)
    g0 = rng.uniform(0, 1, (n, 3))
    g = od.diffuse(A, g0, 5)
    assert np.allclose(od.diffuse(A, 4.5 * g0, 5), g, rtol=1e-12)
    for c in range(3):
        assert np.allclose(od.diffuse(A, g0[:, c], 5), g[:, c], rtol=1e-12)


def test_steps_zero_and_zero_channel():
    n = 50
    _, _, A = random_graph(n, 4, 4)
    g0 = np.zeros((n, 2))
    g0[:, 1] = np.arange(n)
    assert np.array_equal(od.diffuse(A, g0, 0), g0)
    g = od.diffuse(A, g0, 3)
    assert np.all(g[:, 0] == 0) and np.all(np.isfinite(g))


def test_power_method_reaches_dominant_eigenvector():
    """Eq. (8) is the power method: on a symmetric matrix with a spectral gap the
    normalised iterate converges to numpy.linalg.eigh's dominant eigenvector."""
    rng = np.random.default_rng(5)
    n = 40
    B = rng.uniform(0, 1, (n, n))
    M = (B + B.T) / 2 + np.diag(np.linspace(0, 2, n))
    w, V = np.linalg.eigh(M)
    v = V[:, -1] * np.sign(V[:, -1].sum())
    g = od.diffuse(sp.csr_matrix(M), rng.uniform(0.5, 1, n), 200)
    g = g / np.linalg.norm(g)
    assert np.allclose(g, v, atol=1e-10)
    # one more step multiplies the unit iterate by the top eigenvalue
    g1 = od.diffuse(sp.csr_matrix(M), g, 1)
    assert np.linalg.norm(g1) == np.float64(np.linalg.norm(g1))
    assert abs(np.linalg.norm(g1) - w[-1]) < 1e-9 * w[-1]


def test_knn_matches_brute_force():
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, (700, 3))
    idx, dist = graph.knn(x, 10)
    D = np.linalg.norm(x[:, None] - x[None], axis=-1)
    np.fill_diagonal(D, np.inf)
    ref = np.argsort(D, axis=1, kind="stable")[:, :10]
    assert np.array_equal(np.sort(idx, 1), np.sort(ref, 1))
    assert np.allclose(np.sort(dist, 1), np.sort(np.take_along_axis(D, ref, 1), 1))


def test_graph_is_union_symmetric_and_row_stochastic():
    n, k = 400, 6
    x, f, A = random_graph(n, k, 7)
    pat = (A != 0).astype(np.int8)
    idx, dist = graph.knn(x, k)
    # every kNN edge with positive cosine is present in both directions
    fn = f / np.linalg.norm(f, axis=1, keepdims=True)
    for i in range(0, n, 37):
        for j in idx[i]:
            if fn[i] @ fn[j] > 1e-9:
                assert pat[i, j] and pat[j, i]
    assert np.allclose(np.asarray(A.sum(axis=1)).ravel(), 1.0, atol=1e-6)
    sigma = np.median(dist)
    i = 0
    j = [c for c in idx[0] if fn[0] @ fn[c] > 0][0]
    d = np.linalg.norm(x[0] - x[j])
    w = np.exp(-d * d / sigma ** 2) * (fn[0] @ fn[j])
    row = A.getrow(0).toarray().ravel()
    assert abs(row[j] / row.sum() - w / sum(
        np.exp(-np.linalg.norm(x[0] - x[c]) ** 2 / sigma ** 2) * max(0.0, fn[0] @ fn[c])
        for c in np.nonzero(row)[0])) < 1e-6
