"""Pins for the FP64 diffusion oracle (Eq. 8)."""
import numpy as np
import scipy.sparse as sp

from oracle import diffuse as od
from oracle import graph


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


def test_bf16_rounding_matches_library_conversion():
    """On FP32 inputs (where no double rounding can occur) the BF16 rounding
    of the storage option equals torch's float32 -> bfloat16 conversion
    (round to nearest, ties to even), ties and subnormals included."""
    import torch
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(size=20000), rng.normal(size=2000) * 1e-38,
                        rng.uniform(-1, 1, 2000) * 1e30]).astype(np.float32)
    bits = x.view(np.uint32)
    ties = ((bits & ~np.uint32(0xFFFF)) | np.uint32(0x8000)).view(np.float32)  # exact halfway cases
    x = np.concatenate([x, ties, np.float32([0.0, -0.0, 1.0, 2.0 ** -133, 3 * 2.0 ** -134])])
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy().astype(np.float64)
    assert np.array_equal(od.round_bf16(x.astype(np.float64)), ref)


def test_bf16_storage_diffusion_stays_on_the_bf16_grid():
    n = 200
    _, _, A = random_graph(n, 8, 6)
    g0 = np.random.default_rng(7).uniform(0, 1, (n, 2))
    g = od.diffuse(A, od.round_bf16(g0), 3, store="bf16")
    assert np.array_equal(g, od.round_bf16(g))
    ref = od.diffuse(A, od.round_bf16(g0), 3)
    # each step: one relative rounding of at most 2^-9, averaged by a
    # row-stochastic A
    assert np.max(np.abs(g - ref) / np.max(np.abs(ref), axis=0)) <= 3 * 2.0 ** -9
