"""The kNN diffusion graph built on the device (Sec. 3.3) against the FP64
oracle graph: structure (row pointers, columns) bit-exact, values within FP32
rounding of the FP64 weights; then diffusion on it against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2410_14462_amd as lv
from oracle import diffuse as od
from synth import philox, scenes
from synth.scenes import Scene

pytestmark = pytest.mark.gpu


def scene_at(means):
    n = means.shape[0]
    return Scene(np.ascontiguousarray(means, np.float32), np.full((n, 3), 0.01, np.float32),
                 np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)), np.full(n, 0.5, np.float32))


def uniform_points(n, seed):
    return (2.0 * philox.uniform(seed, 0, 3 * n).astype(np.float64) - 1.0).astype(np.float32).reshape(n, 3)


def clustered_points(n, seed):
    """Gaussian blobs of very different widths, plus exact duplicates."""
    z = philox.normal64(seed, 1, 3 * n).reshape(n, 3)
    c = (2.0 * philox.uniform(seed, 2, 3 * 12).astype(np.float64) - 1.0).reshape(12, 3)
    which = (philox.uniform(seed, 3, n).astype(np.float64) * 12).astype(np.int64)
    width = np.array([0.3, 0.01, 0.05, 0.002] * 3)[which][:, None]
    x = (c[which] + width * z).astype(np.float32)
    x[n // 2:n // 2 + 20] = x[:20]  # duplicated centres (distance 0)
    return x


def features(n, D, seed):
    return philox.normal(seed, 0, n * D).reshape(n, D).astype(np.float32)


def compare(x, f, k):
    gs = lv.Scene.from_arrays(scene_at(x))
    G = lv.Graph.knn(gs, torch.as_tensor(f, device="cuda"), k)
    rp, col, val = (t.cpu().numpy() for t in G.csr())
    rrp, rcol, rval = oracle.graph.knn_graph(x, f, k)
    assert np.array_equal(rp, rrp)
    assert np.array_equal(col, rcol)
    err = np.abs(val.astype(np.float64) - rval) - 2e-7 * np.abs(rval)
    assert err.max() <= 1e-9, float(err.max())
    return G, gs, (rp, col, val)


@pytest.mark.parametrize("n,k,D", [(17, 16, 3), (500, 16, 5), (3000, 1, 1), (3000, 32, 8),
                                   (20000, 16, 64), (20001, 7, 2)])
def test_knn_graph_uniform(n, k, D):
    compare(uniform_points(n, n), features(n, D, n + 1), k)


def test_knn_graph_clustered_with_duplicates():
    compare(clustered_points(30000, 4), features(30000, 4, 5), 16)


def test_knn_graph_zero_rows_and_zero_features():
    n = 400
    x = uniform_points(n, 9)
    f = np.ones((n, 3), np.float32)
    f[11] = -1.0          # every weight of row 11 is 0: self-loop
    f[12] = 0.0           # zero feature: cosine 0
    G, gs, (rp, col, val) = compare(x, f, 8)
    cs = col[rp[11]:rp[12]]
    assert 11 in cs and val[rp[11]:rp[12]][list(cs).index(11)] == 1.0


def test_knn_graph_bad_arguments():
    gs = lv.Scene.from_arrays(scene_at(uniform_points(10, 1)))
    f = torch.ones((10, 2), device="cuda")
    for k in (0, 33, 10):
        with pytest.raises(lv.LvError):
            lv.Graph.knn(gs, f, k)


def test_diffusion_on_device_graph():
    n, k = 20000, 16
    x = uniform_points(n, 21)
    f = features(n, 4, 22)
    G, gs, (rp, col, val) = compare(x, f, k)
    g0 = scenes.halfspace_indicator(23, x)
    out = G.diffuse(torch.as_tensor(g0, device="cuda"), 20, scene=gs).cpu().numpy().astype(np.float64)
    rrp, rcol, rval = oracle.graph.knn_graph(x, f, k)
    ref = od.diffuse(od.csr_matrix(n, rrp, rcol, rval), g0, 20)
    err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    print(f"diffusion on the device graph: err {err:.3e}")
    assert err < 1e-5


# ------------------------------------------- the paper's Eq. 7 / Eq. 9 graph
def compare_rbf(x, f, k, b, unary=None, binarize=0.0):
    gs = lv.Scene.from_arrays(scene_at(x))
    P = None if unary is None else torch.as_tensor(unary, device="cuda")
    G = lv.Graph.knn(gs, torch.as_tensor(f, device="cuda"), k, kind="feature_rbf", bandwidth=b, unary=P,
                     binarize=binarize)
    rp, col, val = (t.cpu().numpy() for t in G.csr())
    rrp, rcol, rval = oracle.graph.feature_rbf_graph(x, f, k, b, unary=unary, binarize=binarize)
    assert np.array_equal(rp, rrp)
    assert np.array_equal(col, rcol)
    err = np.abs(val.astype(np.float64) - rval) - 2e-7 * np.abs(rval)
    assert err.max(initial=0.0) <= 1e-9
    return G, gs, (rp, col, val)


@pytest.mark.parametrize("n,k,D,b,with_unary", [(300, 8, 4, 1.0, False), (5000, 16, 32, 0.3, True),
                                                 (20000, 16, 64, 2.0, True)])
def test_feature_rbf_graph(n, k, D, b, with_unary):
    x = uniform_points(n, 70 + n)
    f = features(n, D, 71 + n)
    p = philox.uniform(72, n, n).astype(np.float32) if with_unary else None
    compare_rbf(x, f, k, b, p)


def test_feature_rbf_graph_binarised_and_reachability():
    """The segmentation diffusion of the appendix on synthetic inputs: anchors
    from a mask (the largest 10 % of its positive values), the binarised
    Eq. 7 graph with a unary term, T steps, h = P on the reached nodes.  The
    reached set is a graph property (A >= 0, g0 >= 0), so h is compared
    exactly."""
    n, k, T = 20000, 16, 4
    x = uniform_points(n, 81)
    f = features(n, 16, 82)
    p = philox.uniform(83, 0, n).astype(np.float32)
    G, gs, (rp, col, val) = compare_rbf(x, f, k, 0.5, p, binarize=1e-5)
    assert np.all(val == 1.0)
    # a mask that is positive only in a slab of the scene
    mask = np.where(x[:, 0] > 0.8, philox.uniform(84, 0, n) + 0.1, -1.0).astype(np.float32)
    g0 = lv.anchor_init(torch.as_tensor(mask, device="cuda"), 0.1)
    ref_g0 = oracle.prune.anchor_init(mask, 0.1)
    assert np.array_equal(g0.cpu().numpy(), ref_g0)
    gT = G.diffuse(g0, T)
    h = lv.reach_unary(gT, torch.as_tensor(p, device="cuda")).cpu().numpy()
    ref_gT = od.diffuse(od.csr_matrix(n, rp, col, val), ref_g0.astype(np.float64), T)
    ref_h = oracle.prune.reach_unary(ref_gT, p)
    reached = int(np.count_nonzero(ref_h))
    print(f"reached {reached} of {n} nodes from {np.count_nonzero(ref_g0)} anchors in {T} steps")
    assert 0 < reached < n
    assert np.array_equal(h, ref_h)


@pytest.mark.parametrize("n", [0, 1, 9, 4097, 300001])
def test_anchor_init_matches_oracle(n):
    g = (philox.normal(90, n % 7, max(n, 1))[:n]).astype(np.float32)
    if n > 8:
        g[:4] = 0.0
        g[4:8] = g[8]  # ties
    for frac in (0.1, 0.5, 1.0):
        got = lv.anchor_init(torch.as_tensor(g, device="cuda"), frac).cpu().numpy()
        assert np.array_equal(got, oracle.prune.anchor_init(g, frac)), (n, frac)


def test_graph_opts_bad_arguments():
    gs = lv.Scene.from_arrays(scene_at(uniform_points(50, 1)))
    f = torch.ones((50, 2), device="cuda")
    with pytest.raises(lv.LvError):
        lv.Graph.knn(gs, f, 4, kind="feature_rbf", bandwidth=0.0)
    with pytest.raises(lv.LvError):
        lv.anchor_init(torch.ones(5, device="cuda"), 0.0)
