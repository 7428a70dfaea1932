"""Pins for the FP64 kNN diffusion graph (Sec. 3.3): neighbours against
brute force and a k-d tree, ties by index, the union structure, the weight
formula recomputed independently, row sums and the zero-row self-loop."""
import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist

from oracle import graph

F32 = np.float32


def rand_points(n, seed):
    return np.random.default_rng(seed).uniform(-1, 1, (n, 3)).astype(F32)


@pytest.mark.parametrize("n,k", [(40, 16), (700, 10), (1500, 16)])
def test_knn_matches_brute_force(n, k):
    x = rand_points(n, n)
    idx, d2 = graph.knn(x, k)
    D = cdist(x.astype(np.float64), x.astype(np.float64))
    np.fill_diagonal(D, np.inf)
    ref = np.argsort(D, axis=1, kind="stable")[:, :k]
    assert np.array_equal(idx, ref)
    assert np.allclose(np.sqrt(d2), np.take_along_axis(D, ref, 1), rtol=1e-14, atol=0)


def test_knn_matches_kdtree_at_size():
    x = rand_points(50000, 3)
    idx, d2 = graph.knn(x, 16)
    dist, cand = cKDTree(x.astype(np.float64)).query(x.astype(np.float64), k=17)
    assert np.array_equal(np.sort(idx, 1), np.sort(cand[:, 1:], 1))
    assert abs(graph.median_distance(d2) - np.median(dist[:, 1:])) <= 1e-15


def test_knn_ties_by_index_and_duplicates():
    # points on an integer lattice: many exactly equal distances
    g = np.stack(np.meshgrid(np.arange(4), np.arange(4), np.arange(3), indexing="ij"), -1).reshape(-1, 3)
    x = np.concatenate([g, g[:2]]).astype(F32)  # two duplicated points
    n, k = x.shape[0], 8
    idx, d2 = graph.knn(x, k)
    for r in range(n):
        cands = sorted(((float(np.sum((x[r].astype(np.float64) - x[j]) ** 2)), j)
                        for j in range(n) if j != r))
        assert list(idx[r]) == [j for _, j in cands[:k]], r
    assert d2[n - 2, 0] == 0.0 and idx[n - 2, 0] == 0  # the duplicate of point 0


def test_graph_structure_and_weights():
    n, k = 600, 8
    x = rand_points(n, 11)
    f = np.random.default_rng(12).normal(size=(n, 5)).astype(F32)
    rp, col, val = graph.knn_graph(x, f, k)
    idx, d2 = graph.knn(x, k)
    pairs = {(i, int(j)) for i in range(n) for j in idx[i]}
    union = pairs | {(j, i) for i, j in pairs}
    got = {(i, int(c)) for i in range(n) for c in col[rp[i]:rp[i + 1]]}
    selfs = {(i, i) for i in range(n) if (i, i) in got}
    assert got - selfs <= union and (got - selfs) == {(i, j) for i, j in got - selfs if (j, i) in got}
    assert all(rp[i + 1] - rp[i] == 1 for i, _ in selfs)
    assert all(np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0) for i in range(n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.allclose(np.bincount(rows, weights=val.astype(np.float64), minlength=n), 1.0, atol=1e-6)
    # weights recomputed from their definition, independently of the builder
    sigma = np.median(cdist(x.astype(np.float64), x.astype(np.float64))[np.arange(n)[:, None], idx])
    fn = f.astype(np.float64) / np.linalg.norm(f.astype(np.float64), axis=1, keepdims=True)

    def w(i, j):
        dd = np.linalg.norm(x[i].astype(np.float64) - x[j])
        return np.exp(-dd * dd / sigma ** 2) * max(0.0, float(fn[i] @ fn[j]))
    for i in range(0, n, 29):
        if (i, i) in selfs:
            continue
        cand = sorted(j for a, j in union if a == i)
        raw = np.array([max(w(i, j) if (i, j) in pairs else 0.0, w(j, i) if (j, i) in pairs else 0.0)
                        for j in cand])
        keep = raw > 0
        assert list(col[rp[i]:rp[i + 1]]) == [j for j, k in zip(cand, keep) if k]
        assert np.allclose(val[rp[i]:rp[i + 1]], raw[keep] / raw.sum(), rtol=1e-5, atol=1e-7)


def test_zero_row_gets_self_loop():
    n, k = 60, 4
    x = rand_points(n, 5)
    f = np.ones((n, 2), F32)
    f[7] = -1.0  # opposite to everyone: all of row 7's weights are 0
    rp, col, val = graph.knn_graph(x, f, k)
    cs, vs = col[rp[7]:rp[8]], val[rp[7]:rp[8]]
    assert list(cs) == [7] and vs[0] == 1.0
    assert np.all(val > 0)


# ------------------------------------------------- the paper's Eq. 7 / Eq. 9
def test_feature_rbf_graph_definition():
    n, k, b = 500, 8, 0.7
    x = rand_points(n, 31)
    f = np.random.default_rng(32).normal(size=(n, 6)).astype(F32)
    p = np.random.default_rng(33).uniform(0, 1, n).astype(F32)
    rp, col, val = graph.feature_rbf_graph(x, f, k, b, unary=p)
    A = np.zeros((n, n))
    for i in range(n):
        A[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    assert np.array_equal(A, A.T)  # symmetric bit for bit
    idx, _ = graph.knn(x, k)
    g = f.astype(np.float64) / np.linalg.norm(f.astype(np.float64), axis=1, keepdims=True)
    D = cdist(g, g)
    sf = np.median(D[np.arange(n)[:, None], idx])
    for i in range(0, n, 23):
        for j in idx[i]:
            ref = np.exp(-D[i, j] ** 2 / (float(F32(b)) * sf ** 2)) * np.sqrt(float(p[i]) * float(p[j]))
            assert abs(A[i, j] - ref) <= 1e-6 * ref + 1e-12
    # no self-loops, no row normalisation; unary 1 is the plain kernel
    assert np.all(np.diag(A) == 0)
    rp1, col1, val1 = graph.feature_rbf_graph(x, f, k, b)
    A1 = np.zeros((n, n))
    for i in range(n):
        A1[i, col1[rp1[i]:rp1[i + 1]]] = val1[rp1[i]:rp1[i + 1]]
    sq = np.sqrt(p.astype(np.float64))
    assert np.allclose(A, A1 * sq[:, None] * sq[None, :], rtol=2e-7, atol=1e-12)


def test_feature_rbf_graph_binarised():
    n, k = 400, 10
    x = rand_points(n, 41)
    f = np.random.default_rng(42).normal(size=(n, 3)).astype(F32)
    rp, col, val = graph.feature_rbf_graph(x, f, k, 0.05, binarize=1e-5)
    rpw, colw, valw = graph.feature_rbf_graph(x, f, k, 0.05)
    assert np.all(val == 1.0)
    kept = {(i, int(c)) for i in range(n) for c in col[rp[i]:rp[i + 1]]}
    ref = {(i, int(c)) for i in range(n) for c, v in zip(colw[rpw[i]:rpw[i + 1]], valw[rpw[i]:rpw[i + 1]])
           if float(v) > float(F32(1e-5)) * (1 + 1e-6)}
    assert ref <= kept and len(kept) < len(colw)


def test_anchor_init_and_reach():
    from oracle import prune
    rng = np.random.default_rng(51)
    g = rng.normal(size=1000).astype(F32)
    g0 = prune.anchor_init(g, 0.1)
    npos = int(np.sum(g > 0))
    k = int(np.ceil(0.1 * npos))
    assert np.count_nonzero(g0) == k
    top = np.sort(g[g > 0])[::-1][:k]
    assert np.array_equal(np.sort(g0[g0 != 0])[::-1], top)
    gt = rng.normal(size=(1000, 2)).astype(F32)
    p = rng.uniform(size=1000).astype(F32)
    h = prune.reach_unary(gt, p)
    assert np.array_equal(h[:, 1], np.where(gt[:, 1] > 0, p, 0).astype(F32))
