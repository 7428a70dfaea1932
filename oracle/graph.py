"""kNN diffusion graph over the Gaussian centres, FP64 (test infrastructure
only; see the package docstring).

Graph of the diffusion step (Sec. 3.3, Eq. 8 uses a weighted graph over the
Gaussians): each Gaussian is joined to its k nearest other centres; the
relation is made symmetric by taking the union of the directed pairs
(Sec. 3.3); the weight of a pair is exp(-|x_i - x_j|^2 / sigma^2) *
max(0, cos(f_i, f_j)) (spatial RBF times clipped cosine of the uplifted
features), sigma the median directed kNN distance, the larger of the two
directed weights where both exist; rows are normalised to sum 1, and a row
whose weights are all 0 gets a self-loop of weight 1.

Conventions that make the structure reproducible bit for bit:
* squared distances are FP64, ((dx dx + dy dy) + dz dz) with dx = x_i - x_j
  of the FP32 centres promoted to FP64; neighbours are ordered by (squared
  distance, index), self excluded;
* the union pairs with a positive FP64 weight are stored (a weight is 0
  where the clipped cosine is <= 0 or the exponential underflows), columns
  ascending; a self-loop is the only entry of its row.
"""
import numpy as np
from scipy.spatial import cKDTree


def sq_dist(x, i, j):
    """Squared distances of pairs (i, j) in the fixed FP64 operation order."""
    d = x[i] - x[j]
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def knn(points, k):
    """Directed kNN, self excluded, ordered by (squared distance, index):
    (idx int64 [n, k], d2 float64 [n, k]).  Candidates come from a k-d tree;
    a row is recomputed by brute force when they may not be enough."""
    x = np.asarray(points, np.float32).astype(np.float64)
    n = x.shape[0]
    if n <= k:
        raise ValueError("need more than k points")
    extra = 8
    kk = min(n, k + 1 + extra)
    tree = cKDTree(x)
    dist, cand = tree.query(x, k=kk, workers=-1)
    rows = np.arange(n)[:, None]
    d2 = sq_dist(x, np.broadcast_to(rows, cand.shape), cand)
    d2 = np.where(cand == rows, np.inf, d2)  # self excluded
    order = np.lexsort((cand, d2), axis=1)
    cand = np.take_along_axis(cand, order, 1)
    d2 = np.take_along_axis(d2, order, 1)
    idx, out = cand[:, :k].copy(), d2[:, :k].copy()
    # the tree's farthest candidate bounds what was not returned; rows whose
    # k-th distance is not clearly below it are done again by brute force
    if kk < n:
        bound = dist[:, -1] ** 2 * (1.0 - 1e-9)
        redo = np.nonzero(~(out[:, -1] < bound))[0]
        for r in redo:
            allj = np.arange(n)
            dr = sq_dist(x, np.full(n, r), allj)
            dr[r] = np.inf
            o = np.lexsort((allj, dr))[:k]
            idx[r], out[r] = o, dr[o]
    return idx, out


def median_distance(d2):
    """sigma: median of the directed kNN distances (mean of the two middle
    values for an even count)."""
    return float(np.median(np.sqrt(d2)))


def knn_graph(points, feats, k=16):
    """Returns (row_ptr int32 [n+1], col int32 [nnz], val float32 [nnz])."""
    x = np.asarray(points, np.float32).astype(np.float64)
    n = x.shape[0]
    idx, d2 = knn(x, k)
    sigma = median_distance(d2)
    f = np.asarray(feats, np.float32).astype(np.float64)
    if f.ndim == 1:
        f = f[:, None]
    nrm = np.sqrt(np.sum(f * f, axis=1))
    rows = np.repeat(np.arange(n), k)
    cols = idx.reshape(-1)
    num = np.einsum("ed,ed->e", f[rows], f[cols]) if n * k * f.shape[1] <= (1 << 26) else np.concatenate(
        [np.einsum("ed,ed->e", f[rows[a:a + (1 << 20)]], f[cols[a:a + (1 << 20)]])
         for a in range(0, n * k, 1 << 20)])
    den = nrm[rows] * nrm[cols]
    cos = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    w = np.exp(-d2.reshape(-1) / (sigma * sigma)) * np.maximum(0.0, cos)
    # union of the directed pairs, the larger weight where both exist
    r2 = np.concatenate([rows, cols])
    c2 = np.concatenate([cols, rows])
    w2 = np.concatenate([w, w])
    o = np.lexsort((-w2, c2, r2))          # by row, column, larger weight first
    r2, c2, w2 = r2[o], c2[o], w2[o]
    first = np.ones(r2.size, bool)
    first[1:] = (r2[1:] != r2[:-1]) | (c2[1:] != c2[:-1])
    r2, c2, w2 = r2[first], c2[first], w2[first]
    pos = w2 > 0
    r2, c2, w2 = r2[pos], c2[pos], w2[pos]
    rs = np.bincount(r2, weights=w2, minlength=n)
    zero = np.nonzero(rs <= 0)[0]
    if zero.size:                          # self-loops of weight 1
        r2 = np.concatenate([r2, zero])
        c2 = np.concatenate([c2, zero])
        w2 = np.concatenate([w2, np.ones(zero.size)])
        o = np.lexsort((c2, r2))
        r2, c2, w2 = r2[o], c2[o], w2[o]
        rs = np.bincount(r2, weights=w2, minlength=n)
    val = w2 / rs[r2]
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r2, minlength=n), out=row_ptr[1:])
    return row_ptr.astype(np.int32), c2.astype(np.int32), val.astype(np.float32)


def feature_rbf_graph(points, feats, k, bandwidth, unary=None, binarize=0.0):
    """The paper's weights (Eq. 7 with the feature kernel of Eq. 9, appendix
    on diffusion for segmentation) on the same union pairs:
    A_ij = exp(-|g_i - g_j|^2 / (b s_f^2)) (sqrt(P_i) sqrt(P_j)), g the
    l2-normalised features (a zero feature stays 0), s_f the median of
    |g_i - g_j| over the directed kNN pairs, P = unary (1 if None).  No row
    normalisation and no self-loops; pairs with weight 0 are not stored;
    binarize > 0 keeps the pairs whose weight exceeds it, with value 1.
    Returns (row_ptr int32 [n+1], col int32 [nnz], val float32 [nnz])."""
    x = np.asarray(points, np.float32).astype(np.float64)
    n = x.shape[0]
    idx, _ = knn(x, k)
    f = np.asarray(feats, np.float32).astype(np.float64)
    if f.ndim == 1:
        f = f[:, None]
    nrm = np.sqrt(np.sum(f * f, axis=1))
    g = np.where(nrm[:, None] > 0, f / np.where(nrm > 0, nrm, 1.0)[:, None], 0.0)
    rows = np.repeat(np.arange(n), k)
    cols = idx.reshape(-1)
    fd2 = np.concatenate([np.sum((g[rows[a:a + (1 << 20)]] - g[cols[a:a + (1 << 20)]]) ** 2, axis=1)
                          for a in range(0, n * k, 1 << 20)])
    sf = float(np.median(np.sqrt(fd2)))
    p = np.ones(n) if unary is None else np.asarray(unary, np.float32).astype(np.float64)
    w = np.exp(-fd2 / (float(np.float32(bandwidth)) * (sf * sf))) * (np.sqrt(p[rows]) * np.sqrt(p[cols]))
    r2 = np.concatenate([rows, cols])
    c2 = np.concatenate([cols, rows])
    w2 = np.concatenate([w, w])
    o = np.lexsort((-w2, c2, r2))
    r2, c2, w2 = r2[o], c2[o], w2[o]
    first = np.ones(r2.size, bool)
    first[1:] = (r2[1:] != r2[:-1]) | (c2[1:] != c2[:-1])
    r2, c2, w2 = r2[first], c2[first], w2[first]
    thr = float(np.float32(binarize))
    keep = w2 > thr
    r2, c2, w2 = r2[keep], c2[keep], w2[keep]
    if thr > 0:
        w2 = np.ones_like(w2)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r2, minlength=n), out=row_ptr[1:])
    return row_ptr.astype(np.int32), c2.astype(np.int32), w2.astype(np.float32)
