"""Diffusion-graph input: a k-nearest-neighbour graph over Gaussian centres
(union of the directed kNN relations), edge weight
exp(-|x_i - x_j|^2 / sigma^2) * max(0, cos(f_i, f_j)) with sigma the median
directed kNN distance, rows normalised to sum 1 (a row with no weight gets a
self-loop of weight 1), stored as CSR (int32 row_ptr / col, FP32 values,
columns ascending).  This is input preparation for the diffusion step, built
on the host in FP64."""
import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree


def knn(points, k):
    """Directed kNN (self excluded): (idx [n,k], dist [n,k]) in FP64."""
    pts = np.asarray(points, np.float64)
    tree = cKDTree(pts)
    d, i = tree.query(pts, k=k + 1, workers=-1)
    # drop self (distance 0, normally first); keep k others
    out_i = np.empty((pts.shape[0], k), np.int64)
    out_d = np.empty((pts.shape[0], k))
    self_first = i[:, 0] == np.arange(pts.shape[0])
    out_i[self_first] = i[self_first, 1:]
    out_d[self_first] = d[self_first, 1:]
    bad = np.nonzero(~self_first)[0]
    for r in bad:  # duplicate points: remove self wherever it appears
        keep = i[r] != r
        out_i[r] = i[r][keep][:k]
        out_d[r] = d[r][keep][:k]
    return out_i, out_d


def knn_graph(points, feats, k=16):
    """Returns (row_ptr int32 [n+1], col int32 [nnz], val float32 [nnz])."""
    pts = np.asarray(points, np.float64)
    n = pts.shape[0]
    idx, dist = knn(pts, k)
    sigma = float(np.median(dist))
    f = np.asarray(feats, np.float64)
    if f.ndim == 1:
        f = f[:, None]
    nrm = np.linalg.norm(f, axis=1)
    rows = np.repeat(np.arange(n), k)
    cols = idx.reshape(-1)
    num = np.empty(n * k)
    step = max(1, (1 << 22) // max(1, f.shape[1] * k))  # rows per chunk (bounded temporaries)
    for r0 in range(0, n, step):
        r1 = min(n, r0 + step)
        nb = f[idx[r0:r1]]                                   # [rows, k, D]
        num[r0 * k:r1 * k] = np.einsum("rd,rkd->rk", f[r0:r1], nb).reshape(-1)
    den = nrm[rows] * nrm[cols]
    cos = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    w = np.exp(-(dist.reshape(-1) ** 2) / (sigma * sigma)) * np.maximum(0.0, cos)
    M = sp.coo_matrix((w, (rows, cols)), shape=(n, n)).tocsr()
    M.sum_duplicates()
    S = M.maximum(M.T).tocsr()          # union: w_ij is symmetric in (i, j)
    S.eliminate_zeros()                 # zero-weight edges change nothing
    S.sort_indices()
    rs = np.asarray(S.sum(axis=1)).reshape(-1)
    zero = rs <= 0
    if zero.any():
        S = (S + sp.diags(zero.astype(np.float64))).tocsr()
        S.sort_indices()
        rs = np.asarray(S.sum(axis=1)).reshape(-1)
    S = sp.diags(1.0 / rs) @ S
    S = S.tocsr()
    S.sort_indices()
    return (S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float32))
