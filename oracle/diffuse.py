"""FP64 graph diffusion oracle (test infrastructure only).

Sec. 3.3, Eq. (8): g_{t+1} = A g~_t with g~_t = g_t / ||g_t||_2.  Several
channels (parallel queries, App. A.4) are diffused together, each normalised by
its own norm; a zero-norm channel stays zero.  The result is g_T, the last
product (not normalised).  T = 0 returns g_0.
"""
import numpy as np
import scipy.sparse as sp


def csr_matrix(n, row_ptr, col, val):
    return sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col, np.int64),
                          np.asarray(row_ptr, np.int64)), shape=(n, n))


def diffuse(A, g0, steps):
    """A: scipy CSR (any dtype; used in FP64), g0: [n] or [n, D]."""
    A = A.astype(np.float64)
    g = np.asarray(g0, np.float64)
    squeeze = g.ndim == 1
    if squeeze:
        g = g[:, None]
    for _ in range(steps):
        nrm = np.sqrt(np.sum(g * g, axis=0))
        scale = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 0.0)
        g = A @ (g * scale[None, :])
    return g[:, 0] if squeeze else g
