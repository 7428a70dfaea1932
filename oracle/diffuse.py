"""FP64 graph diffusion oracle (test infrastructure only).

Sec. 3.3, Eq. (8): g_{t+1} = A g~_t with g~_t = g_t / ||g_t||_2.  Several
channels (parallel queries, App. A.4) are diffused together, each normalised by
its own norm; a zero-norm channel stays zero.  The result is g_T, the last
product (not normalised).  T = 0 returns g_0.

Storage precision (the paper states none): with ``store="bf16"`` every
iterate g_{t+1} is rounded to the nearest bfloat16 (ties to even) before the
next step, which is what keeping the signal in BF16 between steps means; the
products and norms stay FP64.
"""
import numpy as np
import scipy.sparse as sp


def csr_matrix(n, row_ptr, col, val):
    return sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col, np.int64),
                          np.asarray(row_ptr, np.int64)), shape=(n, n))


def round_bf16(x):
    """Nearest bfloat16 value (8 significant bits, FP32's exponent range,
    round half to even) of FP64 values, as FP64."""
    x = np.asarray(x, np.float64)
    _, e = np.frexp(x)                        # |x| in [2^(e-1), 2^e)
    ulp = np.ldexp(1.0, np.maximum(e, -125) - 8)  # subnormal spacing below 2^-126
    return np.rint(x / ulp) * ulp             # rint: half to even


def diffuse(A, g0, steps, store=None):
    """A: scipy CSR (any dtype; used in FP64), g0: [n] or [n, D].
    store: None (FP64 iterates) or "bf16" (each iterate rounded to BF16)."""
    if store not in (None, "bf16"):
        raise ValueError(f"unknown storage {store!r}")
    A = A.astype(np.float64)
    g = np.asarray(g0, np.float64)
    squeeze = g.ndim == 1
    if squeeze:
        g = g[:, None]
    for _ in range(steps):
        nrm = np.sqrt(np.sum(g * g, axis=0))
        scale = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 0.0)
        g = A @ (g * scale[None, :])
        if store == "bf16":
            g = round_bf16(g)
    return g[:, 0] if squeeze else g
