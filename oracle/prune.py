"""Weight-based Gaussian filtering, FP64-free plain definition.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.2 (Gaussian filtering): the weight sum beta_i of a Gaussian estimates
its importance; the filter keeps the k Gaussians with the largest beta.  The
order is IEEE 754 totalOrder on the FP32 values (so -0 < +0 and NaNs sit by
their sign and payload), ties to the lower index.
"""
import numpy as np


def total_order_key(values):
    """Unsigned keys whose ascending order is IEEE totalOrder of FP32 values."""
    b = np.ascontiguousarray(values, dtype=np.float32).view(np.uint32).astype(np.uint64)
    neg = (b >> 31) == 1
    return np.where(neg, 0xFFFFFFFF - b, b | 0x80000000).astype(np.uint64)


def keep_top_k(values, k):
    """uint8 mask: 1 for the k largest values in totalOrder, ties to the
    lower index; 0 elsewhere."""
    values = np.asarray(values, dtype=np.float32)
    n = values.shape[0]
    if not 0 <= k <= n:
        raise ValueError("k out of range")
    key = total_order_key(values)
    # descending key, ascending index: lexsort sorts by the last key first
    order = np.lexsort((np.arange(n), -key.astype(np.int64)))
    keep = np.zeros(n, np.uint8)
    keep[order[:k]] = 1
    return keep


def anchor_init(g, fraction):
    """Anchors of a diffusion (appendix on diffusion for segmentation): the
    ceil(fraction * npos) largest of the npos positive values of g keep their
    value (ties to the lower index), every other entry is 0."""
    import math
    g = np.asarray(g, dtype=np.float32)
    npos = int(np.sum(g > 0))
    k = int(math.ceil(float(np.float32(fraction)) * npos))
    return np.where(keep_top_k(g, k) == 1, g, np.float32(0.0)).astype(np.float32)


def reach_unary(gT, unary):
    """h = P where the diffused signal is positive (the nodes reached), else 0."""
    gT = np.asarray(gT, dtype=np.float32)
    p = np.asarray(unary, dtype=np.float32)
    return np.where(gT > 0, p.reshape((-1,) + (1,) * (gT.ndim - 1)), np.float32(0.0)).astype(np.float32)
