"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), vectorised in numpy.

Every random number in the synthetic workloads comes from here.  A stream is
named by a 64-bit key (seed, stream id); element ``i`` of a stream is block
``i`` (counter = (i mod 2^32, i >> 32, 0, 0)), so any slice of any stream can
be regenerated without generating what precedes it.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on uint32 arrays (broadcastable); returns 4 uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32)
    c1 = np.asarray(c1, dtype=np.uint32)
    c2 = np.asarray(c2, dtype=np.uint32)
    c3 = np.asarray(c3, dtype=np.uint32)
    k0 = np.uint32(k0)
    k1 = np.uint32(k1)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0 = np.uint32(k0 + _W0)
                k1 = np.uint32(k1 + _W1)
            p0 = c0.astype(np.uint64) * _M0
            p1 = c2.astype(np.uint64) * _M1
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & _MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & _MASK32).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def blocks(seed, stream, start, count):
    """uint32 array [count, 4]: blocks start..start+count-1 of stream (seed, stream)."""
    idx = np.arange(start, start + count, dtype=np.uint64)
    lo = (idx & _MASK32).astype(np.uint32)
    hi = (idx >> np.uint64(32)).astype(np.uint32)
    z = np.zeros_like(lo)
    out = philox4x32_10(lo, hi, z, z, seed, stream)
    return np.stack(out, axis=-1)


def uniform(seed, stream, count, start=0):
    """count FP32 values in (0, 1): 4 per block, u = ((x >> 8) + 0.5) * 2^-24 (exact)."""
    nb = (count + 3) // 4
    b = blocks(seed, stream, start, nb).reshape(-1)[:count]
    return (((b >> np.uint32(8)).astype(np.float64) + 0.5) * 2.0 ** -24).astype(np.float32)


def normal64(seed, stream, count, start=0):
    """count N(0,1) values in FP64 by Box-Muller: block b gives normals 2b and 2b+1
    from its first two words (u1, u2 = (x + 0.5) * 2^-32)."""
    nb = (count + 1) // 2
    b = blocks(seed, stream, start, nb)
    u1 = (b[:, 0].astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = (b[:, 1].astype(np.float64) + 0.5) * 2.0 ** -32
    r = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    z = np.empty(2 * nb, dtype=np.float64)
    z[0::2] = r * np.cos(th)
    z[1::2] = r * np.sin(th)
    return z[:count]


def normal(seed, stream, count, start=0):
    """N(0,1) drawn in FP64 and rounded to FP32."""
    return normal64(seed, stream, count, start).astype(np.float32)
