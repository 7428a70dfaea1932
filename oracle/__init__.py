"""FP64 CPU oracle for learning-free uplifting and graph diffusion.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2410_14462_amd``) and never imports it.

* ``lv_oracle.c``  -- uplift (Eq. 3 / Eq. 5) and forward render (Eq. 4), plain C:
  FP32 (S32) structure, FP64 values and FP64 skip/stop decisions with a log of
  their margins; see its header for the conventions.
* ``diffuse.py``    -- graph diffusion (Eq. 8) in FP64 on a CSR matrix.
* ``prune.py``      -- weight-based Gaussian filtering (Sec. 3.2).
* ``graph.py``      -- the kNN diffusion graph over the centres (Sec. 3.3).
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from . import graph, prune  # noqa: F401  (oracle.graph, oracle.prune)

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lv_oracle.c")
LIB = os.path.join(HERE, "liblv_oracle.so")

_lib = None


def build(force=False):
    """Compile the C oracle with gcc (no contraction: S32 needs exact FP32 ops)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int
        f64 = ctypes.c_double
        L.orc_uplift_view.argtypes = [i64, P, P, P, P, P, i32, i32, P, i32, P, i64, P, P, P, P, P,
                                      P, P, f64, P, P, i32]
        L.orc_uplift_view.restype = i32
        L.orc_render_view.argtypes = [i64, P, P, P, P, P, i32, i32, P, i32, P, P, P, f64, i32]
        L.orc_render_view.restype = i32
        L.orc_view_structure.argtypes = [i64, P, P, P, P, P, i32, i32, P, P, P, P, P, P]
        L.orc_view_structure.restype = i64
        L.orc_factor32_array.argtypes = [i64, P, P, P]
        L.orc_factor32_array.restype = None
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def cam17(cam):
    """Camera -> the oracle's 17-float layout (R[9], t[3], fx, fy, cx, cy, znear)."""
    return np.concatenate([np.asarray(cam.R, np.float32).reshape(9), np.asarray(cam.t, np.float32),
                           np.array([cam.fx, cam.fy, cam.cx, cam.cy, cam.znear], np.float32)])


def _scene_arrays(scene):
    return (_f32(scene.means), _f32(scene.scales), _f32(scene.quats), _f32(scene.opacity))


# Relative decision margin below which a pixel is ambiguous: an FP32
# evaluation of alpha and T (a few units of 2^-24 per operation, times the
# exponent's size at the 1/255 boundary, ln(255) ~ 5.5) may decide it the
# other way.
AMB_THR = 1e-5


@dataclass
class UpliftResult:
    U: np.ndarray        # [rows, D] sum w F
    A: np.ndarray        # [rows, D] sum w |F|
    beta: np.ndarray     # [n]       sum w
    count: np.ndarray    # [n]       number of (view, pixel) pairs counted
    nnz: int
    P: int
    nvis: int
    rows: np.ndarray     # Gaussian index of each accumulated row
    amb: np.ndarray      # [n] ambiguous pixels at which the Gaussian is flagged
    amb_px: int          # ambiguous pixels over all views
    margin_skip: float   # smallest relative margin of an alpha >= 1/255 decision
    margin_stop: float   # smallest relative margin of a T < 1e-4 decision

    @property
    def strict(self):
        """Gaussians no ambiguous decision touches: their counts, beta and f
        are fixed by the definition at FP32 precision."""
        return self.amb == 0

    @property
    def f(self):
        """Eq. (3): f = U / beta (0 where beta == 0)."""
        b = self.beta[self.rows][:, None]
        with np.errstate(invalid="ignore", divide="ignore"):
            return np.where(b > 0, self.U / np.where(b > 0, b, 1.0), 0.0)

    @property
    def f_count(self):
        """Count-normalised features (appendix, GaussianEditor's aggregation):
        U / count, 0 where count == 0."""
        c = self.count[self.rows][:, None].astype(np.float64)
        with np.errstate(invalid="ignore", divide="ignore"):
            return np.where(c > 0, self.U / np.where(c > 0, c, 1.0), 0.0)

    @property
    def a(self):
        """Convex-combination magnitude sum w|F| / beta (the error scale)."""
        b = self.beta[self.rows][:, None]
        with np.errstate(invalid="ignore", divide="ignore"):
            return np.where(b > 0, self.A / np.where(b > 0, b, 1.0), 0.0)


class Uplifter:
    """Accumulates views one at a time (maps can be produced lazily)."""

    def __init__(self, scene, D, rows=None, nthreads=0, amb_thr=AMB_THR):
        self.scene = scene
        self.arrs = _scene_arrays(scene)
        n = scene.n
        self.D = D
        self.rows = np.arange(n, dtype=np.int64) if rows is None else np.asarray(rows, np.int64)
        if rows is None:
            self.rowmap = None
        else:
            self.rowmap = np.full(n, -1, np.int32)
            self.rowmap[self.rows] = np.arange(len(self.rows), dtype=np.int32)
        nr = len(self.rows)
        self.U = np.zeros((nr, D))
        self.A = np.zeros((nr, D))
        self.beta = np.zeros(n)
        self.count = np.zeros(n, np.int64)
        self.amb = np.zeros(n, np.int32)
        self.margins = np.full(2, np.inf)
        self.stats = np.zeros(4, np.int64)
        self.nthreads = nthreads
        self.amb_thr = amb_thr

    def add_view(self, cam, F, tfinal=False, amb_px=False):
        """Adds one view.  Returns the FP64 final transmittance [H,W] if
        tfinal, the ambiguous-pixel mask [H,W] if amb_px (a tuple if both)."""
        F = _f32(F)
        H, W = cam.height, cam.width
        assert F.shape == (H, W, self.D), (F.shape, (H, W, self.D))
        tf = np.zeros((H, W)) if tfinal else None
        am = np.zeros((H, W), np.uint8) if amb_px else None
        c = cam17(cam)
        rc = lib().orc_uplift_view(self.scene.n, *[_p(a) for a in self.arrs], _p(c), W, H, _p(F),
                                   self.D, _p(self.rowmap), len(self.rows), _p(self.U), _p(self.A),
                                   _p(self.beta), _p(self.count), _p(tf), _p(am), _p(self.amb),
                                   self.amb_thr, _p(self.margins), _p(self.stats), self.nthreads)
        if rc != 0:
            raise MemoryError("oracle: allocation failed")
        out = [x for x in (tf, am) if x is not None]
        return out[0] if len(out) == 1 else (tuple(out) if out else None)

    def result(self):
        return UpliftResult(self.U, self.A, self.beta, self.count, int(self.stats[0]),
                            int(self.stats[1]), int(self.stats[2]), self.rows, self.amb,
                            int(self.stats[3]), float(self.margins[0]), float(self.margins[1]))


def uplift(scene, cams, maps, rows=None, nthreads=0, amb_thr=AMB_THR):
    """Eq. (3) over all views.  maps: sequence (or callable view -> array) of [H,W,D]."""
    get = maps if callable(maps) else (lambda v: maps[v])
    first = np.asarray(get(0)) if len(cams) else np.zeros((1, 1, 1), np.float32)
    up = Uplifter(scene, first.shape[-1], rows, nthreads, amb_thr)
    for v, cam in enumerate(cams):
        up.add_view(cam, first if v == 0 else get(v))
    return up.result()


def render(scene, cam, g, nthreads=0, amb_thr=AMB_THR, amb_px=False):
    """Eq. (4) for one view: returns (F^ [H,W,D], alpha [H,W]) in FP64, and the
    ambiguous-pixel mask [H,W] as a third item if amb_px."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    if g.ndim == 1:
        g = g[:, None]
    D = g.shape[1]
    out = np.zeros((cam.height, cam.width, D))
    alpha = np.zeros((cam.height, cam.width))
    am = np.zeros((cam.height, cam.width), np.uint8)
    rc = lib().orc_render_view(scene.n, *[_p(a) for a in _scene_arrays(scene)], _p(cam17(cam)),
                               cam.width, cam.height, _p(g), D, _p(out), _p(alpha), _p(am),
                               amb_thr, nthreads)
    if rc != 0:
        raise MemoryError("oracle: allocation failed")
    return (out, alpha, am.astype(bool)) if amb_px else (out, alpha)


@dataclass
class ViewStructure:
    visible: np.ndarray   # [n] bool
    depth: np.ndarray     # [n] uint32 key (bits of FP32 view-space z)
    rect: np.ndarray      # [n,4] int32 (x0, y0, x1, y1) tile rectangle
    center: np.ndarray    # [n,2] f32 S32 projected centre (places the rectangle)
    tile_start: np.ndarray  # [TX*TY+1] int64
    ids: np.ndarray       # [P] int32, per tile sorted by (depth, index)


def structure(scene, cam):
    n = scene.n
    arrs = _scene_arrays(scene)
    c = cam17(cam)
    L = lib()
    P = L.orc_view_structure(n, *[_p(a) for a in arrs], _p(c), cam.width, cam.height,
                             None, None, None, None, None, None)
    if P < 0:
        raise MemoryError("oracle: allocation failed")
    TX, TY = -(-cam.width // 16), -(-cam.height // 16)
    vis = np.zeros(n, np.uint8)
    depth = np.zeros(n, np.uint32)
    rect = np.zeros((n, 4), np.int32)
    ctr = np.zeros((n, 2), np.float32)
    ts = np.zeros(TX * TY + 1, np.int64)
    ids = np.zeros(max(P, 1), np.int32)
    L.orc_view_structure(n, *[_p(a) for a in arrs], _p(c), cam.width, cam.height, _p(vis),
                         _p(depth), _p(rect), _p(ctr), _p(ts), _p(ids))
    return ViewStructure(vis.astype(bool), depth, rect, ctr, ts, ids[:P])


def factor32(scales, quats):
    """S32 covariance factor M = R diag(s), [n,3,3]; Sigma = M M^T."""
    s, q = _f32(scales), _f32(quats)
    out = np.zeros((s.shape[0], 3, 3), np.float32)
    lib().orc_factor32_array(s.shape[0], _p(s), _p(q), _p(out))
    return out


def num_threads():
    return int(lib().orc_num_threads())
