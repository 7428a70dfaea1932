"""Shared test helpers: error metrics and device-side map generation."""
import numpy as np


def feature_error(f_gpu, ref, rows=None):
    """e_ic = |f^_ic - f_ic| / a_ic over Gaussians with beta > 0, where
    a_ic = sum w |F_c| / beta (f is a convex combination of the F_c, so
    a_ic >= |f_ic|; for non-negative features this is the relative error)."""
    rows = ref.rows if rows is None else rows
    seen = ref.beta[rows] > 0
    f = np.asarray(f_gpu, np.float64)
    a = ref.a[seen]
    d = np.abs(f[seen] - ref.f[seen])
    with np.errstate(invalid="ignore", divide="ignore"):
        e = np.where(a > 0, d / np.where(a > 0, a, 1.0), d)
    return e


def beta_error(b_gpu, ref):
    seen = ref.beta > 0
    b = np.asarray(b_gpu, np.float64)
    return np.abs(b[seen] - ref.beta[seen]) / ref.beta[seen]


def maps_on_device(w, views, D=None):
    from synth import scenes
    return [scenes.feature_map(w, v, device="cuda", D=D) for v in views]
