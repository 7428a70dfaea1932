"""Shared test helpers: error metrics over the Gaussians the oracle decides
unambiguously, and device-side map generation."""
import numpy as np


def _strict(ref, rows):
    """Gaussians of `rows` with a weight and no ambiguous decision."""
    return (ref.beta[rows] > 0) & ref.strict[rows]


def feature_error(f_gpu, ref, rows=None):
    """e_ic = |f^_ic - f_ic| / a_ic over Gaussians with beta > 0 that no
    ambiguous pixel touches, where a_ic = sum w |F_c| / beta (f is a convex
    combination of the F_c, so a_ic >= |f_ic|; for non-negative features this
    is the relative error)."""
    rows = ref.rows if rows is None else rows
    seen = _strict(ref, rows)
    f = np.asarray(f_gpu, np.float64)
    a = ref.a[seen]
    d = np.abs(f[seen] - ref.f[seen])
    with np.errstate(invalid="ignore", divide="ignore"):
        e = np.where(a > 0, d / np.where(a > 0, a, 1.0), d)
    return e


def beta_error(b_gpu, ref):
    seen = (ref.beta > 0) & ref.strict
    b = np.asarray(b_gpu, np.float64)
    return np.abs(b[seen] - ref.beta[seen]) / ref.beta[seen]


def counts_match(c_gpu, ref):
    """Contribution counts equal on every Gaussian no ambiguous pixel touches;
    prints the ambiguity log (ambiguous pixels, flagged Gaussians, smallest
    skip and stop margins)."""
    c = np.asarray(c_gpu).astype(np.int64)
    s = ref.strict
    print(f"ambiguous pixels {ref.amb_px}, flagged Gaussians {int((~s).sum())}, "
          f"min margins skip {ref.margin_skip:.2e} stop {ref.margin_stop:.2e}", flush=True)
    return bool(np.array_equal(c[s], ref.count[s]))


def maps_on_device(w, views, D=None):
    from synth import scenes
    return [scenes.feature_map(w, v, device="cuda", D=D) for v in views]
