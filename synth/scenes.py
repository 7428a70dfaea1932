"""Seeded synthetic workloads: Gaussian scenes, camera rigs, feature maps,
masks and diffusion seeds.  Holds none of the uplifting arithmetic: it only
draws inputs.  Both the HIP path and the FP64 oracle consume what it returns.

Stream ids: stream = (tensor tag << 20) | view.  Every array is a pure
function of (config seed, tag, view), so tests can rebuild any single view.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import philox

TAG_MEANS, TAG_SCALES, TAG_QUATS, TAG_OPACITY = 1, 2, 3, 4
TAG_MAP_UNIFORM, TAG_MAP_LOWRES, TAG_MASK, TAG_HALFSPACE = 8, 9, 10, 11
TAG_SUBSAMPLE = 12


def stream(tag, view=0):
    return (tag << 20) | view


@dataclass
class Scene:
    means: np.ndarray      # [n,3] f32
    scales: np.ndarray     # [n,3] f32, linear (not log)
    quats: np.ndarray      # [n,4] f32, (w,x,y,z), not normalised
    opacity: np.ndarray    # [n]   f32 in (0,1)

    @property
    def n(self):
        return int(self.means.shape[0])


@dataclass
class Camera:
    R: np.ndarray          # [3,3] f32 world->camera rows (x right, y down, z forward)
    t: np.ndarray          # [3]   f32, x_c = R x_w + t
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.01


@dataclass
class Workload:
    name: str
    seed: int
    n: int
    scale_mu: float
    scale_sd: float
    op_mu: float
    op_sd: float
    m: int
    width: int
    height: int
    fov_deg: float
    D: int
    maps: str              # "uniform" | "lowres_normal"
    radius: float = 4.0
    extra: dict = field(default_factory=dict)


# The five synthetic workloads (sizes and distributions from the benchmark
# configurations; seeds 0..4).
WORKLOADS = {
    "tiny": Workload("uplift-10k-4v-128x128-D8", 0, 10_000, -4.0, 0.5, 0.0, 1.0,
                     4, 128, 128, 60.0, 8, "uniform"),
    "mid": Workload("uplift-200k-50v-512x384-D64+mask", 1, 200_000, -4.0, 0.5, 0.0, 1.0,
                    50, 512, 384, 55.0, 64, "lowres_normal", extra={"mask": True}),
    "large": Workload("uplift-1M-100v-1008x756-D384", 2, 1_000_000, -5.0, 0.7, 0.5, 1.0,
                      100, 1008, 756, 55.0, 384, "lowres_normal"),
    "diffuse": Workload("uplift+diffuse-1M-100v-1008x756-D64", 4, 1_000_000, -5.0, 0.7, 0.5, 1.0,
                        100, 1008, 756, 55.0, 64, "lowres_normal", extra={"steps": 100, "k": 16}),
}


def make_scene(seed, n, scale_mu, scale_sd, op_mu, op_sd):
    """Centres U[-1,1]^3, scales exp(N(mu, sd^2)) per axis, quaternions N(0, I4)
    (uniform rotations once normalised), opacities sigmoid(N(mu, sd^2))."""
    u = philox.uniform(seed, stream(TAG_MEANS), 3 * n).astype(np.float64)
    means = (2.0 * u - 1.0).astype(np.float32).reshape(n, 3)
    z = philox.normal64(seed, stream(TAG_SCALES), 3 * n)
    scales = np.exp(scale_mu + scale_sd * z).astype(np.float32).reshape(n, 3)
    quats = philox.normal(seed, stream(TAG_QUATS), 4 * n).reshape(n, 4)
    zo = philox.normal64(seed, stream(TAG_OPACITY), n)
    opacity = (1.0 / (1.0 + np.exp(-(op_mu + op_sd * zo)))).astype(np.float32)
    return Scene(means, scales, quats, opacity)


def scene_for(w: Workload):
    return make_scene(w.seed, w.n, w.scale_mu, w.scale_sd, w.op_mu, w.op_sd)


def look_at(eye, width, height, fov_deg, znear=0.01):
    """Pinhole camera at `eye` looking at the origin; horizontal field of view;
    principal point at the image centre; fy = fx."""
    eye = np.asarray(eye, dtype=np.float64)
    zc = -eye / np.linalg.norm(eye)
    up = np.array([0.0, 0.0, 1.0])
    xc = np.cross(zc, up)
    if np.linalg.norm(xc) < 1e-9:
        xc = np.cross(zc, np.array([0.0, 1.0, 0.0]))
    xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    R = np.stack([xc, yc, zc])
    t = -R @ eye
    fx = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return Camera(R.astype(np.float32), t.astype(np.float32), float(np.float32(fx)), float(np.float32(fx)),
                  width / 2.0, height / 2.0, width, height, znear)


def fibonacci_eyes(m, radius):
    k = np.arange(m, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / m
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return radius * np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def cameras_for(w: Workload, m=None, width=None, height=None):
    m = w.m if m is None else m
    eyes = fibonacci_eyes(m, w.radius)
    return [look_at(e, width or w.width, height or w.height, w.fov_deg) for e in eyes]


def lowres_shape(width, height, patch=14):
    return (math.ceil(height / patch), math.ceil(width / patch))


def map_uniform(seed, view, H, W, D):
    return philox.uniform(seed, stream(TAG_MAP_UNIFORM, view), H * W * D).reshape(H, W, D)


def map_lowres(seed, view, H, W, D):
    h, w = lowres_shape(W, H)
    return philox.normal(seed, stream(TAG_MAP_LOWRES, view), h * w * D).reshape(h, w, D)


def upsample(low, H, W, device="cpu"):
    """Bilinear, half-pixel centres (align_corners=False), edge clamp.
    low: [h,w,D] (numpy or torch) -> torch [H,W,D] f32 contiguous on `device`."""
    import torch
    x = torch.as_tensor(low, device=device, dtype=torch.float32).permute(2, 0, 1).unsqueeze(0)
    y = torch.nn.functional.interpolate(x, size=(H, W), mode="bilinear", align_corners=False)
    return y[0].permute(1, 2, 0).contiguous()


def feature_map(w: Workload, view, device="cpu", D=None):
    """Full-resolution FP32 map [H,W,D] of `view` as a torch tensor."""
    import torch
    D = w.D if D is None else D
    if w.maps == "uniform":
        return torch.as_tensor(map_uniform(w.seed, view, w.height, w.width, D), device=device)
    return upsample(map_lowres(w.seed, view, w.height, w.width, D), w.height, w.width, device)


def ellipse_mask(seed, view, H, W):
    """[H,W,1] f32: 1 inside a random ellipse (centre uniform over the image,
    semi-axes U(0.1,0.4)*min(W,H), angle U[0,pi)) at pixel centres."""
    u = philox.uniform(seed, stream(TAG_MASK, view), 5).astype(np.float64)
    cx, cy = u[0] * W, u[1] * H
    a = (0.1 + 0.3 * u[2]) * min(W, H)
    b = (0.1 + 0.3 * u[3]) * min(W, H)
    th = u[4] * math.pi
    ys, xs = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    dx, dy = xs - cx, ys - cy
    ex = (dx * math.cos(th) + dy * math.sin(th)) / a
    ey = (-dx * math.sin(th) + dy * math.cos(th)) / b
    return ((ex * ex + ey * ey) <= 1.0).astype(np.float32)[:, :, None]


def halfspace_indicator(seed, means):
    """g0 [n,1] f32 = 1[nu . mu > b], nu uniform on S^2, b ~ U(-0.5, 0.5)."""
    z = philox.normal64(seed, stream(TAG_HALFSPACE), 3)
    nu = z / np.linalg.norm(z)
    b = float(philox.uniform(seed, stream(TAG_HALFSPACE, 1), 1)[0]) - 0.5
    return ((means.astype(np.float64) @ nu) > b).astype(np.float32)[:, None]


def subsample(seed, n, k):
    """k distinct Gaussian indices drawn without replacement (sorted)."""
    keys = philox.blocks(seed, stream(TAG_SUBSAMPLE), 0, n)[:, 0]
    return np.sort(np.argsort(keys, kind="stable")[:k])
