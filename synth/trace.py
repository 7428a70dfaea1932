"""Seeded synthetic serving trace: resident scenes, their camera rigs, a bank
of feature maps and a stream of uplift requests with Poisson arrivals.
Holds none of the uplifting arithmetic.

Scenes: 100k, 500k and 2M Gaussians drawn as the tiny scene (centres
U[-1,1]^3, uniform rotations, opacities sigmoid(N(0,1))) with scales
exp(N(-5, 0.7^2)); seeds 30, 31, 32.  Rig: 200 Fibonacci-sphere poses at
radius 4, 55 deg horizontal FoV, at 512x384, 768x576 and 1008x756.
Requests (seed 33): exponential inter-arrival gaps (Poisson arrivals at
`rate` per second), scene U{3}, D U{1, 3, 16, 64, 384, 512}, resolution
U{3}, 10..200 distinct poses of the rig.  A request's map of pose v is
channels [0, D) of bank map (v mod K) at its resolution; bank maps are
512-channel N(0,1) maps at 1/14 resolution, bilinearly upsampled.
"""
from dataclasses import dataclass

import numpy as np

from . import philox
from .scenes import fibonacci_eyes, look_at, make_scene, map_lowres, stream, upsample

TAG_TRACE, TAG_VIEWS = 20, 21
SCENE_SEEDS = (30, 31, 32)
SCENE_SIZES = (100_000, 500_000, 2_000_000)
RESOLUTIONS = ((512, 384), (768, 576), (1008, 756))
D_CHOICES = (1, 3, 16, 64, 384, 512)
RIG_POSES = 200
BANK_D = 512
TRACE_SEED = 33


@dataclass
class Request:
    arrival: float     # seconds after the start of the trace
    scene: int         # index into SCENE_SIZES
    D: int
    res: int           # index into RESOLUTIONS
    views: list        # rig poses, ascending


def scenes(sizes=SCENE_SIZES):
    return [make_scene(seed, n, -5.0, 0.7, 0.0, 1.0) for seed, n in zip(SCENE_SEEDS, sizes)]


def rig(res):
    W, H = RESOLUTIONS[res]
    return [look_at(e, W, H, 55.0) for e in fibonacci_eyes(RIG_POSES, 4.0)]


def requests(count, rate, seed=TRACE_SEED, min_views=10, max_views=RIG_POSES):
    out = []
    t = 0.0
    for i in range(count):
        u = philox.uniform(seed, stream(TAG_TRACE, i), 5).astype(np.float64)
        t += -np.log(u[0]) / rate
        scene = int(u[1] * len(SCENE_SIZES))
        D = D_CHOICES[int(u[2] * len(D_CHOICES))]
        res = int(u[3] * len(RESOLUTIONS))
        k = min_views + int(u[4] * (max_views - min_views + 1))
        keys = philox.blocks(seed, stream(TAG_VIEWS, i), 0, RIG_POSES)[:, 0]
        views = sorted(np.argsort(keys, kind="stable")[:k].tolist())
        out.append(Request(t, scene, D, res, views))
    return out


def bank(res, K, device="cuda", D=BANK_D, seed=TRACE_SEED):
    """K maps [H, W, D] FP32 at resolution `res` (torch, on `device`)."""
    W, H = RESOLUTIONS[res]
    return [upsample(map_lowres(seed, 1000 * res + k, H, W, D), H, W, device) for k in range(K)]
