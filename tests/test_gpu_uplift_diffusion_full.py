"""Uplift followed by graph diffusion at full size (Sec. 3.2 then Sec. 3.3,
Eq. 8), through the C ABI.

1,000,000 Gaussians (scales exp(N(-5, 0.7^2)), opacities sigmoid(N(0.5, 1))),
D = 64 FP32 features uplifted on the GPU from all 100 views at 1008x756; a
16-NN graph over the centres with weights exp(-d^2 / sigma^2) (sigma the
median kNN distance) times the clipped cosine similarity of the uplifted
features, union-symmetrised and row-normalised (host, FP64, stored FP32 and
BF16); 100 diffusion steps on a D = 1 half-space indicator and on the D = 64
features.  The FP64 oracle diffuses the same CSR: the D = 1 signal in full
and a sample of the 64 channels (each channel is normalised by its own norm,
so channels are independent).
"""
import numpy as np
import pytest
import torch

import paper_2410_14462_amd as lv
from oracle import diffuse as od
from synth import graph, scenes

pytestmark = pytest.mark.gpu

STEPS = 100
CHANNELS = [0, 21, 42, 63]


def rel_err(out, ref):
    """max |out - ref| per channel, relative to that channel's max |ref|."""
    scale = np.maximum(np.max(np.abs(ref), axis=0), 1e-30)
    return np.max(np.abs(out - ref) / scale)


def test_uplift_graph_diffusion_full_size():
    w = scenes.WORKLOADS["large"]
    sc = scenes.scene_for(w)
    cams = scenes.cameras_for(w)
    gs = lv.Scene.from_arrays(sc)
    D = 64
    print("full diffusion: uplift D=64 from 100 views", flush=True)
    acc = lv.Accum(gs, D)
    for v0 in range(0, w.m, 10):
        maps = [scenes.feature_map(w, v, device="cuda", D=D) for v in range(v0, v0 + 10)]
        acc.add(cams[v0:v0 + 10], maps)
        del maps
    f, b = acc.finalize()
    acc.close()
    feats = f.cpu().numpy()
    assert np.isfinite(feats).all() and (b.cpu().numpy() > 0).mean() > 0.2

    print("full diffusion: 16-NN graph", flush=True)
    rp, col, val = graph.knn_graph(sc.means, feats, 16)
    n = sc.n
    print(f"full diffusion: nnz={len(col)}", flush=True)
    mask = scenes.halfspace_indicator(w.seed, sc.means)
    dev = lambda a: torch.as_tensor(a, device="cuda")
    for vdt in ("f32", "bf16"):
        gval = dev(val) if vdt == "f32" else dev(val).to(torch.bfloat16)
        G = lv.Graph(dev(rp), dev(col), gval)
        tdt = torch.float32 if vdt == "f32" else torch.bfloat16
        g_mask = dev(mask).to(tdt)
        g_feat = f.to(tdt)
        out_mask = G.diffuse(g_mask, STEPS, scene=gs).float().cpu().numpy().astype(np.float64)
        out_feat = G.diffuse(g_feat, STEPS, scene=gs).float().cpu().numpy().astype(np.float64)
        G.close()
        aval = val if vdt == "f32" else torch.as_tensor(val).to(torch.bfloat16).float().numpy()
        A = od.csr_matrix(n, rp, col, aval)
        chans = CHANNELS if vdt == "f32" else CHANNELS[:2]
        ref_mask = od.diffuse(A, g_mask.float().cpu().numpy(), STEPS)
        ref_feat = od.diffuse(A, g_feat[:, chans].float().cpu().numpy(), STEPS)
        e_mask, e_feat = rel_err(out_mask, ref_mask), rel_err(out_feat[:, chans], ref_feat)
        print(f"full diffusion {vdt}: mask err {e_mask:.3e}, features err {e_feat:.3e}", flush=True)
        assert np.all(out_mask >= 0)  # A >= 0 and g0 >= 0
        if vdt == "f32":
            assert e_mask < 1e-4 and e_feat < 1e-4
        else:
            # every iterate is rounded to BF16 (relative 2^-9); A is row-stochastic,
            # so a step adds at most that much to the max-norm error
            assert e_mask < STEPS * 2.0 ** -9 and e_feat < STEPS * 2.0 ** -9
