"""Uplift followed by graph construction and diffusion at full size
(Sec. 3.2 then Sec. 3.3, Eq. 8), through the C ABI.

1,000,000 Gaussians (scales exp(N(-5, 0.7^2)), opacities sigmoid(N(0.5, 1))),
100 views at 1008x756.

* Graph parity at full size: the 16-NN graph over the centres with
  synthetic N(0,1) features (64 channels) built on the device against the
  FP64 oracle graph (structure bit-exact, values within FP32 rounding), then
  100 diffusion steps of a half-space indicator (D = 1) and of a sample of
  the 64 channels on it, FP32 and BF16 storage, against the oracle diffusing
  the oracle graph (with BF16 storage: the oracle rounds every iterate to
  BF16 as well).
* The chained path: D = 64 features uplifted on the GPU from all 100 views,
  the device graph built from them, 100 steps on it; the graph checked by
  properties (finite, row-stochastic and union-symmetric), the diffusion of
  the mask and of sampled feature channels against the FP64 oracle on the
  device graph's CSR, a constant signal staying constant.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2410_14462_amd as lv
from oracle import diffuse as od
from synth import philox, scenes

pytestmark = pytest.mark.gpu

STEPS = 100
CHANNELS = [0, 21, 42, 63]


def rel_err(out, ref):
    """max |out - ref| per channel, relative to that channel's max |ref|."""
    scale = np.maximum(np.max(np.abs(ref), axis=0), 1e-30)
    return np.max(np.abs(out - ref) / scale)


@pytest.fixture(scope="module")
def large():
    w = scenes.WORKLOADS["large"]
    sc = scenes.scene_for(w)
    return w, sc, lv.Scene.from_arrays(sc)


def test_graph_and_diffusion_full_size(large):
    w, sc, gs = large
    n, D = sc.n, 64
    feats = philox.normal(w.seed, 77, n * D).reshape(n, D).astype(np.float32)
    print("full graph: device build", flush=True)
    G = lv.Graph.knn(gs, torch.as_tensor(feats, device="cuda"), 16)
    rp, col, val = (t.cpu().numpy() for t in G.csr())
    print(f"full graph: nnz={len(col)}; oracle build", flush=True)
    rrp, rcol, rval = oracle.graph.knn_graph(sc.means, feats, 16)
    assert np.array_equal(rp, rrp) and np.array_equal(col, rcol)
    err = np.abs(val.astype(np.float64) - rval) - 2e-7 * np.abs(rval)
    assert err.max() <= 1e-9
    mask = scenes.halfspace_indicator(w.seed, sc.means)
    dev = lambda a: torch.as_tensor(a, device="cuda")
    for vdt in ("f32", "bf16"):
        tdt = torch.float32 if vdt == "f32" else torch.bfloat16
        Gd = G if vdt == "f32" else lv.Graph(dev(rp), dev(col), dev(val).to(torch.bfloat16))
        g_mask = dev(mask).to(tdt)
        g_feat = dev(feats).to(tdt)
        out_mask = Gd.diffuse(g_mask, STEPS, scene=gs).float().cpu().numpy().astype(np.float64)
        out_feat = Gd.diffuse(g_feat, STEPS, scene=gs).float().cpu().numpy().astype(np.float64)
        aval = rval if vdt == "f32" else torch.as_tensor(rval).to(torch.bfloat16).float().numpy()
        A = od.csr_matrix(n, rrp, rcol, aval)
        chans = CHANNELS if vdt == "f32" else CHANNELS[:2]
        store = None if vdt == "f32" else "bf16"  # BF16: every iterate stored in BF16
        ref_mask = od.diffuse(A, g_mask.float().cpu().numpy(), STEPS, store=store)
        ref_feat = od.diffuse(A, g_feat[:, chans].float().cpu().numpy(), STEPS, store=store)
        e_mask, e_feat = rel_err(out_mask, ref_mask), rel_err(out_feat[:, chans], ref_feat)
        print(f"full diffusion {vdt}: mask err {e_mask:.3e}, features err {e_feat:.3e}", flush=True)
        assert np.all(out_mask >= 0)  # A >= 0 and g0 >= 0
        if vdt == "f32":
            assert e_mask < 1e-4 and e_feat < 1e-4
        else:
            # against the oracle that stores every iterate in BF16 too: the
            # GPU's FP32 sums round to the other BF16 neighbour only near ties
            # (one BF16 ulp, 2^-8 of that element), and the row-stochastic A
            # averages such flips rather than growing them
            assert e_mask <= 2.0 ** -7 and e_feat <= 2.0 ** -7
        if vdt == "bf16":
            Gd.close()
    G.close()


def test_uplift_graph_diffusion_chain(large):
    w, sc, gs = large
    cams = scenes.cameras_for(w)
    D = 64
    print("chain: uplift D=64 from 100 views", flush=True)
    acc = lv.Accum(gs, D)
    for v0 in range(0, w.m, 10):
        maps = [scenes.feature_map(w, v, device="cuda", D=D) for v in range(v0, v0 + 10)]
        acc.add(cams[v0:v0 + 10], maps)
        del maps
    f, b = acc.finalize()
    acc.close()
    assert torch.isfinite(f).all() and (b > 0).float().mean() > 0.2
    G = lv.Graph.knn(gs, f, 16)
    rp, col, val = (t.cpu().numpy() for t in G.csr())
    n = sc.n
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(np.isfinite(val)) and np.all(val >= 0)
    assert np.allclose(np.bincount(rows, weights=val.astype(np.float64), minlength=n), 1.0, atol=1e-5)
    # union-symmetric structure (self-loops aside)
    off = rows != col
    fwd = rows[off].astype(np.int64) * n + col[off]
    bwd = col[off].astype(np.int64) * n + rows[off]
    assert np.array_equal(np.sort(fwd), np.sort(bwd))
    mask = torch.as_tensor(scenes.halfspace_indicator(w.seed, sc.means), device="cuda")
    out = G.diffuse(mask, STEPS, scene=gs)
    assert torch.all(out >= 0) and torch.isfinite(out).all()
    # the FP64 oracle diffusing on the device graph's own CSR: the mask and a
    # sample of the uplifted feature channels
    A = od.csr_matrix(n, rp, col, val)
    e_mask = rel_err(out.cpu().numpy().astype(np.float64), od.diffuse(A, mask.cpu().numpy(), STEPS))
    chans = [0, 31, 63]
    out_f = G.diffuse(f, STEPS, scene=gs).cpu().numpy().astype(np.float64)[:, chans]
    e_feat = rel_err(out_f, od.diffuse(A, f[:, chans].cpu().numpy(), STEPS))
    print(f"chain diffusion vs oracle on the device CSR: mask {e_mask:.3e}, features {e_feat:.3e}",
          flush=True)
    assert e_mask < 1e-4 and e_feat < 1e-4
    ones = G.diffuse(torch.ones((n, 1), device="cuda"), STEPS, scene=gs)
    assert torch.allclose(ones, torch.full_like(ones, n ** -0.5), rtol=1e-4)
    G.close()
