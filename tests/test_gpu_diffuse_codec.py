"""GPU parity of the storage codec and of graph diffusion (Eq. 8)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2410_14462_amd as lv
from oracle import diffuse as od
from oracle import graph
from synth import philox, scenes
from helpers import beta_error, counts_match, feature_error

pytestmark = pytest.mark.gpu


def test_bf16_encode_is_round_to_nearest_even():
    x = torch.as_tensor(philox.normal(30, 0, 4096 * 48).reshape(4096, 48) * 3.0, device="cuda")
    x[0, :4] = torch.tensor([0.0, -0.0, 1e-40, 65504.0])
    y, _ = lv.encode(x, "bf16")
    assert torch.equal(y.view(torch.int16), x.to(torch.bfloat16).view(torch.int16))


def test_fp8_encode_matches_ocp_e4m3fn():
    D = 40
    x = torch.as_tensor(philox.normal(31, 0, 3000 * D).reshape(3000, D), device="cuda")
    x[:, 3] = 0.0                          # all-zero channel: scale 1
    x[:5, 7] = torch.tensor([1e-6, -2e-3, 5e-5, 3.0, -3.0], device="cuda")
    y, sc = lv.encode(x, "fp8")
    # reference on the CPU: FP32 quotients correctly rounded via FP64
    xc = x.cpu().double()
    amax = xc.abs().amax(0)
    ref_scale = torch.where(amax > 0, amax / 448.0, torch.ones_like(amax)).float()
    assert torch.equal(sc.cpu(), ref_scale)
    q = (xc / ref_scale.double()).float().clamp(-448, 448).to(torch.float8_e4m3fn)
    assert torch.equal(y.cpu(), q.view(torch.uint8))


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_low_precision_storage_within_stated_bounds(dtype):
    """D = 384 maps stored in BF16 or FP8 (per-channel absmax scales), FP32
    accumulation.  Against the oracle on the FP32 maps the error obeys the
    closed-form bound (f is a convex combination of the stored values):
    BF16 |df| <= 2^-8 a + 1e-4 a;  FP8 |df| <= 2^-4 a + 2^-10 scale + 1e-4 a.
    Against the oracle on the decoded maps it is the FP32 bar (1e-4)."""
    D = 384
    w = scenes.WORKLOADS["large"]
    sc = scenes.make_scene(w.seed, 20000, w.scale_mu, w.scale_sd, w.op_mu, w.op_sd)
    cams = [scenes.look_at(e, 160, 120, 55.0) for e in scenes.fibonacci_eyes(3, 4.0)]
    low = [scenes.map_lowres(w.seed, v, 120, 160, D) for v in range(3)]
    maps32 = [scenes.upsample(l, 120, 160, "cuda") for l in low]
    enc = [lv.encode(m, dtype) for m in maps32]
    gs = lv.Scene.from_arrays(sc)
    acc = lv.Accum(gs, D)
    if dtype == "bf16":
        acc.add(cams, [e[0] for e in enc], dtype="bf16")
        dec = [e[0].float() for e in enc]
    else:
        scales = torch.stack([e[1] for e in enc]).contiguous()
        acc.add(cams, [e[0] for e in enc], dtype="fp8", scales=scales)
        dec = [e[0].view(torch.float8_e4m3fn).float() * e[1] for e in enc]
    f, b = acc.finalize()
    f = f.cpu().numpy()
    ref32 = oracle.uplift(sc, cams, [m.cpu().numpy() for m in maps32])
    refq = oracle.uplift(sc, cams, [m.cpu().numpy() for m in dec])
    assert feature_error(f, refq).max() < 1e-4
    seen = (ref32.beta > 0) & ref32.strict  # no ambiguous decision
    d = np.abs(f[seen] - ref32.f[seen])
    a = ref32.a[seen]
    if dtype == "bf16":
        bound = 2.0 ** -8 * a + 1e-4 * a
    else:
        smax = max(float(e[1].max()) for e in enc)
        bound = 2.0 ** -4 * a + 2.0 ** -10 * smax + 1e-4 * a
    print(f"{dtype}: max |df|/a = {np.max(d / np.maximum(a, 1e-30)):.3e}")
    assert np.all(d <= bound)


def gpu_graph(n, k, seed, D):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (n, 3))
    feats = rng.normal(size=(n, 8))
    rp, col, val = graph.knn_graph(x, feats, k)
    return rp, col, val


@pytest.mark.parametrize("D,steps", [(1, 10), (3, 5), (64, 20), (70, 3), (8, 0), (8, 6), (12, 4), (4, 6), (16, 5),
                                     (32, 4), (384, 3)])
def test_diffuse_fp32_parity(D, steps):
    n = 5000
    rp, col, val = gpu_graph(n, 16, D, D)
    g0 = philox.uniform(40 + D, 0, n * D).reshape(n, D)
    g0[:, 0] = 0.0  # a zero channel stays zero
    G = lv.Graph(torch.as_tensor(rp, device="cuda"), torch.as_tensor(col, device="cuda"),
                 torch.as_tensor(val, device="cuda"))
    out = G.diffuse(torch.as_tensor(g0, device="cuda"), steps).cpu().numpy().astype(np.float64)
    ref = od.diffuse(od.csr_matrix(n, rp, col, val), g0.astype(np.float64), steps)
    assert np.all(out[:, 0] == 0) or steps == 0
    scale = np.maximum(np.max(np.abs(ref), axis=0), 1e-30)
    err = np.max(np.abs(out - ref) / scale)
    print(f"diffuse D={D} steps={steps}: max err {err:.3e}")
    assert err < 1e-5


@pytest.mark.parametrize("D,gdt", [(64, "f32"), (32, "f32"), (64, "bf16"), (32, "bf16"), (16, "f32")])
def test_diffuse_ragged_degrees(D, gdt):
    """Rows of very different degrees in one wave: empty rows (also at the
    start and end), rows of 1-20 edges and hubs of 100-300 edges (several
    64-edge chunks of a wave's edge range), n not a multiple of any row
    tile; FP32 against the FP64 oracle, BF16 storage against the oracle that
    rounds every iterate to BF16."""
    n, steps = 3001, 4
    rng = np.random.default_rng(7 + D)
    deg = rng.integers(1, 21, n)
    deg[rng.random(n) < 0.3] = 0
    hubs = rng.choice(n, 12, replace=False)
    deg[hubs] = rng.integers(100, 301, 12)
    deg[:3] = 0
    deg[-2:] = 0
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum(deg)
    col = rng.integers(0, n, rp[-1]).astype(np.int32)
    val = rng.uniform(0.1, 1.0, rp[-1]).astype(np.float32)
    g0 = philox.uniform(60 + D, 1, n * D).reshape(n, D)
    dt = torch.float32 if gdt == "f32" else torch.bfloat16
    G = lv.Graph(torch.as_tensor(rp, device="cuda"), torch.as_tensor(col, device="cuda"),
                 torch.as_tensor(val, device="cuda"))
    gin = torch.as_tensor(g0, device="cuda").to(dt)
    out = G.diffuse(gin, steps).float().cpu().numpy().astype(np.float64)
    A = od.csr_matrix(n, rp, col, val)
    if gdt == "f32":
        ref = od.diffuse(A, g0.astype(np.float64), steps)
        tol = 1e-5
    else:
        ref = od.diffuse(A, gin.float().cpu().numpy().astype(np.float64), steps, store="bf16")
        tol = 2.0 ** -7
    assert np.all(out[deg == 0] == 0)
    scale = np.maximum(np.max(np.abs(ref), axis=0), 1e-30)
    err = np.max(np.abs(out - ref) / scale)
    print(f"ragged degrees D={D} {gdt}: max err {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("D,vdt", [(1, "f32"), (64, "f32"), (5, "bf16")])
def test_diffuse_locality_order(D, vdt):
    """With the scene given, rows run in the Morton order of the centres
    (P A P^T, undone on output): same result as the caller's order, and as
    the oracle."""
    sc = scenes.make_scene(12, 6000, -4.0, 0.5, 0.0, 1.0)
    gs = lv.Scene.from_arrays(sc)
    feats = philox.normal(12, 1, sc.n * 8).reshape(sc.n, 8)
    rp, col, val = graph.knn_graph(sc.means, feats, 16)
    dt = torch.float32 if vdt == "f32" else torch.bfloat16
    G = lv.Graph(torch.as_tensor(rp, device="cuda"), torch.as_tensor(col, device="cuda"),
                 torch.as_tensor(val, device="cuda").to(dt))
    g0 = torch.as_tensor(philox.uniform(13, D, sc.n * D).reshape(sc.n, D), device="cuda").to(dt)
    a = G.diffuse(g0, 30, scene=gs).float().cpu().numpy().astype(np.float64)
    b = G.diffuse(g0, 30).float().cpu().numpy().astype(np.float64)
    a2 = G.diffuse(g0, 30, scene=gs).float().cpu().numpy().astype(np.float64)  # cached order
    aval = val if vdt == "f32" else torch.as_tensor(val).to(dt).float().numpy()
    ref = od.diffuse(od.csr_matrix(sc.n, rp, col, aval), g0.float().cpu().numpy(), 30)
    scale = np.max(np.abs(ref), axis=0)
    tol = 1e-5 if vdt == "f32" else 30 * 2.0 ** -9
    assert np.max(np.abs(a - a2) / scale) < (1e-6 if vdt == "f32" else 2.0 ** -7)  # norm sums are atomics
    assert np.max(np.abs(a - ref) / scale) < tol and np.max(np.abs(b - ref) / scale) < tol
    if vdt == "f32":
        assert np.max(np.abs(a - b) / scale) < 1e-5


def test_diffuse_bf16_storage_and_constant_signal():
    n, D, steps = 4000, 16, 10
    rp, col, val = gpu_graph(n, 16, 3, D)
    A = od.csr_matrix(n, rp, col, val)
    G = lv.Graph(torch.as_tensor(rp, device="cuda"), torch.as_tensor(col, device="cuda"),
                 torch.as_tensor(val, device="cuda").to(torch.bfloat16))
    # constant signal: row-stochastic A keeps it constant (up to BF16 rounding)
    ones = torch.ones((n, 1), device="cuda", dtype=torch.bfloat16)
    c = G.diffuse(ones, steps).float().cpu().numpy()
    assert np.allclose(c, 1.0 / np.sqrt(n), rtol=2e-2)
    g0 = philox.uniform(50, 0, n * D).reshape(n, D)
    g0b = torch.as_tensor(g0, device="cuda").to(torch.bfloat16)
    Ab = od.csr_matrix(n, rp, col, torch.as_tensor(val).to(torch.bfloat16).float().numpy())
    for T in (1, 3, 5, steps):
        out = G.diffuse(g0b, T).float().cpu().numpy()
        # the FP64 oracle with each iterate stored in BF16, as the path stores
        # it: the GPU's FP32 sums and norms round to the other neighbour only
        # near BF16 ties, one BF16 ulp (2^-8 relative) of that element, and a
        # row-stochastic A averages such flips instead of growing them
        ref = od.diffuse(Ab, g0b.float().cpu().numpy(), T, store="bf16")
        err = np.max(np.abs(out - ref) / np.max(np.abs(ref), axis=0))
        exact = np.mean(out == ref)
        # and the FP64 iterates without storage rounding: at most 2^-9 per step
        ref64 = od.diffuse(Ab, g0b.float().cpu().numpy(), T)
        err64 = np.max(np.abs(out - ref64) / np.max(np.abs(ref64), axis=0))
        print(f"diffuse bf16 T={T}: max err {err:.3e} vs BF16-stored oracle "
              f"({exact:.4f} of the values equal), {err64:.3e} vs FP64 iterates")
        assert err <= 2.0 ** -7
        assert err64 <= T * 2.0 ** -9 + 2.0 ** -7


def test_large_full_size_precision_sampled():
    """The large configuration at full size: 1,000,000 Gaussians (scales
    exp(N(-5, 0.7^2)), opacities sigmoid(N(0.5, 1))), 1008x756 views, D = 384
    maps (N(0,1) at 1/14 resolution, upsampled), stored FP32 (HWC), BF16 and
    FP8 (pixel blocks) with FP32 accumulation, 5 of the 100 rig views.  The oracle walks every pixel and
    accumulates a 20,000-Gaussian sample (drawn without replacement); counts
    and weight sums are compared for all Gaussians."""
    w = scenes.WORKLOADS["large"]
    sc = scenes.scene_for(w)
    rig = scenes.cameras_for(w)
    views = [0, 20, 40, 60, 80]
    cams = [rig[v] for v in views]
    gs = lv.Scene.from_arrays(sc)
    rows = scenes.subsample(2, sc.n, 20000)
    print("large: maps", flush=True)
    maps32 = [scenes.feature_map(w, v, device="cuda") for v in views]
    results = {}
    for dtype in ("f32", "bf16", "fp8"):
        acc = lv.Accum(gs, w.D, counts=True)
        smax = 0.0
        if dtype == "f32":
            acc.add(cams, maps32)
            dec = maps32
        else:
            # pixel-block storage, the layout the headline bench times
            enc = [lv.encode(m, dtype + "_px8") for m in maps32]
            Wd = maps32[0].shape[1]
            if dtype == "bf16":
                acc.add(cams, [e[0] for e in enc], dtype="bf16_px8")
                dec = [px8_to_hwc(e[0].float(), Wd) for e in enc]
            else:
                scales = torch.stack([e[1] for e in enc]).contiguous()
                acc.add(cams, [e[0] for e in enc], dtype="fp8_px8", scales=scales)
                dec = [px8_to_hwc(e[0].view(torch.float8_e4m3fn).float(), Wd) * e[1] for e in enc]
            if dtype == "fp8":
                smax = max(float(e[1].max()) for e in enc)
            del enc
        f, b = acc.finalize()
        c = acc.counts().cpu().numpy().astype(np.int64)
        f = f.cpu().numpy()[rows]
        b = b.cpu().numpy()
        acc.close()
        print(f"large {dtype}: oracle", flush=True)
        up = oracle.Uplifter(sc, w.D, rows=rows)
        for k, cam in enumerate(cams):
            up.add_view(cam, dec[k].cpu().numpy())
        ref = up.result()
        del dec
        assert counts_match(c, ref)
        assert beta_error(b, ref).max() < 1e-4
        e = feature_error(f, ref)
        print(f"large {dtype} vs decoded maps: max {e.max():.3e}", flush=True)
        assert e.max() < 1e-4
        results[dtype] = (f, smax)
    # low-precision results against the FP32 result's oracle (same rows)
    up = oracle.Uplifter(sc, w.D, rows=rows)
    for k, cam in enumerate(cams):
        up.add_view(cam, maps32[k].cpu().numpy())
    ref32 = up.result()
    seen = (ref32.beta[rows] > 0) & ref32.strict[rows]  # no ambiguous decision
    a = ref32.a[seen]
    for dtype, (f, smax) in results.items():
        d = np.abs(f[seen] - ref32.f[seen])
        bound = {"f32": 1e-4 * a, "bf16": 2.0 ** -8 * a + 1e-4 * a,
                 "fp8": 2.0 ** -4 * a + 2.0 ** -10 * smax + 1e-4 * a}[dtype]
        print(f"large {dtype} vs FP32 maps: max |df|/a {np.max(d / np.maximum(a, 1e-30)):.3e}")
        assert np.all(d <= bound)


def px8_to_hwc(t, W):
    """[H, ceil(W/8), D, 8] -> [H, W, D] (the inverse of px8_reference)."""
    H, W8, D, _ = t.shape
    return t.permute(0, 1, 3, 2).reshape(H, W8 * 8, D)[:, :W]


def px8_reference(a):
    """[H, W, D] -> [H, ceil(W/8), D, 8] (pixels past W zero), on the CPU."""
    H, W, D = a.shape
    W8 = (W + 7) // 8
    p = torch.zeros((H, W8 * 8, D), dtype=a.dtype)
    p[:, :W] = a
    return p.reshape(H, W8, 8, D).permute(0, 1, 3, 2).contiguous()


@pytest.mark.parametrize("dtype", ["f32_px8", "bf16_px8", "fp8_px8"])
def test_pixel_block_encode_bit_exact(dtype):
    """lv_encode_map's pixel-block layout: the HWC encoding's values (BF16
    round to nearest even, FP8 E4M3FN with per-channel absmax scales, FP32
    copied) moved to [H][ceil(W/8)][D][8] with zero padding, bit for bit, on a
    width that is not a multiple of 8."""
    H, W, D = 13, 37, 20
    x = torch.as_tensor(philox.normal(32, 0, H * W * D).reshape(H, W, D), device="cuda")
    x[0, 0, :3] = torch.tensor([0.0, -0.0, 1e-40], device="cuda")
    y, sc = lv.encode(x, dtype)
    assert tuple(y.shape) == (H, (W + 7) // 8, D, 8)
    if dtype == "f32_px8":
        ref = px8_reference(x.cpu())
        assert torch.equal(y.cpu().view(torch.int32), ref.view(torch.int32))
    elif dtype == "bf16_px8":
        ref = px8_reference(x.cpu().to(torch.bfloat16))
        assert torch.equal(y.cpu().view(torch.int16), ref.view(torch.int16))
    else:
        hwc, sc_hwc = lv.encode(x.reshape(H * W, D), "fp8")
        assert torch.equal(sc.cpu(), sc_hwc.cpu())
        ref = px8_reference(hwc.reshape(H, W, D).cpu())
        assert torch.equal(y.cpu(), ref)


@pytest.mark.parametrize("D", [64, 130])
@pytest.mark.parametrize("elem", ["f32", "bf16", "fp8"])
def test_pixel_block_uplift_parity(elem, D):
    """The uplift from pixel-block maps (one vector load per 8 pixels of a
    channel) against the oracle on the decoded maps (counts exact, 1e-4), and
    against the HWC maps of the same values; D = 64 runs the one-group
    quadrant kernel, D = 130 the several-group half-tile kernel.  Ragged
    image (97 x 83).  A channel slice of wider pixel-block maps too."""
    sc = scenes.make_scene(15, 3000, -3.8, 0.5, 0.0, 1.0)
    cams = [scenes.look_at(e, 97, 83, 60.0) for e in scenes.fibonacci_eyes(2, 4.0)]
    gs = lv.Scene.from_arrays(sc)
    Dw = D + 6  # the stored maps hold D + 6 channels; the uplift reads the first D
    src = [torch.as_tensor(philox.normal(150 + D, v, 83 * 97 * Dw).reshape(83, 97, Dw), device="cuda")
           for v in range(2)]
    hwc = [lv.encode(m[..., :D].contiguous(), elem) for m in src]
    px = [lv.encode(m, elem + "_px8") for m in src]
    if elem == "fp8":
        # the scales of the wider map's first D channels are those of the narrower map
        assert all(torch.equal(a[1], b[1][:D]) for a, b in zip(hwc, px))
        scales = torch.stack([e[1] for e in hwc]).contiguous()
        dec = [e[0].view(torch.float8_e4m3fn).float() * e[1] for e in hwc]
    else:
        scales = None
        dec = [e[0].float() for e in hwc]
    ref = oracle.uplift(sc, cams, [d.cpu().numpy() for d in dec])
    outs = {}
    for name, maps, dt in (("hwc", [e[0] for e in hwc], elem),
                           ("px8", [e[0][:, :, :D, :] for e in px], elem + "_px8")):
        acc = lv.Accum(gs, D, counts=True)
        lv.accumulate_sets(cams, [(acc, maps, scales)], dtype=dt)
        f, b = acc.finalize()
        torch.cuda.synchronize()
        assert counts_match(acc.counts().cpu().numpy(), ref), name
        e = feature_error(f.cpu().numpy(), ref)
        print(f"px8 parity {elem} D={D} {name}: max err {e.max():.3e}", flush=True)
        assert e.max() < 1e-4, name
        assert beta_error(b.cpu().numpy(), ref).max() < 1e-4, name
        outs[name] = f.cpu().numpy()
    assert np.abs(outs["hwc"] - outs["px8"]).max() <= 1e-5 * max(1.0, np.abs(outs["hwc"]).max())
