"""Forward render (Eq. 4) through the C ABI: against the FP64 oracle's render,
and as the adjoint of the uplift's raw sums W^T F."""
import numpy as np
import pytest
import torch

import oracle
import paper_2410_14462_amd as lv
from synth import philox, scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    sc = scenes.make_scene(31, 3000, -3.8, 0.5, 0.0, 1.0)
    cams = [scenes.look_at(e, 96, 80, 60.0) for e in scenes.fibonacci_eyes(3, 4.0)]
    cams.append(scenes.look_at([0.3, 0.2, 0.6], 77, 45, 90.0))  # inside the cloud, ragged tiles
    return sc, cams, lv.Scene.from_arrays(sc)


@pytest.mark.parametrize("D", [1, 5, 40, 64, 70])
def test_render_matches_oracle(setup, D):
    sc, cams, gs = setup
    g = philox.normal(40 + D, 0, sc.n * D).reshape(sc.n, D)
    outs, alphas = gs.render(cams, torch.as_tensor(g, device="cuda"))
    for v, cam in enumerate(cams):
        # pixels with an ambiguous skip/stop decision (relative margin below
        # 1e-5) are excluded and counted
        ref, ref_a, amb = oracle.render(sc, cam, g, amb_px=True)
        scale, _ = oracle.render(sc, cam, np.abs(g))  # sum_i w_i(p) |g_i|
        got = outs[v].cpu().numpy().astype(np.float64)
        err = np.abs(got - ref) / np.maximum(scale, 1e-30)
        ok = ~amb
        print(f"render D={D} view {v}: max err {err[ok].max():.3e}, ambiguous pixels {int(amb.sum())}")
        assert amb.sum() <= 0.001 * amb.size
        assert err[ok].max() < 1e-4
        assert np.abs(alphas[v].cpu().numpy() - ref_a)[ok].max() < 1e-5
        assert np.all(ref_a <= 1.0 + 1e-12)


def test_render_is_the_adjoint_of_the_uplift(setup):
    """<W g, F> = <g, W^T F> over all views, with W^T F the uplift's raw sums."""
    sc, cams, gs = setup
    D = 7
    g = torch.as_tensor(philox.normal(50, 0, sc.n * D).reshape(sc.n, D), device="cuda")
    maps = [torch.as_tensor(philox.normal(51, v, c.height * c.width * D).reshape(c.height, c.width, D),
                            device="cuda") for v, c in enumerate(cams)]
    outs, _ = gs.render(cams, g, alpha=False)
    lhs = sum(float((o.double() * m.double()).sum()) for o, m in zip(outs, maps))
    acc = lv.Accum(gs, D)
    acc.add(cams, maps)
    _, _, U = acc.finalize(want_sum=True)
    rhs = float((g.double() * U.double()).sum())
    mag = sum(float((o.double().abs() * m.double().abs()).sum()) for o, m in zip(outs, maps))
    print(f"adjoint: {lhs:.6e} vs {rhs:.6e} (scale {mag:.3e})")
    assert abs(lhs - rhs) <= 1e-5 * mag


def test_render_empty_view_and_bad_args(setup):
    sc, cams, gs = setup
    away = scenes.look_at([0, 0, 40.0], 64, 48, 60.0)
    away.t = -away.t  # the cloud is behind this camera
    # outputs filled with NaN first: the render writes every pixel, zeros
    # where no Gaussian reaches
    out = torch.full((48, 64, 3), float("nan"), device="cuda")
    alpha = torch.full((48, 64), float("nan"), device="cuda")
    outs, alphas = gs.render([away], torch.ones((sc.n, 3), device="cuda"), outs=([out], [alpha]))
    torch.cuda.synchronize()
    assert torch.all(outs[0] == 0) and torch.all(alphas[0] == 0)
    with pytest.raises(lv.LvError):
        gs.render(cams[:1], torch.ones((sc.n + 1, 3), device="cuda"))


def test_render_full_size_view():
    """The render benchmark's configuration on one view: the 1M-Gaussian
    scene, a 1008 x 756 camera of its rig, D = 384 FP32 features, written into
    caller-provided outputs; every pixel against the oracle's render (pixels
    with an ambiguous skip/stop decision excluded and counted)."""
    w = scenes.WORKLOADS["large"]
    sc = scenes.scene_for(w)
    cam = scenes.cameras_for(w)[0]
    gs = lv.Scene.from_arrays(sc)
    D = w.D
    g = np.random.default_rng(2024).standard_normal((sc.n, D), dtype=np.float32)
    out = torch.full((cam.height, cam.width, D), float("nan"), device="cuda")
    alpha = torch.full((cam.height, cam.width), float("nan"), device="cuda")
    outs, alphas = gs.render([cam], torch.as_tensor(g, device="cuda"), outs=([out], [alpha]))
    assert outs[0] is out and alphas[0] is alpha
    got = out.cpu().numpy().astype(np.float64)
    got_a = alpha.cpu().numpy()
    gs.close()
    print("render full-size view: oracle", flush=True)
    ref, ref_a, amb = oracle.render(sc, cam, g, amb_px=True)
    scale, _ = oracle.render(sc, cam, np.abs(g))
    err = np.abs(got - ref) / np.maximum(scale, 1e-30)
    ok = ~amb
    print(f"render full-size view: max err {err[ok].max():.3e}, ambiguous pixels {int(amb.sum())}", flush=True)
    assert amb.sum() <= 0.001 * amb.size
    assert err[ok].max() < 1e-4
    assert np.abs(got_a - ref_a)[ok].max() < 1e-5


def test_render_of_a_scene_without_gaussians():
    """n = 0: no kernel runs, and every output and opacity is set to 0 (the
    outputs are filled with NaN first)."""
    from synth.scenes import Scene
    empty = Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                  np.zeros((0, 4), np.float32), np.zeros(0, np.float32))
    cams = [scenes.look_at([0, 0, 4.0], 64, 48, 60.0), scenes.look_at([0, 4.0, 0.5], 33, 17, 50.0)]
    g0 = lv.Scene.from_arrays(empty)
    outs = [torch.full((c.height, c.width, 5), float("nan"), device="cuda") for c in cams]
    alps = [torch.full((c.height, c.width), float("nan"), device="cuda") for c in cams]
    g0.render(cams, torch.zeros((0, 5), device="cuda"), outs=(outs, alps))
    torch.cuda.synchronize()
    for o, a in zip(outs, alps):
        assert torch.all(o == 0) and torch.all(a == 0)
    g0.close()
