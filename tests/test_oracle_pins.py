"""Pins for the FP64 uplifting oracle: closed forms, invariants, a library
rotation, a finite-difference projection and brute force on tiny scenes.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, a transposed operand, a wrong constant, an off-by-half pixel
centre, a wrong tile bound) breaks at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from synth import philox, scenes
from synth.scenes import Camera, Scene

F32 = np.float32
ALPHA_MAX = float(F32(0.99))
ALPHA_MIN = float(F32(1.0) / F32(255.0))
T_EPS = float(F32(1e-4))


def one_scene(means, scales, quats=None, opacity=None):
    means = np.asarray(means, F32).reshape(-1, 3)
    n = means.shape[0]
    scales = np.asarray(scales, F32).reshape(n, 3)
    quats = np.tile(np.array([1, 0, 0, 0], F32), (n, 1)) if quats is None else np.asarray(quats, F32)
    opacity = np.full(n, 0.5, F32) if opacity is None else np.asarray(opacity, F32).reshape(n)
    return Scene(means, scales, quats, opacity)


def axis_camera(f, W=129, H=129, z0=4.0):
    """Camera at (0,0,-z0) looking along +z (R = I), principal point at the centre."""
    return Camera(np.eye(3, dtype=F32), np.array([0, 0, z0], F32), f, f, W / 2.0, H / 2.0, W, H, 0.01)


# --------------------------------------------------------------------- RNG
def test_philox_known_answers():
    path = __file__.replace("test_oracle_pins.py", "golden/philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(*v[:6])
        assert [int(x) for x in out] == v[6:]


def test_generators_are_counter_based():
    a = philox.normal(7, 3, 1000)
    b = philox.normal(7, 3, 10, start=200)  # blocks 200.. -> normals 400..
    assert np.array_equal(a[400:410], b)
    u = philox.uniform(7, 3, 4001)
    assert u.min() > 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.02


# ------------------------------------------------------------ S32 helpers
def test_covariance_factor_matches_library_rotation():
    """M = R diag(s) against scipy's quaternion rotation, and M M^T against the
    covariance R diag(s)^2 R^T (Sec. 3.1)."""
    rng = np.random.default_rng(3)
    q = rng.normal(size=(500, 4)).astype(F32)
    s = np.exp(rng.normal(-3, 0.7, size=(500, 3))).astype(F32)
    M = oracle.factor32(s, q).astype(np.float64)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]].astype(np.float64)).as_matrix()  # scalar-last
    ref = R * s.astype(np.float64)[:, None, :]
    assert np.max(np.abs(M - ref) / s.max(1)[:, None, None]) < 1e-6
    full = R @ (np.square(s.astype(np.float64))[:, :, None] * np.transpose(R, (0, 2, 1)))
    scale = np.max(np.abs(full), axis=(1, 2))[:, None, None]
    assert np.max(np.abs(M @ M.transpose(0, 2, 1) - full) / scale) < 2e-6


# --------------------------------------------------- single-Gaussian forms
def single_closed_form(cam, u, vx, vy, op, tiles, F):
    """Exact uplift of one Gaussian with diagonal 2D covariance diag(vx, vy):
    alpha(p) = min(0.99, op exp(-dx^2/(2vx) - dy^2/(2vy))) on its tiles, kept
    where alpha >= 1/255.  Returns (beta, U, count, min decision margin)."""
    W, H = cam.width, cam.height
    ys, xs = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    dx, dy = xs - u[0], ys - u[1]
    al = np.minimum(ALPHA_MAX, float(F32(op)) * np.exp(-dx * dx / (2 * vx) - dy * dy / (2 * vy)))
    (tx0, ty0, tx1, ty1) = tiles
    tx, ty = np.floor(xs / 16), np.floor(ys / 16)
    sup = (tx >= tx0) & (tx < tx1) & (ty >= ty0) & (ty < ty1)
    keep = sup & (al >= ALPHA_MIN)
    margin = np.min(np.abs(al[sup] - ALPHA_MIN) / ALPHA_MIN)
    beta = al[keep].sum()
    U = (al[keep][:, None] * F[keep]).sum(0)
    return beta, U, int(keep.sum()), margin


def tiles_for(u, v_max, W, H):
    r = math.ceil(3 * math.sqrt(v_max))
    TX, TY = -(-W // 16), -(-H // 16)
    return (max(0, math.floor((u[0] - r) / 16)), max(0, math.floor((u[1] - r) / 16)),
            min(TX, math.floor((u[0] + r) / 16) + 1), min(TY, math.floor((u[1] + r) / 16) + 1))


@pytest.mark.parametrize("s,op", [(0.05, 0.8), (0.406, 1.0), (0.3, 0.3)])
def test_single_isotropic_on_axis(s, op):
    f, z0 = 100.0, 4.0
    cam = axis_camera(f, z0=z0)
    sc = one_scene([0, 0, 0], [s, s, s], opacity=[op])
    v = (f * float(F32(s)) / z0) ** 2 + float(F32(0.3))
    u = (64.5, 64.5)
    tiles = tiles_for(u, v, 129, 129)
    F = philox.uniform(11, 1, 129 * 129 * 3).reshape(129, 129, 3).astype(np.float64)
    beta, U, cnt, margin = single_closed_form(cam, u, v, v, op, tiles, F)
    assert margin > 1e-4
    r = oracle.uplift(sc, [cam], [F.astype(F32)])
    assert r.count[0] == cnt
    assert r.beta[0] == pytest.approx(beta, rel=1e-9)
    assert np.allclose(r.U[0], U, rtol=1e-9, atol=0)
    st = oracle.structure(sc, cam)
    assert tuple(st.rect[0]) == tiles
    # the centre pixel (64, 64) sits exactly on the mean: alpha = min(0.99, op)
    _, alpha = oracle.render(sc, cam, np.ones((1, 1)))
    assert alpha[64, 64] == min(ALPHA_MAX, float(F32(op)))


def test_tile_support_truncates():
    """s = 0.406: the alpha >= 1/255 disc (radius ~34 px) is wider than the tile
    rectangle grown from ceil(3 sqrt(lambda)) (edges 32.5 / 31.5 px away):
    pixels outside the tiles must not count."""
    f, z0, s = 100.0, 4.0, 0.406
    cam = axis_camera(f, z0=z0)
    sc = one_scene([0, 0, 0], [s, s, s], opacity=[1.0])
    v = (f * float(F32(s)) / z0) ** 2 + float(F32(0.3))
    tiles = tiles_for((64.5, 64.5), v, 129, 129)
    F = np.ones((129, 129, 1))
    b_sup, _, c_sup, _ = single_closed_form(cam, (64.5, 64.5), v, v, 1.0, tiles, F)
    b_all, _, c_all, _ = single_closed_form(cam, (64.5, 64.5), v, v, 1.0, (0, 0, 9, 9), F)
    assert c_all > c_sup  # truncation really happens in this setup
    r = oracle.uplift(sc, [cam], [F.astype(F32)])
    assert r.count[0] == c_sup and r.beta[0] == pytest.approx(b_sup, rel=1e-9)


def test_single_off_axis_shift_and_jacobian():
    """Mean at x = 0.5, z = 4, f = 128: the peak moves by f x / z = 16 px and the
    EWA covariance is s^2 (f/z)^2 diag(1 + (x/z)^2, 1) + 0.3."""
    f, z0, s, op = 128.0, 4.0, 0.1, 0.7
    cam = axis_camera(f, z0=z0)
    sc = one_scene([0.5, 0, 0], [s, s, s], opacity=[op])
    k = (f * float(F32(s)) / z0) ** 2
    vx, vy = k * (1 + 0.125 ** 2) + float(F32(0.3)), k + float(F32(0.3))
    u = (64.5 + 16.0, 64.5)
    tiles = tiles_for(u, max(vx, vy), 129, 129)
    F = philox.uniform(12, 1, 129 * 129 * 2).reshape(129, 129, 2).astype(np.float64)
    beta, U, cnt, margin = single_closed_form(cam, u, vx, vy, op, tiles, F)
    assert margin > 1e-4
    r = oracle.uplift(sc, [cam], [F.astype(F32)])
    assert r.count[0] == cnt and r.beta[0] == pytest.approx(beta, rel=1e-9)
    assert np.allclose(r.U[0], U, rtol=1e-9)
    _, alpha = oracle.render(sc, cam, np.ones((1, 1)))
    assert alpha[64, 80] == pytest.approx(op, rel=1e-7)
    assert np.unravel_index(np.argmax(alpha), alpha.shape) == (64, 80)


def test_jacobian_clamp():
    """Mean at x/z = 5 with f = 20 (limit 1.3 * 64.5 / 20 = 4.1925): the x
    column of the Jacobian uses the clamped 4.1925, not 5."""
    f, z0, s, op = 20.0, 4.0, 1.0, 0.9
    cam = axis_camera(f, z0=z0)
    sc = one_scene([20.0, 0, 0], [s, s, s], opacity=[op])
    lim = float(F32(1.3)) * (64.5 / f)
    k = (f / z0) ** 2
    vx, vy = k * (1 + lim ** 2) + float(F32(0.3)), k + float(F32(0.3))
    u = (f * 5.0 + 64.5, 64.5)
    tiles = tiles_for(u, max(vx, vy), 129, 129)
    F = np.ones((129, 129, 1))
    beta, _, cnt, margin = single_closed_form(cam, u, vx, vy, op, tiles, F)
    assert margin > 1e-4 and cnt > 0
    r = oracle.uplift(sc, [cam], [F.astype(F32)])
    assert r.count[0] == cnt and r.beta[0] == pytest.approx(beta, rel=1e-7)
    # unclamped covariance would give a different weight sum
    vx_u = k * 26 + float(F32(0.3))
    b_u, _, _, _ = single_closed_form(cam, u, vx_u, vy, op, tiles_for(u, vx_u, 129, 129), F)
    assert abs(b_u - beta) / beta > 1e-2


def test_termination_at_T_eps():
    """14 wide Gaussians stacked on the axis with opacity 0.5: alpha = 0.5 at the
    centre pixel, T_k = 2^-k; the 14th would take T to 2^-14 < 1e-4, so exactly
    13 count and the weights are 2^-1 .. 2^-13."""
    n = 14
    means = np.array([[0, 0, 0.1 * k] for k in range(n)], F32)
    sc = one_scene(means, np.full((n, 3), 0.5), opacity=np.full(n, 0.5))
    cam = axis_camera(100.0)
    out, alpha = oracle.render(sc, cam, np.eye(n))
    assert alpha[64, 64] == 1.0 - 2.0 ** -13
    assert np.array_equal(out[64, 64], np.array([2.0 ** -(k + 1) for k in range(13)] + [0.0]))


def test_alpha_clamp_uses_fp32_constants():
    """Two opaque Gaussians: alpha = 0.99f, then T' = (1 - 0.99f)^2 = 9.99998e-5
    < 1e-4f, so the second is excluded (with decimal 0.99 it would count).  The
    margin, 1.9e-6 relative, is below the ambiguity threshold: the pixel is
    reported ambiguous, and the second Gaussian flagged, the first not."""
    means = np.array([[0, 0, 0], [0, 0, 0.1]], F32)
    sc = one_scene(means, np.full((2, 3), 0.5), opacity=np.ones(2))
    cam = axis_camera(100.0)
    out, alpha, amb = oracle.render(sc, cam, np.eye(2), amb_px=True)
    assert alpha[64, 64] == ALPHA_MAX
    assert out[64, 64, 1] == 0.0
    assert amb[64, 64]
    r = oracle.uplift(sc, [cam], [np.ones((129, 129, 1), F32)])
    t_next = (1.0 - ALPHA_MAX) ** 2
    assert r.margin_stop == pytest.approx(abs(t_next - T_EPS) / T_EPS, rel=1e-9)
    assert r.margin_stop < oracle.AMB_THR and r.amb[1] >= 1


# ------------------------------------------------------ decision margins
def _centre_counts(sc, cam):
    up = oracle.Uplifter(sc, 1)
    amb = up.add_view(cam, np.ones((cam.height, cam.width, 1), F32), amb_px=True)
    return up.result(), amb


def test_alpha_next_to_skip_threshold_is_flagged():
    """A Gaussian centred on pixel (64, 64) has alpha = opacity there (power 0).
    With the opacity one FP32 ulp above 1/255 (4.7e-10 above it, relative
    margin 1.2e-7) it counts
    and the pixel is ambiguous; one ulp below, it is skipped and the pixel is
    still ambiguous; 1e-3 above, nothing is ambiguous.  A wide Gaussian in
    front keeps its weight and is not flagged; one behind is flagged (its T
    depends on the decision)."""
    amin32 = F32(1.0) / F32(255.0)
    up1 = float(np.nextafter(amin32, F32(1)))
    dn1 = float(np.nextafter(amin32, F32(0)))
    cam = axis_camera(100.0)
    means = np.array([[0, 0, -0.2], [0, 0, 0], [0, 0, 0.2]], F32)
    scales = np.array([[0.2] * 3, [0.01] * 3, [0.2] * 3], F32)
    for op, counted, ambiguous in ((up1, 1, True), (dn1, 0, True),
                                   (float(amin32) * 1.001, 1, False)):
        sc = one_scene(means, scales, opacity=[0.5, op, 0.5])
        r, amb = _centre_counts(sc, cam)
        # the small Gaussian counts at the centre pixel only (its neighbours
        # see a quarter of the opacity, far below 1/255)
        assert r.count[1] == counted
        assert bool(amb[64, 64]) == ambiguous and amb.sum() == int(ambiguous)
        assert r.amb_px == int(ambiguous)
        if ambiguous:
            assert r.margin_skip == pytest.approx(abs(op - ALPHA_MIN) / ALPHA_MIN, rel=1e-9)
            assert abs(op - ALPHA_MIN) < 1e-9 and r.margin_skip < 2e-7
            assert list(r.amb) == [0, 1, 1]
        else:
            assert r.margin_skip > 1e-4 and not r.amb.any()


def test_transmittance_next_to_stop_threshold_is_flagged():
    """13 stacked wide Gaussians with opacity 0.5 leave T = 2^-13 at the centre
    pixel; a 14th with opacity fl32(1 - 1e-4f 2^13) gives T' within 1e-7 of
    1e-4: the pixel is ambiguous and only the 14th is flagged there."""
    n = 14
    means = np.array([[0, 0, 0.05 * k] for k in range(n)], F32)
    op14 = F32(1.0 - T_EPS * 2.0 ** 13)
    sc = one_scene(means, np.full((n, 3), 0.5), opacity=[0.5] * 13 + [float(op14)])
    cam = axis_camera(100.0)
    r, amb = _centre_counts(sc, cam)
    t_next = 2.0 ** -13 * (1.0 - float(op14))
    assert abs(t_next - T_EPS) / T_EPS < 1e-7
    assert amb[64, 64]
    assert r.margin_stop == pytest.approx(abs(t_next - T_EPS) / T_EPS, rel=1e-6)
    # flags at the centre pixel alone: from the 14th on (the first 13 keep
    # their weights whatever the stop decides)
    _, _, amb_r = oracle.render(sc, cam, np.eye(n), amb_px=True)
    assert np.array_equal(amb_r, amb.astype(bool))
    only = one_scene(means, np.full((n, 3), 0.5), opacity=[0.5] * 13 + [float(op14)])
    ro = oracle.uplift(only, [cam], [np.ones((129, 129, 1), F32)])
    assert ro.amb[13] >= 1
    if amb.sum() == 1:
        assert not ro.amb[:13].any()


def test_depth_order_front_to_back():
    """The nearer Gaussian takes weight alpha, the farther alpha (1 - alpha'),
    whatever their index order."""
    means = np.array([[0, 0, 0.5], [0, 0, 0.0]], F32)  # index 1 is nearer
    sc = one_scene(means, np.full((2, 3), 0.5), opacity=[0.3, 0.6])
    out, _ = oracle.render(sc, axis_camera(100.0), np.eye(2))
    assert out[64, 64, 1] == pytest.approx(float(F32(0.6)), rel=1e-12)
    assert out[64, 64, 0] == pytest.approx(float(F32(0.3)) * (1 - float(F32(0.6))), rel=1e-12)


def test_behind_camera_and_near_plane():
    sc = one_scene([[0, 0, -4.5], [0, 0, -3.995], [0, 0, 0]], np.full((3, 3), 0.05))
    st = oracle.structure(sc, axis_camera(100.0))
    assert list(st.visible) == [False, False, True]


# ------------------------------------------------------------- invariants
@pytest.fixture(scope="module")
def tiny():
    w = scenes.WORKLOADS["tiny"]
    sc = scenes.scene_for(w)
    cams = scenes.cameras_for(w, m=2, width=96, height=80)
    maps = [philox.uniform(21, v, 80 * 96 * 3).reshape(80, 96, 3) for v in range(2)]
    return sc, cams, maps


def test_weights_telescope(tiny):
    sc, cams, maps = tiny
    up = oracle.Uplifter(sc, 3)
    tf = up.add_view(cams[0], maps[0], tfinal=True)
    _, alpha = oracle.render(sc, cams[0], np.ones((sc.n, 1)))
    assert np.max(np.abs(alpha - (1.0 - tf))) < 1e-12
    assert alpha.max() <= 1.0 and alpha.max() > 0.99


def test_constant_map_uplifts_to_constant(tiny):
    sc, cams, _ = tiny
    c = np.array([0.25, -3.0, 7.5], F32)
    r = oracle.uplift(sc, cams, [np.broadcast_to(c, (80, 96, 3))] * 2)
    seen = r.beta > 0
    assert seen.sum() > 0.5 * sc.n
    assert np.allclose(r.f[seen], c.astype(np.float64), rtol=1e-12, atol=1e-12)
    assert np.all(r.f[~seen] == 0)


def test_linearity_channels_and_views(tiny):
    sc, cams, maps = tiny
    r = oracle.uplift(sc, cams, maps)
    r0 = oracle.uplift(sc, cams, [m[:, :, :1] for m in maps])
    assert np.allclose(r.U[:, :1], r0.U, rtol=1e-12, atol=1e-15)
    mix = [(2.0 * m[:, :, 0] - 0.5 * m[:, :, 2])[:, :, None].astype(F32) for m in maps]
    rm = oracle.uplift(sc, cams, mix)
    ref = 2.0 * np.asarray(r.U[:, 0], np.float64) - 0.5 * r.U[:, 2]
    # F32 rounding of the mixed map is the only difference
    assert np.max(np.abs(rm.U[:, 0] - ref)) <= 1e-6 * np.max(r.A[:, 0] + r.A[:, 2])
    a = oracle.uplift(sc, cams[:1], maps[:1])
    b = oracle.uplift(sc, cams[1:], maps[1:])
    assert np.allclose(a.U + b.U, r.U, rtol=1e-12, atol=1e-15)
    assert np.array_equal(a.count + b.count, r.count)


def test_permutation_equivariance(tiny):
    sc, cams, maps = tiny
    # FP32 depth keys do collide (ties go by index); drop every Gaussian that
    # ties with another in some view so that the order is index-free.
    keep = np.ones(sc.n, bool)
    for cam in cams:
        st = oracle.structure(sc, cam)
        d = np.where(st.visible, st.depth.astype(np.int64), -1 - np.arange(sc.n))
        _, inv, cnt = np.unique(d, return_inverse=True, return_counts=True)
        keep &= cnt[inv] == 1
    assert 0 < (~keep).sum() < 50
    sc = Scene(sc.means[keep], sc.scales[keep], sc.quats[keep], sc.opacity[keep])
    perm = np.random.default_rng(5).permutation(sc.n)
    sp = Scene(sc.means[perm], sc.scales[perm], sc.quats[perm], sc.opacity[perm])
    r = oracle.uplift(sc, cams, maps)
    rp = oracle.uplift(sp, cams, maps)
    assert np.array_equal(rp.count, r.count[perm])
    assert np.allclose(rp.U, r.U[perm], rtol=1e-12, atol=1e-15)


def test_adjoint_of_forward_render(tiny):
    """Sec. 3.2 reads the uplift numerator as W^T F with W the forward render of
    Eq. (4): <W g, F> = <g, W^T F> for any g."""
    sc, cams, maps = tiny
    g = np.random.default_rng(9).normal(size=(sc.n, 3))
    r = oracle.uplift(sc, cams, maps)
    lhs = sum(np.sum(oracle.render(sc, cam, g)[0] * maps[v]) for v, cam in enumerate(cams))
    rhs = np.sum(g * r.U)
    assert lhs == pytest.approx(rhs, rel=1e-11)


def test_structure_lists_are_sorted_rect_members(tiny):
    sc, cams, _ = tiny
    st = oracle.structure(sc, cams[0])
    TX = -(-96 // 16)
    for t in range(len(st.tile_start) - 1):
        ids = st.ids[st.tile_start[t]:st.tile_start[t + 1]]
        tx, ty = t % TX, t // TX
        r = st.rect
        members = np.nonzero(st.visible & (r[:, 0] <= tx) & (tx < r[:, 2]) & (r[:, 1] <= ty) & (ty < r[:, 3]))[0]
        assert set(ids.tolist()) == set(members.tolist())
        d, i = st.depth[ids].astype(np.int64), ids.astype(np.int64)
        assert np.all((d[1:] > d[:-1]) | ((d[1:] == d[:-1]) & (i[1:] > i[:-1])))


# ------------------------------------------------------------ brute force
def brute_force(scene, cams, maps):
    """Independent FP64 uplift for tiny scenes: library rotation, finite-difference
    projection Jacobian, every Gaussian at every pixel (no tiles), one global
    depth order per view, decisions in FP64.  Returns (beta, U, count, margin)."""
    n = scene.n
    q = scene.quats.astype(np.float64)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    S = np.square(scene.scales.astype(np.float64))
    cov = R @ (S[:, :, None] * np.transpose(R, (0, 2, 1)))
    D = maps[0].shape[-1]
    beta, U, cnt = np.zeros(n), np.zeros((n, D)), np.zeros(n, np.int64)
    margin = np.inf
    dil = float(F32(0.3))
    for cam, F in zip(cams, maps):
        F = np.asarray(F, np.float64)
        Rc, t = cam.R.astype(np.float64), cam.t.astype(np.float64)

        def proj(x):
            y = Rc @ x + t
            return np.array([cam.fx * y[0] / y[2] + cam.cx, cam.fy * y[1] / y[2] + cam.cy])

        recs = []
        for i in range(n):
            mu = scene.means[i].astype(np.float64)
            z = (Rc @ mu + t)[2]
            if z <= cam.znear:
                continue
            h = 1e-6
            J = np.stack([(proj(mu + h * e) - proj(mu - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
            S2 = J @ cov[i] @ J.T + dil * np.eye(2)
            recs.append((z, i, proj(mu), np.linalg.inv(S2), float(scene.opacity[i])))
        recs.sort(key=lambda r: (r[0], r[1]))
        for py in range(cam.height):
            for px in range(cam.width):
                p = np.array([px + 0.5, py + 0.5])
                T = 1.0
                for (_, i, u, C, op) in recs:
                    d = p - u
                    al = min(ALPHA_MAX, op * math.exp(min(0.0, -0.5 * d @ C @ d)))
                    margin = min(margin, abs(al - ALPHA_MIN) / ALPHA_MIN)
                    if al < ALPHA_MIN:
                        continue
                    Tn = T * (1 - al)
                    margin = min(margin, abs(Tn - 1e-4) / 1e-4)
                    if Tn < float(F32(1e-4)):
                        break
                    beta[i] += al * T
                    U[i] += al * T * F[py, px]
                    cnt[i] += 1
                    T = Tn
    return beta, U, cnt, margin


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_tiny_scenes(seed):
    """Opacities below 0.3 keep every alpha >= 1/255 pixel inside the radius
    3 sqrt(lambda_max), so the tile support changes nothing here."""
    n = 6
    u = philox.uniform(100 + seed, 0, 3 * n).reshape(n, 3).astype(np.float64)
    means = (0.3 * (2 * u - 1)).astype(F32)
    scales = np.exp(-3.6 + 0.4 * philox.normal(100 + seed, 1, 3 * n)).reshape(n, 3).astype(F32)
    quats = philox.normal(100 + seed, 2, 4 * n).reshape(n, 4)
    op = (0.05 + 0.25 * philox.uniform(100 + seed, 3, n)).astype(F32)
    sc = Scene(means, scales, quats, op)
    cams = [scenes.look_at(e, 32, 32, 50.0) for e in scenes.fibonacci_eyes(2, 2.0)]
    maps = [philox.uniform(200 + seed, v, 32 * 32 * 2).reshape(32, 32, 2) for v in range(2)]
    beta, U, cnt, margin = brute_force(sc, cams, maps)
    assert margin > 1e-4
    r = oracle.uplift(sc, cams, maps)
    assert r.amb_px == 0 and min(r.margin_skip, r.margin_stop) == pytest.approx(margin, rel=1e-6)
    assert cnt.sum() > 100
    assert np.array_equal(r.count, cnt)
    assert np.allclose(r.beta, beta, rtol=1e-9, atol=1e-300)
    assert np.allclose(r.U, U, rtol=1e-9, atol=1e-12)


# ------------------------------------------- count normalisation, filtering
def test_count_normalised_single_gaussian():
    """Appendix (GaussianEditor's aggregation): f = U / count, from the closed
    form of one Gaussian; for a constant map it is c beta / count, smaller
    than c because every weight is below 1."""
    f, z0, s, op = 100.0, 4.0, 0.2, 0.7
    cam = axis_camera(f, z0=z0)
    sc = one_scene([0, 0, 0], [s, s, s], opacity=[op])
    v = (f * float(F32(s)) / z0) ** 2 + float(F32(0.3))
    tiles = tiles_for((64.5, 64.5), v, 129, 129)
    F = philox.uniform(12, 1, 129 * 129 * 2).reshape(129, 129, 2).astype(np.float64)
    beta, U, cnt, margin = single_closed_form(cam, (64.5, 64.5), v, v, op, tiles, F)
    assert margin > 1e-4 and cnt > 10
    r = oracle.uplift(sc, [cam], [F.astype(F32)])
    assert np.allclose(r.f_count[0], U / cnt, rtol=1e-9, atol=0)
    c = np.array([2.0, -1.0], F32)
    rc = oracle.uplift(sc, [cam], [np.broadcast_to(c, (129, 129, 2))])
    assert np.allclose(rc.f_count[0], c * beta / cnt, rtol=1e-9)
    assert np.all(np.abs(rc.f_count[0]) < np.abs(c))


def test_count_normalised_unseen_is_zero(tiny):
    sc = one_scene([[0, 0, 0], [100, 0, 0]], [[0.2] * 3, [0.2] * 3])  # the second is out of frame
    r = oracle.uplift(sc, [axis_camera(100.0)], [np.ones((129, 129, 2), F32)])
    assert r.count[0] > 0 and r.count[1] == 0 and np.all(r.f_count[1] == 0)
    sc, cams, maps = tiny
    r = oracle.uplift(sc, cams, maps)
    seen = r.count > 0
    assert np.allclose(r.f_count[seen] * r.count[seen][:, None], r.U[seen], rtol=1e-12)


def _brute_keep(values, k):
    """Sorting (key, index) tuples in Python: the plain definition."""
    import struct
    def tot(x):  # IEEE totalOrder key of an FP32 value
        b = struct.unpack("<I", struct.pack("<f", float(x)))[0]
        return (0xFFFFFFFF - b) if b >> 31 else (b | 0x80000000)
    order = sorted(range(len(values)), key=lambda i: (-tot(values[i]), i))
    keep = np.zeros(len(values), np.uint8)
    keep[order[:k]] = 1
    return keep


@pytest.mark.parametrize("n", [0, 1, 2, 7, 64, 300])
def test_prune_matches_brute_force(n):
    rng = np.random.default_rng(n)
    v = rng.choice(np.array([0.0, -0.0, 0.5, 1.5, 1e-30, 3.0, np.inf], F32), size=n).astype(F32)
    v[: n // 3] = rng.random(n // 3).astype(F32)
    for k in sorted({0, n // 2, n, min(n, 1), max(0, n - 1)}):
        assert np.array_equal(oracle.prune.keep_top_k(v, k), _brute_keep(v, k)), (n, k)


def test_prune_matches_library_sort_and_orders_signed_zero():
    rng = np.random.default_rng(5)
    v = np.round(rng.random(20000) * 300).astype(F32)  # many ties
    k = 10000
    order = np.argsort(-v.astype(np.float64), kind="stable")  # ties keep index order
    ref = np.zeros(v.size, np.uint8)
    ref[order[:k]] = 1
    keep = oracle.prune.keep_top_k(v, k)
    assert np.array_equal(keep, ref) and keep.sum() == k
    assert v[keep == 1].min() >= v[keep == 0].max()
    # totalOrder: +0 above -0, whatever their indices
    z = np.array([-0.0, 0.0, -0.0, 0.0], F32)
    assert np.array_equal(oracle.prune.keep_top_k(z, 2), np.array([0, 1, 0, 1], np.uint8))
    with pytest.raises(ValueError):
        oracle.prune.keep_top_k(z, 5)
