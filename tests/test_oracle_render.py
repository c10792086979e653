"""Pins of the oracle's splatting renderer (Eq. 3-4, 9) and its gradients; CPU only."""
import numpy as np
import pytest

import synthetic as S
from oracle import render as R
from oracle.geometry import pixel_rays
from oracle.grad import autograd_loss_and_grads, fd_gradient, render_view_torch  # noqa: F401
from oracle.keys import project_all


def _sphere_scene(centers, radii, colors, sigma_w2, b1=0.0, omega0=10.0, N=8):
    """Spheres of constant density: W1 = 0 makes sigma = sum_k W2_k cos(omega0 b1) + b2."""
    P = len(centers)
    return dict(P=P, N=N, omega0=omega0, color_mode=0, cmlp_width=0, cmlp_depth=0,
                centers=np.asarray(centers, np.float32),
                scales=np.repeat(np.asarray(radii, np.float32)[:, None], 3, 1),
                quats=np.tile(np.array([1, 0, 0, 0], np.float32), (P, 1)),
                w1=np.zeros((P, N, 3), np.float32), b1=np.full((P, N), b1, np.float32),
                w2=np.asarray(sigma_w2, np.float32)[:, None].repeat(N, 1) / N,
                b2=np.zeros(P, np.float32), colors=np.asarray(colors, np.float32),
                cmlp=None, xi=None)


def test_single_sphere_image_is_analytic():
    """One constant-density sphere: alpha = 1 - exp(-sigma 2 sqrt(r^2 - b^2)) per
    pixel (b: distance between the ray and the centre), C = c alpha, T = 1 - alpha."""
    cam = S.make_cameras([(96, 80)], seed=3)[0]
    r = 0.4
    scene = _sphere_scene([[0.1, -0.2, 0.05]], [r], [[0.2, 0.7, 0.4]], [3.0])
    out = R.render_view(scene, cam, R.RenderOptions(t_eps=0.0))
    rows, cols = np.mgrid[0:80, 0:96]
    o, d = pixel_rays(cam, cols, rows)
    c = scene["centers"][0].astype(float)
    b = np.linalg.norm(np.cross(c - o, d), axis=-1)
    sigma = float(np.sum(scene["w2"][0].astype(float)))
    r64 = float(np.float32(r))
    chord = 2 * np.sqrt(np.maximum(r64 * r64 - b * b, 0.0))
    alpha = np.minimum(1 - np.exp(-sigma * chord), 0.99)
    assert np.max(np.abs(out["T"] - (1 - alpha))) <= 1e-12
    assert np.max(np.abs(out["image"] - alpha[..., None] * scene["colors"][0].astype(float))) <= 1e-12
    assert out["hit_pairs"] == int(np.sum(chord > 0))


def test_two_spheres_composite_by_hand():
    cam = S.make_cameras([(64, 64)], seed=3)[0]
    o = -np.linalg.inv(np.asarray(cam.R, float)) @ np.asarray(cam.t, float)
    fwd = -o / np.linalg.norm(o)
    front, back = (o + 2.6 * fwd), (o + 3.4 * fwd)
    cols = [[1.0, 0.0, 0.0], [0.0, 0.5, 1.0]]  # exact in float32
    both = _sphere_scene([back, front], [0.3, 0.25], [cols[1], cols[0]], [2.0, 4.0])
    a = R.render_view(_sphere_scene([front], [0.25], [cols[0]], [4.0]), cam, R.RenderOptions(t_eps=0))
    b = R.render_view(_sphere_scene([back], [0.3], [cols[1]], [2.0]), cam, R.RenderOptions(t_eps=0))
    ab = R.render_view(both, cam, R.RenderOptions(t_eps=0))
    a1 = 1 - a["T"]
    a2 = 1 - b["T"]
    expect = a1[..., None] * np.array(cols[0]) + ((1 - a1) * a2)[..., None] * np.array(cols[1])
    assert np.max(np.abs(ab["image"] - expect)) <= 1e-12
    assert np.max(np.abs(ab["T"] - (1 - a1) * (1 - a2))) <= 1e-12


def test_invariants_and_background():
    cfg, scene, cams, _ = S.make_workload("C1")
    for bg in ((0, 0, 0), (0.25, 0.5, 1.0)):
        out = R.render_view(scene, cams[0], R.RenderOptions(bg=bg))
        T = out["T"]
        assert np.all((T > 0) & (T <= 1))
        assert np.all(out["image"] >= 0) and np.all(out["image"] <= 1)
    empty = dict(scene)
    empty["centers"] = scene["centers"] + np.float32(100.0)
    out = R.render_view(empty, cams[0], R.RenderOptions(bg=(0.25, 0.5, 1.0)))
    assert np.all(out["image"] == np.array([0.25, 0.5, 1.0])) and out["hit_pairs"] == 0
    # adding a primitive can only lower the transmittance
    sub = S.subset_scene(scene, np.arange(128))
    T_sub = R.render_view(sub, cams[0])["T"]
    assert np.all(out_T_full(scene, cams[0]) <= T_sub + 1e-15)


def out_T_full(scene, cam):
    return R.render_view(scene, cam)["T"]


def test_alpha_is_zero_off_the_ellipsoid_and_clamped():
    """alpha is 0 for rays that miss and for non-positive integrals (Eq. 9)."""
    scene = S.custom_scene(64, 8, seed=5)
    scene["b2"] = np.full(64, -2.0, np.float32)     # makes most integrals negative
    cam = S.make_cameras([(48, 48)], seed=6)[0]
    out = R.render_view(scene, cam)
    assert out["hit_pairs"] > 0
    assert np.all(out["T"] <= 1.0)
    neg = dict(scene)
    neg["b2"] = np.full(64, -50.0, np.float32)
    out2 = R.render_view(neg, cam)
    assert np.all(out2["T"] == 1.0) and np.all(out2["image"] == 0.0)


def test_pixelwise_and_imagewise_renderers_agree():
    cfg, scene, cams, _ = S.make_workload("C1")
    full = R.render_view(scene, cams[0])
    rng = np.random.default_rng(0)
    cols = rng.integers(0, 64, 40)
    rows = rng.integers(0, 64, 40)
    c, t, h = R.render_pixels(scene, cams[0], cols, rows)
    assert np.allclose(c, full["image"][rows, cols], atol=1e-13)
    assert np.allclose(t, full["T"][rows, cols], atol=1e-13)


def test_colour_mlp_scene_numpy_and_torch_agree():
    scene = S.custom_scene(64, 16, color_mode=1, cmlp_width=16, cmlp_depth=2, seed=9)
    cam = S.make_cameras([(40, 32)], seed=10)[0]
    a = R.render_view(scene, cam)
    L, g, imgs = autograd_loss_and_grads(scene, [cam], S.make_targets([cam]))
    assert np.max(np.abs(imgs[0] - a["image"])) < 1e-12


def test_early_termination_bound():
    """Dense scene: termination at T < t_eps changes each pixel by at most
    t_eps * max colour, and some pixels do terminate."""
    scene = S.custom_scene(400, 8, seed=12, scale_lo=0.15, scale_hi=0.4)
    scene["w2"] = scene["w2"] * np.float32(20.0)
    cam = S.make_cameras([(48, 48)], seed=13)[0]
    a = R.render_view(scene, cam, R.RenderOptions(t_eps=1e-3))
    b = R.render_view(scene, cam, R.RenderOptions(t_eps=0.0))
    assert np.sum(b["T"] < 1e-3) > 10
    assert np.max(np.abs(a["image"] - b["image"])) <= 1e-3 * 1.0 + 1e-15
    assert a["hit_pairs"] < b["hit_pairs"]


def _grad_check(scene, cams, targets, keys, n_per_key=6, seed=0, opts=R.RenderOptions(t_eps=0.0)):
    L, g, _ = autograd_loss_and_grads(scene, cams, targets, opts)
    rng = np.random.default_rng(seed)
    for k in keys:
        G = g[k]
        flat = np.abs(G).ravel()
        # elements carrying gradient: sample from the larger half
        cand = np.argsort(flat)[-max(1, len(flat) // 2):]
        for fi in rng.choice(cand, size=min(n_per_key, len(cand)), replace=False):
            idx = np.unravel_index(fi, G.shape)
            fd = fd_gradient(scene, cams, targets, k, idx, rel_step=1e-6, opts=opts)
            assert abs(fd - G[idx]) <= 1e-4 * np.max(np.abs(G)) + 1e-6 * abs(G[idx]), (k, idx, fd, G[idx])


def test_autograd_matches_finite_differences_constant_colour():
    cfg, scene, cams, targets = S.make_workload("C1")
    _grad_check(scene, cams, targets, ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors"])


def test_autograd_matches_finite_differences_colour_mlp():
    scene = S.custom_scene(48, 8, color_mode=1, cmlp_width=16, cmlp_depth=2, seed=15)
    cams = S.make_cameras([(32, 32), (24, 32)], seed=16)
    targets = S.make_targets(cams, seed=17)
    _grad_check(scene, cams, targets, ["centers", "quats", "cmlp", "xi", "w1"], n_per_key=5)


def test_colour_mlp_identity_weights():
    """Colour MLP with identity hidden layers: colour = sigmoid(relu(dir)), dir =
    normalize(x_B - o); with zero weights it is sigmoid(output bias).  Pins the
    packing (each layer W (out x in, row-major) then b) and the activations."""
    from oracle.color import primitive_colors
    from oracle.geometry import camera_center
    scene = S.custom_scene(20, 8, color_mode=1, cmlp_width=16, cmlp_depth=2, seed=131)
    cam = S.make_cameras([(32, 32)], seed=132)[0]
    W0 = np.zeros((16, 11)); W0[:11, :11] = np.eye(11)
    W1 = np.eye(16)
    W2 = np.zeros((3, 16)); W2[:, :3] = np.eye(3)
    vec = np.concatenate([W0.ravel(), np.zeros(16), W1.ravel(), np.zeros(16), W2.ravel(), np.zeros(3)])
    scene["cmlp"] = np.tile(vec, (20, 1)).astype(np.float32)
    dirv = scene["centers"].astype(float) - camera_center(cam)
    dirv /= np.linalg.norm(dirv, axis=1, keepdims=True)
    expect = 1.0 / (1.0 + np.exp(-np.maximum(dirv, 0.0)))
    assert np.max(np.abs(primitive_colors(scene, cam) - expect)) < 1e-12
    bias = np.array([0.3, -1.2, 2.0])
    vec2 = np.zeros_like(vec); vec2[-3:] = bias
    scene["cmlp"] = np.tile(vec2, (20, 1)).astype(np.float32)
    expect2 = 1.0 / (1.0 + np.exp(-bias.astype(np.float32).astype(float)))
    assert np.max(np.abs(primitive_colors(scene, cam) - expect2)) < 1e-12


def test_alpha_min_skips_faint_pairs_by_hand():
    """alpha_min (the 3DGS skip of faint pairs): a pair whose alpha is below
    alpha_min leaves colour and transmittance unchanged but is still a hit.
    Front sphere faint everywhere (skipped at every pixel), back sphere
    faint near its silhouette only; composited by hand from the analytic
    constant-density alphas 1 - exp(-sigma 2 sqrt(r^2 - b^2))."""
    cam = S.make_cameras([(64, 64)], seed=3)[0]
    o = -np.linalg.inv(np.asarray(cam.R, float)) @ np.asarray(cam.t, float)
    fwd = -o / np.linalg.norm(o)
    front, back = o + 2.6 * fwd, o + 3.4 * fwd
    cols = [[1.0, 0.0, 0.0], [0.0, 0.5, 1.0]]
    r_f, r_b, s_f, s_b = 0.25, 0.3, 0.02, 2.0
    scene = _sphere_scene([back, front], [r_b, r_f], [cols[1], cols[0]], [s_b, s_f])
    amin = 0.45
    out = R.render_view(scene, cam, R.RenderOptions(t_eps=0.0, alpha_min=amin))
    rows, cc = np.mgrid[0:64, 0:64]
    oo, d = pixel_rays(cam, cc, rows)

    def analytic(center, r, s_w2):
        b = np.linalg.norm(np.cross(np.asarray(center, np.float32).astype(float) - oo, d), axis=-1)
        r64 = float(np.float32(r))
        sigma = float(np.sum((np.float32(s_w2) * np.ones(8, np.float32) / np.float32(8)).astype(float)))
        chord = 2 * np.sqrt(np.maximum(r64 * r64 - b * b, 0.0))
        return chord > 0, np.minimum(1 - np.exp(-sigma * chord), 0.99)

    hit_f, a_f = analytic(front, r_f, s_f)
    hit_b, a_b = analytic(back, r_b, s_b)
    assert np.all(a_f < amin) and np.any(hit_f)              # front: every pair skipped
    assert np.any(hit_b & (a_b < amin)) and np.any(a_b >= amin)  # back: skipped at the rim only
    use_b = hit_b & (a_b >= amin)
    expect_T = np.where(use_b, 1 - a_b, 1.0)
    expect_C = np.where(use_b, a_b, 0.0)[..., None] * np.array(cols[1])
    assert np.max(np.abs(out["T"] - expect_T)) <= 1e-12
    assert np.max(np.abs(out["image"] - expect_C)) <= 1e-12
    assert out["hit_pairs"] == int(hit_f.sum() + hit_b.sum())
    # the pixel-by-pixel renderer takes the same decisions
    sel = np.random.default_rng(4).integers(0, 64, (2, 48))
    c, t, h = R.render_pixels(scene, cam, sel[0], sel[1], R.RenderOptions(t_eps=0.0, alpha_min=amin))
    assert np.max(np.abs(c - expect_C[sel[1], sel[0]])) <= 1e-12
    assert np.max(np.abs(t - expect_T[sel[1], sel[0]])) <= 1e-12
    assert np.array_equal(h, hit_f[sel[1], sel[0]].astype(int) + hit_b[sel[1], sel[0]].astype(int))


@pytest.mark.parametrize("win", [(24, 24, 16, 16), (16, 32, 16, 16), (41, 7, 23, 19), (48, 48, 16, 16)])
def test_window_render_equals_the_window_of_the_full_view(win):
    """render_window (a window of a view rendered through a shifted camera
    with the primitives whose rectangle meets it) equals that window of the
    full render: image, transmittance, and the hit pairs of its pixels."""
    scene = S.custom_scene(300, 16, color_mode=1, cmlp_width=16, cmlp_depth=2, seed=21)
    cam = S.make_cameras([(64, 64)], seed=22)[0]
    full = R.render_view(scene, cam)
    x0, y0, w, h = win
    w, h = min(w, 64 - x0), min(h, 64 - y0)
    out = R.render_window(scene, cam, x0, y0, w, h)
    assert np.max(np.abs(out["image"] - full["image"][y0:y0 + h, x0:x0 + w])) <= 1e-13
    assert np.max(np.abs(out["T"] - full["T"][y0:y0 + h, x0:x0 + w])) <= 1e-13
    # hit pairs of the window's pixels, counted pixel by pixel
    rows, cols = np.mgrid[y0:y0 + h, x0:x0 + w]
    _, _, hits = R.render_pixels(scene, cam, cols.ravel(), rows.ravel())
    assert out["hit_pairs"] == int(hits.sum()) and out["hit_pairs"] > 0
