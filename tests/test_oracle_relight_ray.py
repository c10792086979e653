"""Pins of the oracle's per-ray relighting colour (colour mode 4: c_dc + a
colour network of the entry point, the ray direction and the light
direction, evaluated per (pixel, primitive) pair); CPU only."""
import numpy as np

import synthetic as S
from oracle.grad import autograd_loss_and_grads, fd_gradient, render_view_torch
from oracle.render import RenderOptions, render_pixels, render_view

OPTS = RenderOptions(t_eps=0.0)


def _reader_network(slot, P, width=4):
    """Depth 1: hidden unit c = relu(input[slot + c] + 1) for c < 3 (the
    inputs lie in [-1, 1]), output c = hidden c - 1, so the colour is
    c_dc + sigmoid(input[slot + c])."""
    W1 = np.zeros((width, 9))
    b1 = np.zeros(width)
    for c in range(3):
        W1[c, slot + c] = 1.0
        b1[c] = 1.0
    W2 = np.zeros((3, width))
    for c in range(3):
        W2[c, c] = 1.0
    b2 = -np.ones(3)
    return np.tile(np.concatenate([W1.ravel(), b1, W2.ravel(), b2]), (P, 1))


def _one_sphere(r=0.3):
    sc = S.custom_scene(1, 8, color_mode=4, cmlp_width=4, cmlp_depth=1, seed=91)
    sc["centers"] = np.array([[0.1, -0.05, 0.2]], np.float32)
    sc["scales"] = np.full((1, 3), r, np.float32)
    sc["quats"] = np.array([[1.0, 0.0, 0.0, 0.0]], np.float32)
    sc["w2"] = sc["w2"] * np.float32(4.0)
    return sc


def _alpha_image(sc, cam):
    """alpha per pixel of the single primitive: the image with colour 1."""
    m0 = dict(sc, color_mode=0, colors=np.ones((1, 3), np.float32), cmlp=None)
    return render_view(m0, cam, OPTS)["image"][..., 0]


def _rays(cam):
    """Unit ray directions of every pixel, by solving R d_world = d_cam."""
    H, W = cam.height, cam.width
    jj, ii = np.mgrid[0:H, 0:W]
    dcam = np.stack([(ii + 0.5 - cam.cx) / cam.fx, (jj + 0.5 - cam.cy) / cam.fy, np.ones((H, W))], -1)
    R = np.asarray(cam.R, np.float64)
    d = np.linalg.solve(R, dcam.reshape(-1, 3).T).T.reshape(H, W, 3)
    o = -np.linalg.solve(R, np.asarray(cam.t, np.float64))
    return o, d / np.linalg.norm(d, axis=-1, keepdims=True)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def test_entry_point_read_by_construction():
    """The network that returns its first three inputs: image / alpha =
    c_dc + sigmoid(entry point), the entry point of a sphere found from the
    ray's closest approach to the centre, on the unit sphere after the
    normalisation."""
    r = 0.5
    sc = _one_sphere(r)
    sc["cmlp"] = _reader_network(0, 1)
    cam = S.make_cameras([(48, 40)], seed=92, lights=True)[0]
    a = _alpha_image(sc, cam)
    img = render_view(sc, cam, OPTS)["image"]
    o, d = _rays(cam)
    xb = sc["centers"][0].astype(np.float64)
    tc = (xb - o) @ d.reshape(-1, 3).T                  # closest approach along each ray
    dist2 = np.sum((xb - o) ** 2) - tc ** 2
    hit = (a.ravel() > 1e-6) & (dist2 < r * r)
    t_in = tc[hit] - np.sqrt(r * r - dist2[hit])
    x_in = (o + t_in[:, None] * d.reshape(-1, 3)[hit] - xb) / r
    assert hit.sum() > 30
    assert np.max(np.abs(np.linalg.norm(x_in, axis=1) - 1.0)) < 1e-9
    got = img.reshape(-1, 3)[hit] / a.ravel()[hit][:, None]
    ref = sc["colors"][0].astype(np.float64) + _sigmoid(x_in)
    assert np.max(np.abs(got - ref)) < 1e-9


def test_ray_and_light_directions_read_by_construction():
    sc = _one_sphere()
    cam = S.make_cameras([(40, 40)], seed=93, lights=True)[0]
    a = _alpha_image(sc, cam)
    hit = a.ravel() > 1e-6
    _, d = _rays(cam)
    sc["cmlp"] = _reader_network(3, 1)
    got = render_view(sc, cam, OPTS)["image"].reshape(-1, 3)[hit] / a.ravel()[hit][:, None]
    ref = sc["colors"][0].astype(np.float64) + _sigmoid(d.reshape(-1, 3)[hit])
    assert np.max(np.abs(got - ref)) < 1e-9
    sc["cmlp"] = _reader_network(6, 1)
    lv = cam.light.astype(np.float64) - sc["centers"][0].astype(np.float64)
    got = render_view(sc, cam, OPTS)["image"].reshape(-1, 3)[hit] / a.ravel()[hit][:, None]
    ref = sc["colors"][0].astype(np.float64) + _sigmoid(lv / np.linalg.norm(lv))
    assert np.max(np.abs(got - ref)) < 1e-9


def test_constant_network_is_a_constant_colour():
    """Zero weights: the colour is c_dc + sigmoid(output bias) for every
    ray, the image of colour mode 0 with that colour."""
    sc = S.custom_scene(30, 8, color_mode=4, cmlp_width=8, cmlp_depth=2, seed=94)
    K = sc["cmlp"].shape[1]
    b_out = np.random.default_rng(95).uniform(-1, 1, (30, 3))
    vec = np.zeros((30, K))
    vec[:, -3:] = b_out
    sc["cmlp"] = vec
    cam = S.make_cameras([(36, 30)], seed=96, lights=True)[0]
    m0 = dict(sc, color_mode=0, colors=(sc["colors"].astype(np.float64) + _sigmoid(b_out)), cmlp=None)
    assert np.max(np.abs(render_view(sc, cam, OPTS)["image"] - render_view(m0, cam, OPTS)["image"])) < 1e-12


def test_pixel_renderer_and_torch_route_agree():
    sc = S.custom_scene(40, 8, color_mode=4, cmlp_width=8, cmlp_depth=2, seed=97)
    cam = S.make_cameras([(30, 26)], seed=98, lights=True)[0]
    full = render_view(sc, cam, RenderOptions())
    cols, rows = np.meshgrid(np.arange(0, 30, 3), np.arange(0, 26, 3))
    c, t, _ = render_pixels(sc, cam, cols.ravel(), rows.ravel(), RenderOptions())
    assert np.max(np.abs(c - full["image"][rows.ravel(), cols.ravel()])) < 1e-12
    import torch
    from oracle.grad import PARAM_KEYS
    params = {k: torch.tensor(np.asarray(sc[k], np.float64)) for k in PARAM_KEYS if sc.get(k) is not None}
    meta = dict(color_mode=4, omega0=sc["omega0"], cmlp_width=8, cmlp_depth=2)
    img_t, _ = render_view_torch(params, meta, cam, RenderOptions())
    assert np.max(np.abs(img_t.numpy() - full["image"])) < 1e-9


def test_autograd_against_finite_differences():
    sc = S.custom_scene(20, 8, color_mode=4, cmlp_width=6, cmlp_depth=2, seed=99)
    sc["w2"] = sc["w2"] * np.float32(6.0)
    cams = S.make_cameras([(26, 22), (22, 26)], seed=100, lights=True)
    tg = S.make_targets(cams, seed=101)
    _, g, _ = autograd_loss_and_grads(sc, cams, tg, OPTS)
    for key in ("colors", "cmlp", "centers", "scales", "quats", "w1"):
        gk = g[key]
        for flat in np.argsort(-np.abs(gk).ravel())[:2]:
            i = np.unravel_index(flat, gk.shape)
            fd = fd_gradient(sc, cams, tg, key, i, opts=OPTS)
            assert abs(fd - gk[i]) <= 2e-5 * abs(gk[i]) + 1e-10, (key, i, fd, gk[i])
