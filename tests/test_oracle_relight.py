"""Pins of the oracle's relighting colour (colour mode 3: c_dc + colour MLP
of view direction, light direction and xi); CPU only."""
import numpy as np

import synthetic as S
from oracle.color import primitive_colors
from oracle.grad import autograd_loss_and_grads, fd_gradient
from oracle.render import RenderOptions


def _scene(P=40, width=14, depth=1, seed=71):
    return S.custom_scene(P, 8, color_mode=3, cmlp_width=width, cmlp_depth=depth, seed=seed)


def test_light_direction_and_offset_by_construction():
    """Depth 1, width 14 with identity first layer and an output layer that
    reads unit 3 + c (the light direction's components): colour_c = c_dc,c +
    sigmoid(relu(light_dir_c)), the light direction normalize(l - x_B)
    computed here independently."""
    sc = _scene()
    P = sc["P"]
    W1 = np.eye(14)
    b1 = np.zeros(14)
    W2 = np.zeros((3, 14))
    for c in range(3):
        W2[c, 3 + c] = 1.0
    b2 = np.zeros(3)
    sc["cmlp"] = np.tile(np.concatenate([W1.ravel(), b1, W2.ravel(), b2]), (P, 1)).astype(np.float32)
    cam = S.make_cameras([(32, 32)], seed=72, lights=True)[0]
    col = primitive_colors(sc, cam)
    x = sc["centers"].astype(np.float64)
    l = cam.light.astype(np.float64)
    ld = (l - x) / np.linalg.norm(l - x, axis=1, keepdims=True)
    ref = sc["colors"].astype(np.float64) + 1.0 / (1.0 + np.exp(-np.maximum(ld, 0.0)))
    assert np.max(np.abs(col - ref)) < 1e-12


def test_without_light_weights_it_is_the_view_colour_mlp_plus_offset():
    """Zero first-layer columns for the light direction: the colour equals
    c_dc plus colour mode 1 with those columns removed."""
    sc = _scene(width=16, depth=2, seed=73)
    P, Wd = sc["P"], 16
    vec = sc["cmlp"].astype(np.float64).copy()
    W1 = vec[:, :14 * Wd].reshape(P, Wd, 14)
    W1[:, :, 3:6] = 0.0
    vec[:, :14 * Wd] = W1.reshape(P, -1)
    sc["cmlp"] = vec
    cam = S.make_cameras([(32, 32)], seed=74, lights=True)[0]
    m1 = dict(sc, color_mode=1, cmlp=np.concatenate([np.delete(W1, [3, 4, 5], axis=2).reshape(P, -1),
                                                     vec[:, 14 * Wd:]], axis=1))
    assert np.max(np.abs(primitive_colors(sc, cam) - (sc["colors"] + primitive_colors(m1, cam)))) < 1e-12


def test_autograd_against_finite_differences():
    sc = _scene(P=25, width=8, depth=2, seed=75)
    sc["w2"] = sc["w2"] * np.float32(6.0)
    cams = S.make_cameras([(28, 24), (24, 28)], seed=76, lights=True)
    tg = S.make_targets(cams, seed=77)
    opts = RenderOptions(t_eps=0.0)
    _, g, _ = autograd_loss_and_grads(sc, cams, tg, opts)
    for key in ("colors", "cmlp", "xi", "centers"):
        gk = g[key]
        for flat in np.argsort(-np.abs(gk).ravel())[:2]:
            i = np.unravel_index(flat, gk.shape)
            fd = fd_gradient(sc, cams, tg, key, i, opts=opts)
            assert abs(fd - gk[i]) <= 2e-5 * abs(gk[i]) + 1e-10, (key, i, fd, gk[i])
