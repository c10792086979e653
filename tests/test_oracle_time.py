"""Pins of the oracle's time-conditioned density (the dynamic-scene
application: the phase of every hidden unit gains xi_t W_t); CPU only."""
import numpy as np

import synthetic as S
from oracle.density import chord_integral, chord_integral_quadrature
from oracle.geometry import intersect_ellipsoid, quat_to_rotmat
from oracle.grad import autograd_loss_and_grads, fd_gradient
from oracle.render import RenderOptions, primitive, render_view


def test_time_zero_is_the_static_density():
    sc = S.custom_scene(120, 8, seed=41, temporal=True)
    cam = S.make_cameras([(48, 40)], seed=42)[0]
    static = dict(sc, wt=None)
    a = render_view(sc, cam)  # time 0
    b = render_view(static, cam)
    assert np.array_equal(a["image"], b["image"])


def test_time_term_is_a_bias_shift_of_the_phase():
    """omega0 (W1 x + b1) + xi W_t equals the static phase with b1 + xi W_t / omega0."""
    sc = S.custom_scene(120, 8, seed=43, temporal=True)
    sc["time"] = 0.37
    cam = S.make_cameras([(48, 40)], seed=44)[0]
    shifted = dict(sc, wt=None, time=0.0,
                   b1=sc["b1"].astype(np.float64) + 0.37 * sc["wt"].astype(np.float64) / sc["omega0"])
    a = render_view(sc, cam)
    b = render_view(shifted, cam)
    assert np.max(np.abs(a["image"] - b["image"])) < 1e-12
    c = render_view(dict(sc, time=0.9), cam)
    assert np.max(np.abs(a["image"] - c["image"])) > 1e-3  # and the time matters


def test_closed_form_with_time_against_quadrature():
    sc = S.custom_scene(5, 16, seed=45, temporal=True)
    sc["time"] = 0.81
    rng = np.random.default_rng(46)
    for p in range(5):
        prim = primitive(sc, p, quat_to_rotmat(sc["quats"][p]))
        for _ in range(4):
            o = np.asarray(prim["center"], float) + rng.normal(size=3) * 2.0
            d = np.asarray(prim["center"], float) + rng.normal(size=3) * 0.02 - o
            d /= np.linalg.norm(d)
            disc, t0, t1 = intersect_ellipsoid(o, d[None], prim["center"], prim["scale"], prim["R"])
            if disc[0] <= 0:
                continue
            exact = chord_integral(o, d[None], t0, t1, prim)[0]
            quad = chord_integral_quadrature(o, d, t0[0], t1[0], prim)
            assert abs(exact - quad) <= 1e-10 * max(1.0, abs(quad))


def test_autograd_of_wt_against_finite_differences():
    sc = S.custom_scene(30, 4, seed=47, temporal=True)
    sc["time"] = 0.6
    sc["w2"] = sc["w2"] * np.float32(6.0)
    cams = S.make_cameras([(32, 24)], seed=48)
    tg = S.make_targets(cams, seed=49)
    opts = RenderOptions(t_eps=0.0)
    _, g, _ = autograd_loss_and_grads(sc, cams, tg, opts)
    gw = g["wt"]
    idx = np.argsort(-np.abs(gw).ravel())[:4]
    for flat in idx:
        i = np.unravel_index(flat, gw.shape)
        fd = fd_gradient(sc, cams, tg, "wt", i, opts=opts)
        assert abs(fd - gw[i]) <= 1e-6 * max(1e-8, abs(gw[i])) + 1e-10, (i, fd, gw[i])
