"""Pins of the oracle's time-dependent zero-order SH coefficient (the
dynamic-scene application: S0 + a degree-4 polynomial + a 4-term Fourier
series of xi_t); CPU only."""
import math

import numpy as np

import synthetic as S
from oracle.grad import autograd_loss_and_grads, fd_gradient
from oracle.render import RenderOptions, render_view

OPTS = RenderOptions(t_eps=0.0)


def _scene(P=40, seed=211):
    sc = S.custom_scene(P, 8, color_mode=2, seed=seed, temporal=True)
    assert sc["sh_t"].shape == (P, 12, 3)
    return sc


def _static_with_shift(sc, shift):
    st = dict(sc, sh_t=None)
    sh = sc["sh"].astype(np.float64).copy()
    sh[:, 0, :] += shift
    st["sh"] = sh
    return st


def _shift_by_loops(sh_t, t):
    """sum_i a_i t^i + sum_i (b_i cos(i t) + c_i sin(i t)), written out
    term by term."""
    P = sh_t.shape[0]
    out = np.zeros((P, 3))
    for p in range(P):
        for c in range(3):
            v = 0.0
            for i in range(1, 5):
                v += float(sh_t[p, i - 1, c]) * t ** i
                v += float(sh_t[p, 3 + i, c]) * math.cos(i * t)
                v += float(sh_t[p, 7 + i, c]) * math.sin(i * t)
            out[p, c] = v
    return out


def test_time_terms_shift_the_zero_order_coefficient():
    """At any time the image equals the static SH image whose zero-order
    coefficient is shifted by the polynomial and Fourier terms."""
    sc = _scene()
    cam = S.make_cameras([(40, 36)], seed=212)[0]
    for t in (0.0, 0.37, 1.0):
        sc["time"] = t
        ref = render_view(_static_with_shift(sc, _shift_by_loops(sc["sh_t"], t)), cam, OPTS)["image"]
        assert np.max(np.abs(render_view(sc, cam, OPTS)["image"] - ref)) < 1e-12, t


def test_single_terms():
    """Only a_3: the shift is a_3 t^3; only c_2: c_2 sin(2 t); only b_4 at
    t = 0: b_4 (cos 0 = 1)."""
    sc = _scene(P=30, seed=213)
    cam = S.make_cameras([(36, 36)], seed=214)[0]
    base = sc["sh_t"].astype(np.float64)
    for k, t, fn in ((2, 0.6, lambda t: t ** 3), (9, 0.8, lambda t: math.sin(2 * t)), (7, 0.0, lambda t: 1.0)):
        one = np.zeros_like(base)
        one[:, k, :] = base[:, k, :]
        sc2 = dict(sc, sh_t=one, time=t)
        ref = render_view(_static_with_shift(sc2, base[:, k, :] * fn(t)), cam, OPTS)["image"]
        assert np.max(np.abs(render_view(sc2, cam, OPTS)["image"] - ref)) < 1e-12, k


def test_autograd_against_finite_differences():
    sc = _scene(P=25, seed=215)
    sc["time"] = 0.43
    sc["w2"] = sc["w2"] * np.float32(6.0)
    cams = S.make_cameras([(28, 24), (24, 28)], seed=216)
    tg = S.make_targets(cams, seed=217)
    _, g, _ = autograd_loss_and_grads(sc, cams, tg, OPTS)
    for key in ("sh_t", "sh", "wt", "centers"):
        gk = g[key]
        for flat in np.argsort(-np.abs(gk).ravel())[:2]:
            i = np.unravel_index(flat, gk.shape)
            fd = fd_gradient(sc, cams, tg, key, i, opts=OPTS)
            assert abs(fd - gk[i]) <= 2e-5 * abs(gk[i]) + 1e-10, (key, i, fd, gk[i])
