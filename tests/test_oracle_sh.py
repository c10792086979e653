"""Pins of the oracle's spherical-harmonics colour (degree 3, 16 basis
functions per channel; the colour the paper adopts for novel-view synthesis,
Sec. 3.1, four bands as in 3DGS, Sec. 3.3 implementation details)."""
import numpy as np
from scipy import special

import synthetic as S
from oracle import render as R
from oracle.color import primitive_colors, sh_basis, view_directions
from oracle.grad import autograd_loss_and_grads
from tests.test_oracle_render import _grad_check

LM = [(0, 0), (1, -1), (1, 0), (1, 1), (2, -2), (2, -1), (2, 0), (2, 1), (2, 2),
      (3, -3), (3, -2), (3, -1), (3, 0), (3, 1), (3, 2), (3, 3)]


def _real_sh_scipy(l, m, d):
    """Real orthonormal harmonics from scipy's complex ones (which carry the
    Condon-Shortley phase): sqrt(2) (-1)^m Re Y_l^m for m > 0,
    sqrt(2) (-1)^m Im Y_l^|m| for m < 0, Y_l^0 for m = 0."""
    theta = np.arccos(np.clip(d[:, 2], -1, 1))      # polar
    phi = np.arctan2(d[:, 1], d[:, 0])              # azimuth
    Y = special.sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return np.sqrt(2) * (-1) ** m * Y.real
    if m < 0:
        return np.sqrt(2) * (-1) ** m * Y.imag
    return Y.real


def _unit(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_basis_matches_scipy_real_harmonics():
    d = _unit(500, 1)
    Y = sh_basis(d)
    for k, (l, m) in enumerate(LM):
        assert np.max(np.abs(Y[:, k] - _real_sh_scipy(l, m, d))) < 1e-12, (l, m)


def test_basis_is_orthonormal_on_the_sphere():
    # Gauss-Legendre in cos(theta) x uniform azimuth: exact for these degrees
    u, wu = np.polynomial.legendre.leggauss(12)
    phi = np.arange(24) * (2 * np.pi / 24)
    U, PHI = np.meshgrid(u, phi, indexing="ij")
    st = np.sqrt(1 - U ** 2)
    d = np.stack([st * np.cos(PHI), st * np.sin(PHI), U], -1).reshape(-1, 3)
    w = (wu[:, None] * np.full(phi.shape, 2 * np.pi / 24)[None, :]).ravel()
    Y = sh_basis(d)
    gram = (Y * w[:, None]).T @ Y
    assert np.max(np.abs(gram - np.eye(16))) < 1e-12


def test_constant_term_only_is_view_independent():
    scene = S.custom_scene(30, 8, color_mode=2, seed=21)
    scene["sh"][:, 1:, :] = 0
    cams = S.make_cameras([(16, 16), (16, 16), (16, 16)], seed=22)
    y00 = _real_sh_scipy(0, 0, np.array([[0.0, 0.0, 1.0]]))[0]
    expect = np.maximum(0.0, 0.5 + y00 * scene["sh"][:, 0, :].astype(float))
    for cam in cams:
        assert np.max(np.abs(primitive_colors(scene, cam) - expect)) < 1e-12


def test_colour_uses_view_direction_and_clamps():
    scene = S.custom_scene(40, 8, color_mode=2, seed=23)
    cam = S.make_cameras([(16, 16)], seed=24)[0]
    d = view_directions(scene, cam)
    pre = 0.5 + np.stack([sum(_real_sh_scipy(l, m, d) * scene["sh"][:, k, c].astype(float)
                              for k, (l, m) in enumerate(LM)) for c in range(3)], -1)
    assert np.max(np.abs(primitive_colors(scene, cam) - np.maximum(pre, 0.0))) < 1e-12


def test_sh_scene_numpy_and_torch_agree():
    scene = S.custom_scene(64, 8, color_mode=2, seed=25)
    cam = S.make_cameras([(40, 32)], seed=26)[0]
    a = R.render_view(scene, cam)
    L, g, imgs = autograd_loss_and_grads(scene, [cam], S.make_targets([cam]))
    assert np.max(np.abs(imgs[0] - a["image"])) < 1e-12
    assert "sh" in g and np.max(np.abs(g["sh"])) > 0


def test_autograd_matches_finite_differences_sh():
    scene = S.custom_scene(48, 8, color_mode=2, seed=27)
    cams = S.make_cameras([(32, 32), (24, 32)], seed=28)
    targets = S.make_targets(cams, seed=29)
    _grad_check(scene, cams, targets, ["centers", "sh", "w1", "scales"], n_per_key=5)
