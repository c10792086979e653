"""Pins of the oracle's Gaussian splats (the 3DGS comparison kernel); CPU only.

Each check comes from outside the oracle's own formulas: numerical
derivatives of the pinhole projection, Monte-Carlo covariance of projected
samples, closed forms of an isotropic splat on the optical axis, a matrix
inverse instead of the closed-form conic, brute force over every pixel, and
compositing by hand."""
import math

import numpy as np

import synthetic as S
from oracle import gaussian as G
from oracle.keys import tile_lists
from oracle.render import RenderOptions


def _scene(centers, sigmas, quats=None, colors=None, opacity=None):
    P = len(centers)
    sig = np.asarray(sigmas, np.float32)
    if sig.ndim == 1:
        sig = np.repeat(sig[:, None], 3, 1)
    q = np.tile(np.array([1, 0, 0, 0], np.float32), (P, 1)) if quats is None else np.asarray(quats, np.float32)
    col = np.full((P, 3), 0.5, np.float32) if colors is None else np.asarray(colors, np.float32)
    op = np.full(P, 0.8, np.float32) if opacity is None else np.asarray(opacity, np.float32)
    return dict(P=P, N=8, omega0=10.0, color_mode=0, primitive=1, centers=np.asarray(centers, np.float32),
                scales=sig, quats=q, colors=col, opacity=op, cmlp=None, xi=None, sh=None)


def _cam_coords(cam, X):
    return X @ np.asarray(cam.R, np.float64).T + np.asarray(cam.t, np.float64)


def _project(cam, Xc):
    return np.stack([cam.fx * Xc[..., 0] / Xc[..., 2] + cam.cx, cam.fy * Xc[..., 1] / Xc[..., 2] + cam.cy], -1)


def test_jacobian_is_the_derivative_of_the_projection():
    """J (rows (j00, 0, j02), (0, j11, j12)) equals central differences of the
    pinhole map at the centre, for centres inside the clamp range."""
    cam = S.make_cameras([(320, 240)], seed=5)[0]
    sc = S.custom_scene(64, 8, primitive=1, scale_lo=0.01, scale_hi=0.05)
    pr = G.project_gaussians(sc, cam)
    j00, j02, j11, j12 = pr["jac"]
    mu = _cam_coords(cam, sc["centers"].astype(np.float64))
    h = 1e-6
    for p in np.nonzero(pr["keep"])[0][:20]:
        Jn = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jn[:, k] = (_project(cam, mu[p] + e) - _project(cam, mu[p] - e)) / (2 * h)
        inside = abs(mu[p, 0] / mu[p, 2]) < 1.3 * cam.cx / cam.fx and abs(mu[p, 1] / mu[p, 2]) < 1.3 * cam.cy / cam.fy
        assert inside
        J = np.array([[j00[p], 0.0, j02[p]], [0.0, j11[p], j12[p]]])
        assert np.allclose(J, Jn, rtol=1e-6, atol=1e-6 * np.abs(Jn).max())


def test_covariance_matches_projected_samples():
    """A small, distant Gaussian: the covariance of its projected samples
    equals J Sigma J^T (the 2D covariance without the low-pass term)."""
    cam = S.make_cameras([(400, 300)], seed=7)[0]
    o = -np.linalg.inv(np.asarray(cam.R, float)) @ np.asarray(cam.t, float)
    c = 0.6 * o  # on the axis, 0.4 of the way to the origin
    c = c + np.array([0.05, -0.03, 0.02])
    q = np.array([[0.8, 0.3, -0.4, 0.33]])
    sc = _scene([c], [[0.004, 0.002, 0.001]], quats=q)
    pr = G.project_gaussians(sc, cam)
    assert pr["keep"][0]
    rng = np.random.default_rng(0)
    from oracle.geometry import quat_to_rotmat
    Rw = quat_to_rotmat(sc["quats"][0])
    Sw = Rw @ np.diag(sc["scales"][0].astype(float) ** 2) @ Rw.T
    X = rng.multivariate_normal(sc["centers"][0].astype(float), Sw, 400_000)
    uv = _project(cam, _cam_coords(cam, X))
    emp = np.cov(uv.T)
    model = pr["cov2d"][0] - G.LOW_PASS * np.eye(2)
    lam = np.linalg.eigvalsh(model).max()
    assert np.max(np.abs(emp - model)) < 0.02 * lam
    # the projected centre is the image of x_B
    assert np.allclose(pr["mean2d"][0], _project(cam, _cam_coords(cam, sc["centers"][0].astype(float))), atol=1e-9)


def test_isotropic_splat_on_the_axis():
    """An isotropic Gaussian at the point the camera looks at: cov2d =
    ((f s / D)^2 + 0.3) I, conic its inverse, radius ceil(3 sqrt(var + sqrt(0.1)))
    (the eigenvalue floor of the square bound), centred at the principal point."""
    cam = S.make_cameras([(200, 200)], seed=2)[0]
    D = 3.0  # cameras sit on the radius-3 sphere looking at the origin
    s = 0.03
    sc = _scene([[0.0, 0.0, 0.0]], [s])
    pr = G.project_gaussians(sc, cam)
    var = (cam.fx * float(np.float32(s)) / D) ** 2 + 0.3
    assert np.allclose(pr["cov2d"][0], var * np.eye(2), rtol=1e-5, atol=1e-6)
    assert np.allclose(pr["conic"][0], [1 / var, 0.0, 1 / var], rtol=1e-5, atol=1e-7)
    assert pr["radius"][0] == math.ceil(3 * math.sqrt(var + math.sqrt(0.1)))
    assert np.allclose(pr["mean2d"][0], [cam.cx, cam.cy], atol=1e-4)


def test_largest_eigenvalue_and_conic_against_linear_algebra():
    cam = S.make_cameras([(320, 240)], seed=5)[0]
    sc = S.custom_scene(200, 8, primitive=1, scale_lo=0.005, scale_hi=0.08)
    pr = G.project_gaussians(sc, cam)
    k = pr["keep"]
    inv = np.linalg.inv(pr["cov2d"][k])
    conic = pr["conic"][k]
    assert np.allclose(conic[:, 0], inv[:, 0, 0], rtol=1e-10)
    assert np.allclose(conic[:, 1], inv[:, 0, 1], rtol=1e-10, atol=1e-14)
    assert np.allclose(conic[:, 2], inv[:, 1, 1], rtol=1e-10)
    lam = np.linalg.eigvalsh(pr["cov2d"][k])[:, 1]
    # the square bound covers 3 sigma of the largest eigenvalue
    assert np.all(pr["radius"][k] >= 3 * np.sqrt(lam) - 1e-9)


def test_alpha_is_the_mahalanobis_gaussian():
    """alpha = o exp(-d^T Sigma2d^-1 d / 2) with the inverse from numpy."""
    cam = S.make_cameras([(160, 120)], seed=4)[0]
    sc = S.custom_scene(50, 8, primitive=1, scale_lo=0.01, scale_hi=0.06)
    pr = G.project_gaussians(sc, cam)
    for p in np.nonzero(pr["nonempty"])[0][:10]:
        x0, x1, y0, y1 = pr["rect"][p]
        rows, cols = np.mgrid[y0:y1 + 1, x0:x1 + 1]
        _, alpha = G.gaussian_alpha(pr, p, cols, rows, sc["opacity"][p], 1.0)
        d = np.stack([cols + 0.5 - pr["mean2d"][p, 0], rows + 0.5 - pr["mean2d"][p, 1]], -1)
        m2 = np.einsum("...i,ij,...j->...", d, np.linalg.inv(pr["cov2d"][p]), d)
        assert np.allclose(alpha, float(sc["opacity"][p]) * np.exp(-0.5 * m2), rtol=1e-10, atol=1e-15)


def test_rectangle_contains_the_three_sigma_ellipse():
    """Brute force over every pixel: a pixel whose centre is within 3 standard
    deviations (Mahalanobis) of a kept Gaussian lies in its rectangle."""
    cam = S.make_cameras([(96, 96)], seed=6)[0]
    sc = S.custom_scene(300, 8, primitive=1, scale_lo=0.01, scale_hi=0.1)
    pr = G.project_gaussians(sc, cam)
    rows, cols = np.mgrid[0:96, 0:96]
    inv = np.linalg.inv(pr["cov2d"])
    for p in np.nonzero(pr["keep"])[0]:
        d = np.stack([cols + 0.5 - pr["mean2d"][p, 0], rows + 0.5 - pr["mean2d"][p, 1]], -1)
        m2 = np.einsum("...i,ij,...j->...", d, inv[p], d)
        inside = m2 <= 9.0
        if not inside.any():
            continue
        assert pr["nonempty"][p]
        x0, x1, y0, y1 = pr["rect"][p]
        assert np.all((cols[inside] >= x0) & (cols[inside] <= x1) & (rows[inside] >= y0) & (rows[inside] <= y1))


def test_near_culling_by_centre_and_clamped_jacobian():
    cam = S.make_cameras([(128, 128)], seed=2)[0]
    Rinv = np.linalg.inv(np.asarray(cam.R, float))
    o = -Rinv @ np.asarray(cam.t, float)
    fwd = Rinv[:, 2]
    right = Rinv[:, 0]
    # centre 0.1 in front of the camera (behind z_near = 0.2) and one far to the side
    sc = _scene([o + 0.1 * fwd, o + 1.0 * fwd + 5.0 * right], [0.01, 0.01])
    pr = G.project_gaussians(sc, cam)
    assert not pr["keep"][0]
    assert pr["keep"][1]
    j00, j02, j11, j12 = pr["jac"]
    mu = _cam_coords(cam, sc["centers"][1].astype(float))
    lim = 1.3 * cam.cx / cam.fx
    assert mu[0] / mu[2] > lim
    assert math.isclose(j02[1], -cam.fx * lim / mu[2], rel_tol=1e-6)


def test_single_gaussian_image_and_two_composited_by_hand():
    cam = S.make_cameras([(80, 64)], seed=3)[0]
    Rinv = np.linalg.inv(np.asarray(cam.R, float))
    o = -Rinv @ np.asarray(cam.t, float)
    fwd = Rinv[:, 2]
    front, back = o + 2.5 * fwd, o + 3.2 * fwd + 0.05 * Rinv[:, 0]
    cols = [[1.0, 0.0, 0.0], [0.0, 0.5, 1.0]]
    opts = RenderOptions(t_eps=0.0, alpha_max=0.99)
    a = G.render_view_gaussian(_scene([front], [0.05], colors=[cols[0]], opacity=[0.7]), cam, opts)
    b = G.render_view_gaussian(_scene([back], [0.08], colors=[cols[1]], opacity=[0.9]), cam, opts)
    both = G.render_view_gaussian(_scene([back, front], [0.08, 0.05], colors=[cols[1], cols[0]],
                                         opacity=[0.9, 0.7]), cam, opts)
    # one Gaussian: image = alpha c with alpha from the inverse covariance, zero outside the rectangle
    sc = _scene([front], [0.05], colors=[cols[0]], opacity=[0.7])
    pr = G.project_gaussians(sc, cam)
    rows, cols_ = np.mgrid[0:64, 0:80]
    d = np.stack([cols_ + 0.5 - pr["mean2d"][0, 0], rows + 0.5 - pr["mean2d"][0, 1]], -1)
    m2 = np.einsum("...i,ij,...j->...", d, np.linalg.inv(pr["cov2d"][0]), d)
    x0, x1, y0, y1 = pr["rect"][0]
    inr = (cols_ >= x0) & (cols_ <= x1) & (rows >= y0) & (rows <= y1)
    alpha = np.where(inr, np.minimum(0.99, float(np.float32(0.7)) * np.exp(-0.5 * m2)), 0.0)
    assert np.max(np.abs(a["image"] - alpha[..., None] * np.array(cols[0]))) < 1e-12
    assert a["hit_pairs"] == int(inr.sum())
    a1, a2 = 1 - a["T"], 1 - b["T"]
    expect = a1[..., None] * np.array(cols[0]) + ((1 - a1) * a2)[..., None] * np.array(cols[1])
    assert np.max(np.abs(both["image"] - expect)) < 1e-12
    assert np.max(np.abs(both["T"] - (1 - a1) * (1 - a2))) < 1e-12


def test_pixel_spot_checks_agree_with_the_image_and_tile_lists_cover_contributors():
    cam = S.make_cameras([(64, 48)], seed=8)[0]
    sc = S.custom_scene(400, 8, primitive=1, scale_lo=0.01, scale_hi=0.08)
    opts = RenderOptions(alpha_min=1 / 255)
    pr = G.project_gaussians(sc, cam, 16, 16)
    img = G.render_view_gaussian(sc, cam, opts, proj=pr)
    rng = np.random.default_rng(1)
    cols = rng.integers(0, 64, 40)
    rows = rng.integers(0, 48, 40)
    c, t, h = G.render_pixels_gaussian(sc, cam, cols, rows, opts, proj=pr)
    assert np.max(np.abs(c - img["image"][rows, cols])) < 1e-12
    assert np.max(np.abs(t - img["T"][rows, cols])) < 1e-12
    # every Gaussian with alpha > 0 at a pixel is in that pixel's tile list
    lists = tile_lists(sc, [cam], 16, 16, projs=[pr])
    for i, j in zip(cols, rows):
        tile = (j // 16) * 4 + i // 16
        ids = {p for _, p in lists[tile]}
        for p in np.nonzero(pr["nonempty"])[0]:
            _, al = G.gaussian_alpha(pr, p, np.array([i]), np.array([j]), sc["opacity"][p], 0.99)
            x0, x1, y0, y1 = pr["rect"][p]
            if al[0] > 0 and x0 <= i <= x1 and y0 <= j <= y1:
                assert p in ids


def test_early_termination_changes_pixels_by_at_most_t_eps():
    cam = S.make_cameras([(48, 48)], seed=9)[0]
    sc = S.custom_scene(600, 8, primitive=1, scale_lo=0.05, scale_hi=0.2)
    sc["opacity"][:] = 0.95
    a = G.render_view_gaussian(sc, cam, RenderOptions(t_eps=1e-3))
    b = G.render_view_gaussian(sc, cam, RenderOptions(t_eps=0.0))
    assert np.max(np.abs(a["image"] - b["image"])) <= 1e-3
    assert a["hit_pairs"] < b["hit_pairs"]


def test_alpha_min_skips_faint_gaussian_pairs_by_hand():
    """alpha_min for Gaussians: inside the rectangle every pixel is a hit, but
    pixels whose alpha is below alpha_min change neither colour nor
    transmittance; composited by hand from o exp(-m^2 / 2) with numpy's
    inverse covariance."""
    cam = S.make_cameras([(80, 64)], seed=3)[0]
    Rinv = np.linalg.inv(np.asarray(cam.R, float))
    o = -Rinv @ np.asarray(cam.t, float)
    fwd = Rinv[:, 2]
    front, back = o + 2.5 * fwd, o + 3.2 * fwd + 0.05 * Rinv[:, 0]
    cols = [[1.0, 0.0, 0.0], [0.0, 0.5, 1.0]]
    amin = 0.3
    opts = RenderOptions(t_eps=0.0, alpha_min=amin)
    sc = _scene([back, front], [0.08, 0.05], colors=[cols[1], cols[0]], opacity=[0.9, 0.7])
    out = G.render_view_gaussian(sc, cam, opts)
    pr = G.project_gaussians(sc, cam)
    rows, cc = np.mgrid[0:64, 0:80]

    def alpha_of(p, op):
        d = np.stack([cc + 0.5 - pr["mean2d"][p, 0], rows + 0.5 - pr["mean2d"][p, 1]], -1)
        m2 = np.einsum("...i,ij,...j->...", d, np.linalg.inv(pr["cov2d"][p]), d)
        x0, x1, y0, y1 = pr["rect"][p]
        inr = (cc >= x0) & (cc <= x1) & (rows >= y0) & (rows <= y1)
        return inr, np.where(inr, np.minimum(0.99, float(np.float32(op)) * np.exp(-0.5 * m2)), 0.0)

    in_b, a_b = alpha_of(0, 0.9)
    in_f, a_f = alpha_of(1, 0.7)
    u_f = in_f & (a_f >= amin)
    u_b = in_b & (a_b >= amin)
    assert np.any(in_f & ~u_f) and np.any(u_f) and np.any(in_b & ~u_b)
    af, ab = np.where(u_f, a_f, 0.0), np.where(u_b, a_b, 0.0)
    expect = af[..., None] * np.array(cols[0]) + ((1 - af) * ab)[..., None] * np.array(cols[1])
    assert np.max(np.abs(out["image"] - expect)) < 1e-12
    assert np.max(np.abs(out["T"] - (1 - af) * (1 - ab))) < 1e-12
    assert out["hit_pairs"] == int(in_f.sum() + in_b.sum())
