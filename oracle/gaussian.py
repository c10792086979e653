"""Gaussian splats through the same tiling, sorting and blending (FP64).

Test infrastructure only (see the package docstring).

The paper measures its renderer against the 3DGS rasterizer on the same
100k random primitives (App. A, integration-cost table).  This module is the
oracle of that second primitive kind: a 3D Gaussian with centre x_B,
standard deviations s_B along the axes of R(q_B) and an opacity o, splatted
as in 3DGS (EWA splatting: the covariance is pushed through the Jacobian of
the perspective projection at the centre, then a 2D Gaussian is evaluated
per pixel).  Everything around it (tile lists, depth keys, front-to-back
blending, alpha clamps, early termination, background, colour modes) is the
framework's, shared with the neural primitives.

Readings (3DGS conventions where the paper defers to 3DGS; all stated so
that the HIP path can follow them bit for bit on the key path):

  * Covariance in camera space Sigma = R_c R diag(s^2) R^T R_c^T.
  * Culling: kept iff the centre's camera depth mu_z > z_near (3DGS culls by
    the centre only) and the 2D covariance below has a positive determinant.
  * Jacobian of (x, y, z) -> (fx x / z + cx, fy y / z + cy) at the centre,
    with x / z clamped to [-1.3 cx / fx, 1.3 (W - cx) / fx] (and likewise
    y / z) -- 3DGS's guard against splats far outside the view; for a
    centred principal point this is +-1.3 tan(fov / 2).
  * 2D covariance J Sigma J^T plus 0.3 px^2 on the diagonal (3DGS's low-pass
    filter).  conic = its inverse.
  * Screen bound: r = ceil(3 sqrt(lambda_max)) with lambda_max = mid +
    sqrt(max(0.1, mid^2 - det)), mid = (a + c) / 2 (3DGS's square bound);
    pixel columns whose centre lies in [u - r, u + r] (u the projected
    centre), i.e. [ceil(u - r - 1/2), floor(u + r - 1/2)], clipped to the
    image; rows alike.  The primitive contributes only inside this
    rectangle, so the image does not depend on the tile shape.
  * Per pixel: d = pixel centre - (u, v); power = -(a' dx^2 + c' dy^2)/2 -
    b' dx dy with conic (a', b', c'); alpha = min(alpha_max, o exp(min(power,
    0))); skipped below alpha_min (3DGS uses 1/255).  A kept Gaussian's conic
    is positive definite (det > 0, a' > 0), so power <= 0 exactly; the clamp
    only keeps a rounding error near the centre from lifting alpha above o
    (3DGS drops such a pixel instead, which rounding could then decide).  Blending and early termination are the framework's (a pixel
    stops after the primitive that takes T below t_eps).
  * A hit pair is a (pixel, primitive) pair with the pixel inside the
    primitive's rectangle and not yet terminated.
  * Opacity is used as given (no activation).

The key path (steps 1-12 of project_gaussians) is evaluated in float64 with
one fixed order of correctly rounded operations and no fused multiply-add.
"""
from __future__ import annotations

import numpy as np

from .color import primitive_colors
from .render import RenderOptions

LOW_PASS = 0.3      # px^2 added to the diagonal of the 2D covariance
CLAMP = 1.3         # Jacobian evaluated with x/z, y/z clamped to 1.3x the view
LAMBDA_FLOOR = 0.1  # floor of the discriminant in the largest eigenvalue


def project_gaussians(scene, cam, tile_w=16, tile_h=16, z_near=0.2):
    """Key path and 2D splat of every Gaussian of `scene` in camera `cam`.

    Returns the fields of keys.project_all (keep, rect, nonempty, trect,
    depth, depth_bits, n_tiles) plus mean2d (P,2) pixel coordinates of the
    projected centre, cov2d (P,2,2) with the low-pass term, conic (P,3)
    (a', b', c') and radius (P,) (pixels)."""
    f64 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    q = f64(scene["quats"])
    xb = f64(scene["centers"])
    s = f64(scene["scales"])
    C = f64(cam.R)
    t = f64(cam.t)
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    W, H = int(cam.width), int(cam.height)
    zn = float(np.float32(z_near))
    P = q.shape[0]

    with np.errstate(all="ignore"):
        # 1. normalised quaternion
        qn = np.sqrt(((q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2]) + q[:, 3] * q[:, 3])
        w = q[:, 0] / qn
        x = q[:, 1] / qn
        y = q[:, 2] / qn
        z = q[:, 3] / qn
        # 2. rotation matrix
        xx = x * x; yy = y * y; zz = z * z
        xy = x * y; xz = x * z; yz = y * z
        wx = w * x; wy = w * y; wz = w * z
        Rp = np.empty((P, 3, 3))
        Rp[:, 0, 0] = 1.0 - 2.0 * (yy + zz)
        Rp[:, 0, 1] = 2.0 * (xy - wz)
        Rp[:, 0, 2] = 2.0 * (xz + wy)
        Rp[:, 1, 0] = 2.0 * (xy + wz)
        Rp[:, 1, 1] = 1.0 - 2.0 * (xx + zz)
        Rp[:, 1, 2] = 2.0 * (yz - wx)
        Rp[:, 2, 0] = 2.0 * (xz - wy)
        Rp[:, 2, 1] = 2.0 * (yz + wx)
        Rp[:, 2, 2] = 1.0 - 2.0 * (xx + yy)
        # 3. camera-frame rotation Rc = C Rp and centre mu = C x_B + t
        Rc = np.empty_like(Rp)
        for i in range(3):
            for j in range(3):
                Rc[:, i, j] = (C[i, 0] * Rp[:, 0, j] + C[i, 1] * Rp[:, 1, j]) + C[i, 2] * Rp[:, 2, j]
        mu = np.empty_like(xb)
        for i in range(3):
            mu[:, i] = ((C[i, 0] * xb[:, 0] + C[i, 1] * xb[:, 1]) + C[i, 2] * xb[:, 2]) + t[i]
        # 4. camera-frame covariance Sigma = Rc diag(s^2) Rc^T
        ss = s * s

        def sig(i, j):
            return (((Rc[:, i, 0] * ss[:, 0]) * Rc[:, j, 0] + (Rc[:, i, 1] * ss[:, 1]) * Rc[:, j, 1])
                    + (Rc[:, i, 2] * ss[:, 2]) * Rc[:, j, 2])

        S = [[sig(i, j) for j in range(3)] for i in range(3)]
        mz = mu[:, 2]
        # 5. near culling by the centre
        keep0 = mz > zn
        # 6. normalised image position, clamped for the Jacobian
        xzr = mu[:, 0] / mz
        yzr = mu[:, 1] / mz
        lxl = -CLAMP * (cx / fx)
        lxh = CLAMP * ((W - cx) / fx)
        lyl = -CLAMP * (cy / fy)
        lyh = CLAMP * ((H - cy) / fy)
        xc = np.minimum(np.maximum(xzr, lxl), lxh) * mz
        yc = np.minimum(np.maximum(yzr, lyl), lyh) * mz
        # 7. Jacobian rows (j00, 0, j02) and (0, j11, j12)
        zz2 = mz * mz
        j00 = fx / mz
        j02 = -(fx * xc) / zz2
        j11 = fy / mz
        j12 = -(fy * yc) / zz2
        # 8. 2D covariance J Sigma J^T (T = J Sigma first), then the low-pass term
        T0 = [j00 * S[0][k] + j02 * S[2][k] for k in range(3)]
        T1 = [j11 * S[1][k] + j12 * S[2][k] for k in range(3)]
        a = (T0[0] * j00 + T0[2] * j02) + LOW_PASS
        b = T0[1] * j11 + T0[2] * j12
        c = (T1[1] * j11 + T1[2] * j12) + LOW_PASS
        # 9. determinant and conic
        det = a * c - b * b
        keep = keep0 & (det > 0.0)
        ia = c / det
        ib = -b / det
        ic = a / det
        # 10. square screen bound from the largest eigenvalue
        mid = 0.5 * (a + c)
        lam = mid + np.sqrt(np.maximum(LAMBDA_FLOOR, mid * mid - det))
        r = np.ceil(3.0 * np.sqrt(lam))
        # 11. projected centre and pixel rectangle
        u = fx * xzr + cx
        v = fy * yzr + cy
        x0 = np.ceil((u - r) - 0.5)
        x1 = np.floor((u + r) - 0.5)
        y0 = np.ceil((v - r) - 0.5)
        y1 = np.floor((v + r) - 0.5)
        x0 = np.where(x0 > 0.0, x0, 0.0)
        x1 = np.where(x1 < W - 1.0, x1, W - 1.0)
        y0 = np.where(y0 > 0.0, y0, 0.0)
        y1 = np.where(y1 < H - 1.0, y1, H - 1.0)
        nonempty = keep & (x0 <= x1) & (y0 <= y1)
    rect = np.zeros((P, 4), dtype=np.int64)
    rect[nonempty, 0] = x0[nonempty].astype(np.int64)
    rect[nonempty, 1] = x1[nonempty].astype(np.int64)
    rect[nonempty, 2] = y0[nonempty].astype(np.int64)
    rect[nonempty, 3] = y1[nonempty].astype(np.int64)
    trect = np.zeros_like(rect)
    trect[:, 0] = rect[:, 0] // tile_w
    trect[:, 1] = rect[:, 1] // tile_w
    trect[:, 2] = rect[:, 2] // tile_h
    trect[:, 3] = rect[:, 3] // tile_h
    n_tiles = np.where(nonempty, (trect[:, 1] - trect[:, 0] + 1) * (trect[:, 3] - trect[:, 2] + 1), 0)
    # 12. depth key: camera-space z rounded to the nearest float32
    depth = mz.astype(np.float32)
    cov2d = np.stack([np.stack([a, b], -1), np.stack([b, c], -1)], -2)
    return dict(keep=keep, rect=rect, nonempty=nonempty, trect=trect, depth=depth,
                depth_bits=depth.view(np.uint32), n_tiles=n_tiles.astype(np.int64),
                mean2d=np.stack([u, v], 1), cov2d=cov2d, conic=np.stack([ia, ib, ic], 1),
                radius=r, jac=(j00, j02, j11, j12))


def gaussian_alpha(proj, p, cols, rows, opacity, alpha_max):
    """power and alpha of Gaussian p at pixels (cols, rows) (centres at
    +0.5).  Returns (power, alpha)."""
    u, v = proj["mean2d"][p]
    ia, ib, ic = proj["conic"][p]
    dx = (np.asarray(cols, dtype=np.float64) + 0.5) - u
    dy = (np.asarray(rows, dtype=np.float64) + 0.5) - v
    power = -0.5 * (ia * dx * dx + ic * dy * dy) - ib * dx * dy
    alpha = np.minimum(alpha_max, float(opacity) * np.exp(np.minimum(power, 0.0)))
    return power, alpha


def depth_order(proj):
    ids = np.nonzero(proj["nonempty"])[0]
    return ids[np.lexsort((ids, proj["depth_bits"][ids]))]


def render_view_gaussian(scene, cam, opts: RenderOptions = RenderOptions(), proj=None):
    """Render one view of Gaussians.  Returns dict(image (H,W,3), T (H,W),
    hit_pairs int)."""
    H, W = cam.height, cam.width
    if proj is None:
        proj = project_gaussians(scene, cam, 16, 16, opts.z_near)
    colors = primitive_colors(scene, cam)
    opac = np.asarray(scene["opacity"], dtype=np.float64)
    img = np.zeros((H, W, 3))
    T = np.ones((H, W))
    done = np.zeros((H, W), dtype=bool)
    hit_pairs = 0
    for p in depth_order(proj):
        x0, x1, y0, y1 = proj["rect"][p]
        rows, cols = np.mgrid[y0:y1 + 1, x0:x1 + 1]
        _, alpha = gaussian_alpha(proj, p, cols, rows, opac[p], opts.alpha_max)
        live = ~done[y0:y1 + 1, x0:x1 + 1]
        hit_pairs += int(live.sum())
        use = live.copy()
        if opts.alpha_min > 0:
            use &= alpha >= opts.alpha_min
        a = np.where(use, alpha, 0.0)
        Tb = T[y0:y1 + 1, x0:x1 + 1]
        img[y0:y1 + 1, x0:x1 + 1] += (a * Tb)[..., None] * colors[p]
        Tn = Tb * (1.0 - a)
        T[y0:y1 + 1, x0:x1 + 1] = Tn
        if opts.t_eps > 0:
            done[y0:y1 + 1, x0:x1 + 1] |= use & (Tn < opts.t_eps)
    img += T[..., None] * np.asarray(opts.bg, dtype=np.float64)
    return dict(image=img, T=T, hit_pairs=hit_pairs)


def render_pixels_gaussian(scene, cam, cols, rows, opts: RenderOptions = RenderOptions(), proj=None):
    """Colour, transmittance and hit count of individual pixels, each on its
    own from every Gaussian whose rectangle contains it (spot checks of large
    images).  Returns (colors (n,3), T (n,), hits (n,))."""
    if proj is None:
        proj = project_gaussians(scene, cam, 16, 16, opts.z_near)
    colors = primitive_colors(scene, cam)
    opac = np.asarray(scene["opacity"], dtype=np.float64)
    order = depth_order(proj)
    rect = proj["rect"][order]
    out_c = np.zeros((len(cols), 3))
    out_t = np.ones(len(cols))
    out_h = np.zeros(len(cols), dtype=np.int64)
    for n, (i, j) in enumerate(zip(cols, rows)):
        sel = order[(rect[:, 0] <= i) & (i <= rect[:, 1]) & (rect[:, 2] <= j) & (j <= rect[:, 3])]
        C = np.zeros(3)
        T = 1.0
        for p in sel:
            out_h[n] += 1
            _, alpha = gaussian_alpha(proj, p, np.array([i]), np.array([j]), opac[p], opts.alpha_max)
            a = float(alpha[0])
            if opts.alpha_min > 0 and a < opts.alpha_min:
                continue
            C += colors[p] * a * T
            T *= 1.0 - a
            if opts.t_eps > 0 and T < opts.t_eps:
                break
        out_c[n] = C + T * np.asarray(opts.bg, dtype=np.float64)
        out_t[n] = T
    return out_c, out_t, out_h
