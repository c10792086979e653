"""Splatting renderer of the oracle (FP64): images, hit-pair counts and loss.

Test infrastructure only (see the package docstring).

Per view and pixel, the primitives whose bounds cover the pixel are taken in
ascending (depth bits, index) order (the tiling/sorting readings in
oracle.keys).  For each one, the ray-ellipsoid intersection gives the chord
[t_in, t_out]; the exact integral of the primitive's density over the chord
(Eq. 7-8) gives alpha = 1 - exp(-max(0, integral)) (Eq. 9); the colours are
blended front to back, C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j) (Eq. 4).

Readings of what the paper leaves open (3DGS conventions, all switchable):
  * alpha_max (default 0.99): alpha is clamped to at most alpha_max;
  * alpha_min (default 0): primitives with alpha < alpha_min are skipped;
  * early termination: after blending a primitive, a pixel whose
    transmittance T fell below t_eps (default 1e-4) takes no further
    primitives (t_eps = 0 disables it);
  * background: C += T_final * bg, bg = 0 by default;
  * a (pixel, primitive) pair is a "hit pair" when the ray meets the
    ellipsoid (disc > 0) and the pixel has not terminated yet; clamped pairs
    (integral <= 0) count as hits.

The image is computed by looping over primitives in depth order and updating
the pixels of each primitive's bounding rectangle at once (every hit pixel lies
in that rectangle).  The loss is the mean absolute error over all pixels,
channels and views.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .color import primitive_colors, ray_colors
from .density import chord_integral
from .geometry import intersect_ellipsoid, pixel_rays, quat_to_rotmat
from .keys import project_all


@dataclasses.dataclass
class RenderOptions:
    z_near: float = 0.2
    t_eps: float = 1e-4
    alpha_min: float = 0.0
    alpha_max: float = 0.99
    bg: tuple = (0.0, 0.0, 0.0)


def primitive(scene, p, R=None):
    """Primitive p of a scene as the dict the density functions take."""
    return dict(center=scene["centers"][p], scale=scene["scales"][p],
                w1=scene["w1"][p], b1=scene["b1"][p], w2=scene["w2"][p],
                b2=scene["b2"][p], omega0=scene["omega0"],
                wt=None if scene.get("wt") is None else scene["wt"][p], time=scene.get("time", 0.0),
                R=quat_to_rotmat(scene["quats"][p]) if R is None else R)


def splat_alpha(o, d, prim, return_t_in=False):
    """disc and alpha (Eq. 9) of one primitive for rays (o, d); alpha is 0
    where the ray misses.  Returns (disc, alpha_unclamped_integral, alpha)
    (and t_in, NaN for misses, with return_t_in)."""
    disc, t_in, t_out = intersect_ellipsoid(o, d, prim["center"], prim["scale"], prim["R"])
    hit = disc > 0
    integral = np.zeros(disc.shape)
    if np.any(hit):
        integral[hit] = chord_integral(o, d[hit], t_in[hit], t_out[hit], prim)
    alpha = np.where(hit, 1.0 - np.exp(-np.maximum(integral, 0.0)), 0.0)
    if return_t_in:
        return disc, integral, alpha, t_in
    return disc, integral, alpha


def pair_colors(scene, p, cam, colors, o, d, t_in, hit):
    """Colour of primitive p for each ray: its per-view colour, or (colour
    mode 4) the per-ray relighting colour at the entry point (0 for misses)."""
    if scene["color_mode"] != 4:
        return np.broadcast_to(colors[p], d.shape)
    out = np.zeros(d.shape)
    if np.any(hit):
        out[hit] = ray_colors(scene, p, cam, o, d[hit], t_in[hit])
    return out


def depth_order(proj):
    """Indices of the primitives with a non-empty rectangle, ascending in
    (depth bits, index)."""
    ids = np.nonzero(proj["nonempty"])[0]
    order = np.lexsort((ids, proj["depth_bits"][ids]))
    return ids[order]


def render_view(scene, cam, opts: RenderOptions = RenderOptions(), return_trace=False):
    """Render one view.  Returns dict(image (H,W,3), T (H,W), hit_pairs int)."""
    H, W = cam.height, cam.width
    proj = project_all(scene, cam, 16, 16, opts.z_near)
    colors = primitive_colors(scene, cam) if scene["color_mode"] != 4 else None
    Rs = quat_to_rotmat(scene["quats"])
    img = np.zeros((H, W, 3))
    T = np.ones((H, W))
    done = np.zeros((H, W), dtype=bool)
    hit_pairs = 0
    for p in depth_order(proj):
        x0, x1, y0, y1 = proj["rect"][p]
        rows, cols = np.mgrid[y0:y1 + 1, x0:x1 + 1]
        o, d = pixel_rays(cam, cols, rows)
        disc, _, alpha, t_in = splat_alpha(o, d, primitive(scene, p, Rs[p]), return_t_in=True)
        live = ~done[y0:y1 + 1, x0:x1 + 1]
        hit = (disc > 0) & live
        hit_pairs += int(hit.sum())
        alpha = np.minimum(alpha, opts.alpha_max)
        use = hit & (alpha >= opts.alpha_min) if opts.alpha_min > 0 else hit
        a = np.where(use, alpha, 0.0)
        Tb = T[y0:y1 + 1, x0:x1 + 1]
        img[y0:y1 + 1, x0:x1 + 1] += (a * Tb)[..., None] * pair_colors(scene, p, cam, colors, o, d, t_in, disc > 0)
        Tn = Tb * (1.0 - a)
        T[y0:y1 + 1, x0:x1 + 1] = Tn
        if opts.t_eps > 0:
            done[y0:y1 + 1, x0:x1 + 1] |= use & (Tn < opts.t_eps)
    img += T[..., None] * np.asarray(opts.bg, dtype=np.float64)
    return dict(image=img, T=T, hit_pairs=hit_pairs)


def render_views(scene, cams, opts: RenderOptions = RenderOptions()):
    return [render_view(scene, c, opts) for c in cams]


def render_pixels(scene, cam, cols, rows, opts: RenderOptions = RenderOptions(), proj=None):
    """Colour and transmittance of individual pixels, each computed on its
    own from all primitives whose rectangle contains it (for spot checks of
    images too large to render whole).  Returns (colors (n,3), T (n,), hits (n,))."""
    if proj is None:
        proj = project_all(scene, cam, 16, 16, opts.z_near)
    colors = primitive_colors(scene, cam) if scene["color_mode"] != 4 else None
    order = depth_order(proj)
    rect = proj["rect"][order]
    out_c = np.zeros((len(cols), 3))
    out_t = np.ones(len(cols))
    out_h = np.zeros(len(cols), dtype=np.int64)
    for n, (i, j) in enumerate(zip(cols, rows)):
        sel = order[(rect[:, 0] <= i) & (i <= rect[:, 1]) & (rect[:, 2] <= j) & (j <= rect[:, 3])]
        o, d = pixel_rays(cam, np.array([i]), np.array([j]))
        C = np.zeros(3)
        T = 1.0
        for p in sel:
            disc, _, alpha, t_in = splat_alpha(o, d, primitive(scene, p), return_t_in=True)
            if disc[0] <= 0:
                continue
            out_h[n] += 1
            a = min(alpha[0], opts.alpha_max)
            if opts.alpha_min > 0 and a < opts.alpha_min:
                continue
            C += pair_colors(scene, p, cam, colors, o, d, t_in, disc > 0)[0] * a * T
            T *= 1.0 - a
            if opts.t_eps > 0 and T < opts.t_eps:
                break
        out_c[n] = C + T * np.asarray(opts.bg, dtype=np.float64)
        out_t[n] = T
    return out_c, out_t, out_h


def window_camera(cam, x0, y0, w, h):
    """The camera of a w x h window of `cam`'s image whose top-left pixel is
    (x0, y0): the same pose and focal lengths, the principal point moved by
    (-x0, -y0).  Its pixel (i, j) has the ray of `cam`'s pixel (x0+i, y0+j)
    (exactly, when cx - x0 and cy - y0 are exact in float32)."""
    import dataclasses as _dc
    return _dc.replace(cam, width=int(w), height=int(h), cx=float(cam.cx) - x0, cy=float(cam.cy) - y0)


def render_window(scene, cam, x0, y0, w, h, opts: RenderOptions = RenderOptions(), proj=None):
    """Image, transmittance and hit-pair count of the w x h window at (x0, y0)
    of view `cam`, without rendering the whole view: the primitives whose
    rectangle in `cam` meets the window (in index order, so their depth
    order is kept) rendered through the window's camera.  Every pixel a
    primitive hits lies inside its rectangle, so the window's pixels see
    exactly the pairs they see in the full view.  Returns
    dict(image (h,w,3), T (h,w), hit_pairs, primitives)."""
    if proj is None:
        proj = project_all(scene, cam, 16, 16, opts.z_near)
    r = proj["rect"]
    meets = proj["nonempty"] & (r[:, 0] <= x0 + w - 1) & (r[:, 1] >= x0) & (r[:, 2] <= y0 + h - 1) & (r[:, 3] >= y0)
    ids = np.nonzero(meets)[0]
    sub = dict(scene)
    for k, v in scene.items():
        if isinstance(v, np.ndarray) and v.ndim >= 1 and v.shape[0] == scene["P"] and k != "P":
            sub[k] = v[ids]
    sub["P"] = len(ids)
    wcam = window_camera(cam, x0, y0, w, h)
    if len(ids) == 0:
        T = np.ones((h, w))
        return dict(image=T[..., None] * np.asarray(opts.bg, dtype=np.float64), T=T, hit_pairs=0, primitives=0)
    out = render_view(sub, wcam, opts)
    out["primitives"] = len(ids)
    return out


def l1_loss(images, targets):
    """Mean absolute error over all views, pixels and channels, and its
    gradient with respect to each image (sign(C - target) / count)."""
    n = sum(int(np.asarray(t).size) for t in targets)
    L = sum(float(np.abs(np.asarray(i, dtype=np.float64) - np.asarray(t, dtype=np.float64)).sum())
            for i, t in zip(images, targets)) / n
    grads = [np.sign(np.asarray(i, dtype=np.float64) - np.asarray(t, dtype=np.float64)) / n
             for i, t in zip(images, targets)]
    return L, grads
