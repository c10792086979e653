"""Gradients of the oracle's L1 loss, by two independent routes (FP64).

Test infrastructure only (see the package docstring).

Route 1 re-implements the renderer of oracle.render in torch.float64 on the
CPU and differentiates it with autograd.  It is written separately from the
numpy renderer: the chord integral uses the antiderivative literally,
S(t_out) - S(t_in) (Eq. 7-8), instead of the midpoint form, so agreement of
the two renderers also checks both integral forms.  Discrete decisions
(culling, rectangles, depth order, termination) are taken from the numpy key
path and carry no gradient.

Route 2 is central finite differences of the numpy renderer's loss.

The paper's renderer is differentiable (Sec. 6: a differentiable
splatting-based renderer) but its adjoint is not described; these routes
define the reference gradient of the loss with respect to centres, scales,
raw quaternions, W1, b1, W2, b2 and colours (or colour-MLP weights).
"""
from __future__ import annotations

import numpy as np
import torch

from .keys import project_all
from .render import RenderOptions, depth_order, l1_loss, render_views

PARAM_KEYS = ("centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors", "cmlp", "xi", "sh", "wt", "sh_t")


def _rotmat_t(q):
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def _sh_basis_t(d):
    """Real spherical harmonics of degrees 0..3 (the 16 of oracle.color.sh_basis),
    written again for autograd."""
    x, y, z = d.unbind(-1)
    pi = np.pi
    c0 = 0.5 * np.sqrt(1 / pi)
    c1 = np.sqrt(3 / (4 * pi))
    c2a, c2b, c2c = 0.5 * np.sqrt(15 / pi), 0.25 * np.sqrt(5 / pi), 0.25 * np.sqrt(15 / pi)
    c3a, c3b = 0.25 * np.sqrt(35 / (2 * pi)), 0.5 * np.sqrt(105 / pi)
    c3c, c3d, c3e = 0.25 * np.sqrt(21 / (2 * pi)), 0.25 * np.sqrt(7 / pi), 0.25 * np.sqrt(105 / pi)
    return torch.stack([
        torch.full_like(x, c0), c1 * y, c1 * z, c1 * x,
        c2a * x * y, c2a * y * z, c2b * (3 * z * z - 1), c2a * x * z, c2c * (x * x - y * y),
        c3a * y * (3 * x * x - y * y), c3b * x * y * z, c3c * y * (5 * z * z - 1), c3d * (5 * z ** 3 - 3 * z),
        c3c * x * (5 * z * z - 1), c3e * z * (x * x - y * y), c3a * x * (x * x - 3 * y * y)], -1)


def _colors_t(params, meta, o, cam=None):
    if meta["color_mode"] == 0:
        return params["colors"]
    dirv = params["centers"] - o
    dirv = dirv / torch.linalg.norm(dirv, dim=1, keepdim=True)
    if meta["color_mode"] == 2:
        sh = params["sh"]
        if params.get("sh_t") is not None:
            # time-dependent zero-order coefficient: polynomial and Fourier terms
            t = float(meta.get("time", 0.0))
            basis = torch.tensor([t, t * t, t ** 3, t ** 4] + [float(np.cos(i * t)) for i in (1, 2, 3, 4)] +
                                 [float(np.sin(i * t)) for i in (1, 2, 3, 4)], dtype=torch.float64)
            s0 = sh[:, 0, :] + torch.einsum("k,pkc->pc", basis, params["sh_t"])
            sh = torch.cat([s0[:, None, :], sh[:, 1:, :]], 1)
        return torch.relu(0.5 + torch.einsum("pk,pkc->pc", _sh_basis_t(dirv), sh))
    parts = [dirv]
    if meta["color_mode"] == 3:
        ld = torch.tensor(np.asarray(cam.light, dtype=np.float32).astype(np.float64)) - params["centers"]
        parts.append(ld / torch.linalg.norm(ld, dim=1, keepdim=True))
    h = torch.cat(parts + [params["xi"]], 1)
    vec = params["cmlp"]
    width, depth = meta["cmlp_width"], meta["cmlp_depth"]
    dims = [h.shape[1]] + [width] * depth + [3]
    pos = 0
    for li, (a, b) in enumerate(zip(dims[:-1], dims[1:])):
        Wm = vec[:, pos:pos + a * b].reshape(-1, b, a)
        pos += a * b
        bb = vec[:, pos:pos + b]
        pos += b
        h = torch.einsum("poi,pi->po", Wm, h) + bb
        if li + 1 < len(dims) - 1:
            h = torch.relu(h)
    if meta["color_mode"] == 3:
        return params["colors"] + torch.sigmoid(h)
    return torch.sigmoid(h)


def _mlp_t(vec, width, depth, h):
    """The packed colour network of one primitive on inputs h (..., n_in):
    ReLU hidden layers, sigmoid output."""
    dims = [h.shape[-1]] + [width] * depth + [3]
    pos = 0
    for li, (a, b) in enumerate(zip(dims[:-1], dims[1:])):
        Wm = vec[pos:pos + a * b].reshape(b, a)
        pos += a * b
        bb = vec[pos:pos + b]
        pos += b
        h = h @ Wm.T + bb
        if li + 1 < len(dims) - 1:
            h = torch.relu(h)
    return torch.sigmoid(h)


def render_view_torch(params, meta, cam, opts: RenderOptions = RenderOptions(), proj=None):
    """Differentiable float64 render of one view (route 1)."""
    if proj is None:
        np_scene = {k: (params[k].detach().numpy() if params.get(k) is not None else None)
                    for k in PARAM_KEYS}
        proj = project_all(np_scene, cam, 16, 16, opts.z_near)
    H, W = cam.height, cam.width
    Rinv = torch.linalg.inv(torch.tensor(np.asarray(cam.R, dtype=np.float64)))
    tc = torch.tensor(np.asarray(cam.t, dtype=np.float64))
    o = -Rinv @ tc
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    Rp = _rotmat_t(params["quats"])
    per_ray = meta["color_mode"] == 4
    colors = None if per_ray else _colors_t(params, meta, o, cam)
    om = float(meta["omega0"])
    img = torch.zeros(H, W, 3, dtype=torch.float64)
    T = torch.ones(H, W, dtype=torch.float64)
    done = torch.zeros(H, W, dtype=torch.bool)
    for p in depth_order(proj):
        x0, x1, y0, y1 = (int(v) for v in proj["rect"][p])
        jj, ii = torch.meshgrid(torch.arange(y0, y1 + 1, dtype=torch.float64),
                                torch.arange(x0, x1 + 1, dtype=torch.float64), indexing="ij")
        dc = torch.stack([(ii + 0.5 - cx) / fx, (jj + 0.5 - cy) / fy, torch.ones_like(ii)], -1)
        d = dc @ Rinv.T
        d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
        xb, s, R = params["centers"][p], params["scales"][p], Rp[p]
        op = ((o - xb) @ R) / s
        dp = (d @ R) / s
        A = (dp * dp).sum(-1)
        B = dp @ op
        Cq = op @ op - 1.0
        disc = B * B - A * Cq
        live = ~done[y0:y1 + 1, x0:x1 + 1]
        hit = (disc > 0) & live
        if not bool(hit.any()):
            continue
        sq = torch.sqrt(torch.where(disc > 0, disc, torch.ones_like(disc)))
        t_in = (-B - sq) / A
        t_out = (-B + sq) / A
        m = torch.max(s)
        a = (d @ params["w1"][p].T) / m                      # (..., N)
        c = ((o - xb) @ params["w1"][p].T) / m + params["b1"][p]
        w2 = params["w2"][p]
        tph = float(meta.get("time", 0.0)) * params["wt"][p] if params.get("wt") is not None else 0.0
        tiny = a.abs() < 1e-9
        a_safe = torch.where(tiny, torch.ones_like(a), a)

        def S(t):
            return (w2 * torch.sin(om * (a_safe * t[..., None] + c) + tph) / (om * a_safe))

        lit = S(t_out) - S(t_in)
        lim = w2 * torch.cos(om * (a * (0.5 * (t_in + t_out))[..., None] + c) + tph) * (t_out - t_in)[..., None]
        integral = torch.where(tiny, lim, lit).sum(-1) + params["b2"][p] * (t_out - t_in)
        alpha = 1.0 - torch.exp(-torch.clamp(integral, min=0.0))
        alpha = torch.clamp(alpha, max=opts.alpha_max)
        use = hit
        if opts.alpha_min > 0:
            use = use & (alpha.detach() >= opts.alpha_min)
        alpha = torch.where(use, alpha, torch.zeros_like(alpha))
        if per_ray:
            # relighting colour per ray at the entry point (colour mode 4)
            x_in = (o + t_in[..., None] * d - xb) / m
            lv = torch.tensor(np.asarray(cam.light, dtype=np.float32).astype(np.float64)) - xb
            lv = lv / torch.linalg.norm(lv)
            inp = torch.cat([x_in, d, lv.expand(d.shape)], -1)
            col = params["colors"][p] + _mlp_t(params["cmlp"][p], meta["cmlp_width"], meta["cmlp_depth"], inp)
        else:
            col = colors[p]
        Tb = T[y0:y1 + 1, x0:x1 + 1]
        img = img.clone()
        img[y0:y1 + 1, x0:x1 + 1] = img[y0:y1 + 1, x0:x1 + 1] + (alpha * Tb)[..., None] * col
        Tn = Tb * (1.0 - alpha)
        T = T.clone()
        T[y0:y1 + 1, x0:x1 + 1] = Tn
        if opts.t_eps > 0:
            done[y0:y1 + 1, x0:x1 + 1] |= use & (Tn.detach() < opts.t_eps)
    img = img + T[..., None] * torch.tensor(opts.bg, dtype=torch.float64)
    return img, T


def autograd_loss_and_grads(scene, cams, targets, opts: RenderOptions = RenderOptions()):
    """Route 1: loss and d loss / d params (numpy float64 arrays)."""
    meta = dict(color_mode=scene["color_mode"], omega0=scene["omega0"], time=scene.get("time", 0.0),
                cmlp_width=scene.get("cmlp_width", 0), cmlp_depth=scene.get("cmlp_depth", 0))
    params = {}
    for k in PARAM_KEYS:
        if scene.get(k) is not None:
            params[k] = torch.tensor(np.asarray(scene[k], dtype=np.float64), requires_grad=True)
    total = torch.zeros((), dtype=torch.float64)
    n = 0
    images = []
    for cam, tgt in zip(cams, targets):
        img, _ = render_view_torch(params, meta, cam, opts)
        images.append(img.detach().numpy())
        total = total + (img - torch.tensor(np.asarray(tgt, dtype=np.float64))).abs().sum()
        n += int(np.asarray(tgt).size)
    loss = total / n
    loss.backward()
    grads = {k: (v.grad.numpy().copy() if v.grad is not None else np.zeros(v.shape))
             for k, v in params.items()}
    return float(loss.detach()), grads, images


def numpy_loss(scene, cams, targets, opts: RenderOptions = RenderOptions()):
    """L1 loss of the numpy renderer."""
    imgs = [r["image"] for r in render_views(scene, cams, opts)]
    return l1_loss(imgs, targets)[0]


def fd_gradient(scene, cams, targets, key, index, rel_step=1e-6, opts: RenderOptions = RenderOptions()):
    """Route 2: central difference of the numpy loss in one parameter element,
    step h = rel_step * max(1, |theta|)."""
    base = np.asarray(scene[key], dtype=np.float64)
    h = rel_step * max(1.0, abs(float(base[index])))
    vals = []
    for sgn in (+1.0, -1.0):
        arr = base.copy()
        arr[index] += sgn * h
        sc = dict(scene)
        sc[key] = arr
        vals.append(numpy_loss(sc, cams, targets, opts))
    return (vals[0] - vals[1]) / (2.0 * h)
