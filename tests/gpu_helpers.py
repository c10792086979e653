"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and fetch its results; compare against the oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

import paper_2510_08491_amd as snp
from oracle.grad import autograd_loss_and_grads
from oracle.render import RenderOptions, render_view

IMG_TOL = 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def config_for(scene, tile=(16, 16, 1), persistent=0, t_eps=1e-4, alpha_min=0.0, alpha_max=0.99, bg=(0, 0, 0),
               fwd_cache=1, bin_order=0):
    return snp.RenderConfig(n_hidden=int(scene["N"]), omega0=float(scene["omega0"]),
                            primitive=int(scene.get("primitive", 0)), bin_order=bin_order,
                            time=float(scene.get("time", 0.0)),
                            color_mode=int(scene["color_mode"]), cmlp_width=int(scene.get("cmlp_width", 0)),
                            cmlp_depth=int(scene.get("cmlp_depth", 0)), tile_w=tile[0], tile_h=tile[1],
                            px_per_lane=tile[2], bwd_batch=tile[3] if len(tile) > 3 else 0, t_eps=t_eps,
                            alpha_min=alpha_min, alpha_max=alpha_max, bg=tuple(bg), persistent=persistent,
                            fwd_cache=fwd_cache)


def options_for(cfg: snp.RenderConfig) -> RenderOptions:
    return RenderOptions(z_near=cfg.z_near, t_eps=cfg.t_eps, alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max,
                         bg=tuple(cfg.bg))


def run_forward(scene, cams, cfg, count_pairs=True, capacity=None):
    """preprocess, bin, sort, forward.  Returns dict of numpy results."""
    params = snp.params_to_device(scene)
    rast = snp.Rasterizer(cfg, scene["P"], cams, capacity=capacity)
    inst = rast.prepare(params)
    images, T = rast.new_images()
    rast.forward(params, images, T, count_pairs=count_pairs)
    _, inst2, pairs = rast.read_status()
    torch.cuda.synchronize()
    n = min(inst, rast.capacity)
    out = dict(rast=rast, params=params, images_t=images, T_t=T, instances=inst, hit_pairs=pairs,
               images=[im.cpu().numpy() for im in rast.split_images(images)],
               keys=rast.keys(n).cpu().numpy().view(np.uint64), values=rast.values(n).cpu().numpy().view(np.uint32),
               ranges=rast.ranges().cpu().numpy().astype(np.int64), rects=rast.rects().cpu().numpy(),
               depth_bits=rast.depth_bits().cpu().numpy().view(np.uint32),
               tile_counts=rast.tile_counts().cpu().numpy())
    Ts, off = [], 0
    Tn = T.cpu().numpy()
    for c in cams:
        Ts.append(Tn[off:off + c.width * c.height].reshape(c.height, c.width))
        off += c.width * c.height
    out["T"] = Ts
    return out


def run_backward(fw, targets, n_norm=None):
    """L1 loss against the targets and the gradients of every parameter."""
    rast = fw["rast"]
    tg = torch.from_numpy(np.concatenate([np.asarray(t, np.float32).ravel() for t in targets])).cuda()
    loss, dL = rast.loss_l1(fw["images_t"], tg, n_norm=n_norm)
    grads = snp.zeros_like_params(fw["params"])
    rast.backward(fw["params"], fw["images_t"], dL, grads)
    torch.cuda.synchronize()
    return float(loss.item()), {k: v.cpu().numpy() for k, v in grads.items()}


def grad_close(g, ref, rel=1e-3, elem_rel=1e-3, elem_floor=1e-2, kink=None):
    """Gradient acceptance: max |g - ref| <= rel * max |ref| over the tensor,
    and elementwise relative error <= elem_rel on the elements with
    |ref| >= elem_floor * max |ref| (minus those flagged in `kink`)."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.max(np.abs(ref))
    if scale == 0:
        return np.max(np.abs(g)) == 0, 0.0, 0.0
    err = np.max(np.abs(g - ref)) / scale
    big = np.abs(ref) >= elem_floor * scale
    if kink is not None:
        big &= ~kink
    e_rel = np.max(np.abs(g - ref)[big] / np.abs(ref[big])) if np.any(big) else 0.0
    return (err <= rel and e_rel <= elem_rel), err, e_rel


def pairs_must_match(cfg, oracle_T_min):
    """Hit pairs are decided in float64 on both sides, so their counts are
    equal -- unless a pixel's transmittance came near the early-termination
    threshold, where float32 and float64 may stop at different primitives."""
    return cfg.t_eps == 0 or oracle_T_min > 2.0 * cfg.t_eps


def check_images(fw, scene, cams, cfg, tol=IMG_TOL):
    """Every view against the oracle's full render (image and T within tol),
    and the hit-pair count (equal, see pairs_must_match)."""
    opts = options_for(cfg)
    pairs, tmin = 0, 1.0
    for v, cam in enumerate(cams):
        ref = render_view(scene, cam, opts)
        err = np.max(np.abs(fw["images"][v] - ref["image"]))
        terr = np.max(np.abs(fw["T"][v] - ref["T"]))
        say(f"  view {v} {cam.width}x{cam.height}: image err {err:.2e}, T err {terr:.2e}")
        assert err <= tol and terr <= tol
        pairs += ref["hit_pairs"]
        tmin = min(tmin, float(ref["T"].min()))
    say(f"  hit pairs gpu {fw['hit_pairs']} oracle {pairs}")
    if pairs_must_match(cfg, tmin):
        assert fw["hit_pairs"] == pairs
    else:
        assert abs(fw["hit_pairs"] - pairs) <= 1e-3 * pairs + 2


def grad_parity(scene, cams, targets, cfg, keys, ref=None, fw=None):
    """HIP loss and gradients (through the C ABI) against the oracle's
    float64 autograd route; `ref` may carry a precomputed (loss, grads)."""
    fw = run_forward(scene, cams, cfg) if fw is None else fw
    loss, g = run_backward(fw, targets)
    if ref is None:
        L_ref, g_ref, _ = autograd_loss_and_grads(scene, cams, targets, options_for(cfg))
    else:
        L_ref, g_ref = ref
    say(f"  loss gpu {loss:.8f} oracle {L_ref:.8f}")
    assert abs(loss - L_ref) <= 1e-5
    bad = []
    for k in keys:
        ok, err, erel = grad_close(g[k], g_ref[k])
        worst = np.unravel_index(np.argmax(np.abs(g[k] - g_ref[k])), g[k].shape)
        say(f"  grad {k}: max err / max {err:.2e}, elementwise rel {erel:.2e}, worst at {worst}")
        if not ok:
            bad.append(k)
    assert not bad, bad
