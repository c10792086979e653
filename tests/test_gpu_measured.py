"""Parity at the launch configuration the benchmark times: density width
N = 16, colour MLP width 32 depth 2, 16x16 tiles with one pixel per thread,
backward batches of 8 instances, persistent launches whose work queue hands
out the heaviest tiles first -- with the forward's pair cache and without it
(re-evaluating every pair, as the 1M-primitive step runs).  Images, hit
pairs (total and per tile) and every gradient against the FP64 oracle, and
the first 1000 primitives of the 1920x1080 scene at a quarter of its
resolution against the oracle's gradients."""
import numpy as np
import pytest
import torch

import synthetic as S
from oracle.grad import autograd_loss_and_grads
from oracle.keys import project_all
from oracle.render import render_window
from tests.gpu_helpers import (IMG_TOL, check_images, config_for, grad_parity, options_for, run_forward, say)

pytestmark = pytest.mark.gpu

BENCH_TILE = (16, 16, 1, 8)
ALL_KEYS = ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "cmlp", "xi"]


@pytest.fixture(autouse=True)
def _announce(request):
    say(f"[gpu-test] {request.node.name}")
    yield
    torch.cuda.synchronize()


def _bench_scene():
    scene = S.custom_scene(1500, 16, color_mode=1, cmlp_width=32, cmlp_depth=2, seed=301)
    cams = S.make_cameras([(96, 72), (128, 72), (64, 48), (80, 80)], seed=302)
    return scene, cams, S.make_targets(cams, seed=303)


_REF = {}


def _oracle_grads(name, scene, cams, targets, cfg):
    if name not in _REF:
        L_ref, g_ref, _ = autograd_loss_and_grads(scene, cams, targets, options_for(cfg))
        _REF[name] = (L_ref, g_ref)
    return _REF[name]


@pytest.mark.parametrize("fwd_cache", [1, 0])
def test_bench_launch_images_pairs_and_gradients(fwd_cache):
    scene, cams, targets = _bench_scene()
    cfg = config_for(scene, tile=BENCH_TILE, persistent=1, fwd_cache=fwd_cache)
    fw = run_forward(scene, cams, cfg)
    assert fw["rast"].fwd_cache == bool(fwd_cache)
    check_images(fw, scene, cams, cfg)
    grad_parity(scene, cams, targets, cfg, ALL_KEYS, ref=_oracle_grads("bench", scene, cams, targets, cfg))


def test_bench_launch_per_tile_pairs_and_windows():
    """The per-tile hit-pair counts of a counting forward and the images of
    whole tiles against the oracle's render of each tile's window."""
    scene, cams, _ = _bench_scene()
    cfg = config_for(scene, tile=BENCH_TILE, persistent=1)
    fw = run_forward(scene, cams, cfg)
    tp = fw["rast"].tile_pairs().cpu().numpy().astype(np.int64)
    assert tp.sum() == fw["hit_pairs"]
    opts = options_for(cfg)
    base = 0
    for v, cam in enumerate(cams):
        ntx, nty = (cam.width + 15) // 16, (cam.height + 15) // 16
        proj = project_all(scene, cam, 16, 16, cfg.z_near)
        for t in range(ntx * nty):
            ty, tx = divmod(t, ntx)
            x0, y0 = 16 * tx, 16 * ty
            w, h = min(16, cam.width - x0), min(16, cam.height - y0)
            ref = render_window(scene, cam, x0, y0, w, h, opts, proj=proj)
            err = np.max(np.abs(fw["images"][v][y0:y0 + h, x0:x0 + w] - ref["image"]))
            assert err <= IMG_TOL, (v, t, err)
            assert tp[base + t] == ref["hit_pairs"], (v, t, tp[base + t], ref["hit_pairs"])
        base += ntx * nty
    say(f"  {base} tiles: per-tile hit pairs equal to the oracle's")


@pytest.mark.parametrize("fwd_cache", [1, 0])
def test_c3_subset_quarter_resolution_gradients(fwd_cache):
    """The first 1000 primitives of the 1920x1080 scene (200k primitives,
    N = 16, colour MLP W32 D2) seen by its camera at 480x270: every gradient
    against the oracle's float64 autograd route."""
    _, scene, _, _ = S.make_workload("C3")
    sub = S.subset_scene(scene, np.arange(1000))
    del scene
    cams = S.make_cameras([(480, 270)], seed=S.scenes.CAMERA_SEED)
    targets = S.make_targets(cams, seed=S.scenes.TARGET_SEED)
    cfg = config_for(sub, tile=BENCH_TILE, persistent=1, fwd_cache=fwd_cache)
    fw = run_forward(sub, cams, cfg)
    check_images(fw, sub, cams, cfg)
    grad_parity(sub, cams, targets, cfg, ALL_KEYS, fw=fw, ref=_oracle_grads("c3sub", sub, cams, targets, cfg))


def test_splat_render_backward_after_a_second_render():
    """Two renders on one Rasterizer, then the first one's backward: the
    backward sees that the workspace now holds the second render and
    restores the first before differentiating it."""
    import paper_2510_08491_amd as snp
    scene, cams, targets = _bench_scene()
    cfg = config_for(scene, tile=BENCH_TILE, persistent=1)
    # the Gaussians' opacity is not an input of the neural primitives
    p1 = {k: v for k, v in snp.params_to_device(scene).items() if k != "opacity"}
    scene2 = dict(scene)
    scene2["centers"] = scene["centers"] + np.float32(0.05)
    p2 = {k: v for k, v in snp.params_to_device(scene2).items() if k != "opacity"}
    for p in (p1, p2):
        for t in p.values():
            t.requires_grad_(True)
    tg = torch.from_numpy(np.concatenate([t.ravel() for t in targets])).cuda()
    rast = snp.Rasterizer(cfg, scene["P"], cams)
    img1, _ = snp.splat_render(rast, p1)
    img2, _ = snp.splat_render(rast, p2)
    (img1 - tg).abs().mean().backward()
    g_late = {k: v.grad.clone() for k, v in p1.items()}
    for t in p1.values():
        t.grad = None
    fresh = snp.Rasterizer(cfg, scene["P"], cams)
    img1b, _ = snp.splat_render(fresh, p1)
    assert torch.equal(img1, img1b)
    (img1b - tg).abs().mean().backward()
    for k, v in p1.items():
        a, b = g_late[k].double(), v.grad.double()
        assert torch.max(torch.abs(a - b)) <= 1e-5 * torch.max(torch.abs(b)) + 1e-12, k
    del img2
