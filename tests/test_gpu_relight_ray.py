"""Per-ray relighting colour (colour mode 4: c_dc + a colour network of the
ray's entry point, the ray direction and the light direction, evaluated per
(pixel, primitive) pair inside the rasterizers) through the C ABI: images,
hit pairs and every gradient -- the network's weights, c_dc, and the
geometry through the entry point, the direction and the light direction --
against the FP64 oracle."""
import pytest
import torch

import synthetic as S
from tests.gpu_helpers import check_images, config_for, grad_parity, run_forward, say

pytestmark = pytest.mark.gpu

KEYS = ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors", "cmlp"]


@pytest.fixture(autouse=True)
def _announce(request):
    say(f"[gpu-test] {request.node.name}")
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("N,persistent,fwd_cache", [(8, 1, 1), (16, 0, 0), (16, 1, 1)])
def test_per_ray_colour_image_and_gradients(N, persistent, fwd_cache):
    scene = S.custom_scene(300, N, color_mode=4, cmlp_width=16, cmlp_depth=1, seed=191 + N)
    cams = S.make_cameras([(64, 56), (56, 64), (48, 40)], seed=192, lights=True)
    targets = S.make_targets(cams, seed=193)
    cfg = config_for(scene, tile=(16, 16, 1), persistent=persistent, fwd_cache=fwd_cache)
    fw = run_forward(scene, cams, cfg)
    check_images(fw, scene, cams, cfg)
    grad_parity(scene, cams, targets, cfg, KEYS, fw=fw)


def test_per_ray_colour_dense_scene_with_termination():
    """Larger primitives so that pixels terminate: the colour of every pair
    up to termination, and alpha_max clamps."""
    scene = S.custom_scene(200, 8, color_mode=4, cmlp_width=16, cmlp_depth=1, seed=197, scale_lo=0.1, scale_hi=0.35)
    scene["w2"] = scene["w2"] * 8
    cams = S.make_cameras([(48, 48), (40, 56)], seed=198, lights=True)
    targets = S.make_targets(cams, seed=199)
    cfg = config_for(scene, tile=(16, 16, 1), persistent=1, alpha_max=0.9)
    fw = run_forward(scene, cams, cfg)
    check_images(fw, scene, cams, cfg)
    grad_parity(scene, cams, targets, cfg, KEYS, fw=fw)
