"""The per-(primitive, view) colour network on the device (its forward and
adjoint run as 16x16x4 products over 16 views per wave) against the float64
oracle, in the shapes the other tests leave out: three hidden layers of 32
units, the relighting inputs, and more than 16 views, so that each wave takes
a second, partly filled block of views (Sec. 3.1 colour; the appendix on
relighting for colour mode 3)."""
import pytest

import synthetic as S
from tests.gpu_helpers import check_images, config_for, grad_parity, run_forward

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("color_mode,width,depth,n_views", [(1, 32, 3, 20), (3, 32, 2, 18), (1, 16, 1, 17)])
def test_colour_network_many_views(color_mode, width, depth, n_views):
    scene = S.custom_scene(150, 8, color_mode=color_mode, cmlp_width=width, cmlp_depth=depth, seed=311 + n_views)
    sizes = [(24 + 8 * (i % 3), 24 + 8 * ((i + 1) % 3)) for i in range(n_views)]
    cams = S.make_cameras(sizes, seed=312 + n_views, lights=color_mode == 3)
    targets = S.make_targets(cams, seed=313 + n_views)
    cfg = config_for(scene, tile=(16, 16, 1), persistent=1)
    fw = run_forward(scene, cams, cfg)
    check_images(fw, scene, cams, cfg)
    keys = ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "cmlp", "xi"]
    if color_mode == 3:
        keys.append("colors")
    grad_parity(scene, cams, targets, cfg, keys, fw=fw)
