"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: tile lists, sort order, rectangles and depth keys bit-exact; images and
transmittance within 1e-4 max abs; gradients within 1e-3 (max error over a
tensor relative to its largest entry, and elementwise on entries above 1% of
it); hit-pair counts equal (both sides decide a hit with a float64
discriminant near the silhouette), except in scenes whose pixels come near
the early-termination threshold."""
import numpy as np
import pytest
import torch

import synthetic as S
from oracle.grad import autograd_loss_and_grads
from oracle.keys import project_all, sorted_instances, tile_lists, tile_ranges
from oracle.render import render_pixels, render_view
from tests.gpu_helpers import (IMG_TOL, check_images, config_for, grad_close, grad_parity, options_for,
                               run_backward, run_forward, say)

pytestmark = pytest.mark.gpu



@pytest.fixture(autouse=True)
def _announce(request):
    say(f"[gpu-test] {request.node.name}")
    yield
    torch.cuda.synchronize()


def _check_keys(fw, scene, cams, cfg):
    lists = tile_lists(scene, cams, cfg.tile_w, cfg.tile_h, cfg.z_near)
    keys, vals = sorted_instances(lists)
    ranges = tile_ranges(lists)
    assert fw["instances"] == len(keys)
    assert np.array_equal(fw["keys"], keys)
    assert np.array_equal(fw["values"], vals)
    # empty tiles have no unique position: compare non-empty ranges exactly
    nonempty = ranges[:, 1] > ranges[:, 0]
    assert np.array_equal(fw["ranges"][nonempty], ranges[nonempty])
    assert np.all(fw["ranges"][~nonempty, 0] == fw["ranges"][~nonempty, 1])
    for v, cam in enumerate(cams):
        pr = project_all(scene, cam, cfg.tile_w, cfg.tile_h, cfg.z_near)
        ne = pr["nonempty"]
        assert np.array_equal(fw["tile_counts"][v], pr["n_tiles"].astype(np.int32))
        assert np.array_equal(fw["rects"][v][ne], pr["rect"][ne].astype(np.int32))
        assert np.array_equal(fw["depth_bits"][v][ne], pr["depth_bits"][ne])


def test_wave_reduction_selftest():
    import ctypes as C
    from paper_2510_08491_amd import _lib
    x = torch.randn(64 * 8, device="cuda")
    y = torch.empty_like(x)
    _lib.check(_lib.lib().snp_selftest_wave_sum(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 8,
                                                 C.c_void_p(torch.cuda.current_stream().cuda_stream)), "selftest")
    torch.cuda.synchronize()
    ref = x.view(8, 64).double().sum(1)
    assert torch.allclose(y.view(8, 64)[:, 0].double(), ref, atol=1e-4)


def test_c1_keys_and_image():
    cfg0, scene, cams, _ = S.make_workload("C1")
    cfg = config_for(scene)
    fw = run_forward(scene, cams, cfg)
    _check_keys(fw, scene, cams, cfg)
    check_images(fw, scene, cams, cfg)


@pytest.mark.parametrize("tile", [(16, 16, 1), (16, 16, 2), (16, 16, 4), (8, 8, 1), (32, 16, 2), (32, 16, 4)])
def test_tile_shapes_ragged_image(tile):
    """A 200 x 120 image (not a multiple of any tile) with 1500 primitives."""
    scene = S.custom_scene(1500, 16, seed=51)
    cams = S.make_cameras([(200, 120)], seed=52)
    cfg = config_for(scene, tile=tile)
    fw = run_forward(scene, cams, cfg)
    _check_keys(fw, scene, cams, cfg)
    check_images(fw, scene, cams, cfg)


@pytest.mark.parametrize("N", [4, 8, 32])
def test_hidden_widths_with_gradients(N):
    scene = S.custom_scene(800, N, seed=60 + N, omega0=30.0 if N == 32 else 10.0)
    cams = S.make_cameras([(96, 80)], seed=61)
    cfg = config_for(scene, tile=(16, 16, 2))
    fw = run_forward(scene, cams, cfg)
    check_images(fw, scene, cams, cfg)
    small = S.subset_scene(scene, np.arange(200))
    small["N"], small["omega0"] = scene["N"], scene["omega0"]
    grad_parity(small, cams, S.make_targets(cams, seed=62), config_for(small, tile=(16, 16, 1)),
                 ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors"])


def test_multiview_batched_and_persistent():
    scene = S.custom_scene(1200, 16, seed=71)
    cams = S.make_cameras([(96, 64), (130, 70), (64, 64), (40, 90)], seed=72)
    a = run_forward(scene, cams, config_for(scene, persistent=0))
    b = run_forward(scene, cams, config_for(scene, persistent=1))
    _check_keys(a, scene, cams, config_for(scene))
    for v in range(len(cams)):
        assert np.array_equal(a["images"][v], b["images"][v])
    check_images(b, scene, cams, config_for(scene, persistent=1))


@pytest.mark.parametrize("width,depth,N", [(16, 2, 16), (32, 2, 16), (32, 3, 32)])
def test_colour_mlp_image(width, depth, N):
    scene = S.custom_scene(1500, N, color_mode=1, cmlp_width=width, cmlp_depth=depth, seed=81)
    cams = S.make_cameras([(120, 90), (64, 48)], seed=82)
    cfg = config_for(scene, tile=(16, 16, 2))
    fw = run_forward(scene, cams, cfg)
    check_images(fw, scene, cams, cfg)


def test_dense_scene_early_termination():
    scene = S.custom_scene(400, 8, seed=12, scale_lo=0.15, scale_hi=0.4)
    scene["w2"] = scene["w2"] * np.float32(20.0)
    cams = S.make_cameras([(48, 48)], seed=13)
    for t_eps in (1e-4, 0.0):
        cfg = config_for(scene, t_eps=t_eps)
        fw = run_forward(scene, cams, cfg)
        assert np.sum(fw["T"][0] < 1e-3) > 10
        check_images(fw, scene, cams, cfg)


def test_background_alpha_min_alpha_max():
    scene = S.custom_scene(600, 8, seed=91, scale_lo=0.1, scale_hi=0.3)
    scene["w2"] = scene["w2"] * np.float32(8.0)
    cams = S.make_cameras([(64, 56)], seed=92)
    cfg = config_for(scene, alpha_min=1.0 / 255.0, alpha_max=0.5, bg=(0.25, 0.5, 1.0))
    fw = run_forward(scene, cams, cfg)
    check_images(fw, scene, cams, cfg)


@pytest.mark.parametrize("fwd_cache", [1, 0])
def test_c1_gradients(fwd_cache):
    _, scene, cams, targets = S.make_workload("C1")
    cfg = config_for(scene, fwd_cache=fwd_cache)
    grad_parity(scene, cams, targets, cfg, ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors"])


@pytest.mark.parametrize("tile,fwd_cache", [((16, 16, 1), 1), ((16, 16, 4), 1), ((32, 16, 2), 1), ((32, 16, 2, 4), 0),
                                            ((16, 16, 4, 16), 1), ((8, 8, 1, 32), 1), ((16, 16, 2, 8), 0)])
def test_gradients_multiview_tiles(tile, fwd_cache):
    scene = S.custom_scene(400, 8, seed=101)
    cams = S.make_cameras([(72, 56), (48, 64)], seed=102)
    targets = S.make_targets(cams, seed=103)
    cfg = config_for(scene, tile=tile, persistent=1, fwd_cache=fwd_cache)
    grad_parity(scene, cams, targets, cfg, ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors"])


def test_cached_and_recomputed_backward_agree():
    """The backward from the forward's stored integrals, the one that
    re-evaluates them, and one with only the leading instances cached give
    the same gradients (up to the rounding of d loss / d H); a cache budget
    of nothing drops the cache."""
    import paper_2510_08491_amd as snp
    scene = S.custom_scene(1500, 16, color_mode=1, cmlp_width=16, cmlp_depth=2, seed=131)
    cams = S.make_cameras([(160, 120), (96, 128)], seed=132)
    targets = S.make_targets(cams, seed=133)
    out = {}
    n_inst = None
    for mode in ("full", "none", "part"):
        cfg = config_for(scene, tile=(16, 16, 2), persistent=1, fwd_cache=0 if mode == "none" else 1)
        if mode == "part":  # the leading ~40% of the instances only
            cfg.fwd_cache_budget = int(0.4 * n_inst) * 4 * 16 * 16
        fw = run_forward(scene, cams, cfg)
        rast = fw["rast"]
        if mode == "full":
            n_inst = fw["instances"]
            assert rast.cached_instances == rast.capacity
        elif mode == "none":
            assert not rast.fwd_cache and rast.cached_instances == 0
        else:
            assert 0 < rast.cached_instances < fw["instances"], (rast.cached_instances, fw["instances"])
        out[mode] = (fw["images"], run_backward(fw, targets))
    for mode in ("none", "part"):
        for a, b in zip(out["full"][0], out[mode][0]):
            assert np.array_equal(a, b)
        assert out["full"][1][0] == out[mode][1][0]
        for k, g in out["full"][1][1].items():
            ok, err, erel = grad_close(g, out[mode][1][1][k], rel=1e-5, elem_rel=1e-4)
            say(f"  {k}: cached vs {mode} {err:.2e} / {erel:.2e}")
            assert ok, (mode, k, err, erel)
    cfg = config_for(scene, tile=(16, 16, 2), fwd_cache=1)
    cfg.fwd_cache_budget = 0
    rast = snp.Rasterizer(cfg, scene["P"], cams)
    assert not rast.fwd_cache and rast.layout.ahat_cache_bytes == 0


@pytest.mark.parametrize("tile,fwd_cache", [((16, 16, 2), 1), ((32, 16, 2, 8), 1), ((16, 16, 1, 8), 0)])
def test_colour_mlp_gradients(tile, fwd_cache):
    scene = S.custom_scene(300, 16, color_mode=1, cmlp_width=16, cmlp_depth=2, seed=111)
    cams = S.make_cameras([(64, 48), (48, 40), (56, 56)], seed=112)
    targets = S.make_targets(cams, seed=113)
    cfg = config_for(scene, tile=tile, fwd_cache=fwd_cache)
    grad_parity(scene, cams, targets, cfg, ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "cmlp", "xi"])


@pytest.mark.parametrize("name", ["C2", "C3"])
def test_full_size_sampled(name):
    """Full-size configurations: sampled pixels against the oracle computed
    pixel by pixel, and the instance lists of sampled tiles bit-exact."""
    cfg0, scene, cams, _ = S.make_workload(name)
    cfg = config_for(scene, tile=(16, 16, 2))
    fw = run_forward(scene, cams, cfg)
    cam = cams[0]
    rng = np.random.default_rng(7)
    cols = rng.integers(0, cam.width, 24)
    rows = rng.integers(0, cam.height, 24)
    pr = project_all(scene, cam, cfg.tile_w, cfg.tile_h, cfg.z_near)
    c, t, h = render_pixels(scene, cam, cols, rows, options_for(cfg), proj=pr)
    err = np.max(np.abs(fw["images"][0][rows, cols] - c))
    terr = np.max(np.abs(fw["T"][0][rows, cols] - t))
    say(f"  {name}: sampled image err {err:.2e}, T err {terr:.2e}, instances {fw['instances']}, pairs {fw['hit_pairs']}")
    assert err <= IMG_TOL and terr <= IMG_TOL
    ntx = (cam.width + cfg.tile_w - 1) // cfg.tile_w
    ids = np.nonzero(pr["nonempty"])[0]
    tr = pr["trect"][ids]
    for g in rng.integers(0, fw["ranges"].shape[0], 6):
        ty, tx = divmod(int(g), ntx)
        sel = (tr[:, 0] <= tx) & (tx <= tr[:, 1]) & (tr[:, 2] <= ty) & (ty <= tr[:, 3])
        lst = sorted(zip(pr["depth_bits"][ids][sel].tolist(), ids[sel].tolist()))
        s, e = fw["ranges"][g]
        assert fw["values"][s:e].tolist() == [p for _, p in lst]


@pytest.mark.parametrize("fwd_cache", [1, 0])
def test_time_conditioned_density_image_and_gradients(fwd_cache):
    """The dynamic-scene density (phase + xi_t W_t): image and every gradient,
    W_t included, against the oracle."""
    scene = S.custom_scene(400, 8, seed=151, temporal=True)
    scene["time"] = 0.63
    cams = S.make_cameras([(72, 56), (48, 64)], seed=152)
    targets = S.make_targets(cams, seed=153)
    cfg = config_for(scene, tile=(16, 16, 1), persistent=1, fwd_cache=fwd_cache)
    fw = run_forward(scene, cams, cfg)
    check_images(fw, scene, cams, cfg)
    grad_parity(scene, cams, targets, cfg, ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors", "wt"])


@pytest.mark.parametrize("fwd_cache,time", [(1, 0.63), (0, 1.0)])
def test_dynamic_scene_sh_image_and_gradients(fwd_cache, time):
    """The dynamic-scene application whole: the time-conditioned density and
    the degree-3 SH colour whose zero-order coefficient follows the
    polynomial and Fourier terms of xi_t; image and every gradient, W_t and
    the time coefficients included, against the oracle."""
    scene = S.custom_scene(400, 8, color_mode=2, seed=155, temporal=True)
    scene["time"] = time
    cams = S.make_cameras([(72, 56), (48, 64)], seed=156)
    targets = S.make_targets(cams, seed=157)
    cfg = config_for(scene, tile=(16, 16, 1), persistent=1, fwd_cache=fwd_cache)
    fw = run_forward(scene, cams, cfg)
    check_images(fw, scene, cams, cfg)
    grad_parity(scene, cams, targets, cfg, ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "sh", "wt", "sh_t"])


@pytest.mark.parametrize("tile", [(16, 16, 1), (8, 8, 1), (32, 16, 2)])
def test_both_binning_orders_give_the_oracle_lists(tile):
    """Depth sort of the pairs then a tile-bit sort of the instances, and one
    sort over all key bits: the same keys, values and ranges (the oracle's),
    bit for bit, on views whose tile counts need one, two and three digits of
    tile bits."""
    scene = S.custom_scene(1200, 8, seed=141)
    cams = S.make_cameras([(64, 48), (200, 120), (120, 90), (48, 40)], seed=142)
    out = {}
    for order in (1, 2):
        cfg = config_for(scene, tile=tile, persistent=1, bin_order=order)
        fw = run_forward(scene, cams, cfg)
        _check_keys(fw, scene, cams, cfg)
        out[order] = fw
    for k in ("keys", "values", "ranges"):
        assert np.array_equal(out[1][k], out[2][k])
    for a, b in zip(out[1]["images"], out[2]["images"]):
        assert np.array_equal(a, b)


def test_capacity_overflow_is_reported_then_grown():
    import paper_2510_08491_amd as snp
    from paper_2510_08491_amd import _lib
    _, scene, cams, _ = S.make_workload("C1")
    cfg = config_for(scene)
    params = snp.params_to_device(scene)
    rast = snp.Rasterizer(cfg, scene["P"], cams, capacity=16)
    rast.preprocess(params)
    rast.bin()
    code, inst, _ = rast.read_status(raise_on_error=False)
    assert code == _lib.SNP_ERR_CAPACITY and inst > 16
    fw = run_forward(scene, cams, cfg, capacity=16)
    assert fw["rast"].capacity >= fw["instances"]
    check_images(fw, scene, cams, cfg)


@pytest.mark.parametrize("width,depth,n_views", [(32, 2, 3), (32, 3, 18), (16, 1, 17)])
def test_colour_mlp_gradients_widths_and_view_chunks(width, depth, n_views):
    """Colour-MLP shapes of the workloads and view counts beyond one chunk
    of 16 views in the colour backward."""
    scene = S.custom_scene(200, 8, color_mode=1, cmlp_width=width, cmlp_depth=depth, seed=141 + depth)
    sizes = [(40, 32), (32, 40), (36, 36)] * 6
    cams = S.make_cameras(sizes[:n_views], seed=142)
    targets = S.make_targets(cams, seed=143)
    cfg = config_for(scene, tile=(16, 16, 1), persistent=1)
    grad_parity(scene, cams, targets, cfg, ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "cmlp", "xi"])


@pytest.mark.parametrize("fwd_cache", [1, 0])
def test_sh_colour_image_and_gradients(fwd_cache):
    """Degree-3 spherical-harmonics colour (the paper's novel-view colour):
    images and every gradient, SH coefficients included."""
    scene = S.custom_scene(300, 8, omega0=30.0, color_mode=2, seed=151)
    cams = S.make_cameras([(64, 48), (48, 56), (40, 40)], seed=152)
    targets = S.make_targets(cams, seed=153)
    cfg = config_for(scene, tile=(16, 16, 1), persistent=1, fwd_cache=fwd_cache)
    fw = run_forward(scene, cams, cfg)
    check_images(fw, scene, cams, cfg)
    grad_parity(scene, cams, targets, cfg, ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "sh"])


def test_graph_replay_matches_eager():
    import paper_2510_08491_amd as snp
    scene = S.custom_scene(600, 16, color_mode=1, cmlp_width=16, cmlp_depth=2, seed=121)
    cams = S.make_cameras([(80, 64), (64, 64), (96, 48)], seed=122)
    targets = S.make_targets(cams, seed=123)
    cfg = config_for(scene, tile=(16, 16, 2), persistent=1)
    params = snp.params_to_device(scene)
    rast = snp.Rasterizer(cfg, scene["P"], cams)
    rast.prepare(params)
    tg = torch.from_numpy(np.concatenate([t.ravel() for t in targets])).cuda()
    n = float(tg.numel())
    # eager step through the C ABI
    images, T = rast.new_images()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    dL = torch.empty_like(images)
    grads = snp.zeros_like_params(params)
    rast.step(params, images, T, tg, n, loss, dL, grads)
    torch.cuda.synchronize()
    ref_img, ref_g, ref_loss = images.clone(), {k: v.clone() for k, v in grads.items()}, loss.item()
    step = snp.GraphStep(rast, params, tg, n)
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        step.launch()
        torch.cuda.synchronize()
        assert torch.equal(step.images, ref_img), rep
        assert abs(step.loss.item() - ref_loss) <= 1e-12
        for k in ref_g:
            ok, err, erel = grad_close(step.grads[k].cpu().numpy(), ref_g[k].cpu().numpy(), rel=1e-4, elem_rel=1e-3)
            assert ok, (rep, k, err, erel)
        del junk
    # and the eager result itself matches the oracle
    fw_imgs = rast.split_images(ref_img)
    opts = options_for(cfg)
    for v, cam in enumerate(cams):
        assert np.max(np.abs(fw_imgs[v].cpu().numpy() - render_view(scene, cam, opts)["image"])) <= IMG_TOL


def test_central_differences_full_hd_subset():
    """Gradients of the HIP backward against central finite differences of
    the HIP forward + float64-accumulated L1 loss, on the first 1000
    primitives of the 1920x1080 scene at full resolution, for the entries
    with the largest gradients of several parameter tensors.  Density and
    colour-MLP parameters move the loss smoothly: 1e-3.  A finite step of a
    centre or scale moves silhouette pixels across the ellipsoid's edge,
    where the chord length has a square-root edge and L1 has kinks, so the
    difference quotient itself is only good to about 1e-2 there: 2e-2."""
    import paper_2510_08491_amd as snp
    _, scene, cams, targets = S.make_workload("C3")
    sub = S.subset_scene(scene, np.arange(1000))
    cfg = config_for(sub, tile=(16, 16, 1), persistent=1)
    params = snp.params_to_device(sub)
    rast = snp.Rasterizer(cfg, sub["P"], cams)
    tg = torch.from_numpy(np.concatenate([t.ravel() for t in targets])).cuda()

    def loss_of():
        rast.prepare(params)
        images, T = rast.new_images()
        rast.forward(params, images, T)
        loss, dL = rast.loss_l1(images, tg)
        return loss, images, dL

    loss, images, dL = loss_of()
    grads = snp.zeros_like_params(params)
    rast.backward(params, images, dL, grads)
    torch.cuda.synchronize()
    checked = 0
    for key, h in (("centers", 1e-3), ("scales", 1e-4), ("w1", 1e-3), ("b1", 1e-3), ("w2", 1e-3), ("cmlp", 1e-3)):
        g = grads[key].view(-1)
        for idx in torch.topk(g.abs(), 2).indices.tolist():
            flat = params[key].view(-1)
            x0 = flat[idx].item()
            flat[idx] = x0 + h
            lp = loss_of()[0].item()
            flat[idx] = x0 - h
            lm = loss_of()[0].item()
            flat[idx] = x0
            fd = (lp - lm) / (2 * h)
            an = g[idx].item()
            say(f"  {key}[{idx}]: analytic {an:.6e} central difference {fd:.6e} rel {abs(fd - an) / abs(an):.2e}")
            tol = 2e-2 if key in ("centers", "scales") else 1e-3
            assert abs(fd - an) <= tol * abs(an), (key, idx, an, fd)
            checked += 1
    assert checked == 12


@pytest.mark.parametrize("primitive", [0, 1])
def test_degenerate_scenes(primitive):
    """Every primitive culled (zero instances: background, T = 1, zero
    gradients); one primitive covering a whole view; 1x1 and 3x17 views
    batched with a larger one."""
    import paper_2510_08491_amd as snp
    cams = S.make_cameras([(48, 40), (1, 1), (3, 17)], seed=161)
    # all culled: every centre just in front of camera 0, inside its near plane
    scene = S.custom_scene(20, 8, seed=162, primitive=primitive)
    Rinv = np.linalg.inv(np.asarray(cams[0].R, np.float64))
    o = -Rinv @ np.asarray(cams[0].t, np.float64)
    scene["centers"] = np.tile((o + 0.05 * Rinv[:, 2]).astype(np.float32), (20, 1))
    scene["scales"] = np.full((20, 3), 0.01, np.float32)
    cfg = config_for(scene, persistent=1, bg=(0.25, 0.5, 1.0))
    fw = run_forward(scene, cams[:1], cfg)
    assert fw["instances"] == 0 and fw["hit_pairs"] == 0
    assert np.all(fw["T"][0] == 1.0)
    assert np.allclose(fw["images"][0], np.array([0.25, 0.5, 1.0], np.float32))
    if primitive == 0:
        targets = S.make_targets(cams[:1], seed=163)
        _, g = run_backward(fw, targets)
        assert all(np.all(v == 0) for v in g.values())
    # one primitive covering all of camera 0's view, plus tiny views
    big = S.custom_scene(1, 8, seed=164, primitive=primitive)
    big["centers"] = np.zeros((1, 3), np.float32)
    big["scales"] = np.full((1, 3), 0.9 if primitive == 0 else 0.3, np.float32)
    if primitive == 1:
        big["opacity"][:] = np.float32(0.8)
    cfg = config_for(big, tile=(16, 16, 1), persistent=1)
    fw = run_forward(big, cams, cfg)
    if primitive == 0:
        _check_keys(fw, big, cams, cfg)
        check_images(fw, big, cams, cfg)
    assert fw["tile_counts"][0][0] == 3 * 3  # 48x40 in 16x16 tiles, all covered
    assert fw["instances"] >= 9


@pytest.mark.parametrize("width,depth,fwd_cache", [(16, 2, 1), (32, 1, 0)])
def test_relighting_colour_image_and_gradients(width, depth, fwd_cache):
    """Colour mode 3 (c_dc + colour network of view and light direction and
    xi, one point light per view): image and every gradient, the light
    direction's chain to the centres included, against the oracle."""
    scene = S.custom_scene(300, 8, color_mode=3, cmlp_width=width, cmlp_depth=depth, seed=171)
    cams = S.make_cameras([(64, 56), (56, 64), (48, 48)], seed=172, lights=True)
    targets = S.make_targets(cams, seed=173)
    cfg = config_for(scene, tile=(16, 16, 1), persistent=1, fwd_cache=fwd_cache)
    fw = run_forward(scene, cams, cfg)
    check_images(fw, scene, cams, cfg)
    grad_parity(scene, cams, targets, cfg, ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors", "cmlp",
                                             "xi"])


def test_large_image_many_tiles():
    """One 8192x4096 view (131072 tiles: 17 tile bits, three instance-sort
    passes): rectangles, depth keys and tile counts of every primitive, the
    lists of sampled tiles and sampled pixels against the oracle."""
    scene = S.custom_scene(3000, 8, seed=181, scale_lo=0.01, scale_hi=0.1)
    cams = S.make_cameras([(8192, 4096)], seed=182)
    cfg = config_for(scene, tile=(16, 16, 1), persistent=1)
    fw = run_forward(scene, cams, cfg)
    cam = cams[0]
    pr = project_all(scene, cam, cfg.tile_w, cfg.tile_h, cfg.z_near)
    ne = pr["nonempty"]
    assert np.array_equal(fw["tile_counts"][0], pr["n_tiles"].astype(np.int32))
    assert np.array_equal(fw["rects"][0][ne], pr["rect"][ne].astype(np.int32))
    assert np.array_equal(fw["depth_bits"][0][ne], pr["depth_bits"][ne])
    assert fw["instances"] == int(pr["n_tiles"].sum())
    rng = np.random.default_rng(183)
    ntx = (cam.width + 15) // 16
    ids = np.nonzero(ne)[0]
    tr = pr["trect"][ids]
    busy = np.nonzero(fw["ranges"][:, 1] > fw["ranges"][:, 0])[0]
    for g in rng.choice(busy, 12, replace=False):
        ty, tx = divmod(int(g), ntx)
        sel = (tr[:, 0] <= tx) & (tx <= tr[:, 1]) & (tr[:, 2] <= ty) & (ty <= tr[:, 3])
        lst = sorted(zip(pr["depth_bits"][ids][sel].tolist(), ids[sel].tolist()))
        s, e = fw["ranges"][g]
        assert fw["values"][s:e].tolist() == [p for _, p in lst]
    cols = rng.integers(2048, 6144, 40)
    rows = rng.integers(1024, 3072, 40)
    c, t, _ = render_pixels(scene, cam, cols, rows, options_for(cfg), proj=pr)
    err = np.max(np.abs(fw["images"][0][rows, cols] - c))
    say(f"  instances {fw['instances']}, sampled image err {err:.2e}")
    assert err <= IMG_TOL and np.max(np.abs(fw["T"][0][rows, cols] - t)) <= IMG_TOL


def test_autotuner_picks_a_measured_shape():
    """The autotuner times each candidate on a forward + backward, checks
    that all render the same image, and returns one of the candidates."""
    import paper_2510_08491_amd as snp
    from paper_2510_08491_amd import tuning
    _, scene, cams, targets = S.make_workload("C1")
    cfg = config_for(scene, persistent=1)
    params = snp.params_to_device(scene)
    tg = torch.from_numpy(np.concatenate([t.ravel() for t in targets])).cuda()
    best, table = tuning.autotune(cfg, scene["P"], cams, params, tg, reps=1, shapes=[(16, 16, 1), (8, 8, 1)],
                                  write=False, log=say)
    assert best[:3] in [(16, 16, 1), (8, 8, 1)]
    assert all(v["img_diff"] <= 1e-5 for v in table.values())
