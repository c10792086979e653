"""Host-side logic of bench.py (CPU only): the frozen per-pair operation
counts behind the roofline line, the traffic figure's source-hash gate, the
workload descriptions, and the synthetic workloads each bench line runs."""
import hashlib
import os

import numpy as np
import pytest

import bench
import synthetic as S


def test_per_pair_slot_counts():
    """The counts the roofline divides by: forward 50 + 11N VALU and 3N + 3
    transcendentals per hit pair, backward 82 slots per cached hit pair and
    32N + 60 VALU + 6N + 1 transcendentals per live pair; the per-ray colour
    (W = 16) adds 10W + 15 VALU and 7 transcendentals, and 21 + 19W more per
    listed pair."""
    s = lambda vt: bench.slots(vt)
    ops = bench.ops_per_pair(16)
    assert (s(ops["fwd"]), s(ops["bwd_hit_cached"]), s(ops["bwd_hit"]), s(ops["bwd_live"])) == (430, 82, 455, 960)
    ops32 = bench.ops_per_pair(32)
    assert (s(ops32["fwd"]), s(ops32["bwd_hit"]), s(ops32["bwd_live"])) == (798, 823, 1856)
    ray = bench.ops_per_pair(16, ray_colour_width=16)
    assert (s(ray["fwd"]), s(ray["bwd_hit_cached"]), s(ray["bwd_live"])) == (633, 285, 1488)
    assert bench.PEAK_SLOTS == pytest.approx(78.6432e12)


def _fake_root(tmp_path, raster, internal, bwd_bytes, sha=None):
    csrc = tmp_path / "paper_2510_08491_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "raster.hip").write_bytes(raster)
    (csrc / "snp_internal.h").write_bytes(internal)
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = sha or hashlib.sha256(raster + internal).hexdigest()
    (prof / "c4_render_traffic.md").write_text(
        f"# traffic\n\n    source_sha256 {sha}\n    render_bwd_bytes {bwd_bytes:.6e}\n    render_fwd_bytes 1.0e+11\n")
    return str(tmp_path)


def test_traffic_is_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    root = _fake_root(tmp_path, b"kernel source", b"header", 1.8e11)
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.measured_traffic("C4", "render_bwd", True) == pytest.approx(1.8e11)
    assert bench.measured_traffic("C4", "render_fwd", True) == pytest.approx(1.0e11)
    # no figures for the recompute variant or another workload
    assert bench.measured_traffic("C4", "render_bwd", False) is None
    assert bench.measured_traffic("C5", "render_bwd", True) is None
    # an edited rasterizer source voids the figure
    with open(os.path.join(root, "paper_2510_08491_amd", "csrc", "raster.hip"), "ab") as f:
        f.write(b" ")
    assert bench.measured_traffic("C4", "render_bwd", True) is None


@pytest.mark.parametrize("name", ["C3", "C4", "C5", "R", "L", "D"])
def test_workload_names_and_small_scenes(name):
    cfg, scene, cams, targets = S.make_workload(name, n_prims=64, sizes=[(32, 24), (24, 32)])
    desc = bench.workload_name(name, cams)
    assert f"N={cfg.n_hidden}" in desc
    assert scene["P"] == 64 and scene["color_mode"] == cfg.color_mode
    assert len(targets) == 2 and targets[0].shape == (24, 32, 3)
    if cfg.color_mode in (3, 4):
        assert all(c.light is not None for c in cams)
    if name == "D":
        assert scene["time"] == 0.5 and scene["wt"].shape == (64, 16) and scene["sh_t"].shape == (64, 12, 3)
    else:
        assert scene["wt"] is None
    assert np.all(np.isfinite(scene["centers"])) and np.all(scene["scales"] > 0)


def test_oracle_check_of_the_bench_on_oracle_images():
    """The bench's tile check, fed with the oracle's own images and per-tile
    hit-pair counts, reports no error and equal counts; a perturbed pixel of
    a checked tile is reported."""
    import torch

    from oracle.render import RenderOptions, render_view, render_window
    from paper_2510_08491_amd.render import RenderConfig

    _, scene, cams, _ = S.make_workload("C4", n_prims=300, sizes=[(48, 32), (32, 48)])
    cfg = RenderConfig(n_hidden=scene["N"], color_mode=scene["color_mode"], cmlp_width=scene["cmlp_width"],
                       cmlp_depth=scene["cmlp_depth"], tile_w=16, tile_h=16)
    opts = RenderOptions(z_near=cfg.z_near, t_eps=cfg.t_eps, alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max,
                         bg=tuple(cfg.bg))
    imgs, pairs = [], []
    for cam in cams:
        imgs.append(render_view(scene, cam, opts)["image"].ravel())
        for ty in range((cam.height + 15) // 16):
            for tx in range((cam.width + 15) // 16):
                w, h = min(16, cam.width - 16 * tx), min(16, cam.height - 16 * ty)
                pairs.append(render_window(scene, cam, 16 * tx, 16 * ty, w, h, opts)["hit_pairs"])
    images = torch.from_numpy(np.concatenate(imgs).astype(np.float32))
    tile_pairs = np.array(pairs)
    r = bench.oracle_check(scene, cams, cfg, images, tile_pairs, 16, per_view=3)
    assert r["tiles"] == 6 and r["hit_pairs_equal"] and r["hit_pairs_gpu"] == r["hit_pairs_oracle"] > 0
    assert r["max_img_err"] < 1e-6
    # one checked tile's pixel off by 1e-3
    v, t, _ = r["tiles_view_tile_primitives"][0]
    ntx = (cams[v].width + 15) // 16
    ty, tx = divmod(t, ntx)
    off = sum(c.width * c.height for c in cams[:v])
    images[3 * (off + (16 * ty) * cams[v].width + 16 * tx)] += 1e-3
    assert bench.oracle_check(scene, cams, cfg, images, tile_pairs, 16, per_view=3)["max_img_err"] > 9e-4


class _FakeRasterizer:
    """Stands in for the device rasterizer: its step writes the oracle's
    full-view images and gradients (so the windowed check must reproduce
    them from windows alone)."""
    full = None

    def __init__(self, cfg, P, cams):
        pass

    def prepare(self, params):
        return 1

    def _alloc(self, n):
        pass

    def new_images(self):
        import torch
        return torch.zeros(_FakeRasterizer.full["n_img"], dtype=torch.float32), None

    def step(self, params, images, T, tg, n_norm, loss, dL, grads):
        import torch
        images.copy_(torch.from_numpy(_FakeRasterizer.full["images"]))
        for k, g in _FakeRasterizer.full["grads"].items():
            if k in grads:
                grads[k].copy_(torch.from_numpy(g))


def test_windowed_gradients_sum_to_the_full_view_gradients(monkeypatch):
    """The bench's gradient check builds each sampled primitive's gradient
    from the windows of its rectangles alone; on a small scene it must equal
    the oracle's full-view autograd gradient (the windowing argument: a
    primitive changes only the pixels inside its rectangle)."""
    import types

    import torch

    from oracle.grad import PARAM_KEYS, autograd_loss_and_grads
    from oracle.render import RenderOptions
    from paper_2510_08491_amd.render import RenderConfig

    _, scene, cams, targets = S.make_workload("C4", n_prims=120, sizes=[(40, 32), (32, 40)])
    cfg = RenderConfig(n_hidden=scene["N"], color_mode=scene["color_mode"], cmlp_width=scene["cmlp_width"],
                       cmlp_depth=scene["cmlp_depth"], tile_w=16, tile_h=16)
    opts = RenderOptions(z_near=cfg.z_near, t_eps=cfg.t_eps, alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max,
                         bg=tuple(cfg.bg))
    # the oracle's windows first: its workers are forked, which a process
    # that has already run an autograd backward cannot do safely
    ref = bench.oracle_grad_reference(scene, cams, targets, 6)
    _, g, imgs = autograd_loss_and_grads(scene, cams, targets, opts)
    flat = np.concatenate([np.asarray(i).ravel() for i in imgs]).astype(np.float32)
    _FakeRasterizer.full = {"n_img": flat.size, "images": flat,
                            "grads": {k: np.asarray(v, np.float32) for k, v in g.items()}}
    snp = types.SimpleNamespace(
        Rasterizer=_FakeRasterizer,
        zeros_like_params=lambda params: {k: torch.zeros_like(v) for k, v in params.items()})
    monkeypatch.setattr(torch.cuda, "synchronize", lambda: None)
    monkeypatch.setattr(torch.cuda, "empty_cache", lambda: None)
    params = {k: torch.from_numpy(np.asarray(scene[k], np.float32)) for k in PARAM_KEYS if scene.get(k) is not None}
    n_norm = float(sum(t.size for t in targets))
    real_zeros = torch.zeros
    monkeypatch.setattr(torch, "zeros", lambda *a, **kw: real_zeros(*a, **{k: v for k, v in kw.items() if k != "device"}))
    r = bench.oracle_grad_check(snp, torch, cfg, scene, cams, targets, params, None, n_norm, ref)
    assert r["windows"] > 6 and not r["sign_flip_pixels"] and r["compared"] == 6
    # float32 copies of the full-view gradients against the float64 windows
    assert max(r["worst_per_primitive_err"].values()) < 1e-6, r
    assert max(r["normwise_err"].values()) < 1e-6, r
