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
