"""snp_step_static (the training step whose workspace is the library's static
device scratch, for callers that cannot allocate) against snp_step with a
caller-owned workspace: two calls in a row, the second on a smaller scene,
each compared with its own snp_step run -- images and transmittance bitwise,
the loss to 1e-12, every gradient within 1e-5 of the tensor's largest entry
(the backward's float atomics make the sums order-dependent), and the
counters the static call hands back (instances equal, no overflow)."""
import numpy as np
import pytest
import torch

import paper_2510_08491_amd as snp
import synthetic as S
from tests.gpu_helpers import config_for, say

pytestmark = pytest.mark.gpu

KEYS = ["centers", "scales", "quats", "w1", "b1", "w2", "b2", "cmlp", "xi"]


def _case(P, sizes, seed):
    scene = S.custom_scene(P, 16, color_mode=1, cmlp_width=32, cmlp_depth=2, seed=seed)
    cams = S.make_cameras(sizes, seed=seed + 1)
    targets = S.make_targets(cams, seed=seed + 2)
    return scene, cams, targets


def _run(scene, cams, targets, cfg, static):
    params = {k: v for k, v in snp.params_to_device(scene).items() if k != "opacity"}
    npix = sum(c.width * c.height for c in cams)
    tg = torch.from_numpy(np.concatenate([t.ravel() for t in targets])).cuda()
    images = torch.full((3 * npix,), -1.0, dtype=torch.float32, device="cuda")
    T = torch.full((npix,), -1.0, dtype=torch.float32, device="cuda")
    dL = torch.empty_like(images)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grads = snp.zeros_like_params(params)
    for g in grads.values():
        g.fill_(7.0)  # the step zeroes the gradients itself
    if static:
        counters = torch.full((8,), -1, dtype=torch.int64, device="cuda")
        snp.step_static(cfg, params, cams, images, T, tg, 3 * npix, loss, dL, grads, counters)
        torch.cuda.synchronize()
        cnt = counters.cpu().numpy()
        inst, overflow = int(cnt[0]), int(cnt[1])
    else:
        rast = snp.Rasterizer(cfg, scene["P"], cams)
        rast.prepare(params)  # sizes the workspace for the instances
        rast.step(params, images, T, tg, 3 * npix, loss, dL, grads)
        c = rast.counters()
        inst, overflow = int(c["instances"]), int(c["overflow"])
    torch.cuda.synchronize()
    return dict(images=images.cpu(), T=T.cpu(), loss=float(loss.item()), inst=inst, overflow=overflow,
                grads={k: v.cpu().double() for k, v in grads.items()})


def _compare(name, ref, got):
    say(f"  {name}: instances {ref['inst']} / {got['inst']}, loss {ref['loss']:.10f} / {got['loss']:.10f}")
    assert got["overflow"] == 0 and ref["overflow"] == 0
    assert got["inst"] == ref["inst"] > 0
    assert torch.equal(got["images"], ref["images"])
    assert torch.equal(got["T"], ref["T"])
    assert abs(got["loss"] - ref["loss"]) <= 1e-12 * max(1.0, abs(ref["loss"]))
    for k in KEYS:
        a, b = got["grads"][k], ref["grads"][k]
        scale = float(torch.max(torch.abs(b)))
        err = float(torch.max(torch.abs(a - b)))
        say(f"    grad {k}: max |static - workspace| / max {err / max(scale, 1e-30):.2e}")
        assert err <= 1e-5 * scale + 1e-12, k


@pytest.mark.parametrize("fwd_cache", [1, 0])
def test_static_scratch_step_matches_workspace_step(fwd_cache):
    big = _case(1200, [(160, 120), (96, 64)], seed=411)
    small = _case(300, [(64, 48)], seed=421)
    for name, (scene, cams, targets) in (("first call", big), ("second call, smaller", small)):
        cfg = config_for(scene, tile=(16, 16, 1, 8), persistent=1, fwd_cache=fwd_cache)
        say(f"[no-alloc] {name}: P={scene['P']} views={[(c.width, c.height) for c in cams]} fwd_cache={fwd_cache}")
        got = _run(scene, cams, targets, cfg, static=True)
        ref = _run(scene, cams, targets, cfg, static=False)
        _compare(name, ref, got)


def test_static_scratch_rejects_a_step_that_does_not_fit():
    """A step whose fixed arrays exceed the 64 MiB scratch is refused before
    anything is enqueued."""
    scene = S.custom_scene(200000, 16, color_mode=0, seed=431)
    cams = S.make_cameras([(64, 64)], seed=432)
    cfg = config_for(scene, tile=(16, 16, 1, 8), persistent=1, fwd_cache=0)
    params = {k: v for k, v in snp.params_to_device(scene).items() if k != "opacity"}
    images = torch.zeros(3 * 64 * 64, device="cuda")
    T = torch.zeros(64 * 64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grads = snp.zeros_like_params(params)
    with pytest.raises(snp.SnpError) as e:
        snp.step_static(cfg, params, cams, images, T, torch.zeros_like(images), 3 * 64 * 64, loss,
                        torch.zeros_like(images), grads)
    assert e.value.code == snp._lib.SNP_ERR_TOO_LARGE
