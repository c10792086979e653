"""Parity of the training-step extras (Adam, scale regulariser, population
control) through the C ABI with the FP64 oracle."""
import numpy as np
import pytest
import torch

import paper_2510_08491_amd as snp
from paper_2510_08491_amd import train as TR
import synthetic as S
from oracle import train as T
from oracle.keys import project_all
from tests.gpu_helpers import config_for, say

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    say(f"[gpu-test] {request.node.name}")
    yield
    torch.cuda.synchronize()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_adam_groups_and_log_space_against_oracle():
    rng = np.random.default_rng(301)
    P, N = 3000, 16
    params = {"centers": rng.uniform(-1, 1, (P, 3)), "scales": np.exp(rng.uniform(-4, -1.5, (P, 3))),
              "quats": rng.standard_normal((P, 4)), "w1": rng.uniform(-0.3, 0.3, (P, N, 3)), "b2": np.zeros(P)}
    dev = {k: _dev(v) for k, v in params.items()}
    opt = TR.Adam(dev)
    ref = {k: (np.asarray(v, np.float32).astype(np.float64), np.zeros(np.shape(v)), np.zeros(np.shape(v)))
           for k, v in params.items()}
    for step in range(1, 4):
        grads = {k: rng.standard_normal(np.shape(v)) * 10.0 ** rng.uniform(-6, -1) for k, v in params.items()}
        opt.step({k: _dev(g) for k, g in grads.items()})
        for k in params:
            p, m, v = ref[k]
            g = np.asarray(grads[k], np.float32).astype(np.float64)
            ref[k] = T.adam_step(p, g, m, v, step, TR.PAPER_LRS[k], log_space=(k == "scales"))
        torch.cuda.synchronize()
        for k in params:
            p, m, v = ref[k]
            pg = dev[k].cpu().numpy().astype(np.float64)
            lr = TR.PAPER_LRS[k]
            err = np.max(np.abs(pg - p) / (2e-6 * np.abs(p) + 1e-5 * lr))
            # moments: normwise (0.9 m + 0.1 g can cancel, so elementwise relative error is unbounded)
            merr = np.max(np.abs(opt.m[k].cpu().numpy() - m)) / (1e-5 * np.max(np.abs(m)))
            verr = np.max(np.abs(opt.v[k].cpu().numpy() - v)) / (1e-5 * np.max(np.abs(v)))
            say(f"  step {step} {k}: param err/tol {err:.2f}, m {merr:.2f}, v {verr:.2f}")
            assert err <= 1 and merr <= 1 and verr <= 1


def test_scale_regularizer_against_oracle():
    rng = np.random.default_rng(311)
    P = 20000
    s = np.exp(rng.uniform(-5, -1, (P, 3))).astype(np.float32)
    s[:10] = np.float32(0.125)  # isotropic
    _, scene, cams, _ = S.make_workload("C1")
    rast = snp.Rasterizer(config_for(scene), scene["P"], cams)
    g = torch.zeros(P, 3, device="cuda")
    loss = TR.scale_regularizer(rast, _dev(s), 0.3, g)
    L_ref, g_ref = T.scale_regularizer(s.astype(np.float64), 0.3)
    gg = g.cpu().numpy()
    say(f"  loss gpu {loss.item():.10e} oracle {L_ref:.10e}")
    assert abs(loss.item() - L_ref) <= 1e-6 * L_ref
    assert np.all(gg[:10] == 0)
    assert np.max(np.abs(gg - g_ref)) <= 1e-5 * np.max(np.abs(g_ref))


def test_densify_accumulate_against_oracle():
    rng = np.random.default_rng(321)
    scene = S.custom_scene(2000, 8, seed=322)
    cams = S.make_cameras([(96, 64), (64, 80)], seed=323)
    cfg = config_for(scene)
    params = snp.params_to_device(scene)
    rast = snp.Rasterizer(cfg, scene["P"], cams)
    rast.prepare(params)
    P, N = scene["P"], 8
    acc0 = rng.uniform(0, 1e-3, P)
    cnt0 = rng.integers(0, 5, P).astype(np.float64)
    acc, cnt = _dev(acc0), _dev(cnt0)
    grads = {"w1": rng.standard_normal((P, N, 3)) * 1e-4, "b1": rng.standard_normal((P, N)) * 1e-4,
             "w2": rng.standard_normal((P, N)) * 1e-4, "b2": rng.standard_normal(P) * 1e-4}
    TR.densify_accumulate(rast, {k: _dev(v) for k, v in grads.items()}, acc, cnt)
    tc = np.stack([project_all(scene, c, cfg.tile_w, cfg.tile_h, cfg.z_near)["n_tiles"] for c in cams])
    a_ref, c_ref = T.densify_accumulate(np.asarray(acc0, np.float32), np.asarray(cnt0, np.float32),
                                        {k: np.asarray(v, np.float32) for k, v in grads.items()}, tc, N)
    ag, cg = acc.cpu().numpy(), cnt.cpu().numpy()
    say(f"  visible {int((cg - cnt0).sum())} of {P}")
    assert np.array_equal(cg, c_ref)
    assert np.max(np.abs(ag - a_ref) / np.abs(a_ref)) <= 1e-6


def test_densify_plan_and_apply_against_oracle():
    rng = np.random.default_rng(331)
    P, N, K = 5000, 8, 40
    scales = np.exp(rng.uniform(np.log(2e-3), np.log(0.8), (P, 3)))
    cnt = rng.integers(0, 4, P).astype(np.float64)
    stat = 10.0 ** rng.uniform(-7, -3, P)
    # keep every statistic and scale clear of the thresholds (a float32 and a
    # float64 comparison could otherwise disagree)
    for thr in (1e-4, 2e-6):
        near = np.abs(stat / thr - 1) < 1e-3
        stat[near] *= 1.01
    for thr in (1e-2, 0.5):
        near = np.abs(scales.max(1) / thr - 1) < 1e-3
        scales[near] *= 1.01
    acc = stat * cnt
    scales = scales.astype(np.float32)
    acc = acc.astype(np.float32)
    params = {"centers": rng.uniform(-1, 1, (P, 3)), "scales": scales, "quats": rng.standard_normal((P, 4)),
              "w1": rng.standard_normal((P, N, 3)), "b2": rng.standard_normal(P), "cmlp": rng.standard_normal((P, K))}
    params = {k: np.asarray(v, np.float32) for k, v in params.items()}
    state = {"m_centers": rng.standard_normal((P, 3)).astype(np.float32),
             "v_w1": rng.uniform(0, 1, (P, N, 3)).astype(np.float32)}
    noise = rng.standard_normal((P, 2, 3)).astype(np.float32)
    act_ref = T.densify_actions(scales.astype(np.float64), acc.astype(np.float64), cnt)
    new_p, new_s, act = TR.densify({k: _dev(v) for k, v in params.items()}, {k: _dev(v) for k, v in state.items()},
                                   _dev(acc), _dev(cnt), _dev(noise))
    torch.cuda.synchronize()
    counts = np.bincount(act_ref, minlength=4)
    say(f"  prune {counts[0]} keep {counts[1]} clone {counts[2]} split {counts[3]} -> {new_p['centers'].shape[0]}")
    assert np.all(counts > 0)
    assert np.array_equal(act.cpu().numpy(), act_ref)
    p_ref, s_ref = T.densify_apply({k: v.astype(np.float64) for k, v in params.items()},
                                   {k: v.astype(np.float64) for k, v in state.items()}, act_ref,
                                   noise.astype(np.float64))
    for k in params:
        got = new_p[k].cpu().numpy().astype(np.float64)
        assert got.shape == p_ref[k].shape, k
        if k == "centers":
            assert np.max(np.abs(got - p_ref[k])) <= 1e-6
        elif k == "scales":
            assert np.max(np.abs(got - p_ref[k]) / p_ref[k]) <= 2e-7
        else:
            assert np.array_equal(got, p_ref[k]), k
    for k in state:
        assert np.array_equal(new_s[k].cpu().numpy().astype(np.float64), s_ref[k]), k


def test_densify_everything_pruned_and_empty_adam_group():
    """All primitives pruned: zero rows, no kernel writes; an empty tensor in
    an Adam step is allowed and the others still update."""
    P = 64
    scales = np.full((P, 3), 0.9, np.float32)  # above the pruning scale
    params = {"centers": np.zeros((P, 3), np.float32), "scales": scales,
              "quats": np.tile(np.array([1, 0, 0, 0], np.float32), (P, 1))}
    new_p, new_s, act = TR.densify({k: _dev(v) for k, v in params.items()}, {}, _dev(np.ones(P)),
                                   _dev(np.ones(P)), _dev(np.zeros((P, 2, 3))))
    torch.cuda.synchronize()
    assert np.all(act.cpu().numpy() == T.PRUNE) and new_p["centers"].shape == (0, 3)
    dev = {"centers": _dev(np.ones((5, 3))), "b2": torch.zeros(0, device="cuda")}
    opt = TR.Adam(dev)
    opt.step({"centers": _dev(np.ones((5, 3))), "b2": torch.zeros(0, device="cuda")})
    torch.cuda.synchronize()
    assert np.allclose(dev["centers"].cpu().numpy(), 1.0 - TR.PAPER_LRS["centers"], rtol=0, atol=1e-7)
