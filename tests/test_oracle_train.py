"""Pins of the oracle's training-step extras (Adam, scale regulariser,
population control); CPU only.  Adam is checked against torch.optim.Adam and
its first-step closed form, the regulariser against autograd of torch.std and
a closed form, the rotation of split children against scipy's rotations, and
the rest by brute force."""
import math

import numpy as np
import torch
from scipy.spatial.transform import Rotation

from oracle import train as T


def test_adam_matches_torch_over_several_steps():
    rng = np.random.default_rng(0)
    groups = [(rng.standard_normal(37), 1.6e-4), (rng.standard_normal((11, 3)), 5e-3), (rng.standard_normal(5), 1e-3)]
    tparams = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p, _ in groups]
    opt = torch.optim.Adam([{"params": [t], "lr": lr} for t, (_, lr) in zip(tparams, groups)],
                           betas=(0.9, 0.999), eps=1e-15)
    state = [(p.copy(), np.zeros_like(p), np.zeros_like(p)) for p, _ in groups]
    for step in range(1, 6):
        grads = [rng.standard_normal(p.shape) for p, _ in groups]
        for t, g in zip(tparams, grads):
            t.grad = torch.tensor(g)
        opt.step()
        state = [T.adam_step(p, g, m, v, step, lr) for (p, m, v), g, (_, lr) in zip(state, grads, groups)]
        for (p, _, _), t in zip(state, tparams):
            assert np.allclose(p, t.detach().numpy(), rtol=0, atol=1e-14)


def test_adam_first_step_moves_by_the_learning_rate():
    """After one step m_hat = g and v_hat = g^2, so every entry moves by lr
    against the sign of its gradient (|g| >> eps)."""
    rng = np.random.default_rng(1)
    p = rng.standard_normal(100)
    g = rng.standard_normal(100)
    p1, m, v = T.adam_step(p, g, np.zeros(100), np.zeros(100), 1, 2e-3)
    assert np.allclose(p1 - p, -2e-3 * np.sign(g), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_in_log_space_is_adam_on_the_logarithm():
    rng = np.random.default_rng(2)
    s = np.exp(rng.uniform(-4, -1, (20, 3)))
    t = torch.tensor(np.log(s), requires_grad=True)
    opt = torch.optim.Adam([t], lr=5e-3, betas=(0.9, 0.999), eps=1e-15)
    m = np.zeros_like(s)
    v = np.zeros_like(s)
    for step in range(1, 4):
        g = rng.standard_normal(s.shape)
        t.grad = torch.tensor(g * np.exp(t.detach().numpy()))  # chain rule d/dlog s = g s
        opt.step()
        s, m, v = T.adam_step(s, g, m, v, step, 5e-3, log_space=True)
        assert np.allclose(s, np.exp(t.detach().numpy()), rtol=1e-13)


def test_scale_regularizer_against_autograd_and_closed_form():
    rng = np.random.default_rng(3)
    s = np.exp(rng.uniform(-4, -1, (50, 3)))
    s[0] = [0.125, 0.125, 0.125]  # isotropic (exact mean): no loss, no gradient
    loss, grad = T.scale_regularizer(s, 0.7)
    ts = torch.tensor(s, requires_grad=True)
    ref = 0.7 * torch.std(ts, dim=1, unbiased=False).mean()
    ref.backward()
    assert math.isclose(loss, ref.item(), rel_tol=1e-13)
    g_ref = ts.grad.numpy()
    assert np.allclose(grad[1:], g_ref[1:], rtol=1e-10, atol=1e-15)
    assert np.all(grad[0] == 0)
    a, b = 0.02, 0.05  # (a, a, b): std = |b - a| sqrt(2) / 3
    l2, _ = T.scale_regularizer(np.array([[a, a, b]]), 1.0)
    assert math.isclose(l2, abs(b - a) * math.sqrt(2) / 3, rel_tol=1e-13)


def test_accumulate_by_brute_force():
    rng = np.random.default_rng(4)
    P, N, V = 30, 8, 3
    grads = {"w1": rng.standard_normal((P, N, 3)), "b1": rng.standard_normal((P, N)),
             "w2": rng.standard_normal((P, N)), "b2": rng.standard_normal(P)}
    tc = rng.integers(0, 3, (V, P)) * (rng.uniform(size=(V, P)) < 0.3)
    acc, cnt = T.densify_accumulate(np.full(P, 0.5), np.full(P, 2.0), grads, tc, N)
    for p in range(P):
        vals = list(grads["w1"][p].ravel()) + list(grads["b1"][p]) + list(grads["w2"][p]) + [grads["b2"][p]]
        assert math.isclose(acc[p], 0.5 + math.sqrt(sum(x * x for x in vals)), rel_tol=1e-13)
        assert cnt[p] == 2.0 + (1.0 if any(tc[v][p] > 0 for v in range(V)) else 0.0)


def test_actions_cover_every_rule():
    s = np.array([[0.6, 0.1, 0.1],      # too large: prune even with a high gradient
                  [0.05, 0.05, 0.05],   # visible, low gradient: prune
                  [0.005, 0.008, 0.01], # high gradient, small: clone
                  [0.05, 0.02, 0.03],   # high gradient, large: split
                  [0.05, 0.02, 0.03],   # ordinary: keep
                  [0.05, 0.02, 0.03]])  # never visible: keep
    acc = np.array([1.0, 1e-6, 3e-4, 3e-4, 5e-5, 0.0])
    cnt = np.array([1.0, 1.0, 2.0, 2.0, 1.0, 0.0])
    act = T.densify_actions(s, acc, cnt)
    assert act.tolist() == [T.PRUNE, T.PRUNE, T.CLONE, T.SPLIT, T.KEEP, T.KEEP]


def test_apply_clone_split_prune_by_hand():
    rng = np.random.default_rng(5)
    P = 4
    q = rng.standard_normal((P, 4))
    params = {"centers": rng.standard_normal((P, 3)), "scales": np.exp(rng.uniform(-4, -1, (P, 3))), "quats": q,
              "w1": rng.standard_normal((P, 8, 3))}
    moments = {"m_centers": rng.standard_normal((P, 3))}
    act = np.array([T.KEEP, T.CLONE, T.PRUNE, T.SPLIT])
    noise = rng.standard_normal((P, 2, 3))
    out, mo = T.densify_apply(params, moments, act, noise)
    assert out["centers"].shape == (5, 3)
    # rows: 0 keep p0; 1, 2 clone p1; 3, 4 children of p3
    for k in params:
        assert np.array_equal(out[k][0], params[k][0])
        assert np.array_equal(out[k][1], params[k][1]) and np.array_equal(out[k][2], params[k][1])
    Rq = Rotation.from_quat(q[3, [1, 2, 3, 0]]).as_matrix()  # scipy takes (x, y, z, w)
    for r, c in ((3, 0), (4, 1)):
        assert np.allclose(out["centers"][r], params["centers"][3] + Rq @ (params["scales"][3] * noise[3, c]),
                           atol=1e-12)
        assert np.allclose(out["scales"][r], params["scales"][3] / 1.6)
        assert np.array_equal(out["w1"][r], params["w1"][3]) and np.array_equal(out["quats"][r], q[3])
    assert np.array_equal(mo["m_centers"][0], moments["m_centers"][0])
    assert np.array_equal(mo["m_centers"][1], moments["m_centers"][1])
    assert np.all(mo["m_centers"][2:] == 0)
