"""Training-step extras after the backward (FP64): Adam, the scale
regulariser and population control.

Test infrastructure only (see the package docstring).

The paper trains with Adam (Kingma & Ba) at per-group learning rates (means
1.6e-4, scales 5e-3, quaternions 1e-3, SH 2.5e-3, MLP 1e-3; App. on
hyperparameters), adds to the 3DGS loss a regulariser that penalises the
standard deviation of each primitive's scale components (Sec. 3.3,
"Training"), and controls the population by the gradient magnitude of the
primitives' network weights: primitives whose gradient exceeds a threshold
are duplicated or split, those with low gradient are pruned, with a growing
scale threshold 1e-2 and a pruning scale threshold 0.5 (Sec. 3.3, "Population
Control"; App. on hyperparameters).  Readings of what it leaves open:

  * Adam as in Kingma & Ba's algorithm: m = b1 m + (1 - b1) g,
    v = b2 v + (1 - b2) g^2, theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
    b1 = 0.9, b2 = 0.999, eps = 1e-15 (3DGS's choice).  A group may be
    optimised in log space (3DGS's scale parameterisation): theta = log p,
    its gradient g p, and p = exp(theta) afterwards.
  * Regulariser: weight * (1/P) sum_p std(s_p), the population standard
    deviation of the three components; its gradient at std = 0 is taken as 0.
  * Gradient statistic: per step, the L2 norm of a primitive's density-MLP
    weight gradient (W1, b1, W2, b2) is added to an accumulator and a
    visibility count is incremented if the primitive covers a tile of any
    view; the statistic is accumulator / count (0 if never visible).
  * Decision per primitive, in this order: prune if max(s) > prune_scale;
    prune if visible and statistic < prune_threshold; if statistic >
    densify_threshold, clone if max(s) <= grow_scale, else split; else keep.
  * Clone: the primitive and an identical copy.  Split (3DGS): two children
    at x + R diag(s) u_k with standard normal u_k (passed in, one per child),
    scales s / 1.6, everything else copied.
  * Output order: the primitives in index order, each followed by its copy
    (clone) or replaced by its two children (split).  Optimizer moments stay
    with the row that continues the original (a kept primitive, the first row
    of a clone) and are zero for new rows (the clone's copy, both children).
"""
from __future__ import annotations

import numpy as np

from .geometry import quat_to_rotmat

PRUNE, KEEP, CLONE, SPLIT = 0, 1, 2, 3


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15, log_space=False):
    """One Adam step (Kingma & Ba, Algorithm 1) for one parameter group.
    Returns (param, m, v) as new float64 arrays."""
    p = np.asarray(param, np.float64)
    g = np.asarray(grad, np.float64)
    theta = np.log(p) if log_space else p
    if log_space:
        g = g * p  # d loss / d log p
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    theta = theta - lr * m_hat / (np.sqrt(v_hat) + eps)
    return (np.exp(theta) if log_space else theta), m, v


def scale_regularizer(scales, weight):
    """weight * mean over primitives of the population std of the scale
    components.  Returns (loss, d loss / d scales)."""
    s = np.asarray(scales, np.float64)
    P = s.shape[0]
    mean = s.mean(axis=1, keepdims=True)
    dev = s - mean
    std = np.sqrt((dev * dev).sum(axis=1) / 3.0)
    loss = weight * std.sum() / P
    with np.errstate(invalid="ignore", divide="ignore"):
        grad = np.where(std[:, None] > 0.0, weight / P * dev / (3.0 * std[:, None]), 0.0)
    return loss, grad


def mlp_grad_norm(grads, P, N):
    """L2 norm of each primitive's density-MLP weight gradient (W1, b1, W2, b2)."""
    parts = [np.asarray(grads[k], np.float64).reshape(P, -1) for k in ("w1", "b1", "w2", "b2")]
    return np.sqrt(sum((x * x).sum(axis=1) for x in parts))


def densify_accumulate(acc, count, grads, tile_counts, N):
    """acc += ||grad MLP||, count += visible (tile_counts (V, P) > 0 in any view)."""
    P = np.asarray(acc).shape[0]
    vis = (np.asarray(tile_counts).reshape(-1, P) > 0).any(axis=0)
    return np.asarray(acc, np.float64) + mlp_grad_norm(grads, P, N), np.asarray(count, np.float64) + vis


def densify_actions(scales, acc, count, densify_threshold=1e-4, prune_threshold=2e-6, grow_scale=1e-2,
                    prune_scale=0.5):
    """Action per primitive (PRUNE, KEEP, CLONE, SPLIT) by the rule above."""
    s = np.asarray(scales, np.float64)
    cnt = np.asarray(count, np.float64)
    stat = np.where(cnt > 0, np.asarray(acc, np.float64) / np.maximum(cnt, 1.0), 0.0)
    smax = s.max(axis=1)
    act = np.full(s.shape[0], KEEP, dtype=np.int32)
    dens = stat > densify_threshold
    act[dens] = np.where(smax[dens] <= grow_scale, CLONE, SPLIT)
    act[(cnt > 0) & (stat < prune_threshold)] = PRUNE
    act[smax > prune_scale] = PRUNE
    return act


def densify_apply(params, moments, actions, noise, shrink=1.6):
    """New parameter arrays after population control.

    params: dict of (P, ...) arrays (must hold centers, scales, quats);
    moments: dict of (P, ...) optimizer-state arrays; noise: (P, 2, 3)
    standard normals for the two children of a split.  Returns (params,
    moments) with the output rows in the documented order."""
    P = len(actions)
    rows, state_src, child = [], [], []
    for p in range(P):
        a = int(actions[p])
        if a == KEEP:
            rows.append(p); state_src.append(p); child.append(-1)
        elif a == CLONE:
            rows += [p, p]; state_src += [p, -1]; child += [-1, -1]
        elif a == SPLIT:
            rows += [p, p]; state_src += [-1, -1]; child += [0, 1]
    rows = np.array(rows, dtype=np.int64)
    out = {k: np.asarray(v, np.float64)[rows].copy() for k, v in params.items()}
    R = quat_to_rotmat(np.asarray(params["quats"], np.float64))
    s = np.asarray(params["scales"], np.float64)
    x = np.asarray(params["centers"], np.float64)
    for r, (p, c) in enumerate(zip(rows, child)):
        if c >= 0:
            out["centers"][r] = x[p] + R[p] @ (s[p] * np.asarray(noise, np.float64)[p, c])
            out["scales"][r] = s[p] / shrink
    mo = {}
    for k, v in moments.items():
        v = np.asarray(v, np.float64)
        o = np.zeros((len(rows),) + v.shape[1:])
        for r, src in enumerate(state_src):
            if src >= 0:
                o[r] = v[src]
        mo[k] = o
    return out, mo
