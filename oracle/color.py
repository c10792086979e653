"""Per-(primitive, view) colour (FP64).

Test infrastructure only (see the package docstring).

The paper's novel-view-synthesis colour is spherical harmonics (Sec. 3.1);
its relighting application uses a per-primitive colour network (App. D.2,
Eq. 14) whose inputs include the view direction relative to the primitive.
The workloads here use either a constant RGB per primitive or such a
per-primitive colour MLP, evaluated once per (primitive, view):

    input  = [normalize(x_B - o_v) (3), xi_p (8)]
    hidden = ReLU(W h + b), `depth` layers of `width` units
    colour = sigmoid(W h + b), 3 units

Weights are stored per primitive, layer after layer, each layer as W
(out x in, row-major) followed by b (out).
"""
from __future__ import annotations

import numpy as np

from .geometry import camera_center


def unpack_cmlp(vec, width, depth, n_in=11):
    """Split one primitive's packed weight vector into [(W, b), ...]."""
    vec = np.asarray(vec, dtype=np.float64)
    dims = [n_in] + [width] * depth + [3]
    layers, pos = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        W = vec[..., pos:pos + a * b].reshape(vec.shape[:-1] + (b, a))
        pos += a * b
        bb = vec[..., pos:pos + b]
        pos += b
        layers.append((W, bb))
    assert pos == vec.shape[-1], (pos, vec.shape)
    return layers


def mlp_forward(x, layers):
    """Plain MLP: ReLU hidden layers, sigmoid output.  x (..., n_in)."""
    h = np.asarray(x, dtype=np.float64)
    for i, (W, b) in enumerate(layers):
        h = np.einsum("...oi,...i->...o", W, h) + b
        if i + 1 < len(layers):
            h = np.maximum(h, 0.0)
    return 1.0 / (1.0 + np.exp(-h))


def primitive_colors(scene, cam):
    """Colour (P, 3) of every primitive as seen from camera `cam`."""
    if scene["color_mode"] == 0:
        return np.asarray(scene["colors"], dtype=np.float64)
    o = camera_center(cam)
    dirv = np.asarray(scene["centers"], dtype=np.float64) - o
    dirv /= np.linalg.norm(dirv, axis=1, keepdims=True)
    x = np.concatenate([dirv, np.asarray(scene["xi"], dtype=np.float64)], axis=1)
    layers = unpack_cmlp(scene["cmlp"], scene["cmlp_width"], scene["cmlp_depth"], x.shape[1])
    return mlp_forward(x, layers)
