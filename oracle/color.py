"""Per-(primitive, view) colour (FP64).

Test infrastructure only (see the package docstring).

The paper's novel-view-synthesis colour is spherical harmonics of four
bands, as in 3DGS (Sec. 3.1 and Sec. 3.3, implementation details); its
relighting application uses a per-primitive colour network (App. D.2,
Eq. 14) whose inputs include the view direction relative to the primitive.
The workloads here use a constant RGB per primitive, degree-3 spherical
harmonics, or such a per-primitive colour MLP, evaluated once per
(primitive, view).

Relighting colour (the relighting application): a constant colour c_dc plus
the per-primitive colour network of the view direction, the direction from
the primitive to the view's light and xi, evaluated once per (primitive,
view) (the paper evaluates it per ray; with a point light at l_v):

    input  = [normalize(x_B - o_v) (3), normalize(l_v - x_B) (3), xi_p (8)]
    colour = c_dc + sigmoid(MLP(input))

Per-ray relighting colour (colour mode 4; the relighting application's
colour per view ray, at the ray's entry point into the bounding ellipsoid):
for a ray o + t d (d unit) entering the ellipsoid at t_in,

    input  = [(o + t_in d - x_B) / max(s_B) (3), d (3), normalize(l_v - x_B) (3)]
    colour = c_dc + sigmoid(MLP(input))

The entry point is normalised as the density network's input (Eq. 5), so it
lies in the unit ball; the light direction is taken relative to the
primitive's centre, as the paper states.  There is no xi input.

Spherical harmonics: with d = normalize(x_B - o_v) and the 16 real
orthonormal harmonics Y_k(d) of degrees 0..3 (order (l, m) = (0,0),
(1,-1), (1,0), (1,1), (2,-2), ..., (3,3); real forms sqrt(2) (-1)^m Re/Im of
the complex harmonics, which cancels the Condon-Shortley phase),

    colour_c = max(0, 1/2 + sum_k Y_k(d) sh[k, c])

(the offset of one half and the clamp at zero are the 3DGS convention the
paper says it follows).  In the dynamic-scene application the zero-order
coefficient is a function of the time xi_t in [0, 1]: S0 plus a polynomial
and a Fourier series, n = l = 4,

    sh[0, c](xi_t) = S0_c + sum_{i=1..4} a_ic xi_t^i
                          + sum_{i=1..4} (b_ic cos(i xi_t) + c_ic sin(i xi_t))

(reading: the sums start at i = 1, a constant term would repeat S0;
frequencies i in radians, as printed), with the coefficients stored per
primitive as sh_t[12][3]: a_1..a_4, b_1..b_4, c_1..c_4.  Colour MLP:

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


def sh_basis(d):
    """The 16 real spherical harmonics of degrees 0..3 at unit vectors d
    (..., 3), as polynomials in (x, y, z) -> (..., 16)."""
    d = np.asarray(d, dtype=np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    pi = np.pi
    one = np.ones_like(x)
    return np.stack([
        0.5 * np.sqrt(1 / pi) * one,
        np.sqrt(3 / (4 * pi)) * y,
        np.sqrt(3 / (4 * pi)) * z,
        np.sqrt(3 / (4 * pi)) * x,
        0.5 * np.sqrt(15 / pi) * x * y,
        0.5 * np.sqrt(15 / pi) * y * z,
        0.25 * np.sqrt(5 / pi) * (3 * z * z - 1),
        0.5 * np.sqrt(15 / pi) * x * z,
        0.25 * np.sqrt(15 / pi) * (x * x - y * y),
        0.25 * np.sqrt(35 / (2 * pi)) * y * (3 * x * x - y * y),
        0.5 * np.sqrt(105 / pi) * x * y * z,
        0.25 * np.sqrt(21 / (2 * pi)) * y * (5 * z * z - 1),
        0.25 * np.sqrt(7 / pi) * (5 * z ** 3 - 3 * z),
        0.25 * np.sqrt(21 / (2 * pi)) * x * (5 * z * z - 1),
        0.25 * np.sqrt(105 / pi) * z * (x * x - y * y),
        0.25 * np.sqrt(35 / (2 * pi)) * x * (x * x - 3 * y * y),
    ], axis=-1)


def time_basis(time):
    """The 12 functions of xi_t the time-dependent zero-order coefficient
    combines: xi^1..xi^4, cos(i xi), sin(i xi) for i = 1..4."""
    t = float(time)
    return np.array([t ** i for i in range(1, 5)] + [np.cos(i * t) for i in range(1, 5)] +
                    [np.sin(i * t) for i in range(1, 5)])


def time_sh0(sh_t, time):
    """P_n(xi_t) + F_l(xi_t) per primitive and channel (P, 3) from the
    coefficients sh_t (P, 12, 3)."""
    return np.einsum("k,pkc->pc", time_basis(time), np.asarray(sh_t, dtype=np.float64))


def view_directions(scene, cam):
    """normalize(x_B - o_v) for every primitive, (P, 3)."""
    o = camera_center(cam)
    dirv = np.asarray(scene["centers"], dtype=np.float64) - o
    return dirv / np.linalg.norm(dirv, axis=1, keepdims=True)


def primitive_colors(scene, cam):
    """Colour (P, 3) of every primitive as seen from camera `cam`."""
    if scene["color_mode"] == 0:
        return np.asarray(scene["colors"], dtype=np.float64)
    dirv = view_directions(scene, cam)
    if scene["color_mode"] == 2:
        Y = sh_basis(dirv)                                        # (P, 16)
        sh = np.array(scene["sh"], dtype=np.float64)              # (P, 16, 3)
        if scene.get("sh_t") is not None:
            sh[:, 0, :] += time_sh0(scene["sh_t"], scene.get("time", 0.0))
        return np.maximum(0.0, 0.5 + np.einsum("pk,pkc->pc", Y, sh))
    parts = [dirv]
    if scene["color_mode"] == 3:
        ld = np.asarray(cam.light, dtype=np.float32).astype(np.float64) - np.asarray(scene["centers"], dtype=np.float64)
        parts.append(ld / np.linalg.norm(ld, axis=1, keepdims=True))
    x = np.concatenate(parts + [np.asarray(scene["xi"], dtype=np.float64)], axis=1)
    layers = unpack_cmlp(scene["cmlp"], scene["cmlp_width"], scene["cmlp_depth"], x.shape[1])
    c = mlp_forward(x, layers)
    if scene["color_mode"] == 3:
        c = c + np.asarray(scene["colors"], dtype=np.float64)
    return c


def ray_colors(scene, p, cam, o, d, t_in):
    """Per-ray relighting colour (colour mode 4) of primitive p for rays
    o + t d (d (..., 3) unit) entering its ellipsoid at t_in (...)."""
    xb = np.asarray(scene["centers"][p], dtype=np.float64)
    m = float(np.max(np.asarray(scene["scales"][p], dtype=np.float64)))
    d = np.asarray(d, dtype=np.float64)
    x_in = (np.asarray(o, dtype=np.float64) + np.asarray(t_in, dtype=np.float64)[..., None] * d - xb) / m
    ld = np.asarray(cam.light, dtype=np.float32).astype(np.float64) - xb
    ld = ld / np.linalg.norm(ld)
    x = np.concatenate([x_in, d, np.broadcast_to(ld, d.shape)], axis=-1)
    layers = unpack_cmlp(scene["cmlp"][p], scene["cmlp_width"], scene["cmlp_depth"], 9)
    return np.asarray(scene["colors"][p], dtype=np.float64) + mlp_forward(x, layers)
