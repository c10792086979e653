"""Neural density field of one primitive and its exact line integral (FP64).

Test infrastructure only (see the package docstring).

Eq. 5: sigma(x) = f_sigma((x - x_B) / ||s_B||_inf).
Eq. 6: f_sigma(x) = W2 cos(omega0 (W1 x + b1)) + b2, W1 (N x 3), b1 (N),
       W2 (1 x N), b2 scalar; omega0 multiplies b1 as printed in Eq. 6.
Eq. 7: the integral of sigma along the chord [t_in, t_out] equals
       S(t_out) - S(t_in) with S an antiderivative in t.
Eq. 8: S(t) = [W2 / (omega0 W1 d)] sin(omega0 (t W1 d + W1 o + b1)) + t b2.
       The paper prints S without the normalisation of Eq. 5 and says that
       it is absorbed into W1 and b1.  Here it is applied explicitly: with
       m = ||s||_inf,  a_k = W1_k . d / m  and  c_k = W1_k . (o - x_B) / m + b1_k
       the argument is omega0 (a_k t + c_k).  For x_B = 0 and m = 1 this is
       Eq. 8 verbatim.

Time-conditioned density (the dynamic-scene application): with a time
xi_t in [0, 1] and a per-primitive temporal weight W_t (N,), the phase of
unit k gains xi_t W_t,k, added to omega0 (W1 x + b1) unscaled as printed:
f_sigma(x, xi_t) = W2 cos(omega0 (W1 x + b1) + xi_t W_t) + b2.  It is a
constant along the ray, so the antiderivative keeps its form with the
shifted phase.

A primitive is passed as a dict with keys center (3,), scale (3,), w1 (N,3),
b1 (N,), w2 (N,), b2 (scalar) and omega0; optionally wt (N,) and time.
"""
from __future__ import annotations

import numpy as np


def _unpack(prim):
    c = np.asarray(prim["center"], dtype=np.float64)
    s = np.asarray(prim["scale"], dtype=np.float64)
    m = float(np.max(s))
    w1 = np.asarray(prim["w1"], dtype=np.float64)
    b1 = np.asarray(prim["b1"], dtype=np.float64)
    w2 = np.asarray(prim["w2"], dtype=np.float64)
    b2 = float(prim["b2"])
    return c, m, w1, b1, w2, b2, float(prim["omega0"])


def time_phase(prim):
    """xi_t W_t (N,) of the time-conditioned density; zero without W_t."""
    if prim.get("wt") is None:
        return 0.0
    return float(prim.get("time", 0.0)) * np.asarray(prim["wt"], dtype=np.float64)


def density(x, prim):
    """sigma(x) of Eq. 5-6 at points x (..., 3) (with the time term if any)."""
    c, m, w1, b1, w2, b2, om = _unpack(prim)
    u = (np.asarray(x, dtype=np.float64) - c) / m
    return np.cos(om * (u @ w1.T + b1) + time_phase(prim)) @ w2 + b2


def _phase_coefficients(o, d, prim):
    """a_k (..., N) and c_k (N,) such that the phase along o + t d is
    omega0 (a_k t + c_k)."""
    c, m, w1, b1, _, _, _ = _unpack(prim)
    a = (np.asarray(d, dtype=np.float64) @ w1.T) / m
    cc = (np.asarray(o, dtype=np.float64) - c) @ w1.T / m + b1
    return a, cc


def antiderivative(t, o, d, prim):
    """S(t; o, d) of Eq. 8 (normalisation made explicit); t (...), d (..., 3)."""
    _, _, _, _, w2, b2, om = _unpack(prim)
    a, cc = _phase_coefficients(o, d, prim)
    t = np.asarray(t, dtype=np.float64)[..., None]
    return np.sum(w2 * np.sin(om * (a * t + cc) + time_phase(prim)) / (om * a), axis=-1) + b2 * t[..., 0]


def chord_integral_literal(o, d, t_in, t_out, prim):
    """Eq. 7 evaluated literally as S(t_out) - S(t_in)."""
    return antiderivative(t_out, o, d, prim) - antiderivative(t_in, o, d, prim)


def _sinc(h):
    """sin(h)/h with sinc(0) = 1 (Taylor series near 0)."""
    h = np.asarray(h, dtype=np.float64)
    small = np.abs(h) < 1e-4
    hs = np.where(small, 1.0, h)
    return np.where(small, 1.0 - h * h / 6.0, np.sin(hs) / hs)


def chord_integral(o, d, t_in, t_out, prim):
    """Exact integral of sigma over [t_in, t_out] along o + t d (Eq. 7-8).

    Same value as S(t_out) - S(t_in), rearranged with the identity
    sin(u + v) - sin(u - v) = 2 cos(u) sin(v): with the chord midpoint
    t_mid = (t_in + t_out)/2 and length L = t_out - t_in,

        S(t_out) - S(t_in) = sum_k W2_k L cos(omega0 (a_k t_mid + c_k))
                                        sinc(omega0 a_k L / 2)  +  b2 L,

    which stays finite as a_k -> 0 (where Eq. 8 divides by zero) and keeps
    the cosine argument at the chord midpoint, inside the unit ball.
    """
    c, m, w1, b1, w2, b2, om = _unpack(prim)
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    t_in = np.asarray(t_in, dtype=np.float64)
    t_out = np.asarray(t_out, dtype=np.float64)
    L = t_out - t_in
    t_mid = 0.5 * (t_in + t_out)
    p_mid = (o + t_mid[..., None] * d - c) / m      # midpoint in MLP coordinates
    phase = om * (p_mid @ w1.T + b1) + time_phase(prim)
    a = (d @ w1.T) / m
    h = 0.5 * om * a * L[..., None]
    return np.sum(w2 * np.cos(phase) * _sinc(h), axis=-1) * L + b2 * L


def chord_integral_quadrature(o, d, t0, t1, prim, n_nodes=64, n_panels=16, inside=None):
    """Composite Gauss-Legendre quadrature of sigma(o + t d) over [t0, t1]
    (a direct numerical evaluation of the integral in Eq. 3/7).

    If `inside` is a callable x -> bool mask, the integrand is
    sigma(x) * 1[inside(x)] (density restricted to the bounding ellipsoid).
    Scalar t0/t1 and a single direction d (3,).
    """
    xg, wg = np.polynomial.legendre.leggauss(n_nodes)
    edges = np.linspace(float(t0), float(t1), n_panels + 1)
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        t = 0.5 * (b - a) * xg + 0.5 * (a + b)
        x = np.asarray(o, dtype=np.float64) + t[:, None] * np.asarray(d, dtype=np.float64)
        f = density(x, prim)
        if inside is not None:
            f = f * inside(x)
        total += 0.5 * (b - a) * np.sum(wg * f)
    return total
