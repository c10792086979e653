"""Pins of the oracle's density field and chord integral (Eq. 5-8) against
quadrature, calculus identities and special cases; CPU only."""
import json
import math
import os

import numpy as np
import pytest

from oracle import density as D
from oracle.geometry import intersect_ellipsoid, quat_to_rotmat

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_prim(rng, N=16, omega0=10.0, scale=None):
    s = np.exp(rng.uniform(np.log(0.02), np.log(0.2), 3)) if scale is None else np.asarray(scale, float)
    q = rng.standard_normal(4)
    return dict(center=rng.uniform(-1, 1, 3), scale=s, R=quat_to_rotmat(q), q=q,
                w1=rng.uniform(-1 / 3, 1 / 3, (N, 3)), b1=rng.uniform(-np.pi, np.pi, N),
                w2=rng.uniform(0, 1 / 8, N), b2=rng.uniform(-0.5, 0.5), omega0=omega0)


def ray_through(rng, prim, o=None):
    """A camera-like origin and a unit direction aimed at a random point
    inside the ellipsoid."""
    o = rng.standard_normal(3) * 3 if o is None else o
    u = rng.standard_normal(3)
    u = u / np.linalg.norm(u) * rng.uniform(0, 0.95) ** (1 / 3)
    target = prim["center"] + prim["R"] @ (prim["scale"] * u)
    d = target - o
    return o, d / np.linalg.norm(d)


@pytest.mark.parametrize("N,omega0", [(4, 1.0), (8, 10.0), (16, 10.0), (32, 30.0)])
def test_closed_form_matches_gauss_legendre(N, omega0):
    rng = np.random.default_rng(100 + N)
    for _ in range(20):
        prim = random_prim(rng, N, omega0)
        o, d = ray_through(rng, prim)
        disc, t0, t1 = intersect_ellipsoid(o, d[None], prim["center"], prim["scale"], prim["R"])
        assert disc[0] > 0
        exact = D.chord_integral(o, d[None], t0, t1, prim)[0]
        quad = D.chord_integral_quadrature(o, d, t0[0], t1[0], prim, n_nodes=64, n_panels=16)
        scale = np.sum(np.abs(prim["w2"])) * (t1[0] - t0[0]) + abs(prim["b2"]) * (t1[0] - t0[0])
        assert abs(exact - quad) <= 1e-12 * scale


def test_density_vanishes_outside_chord():
    """Integrating sigma * 1[x in B] over [0, 10] equals the chord integral, so the
    bounds t_in, t_out found by the intersection are exactly where B starts and ends."""
    rng = np.random.default_rng(7)
    for _ in range(10):
        prim = random_prim(rng, 8)
        o, d = ray_through(rng, prim)
        _, t0, t1 = intersect_ellipsoid(o, d[None], prim["center"], prim["scale"], prim["R"])

        def inside(x):
            u = ((x - prim["center"]) @ prim["R"]) / prim["scale"]
            return (np.sum(u * u, axis=-1) <= 1.0).astype(float)

        edges = [0.0, t0[0], t1[0], 10.0]
        parts = [D.chord_integral_quadrature(o, d, a, b, prim, 64, 16, inside=inside)
                 for a, b in zip(edges[:-1], edges[1:])]
        assert abs(parts[0]) == 0.0 and abs(parts[2]) == 0.0
        exact = D.chord_integral(o, d[None], t0, t1, prim)[0]
        assert abs(parts[1] - exact) <= 1e-11
        # just inside / just outside the endpoints
        for t, sgn in ((t0[0], +1), (t1[0], -1)):
            assert inside(o + (t + sgn * 1e-7) * d) == 1.0
            assert inside(o + (t - sgn * 1e-7) * d) == 0.0


def test_antiderivative_derivative_is_density():
    """Fundamental theorem of calculus (Eq. 7): dS/dt = sigma(o + t d)."""
    rng = np.random.default_rng(3)
    for _ in range(10):
        prim = random_prim(rng, 16)
        o, d = ray_through(rng, prim)
        for t in rng.uniform(1.0, 5.0, 5):
            h = 1e-5
            dS = (D.antiderivative(t + h, o, d[None], prim)[0] - D.antiderivative(t - h, o, d[None], prim)[0]) / (2 * h)
            sig = D.density(o + t * d, prim)
            assert abs(dS - sig) <= 1e-6 * max(1.0, abs(sig))


def test_literal_and_midpoint_forms_agree():
    rng = np.random.default_rng(11)
    for N in (4, 8, 16, 32):
        prim = random_prim(rng, N)
        o = rng.standard_normal(3) * 3
        ds, t0s, t1s = [], [], []
        for _ in range(200):
            _, d = ray_through(rng, prim, o)
            ds.append(d)
        ds = np.array(ds)
        _, t0, t1 = intersect_ellipsoid(o, ds, prim["center"], prim["scale"], prim["R"])
        a = D.chord_integral(o, ds, t0, t1, prim)
        b = D.chord_integral_literal(o, ds, t0, t1, prim)
        assert np.max(np.abs(a - b)) <= 1e-10


def test_zero_frequency_gives_constant_density():
    """W1 = 0: sigma is the constant sum_k W2_k cos(omega0 b1_k) + b2, so the
    integral is that constant times the chord length."""
    rng = np.random.default_rng(5)
    prim = random_prim(rng, 8)
    prim["w1"] = np.zeros_like(prim["w1"])
    sigma0 = float(np.sum(prim["w2"] * np.cos(prim["omega0"] * prim["b1"])) + prim["b2"])
    o, d = ray_through(rng, prim)
    _, t0, t1 = intersect_ellipsoid(o, d[None], prim["center"], prim["scale"], prim["R"])
    got = D.chord_integral(o, d[None], t0, t1, prim)[0]
    assert abs(got - sigma0 * (t1[0] - t0[0])) <= 1e-14


def test_frequency_orthogonal_to_ray_limit():
    """a_k = 0 (W1_k orthogonal to d): the k-th term is W2_k L cos(phase), the
    limit of Eq. 8 where it divides by zero; checked against quadrature."""
    rng = np.random.default_rng(9)
    prim = random_prim(rng, 8)
    o, d = ray_through(rng, prim)
    for k in range(8):
        w = prim["w1"][k]
        prim["w1"][k] = w - (w @ d) * d
    _, t0, t1 = intersect_ellipsoid(o, d[None], prim["center"], prim["scale"], prim["R"])
    got = D.chord_integral(o, d[None], t0, t1, prim)[0]
    quad = D.chord_integral_quadrature(o, d, t0[0], t1[0], prim)
    assert abs(got - quad) <= 1e-12


def test_unit_normalisation_reduces_to_printed_eq8():
    """x_B = 0 and ||s||_inf = 1: the normalised antiderivative is Eq. 8 as printed,
    S(t) = [W2 / (omega0 W1 d)] sin(omega0 (t W1 d + W1 o + b1)) + t b2."""
    rng = np.random.default_rng(13)
    prim = random_prim(rng, 8, scale=[1.0, 0.5, 0.25])
    prim["center"] = np.zeros(3)
    o = np.array([0.3, -2.0, 0.7])
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    for t in (0.5, 1.25, 2.0):
        w1d = prim["w1"] @ d
        printed = np.sum(prim["w2"] / (prim["omega0"] * w1d) *
                         np.sin(prim["omega0"] * (t * w1d + prim["w1"] @ o + prim["b1"]))) + t * prim["b2"]
        assert abs(D.antiderivative(t, o, d[None], prim)[0] - printed) <= 1e-12


def test_endpoint_derivatives_are_densities():
    """d integral / d t_out = sigma(o + t_out d), d integral / d t_in = -sigma(o + t_in d)."""
    rng = np.random.default_rng(17)
    prim = random_prim(rng, 16)
    o, d = ray_through(rng, prim)
    _, t0, t1 = intersect_ellipsoid(o, d[None], prim["center"], prim["scale"], prim["R"])
    h = 1e-6
    f = lambda a, b: D.chord_integral(o, d[None], np.array([a]), np.array([b]), prim)[0]
    g_out = (f(t0[0], t1[0] + h) - f(t0[0], t1[0] - h)) / (2 * h)
    g_in = (f(t0[0] + h, t1[0]) - f(t0[0] - h, t1[0])) / (2 * h)
    assert abs(g_out - D.density(o + t1[0] * d, prim)) <= 1e-7
    assert abs(g_in + D.density(o + t0[0] * d, prim)) <= 1e-7


def test_parameter_layout_matches_paper_counts():
    """App. C: 41 MLP parameters at N = 8 (W1 N x 3, b1 N, W2 N, b2 1), 10 geometry
    parameters, 48 SH coefficients, 99 in total; the memory column of the network
    configuration table scales like (5N + 1 + 10 + 48) floats per primitive."""
    g = json.load(open(os.path.join(GOLDEN, "paper_param_counts.json")))
    N = g["n_hidden"]
    assert 3 * N + N + N + 1 == g["mlp_params"]
    assert 3 + 3 + 4 == g["geometry_params"]
    assert g["mlp_params"] + g["geometry_params"] + g["sh_params"] == g["total_params"]
    mem = {int(k): v for k, v in g["memory_mb_by_n_hidden"].items()}
    floats = {n: 5 * n + 1 + 10 + 48 for n in mem}
    ratios = [mem[n] / floats[n] for n in sorted(mem)]
    assert max(ratios) / min(ratios) < 1.01
    # the same primitive count at 4 bytes per float (MB = 1e6 bytes)
    prims = mem[8] * 1e6 / (4 * floats[8])
    assert 2.0e5 < prims < 2.6e5
