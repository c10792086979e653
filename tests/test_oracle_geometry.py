"""Pins of the oracle's rotations, rays, intersection and key path; CPU only."""
import numpy as np
import pytest

import synthetic as S
from oracle.geometry import camera_center, intersect_ellipsoid, pixel_rays, quat_to_rotmat
from oracle.keys import project_all, sorted_instances, tile_lists, tile_ranges


def test_rotation_matrix_properties():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((100, 4)) * rng.uniform(0.1, 10, (100, 1))
    R = quat_to_rotmat(q)
    eye = np.broadcast_to(np.eye(3), R.shape)
    assert np.allclose(R @ np.swapaxes(R, 1, 2), eye, atol=1e-14)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-14)
    assert np.allclose(quat_to_rotmat(-q), R, atol=1e-15)
    assert np.allclose(quat_to_rotmat([1, 0, 0, 0]), np.eye(3))
    # 90 degrees about z maps x to y
    c = np.cos(np.pi / 4)
    Rz = quat_to_rotmat([c, 0, 0, c])
    assert np.allclose(Rz @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    # matches Rodrigues' formula
    for qq in q[:10]:
        qq = qq / np.linalg.norm(qq)
        ang = 2 * np.arccos(np.clip(qq[0], -1, 1))
        axis = qq[1:] / np.linalg.norm(qq[1:])
        K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
        Rr = np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K
        assert np.allclose(quat_to_rotmat(qq), Rr, atol=1e-12)


def test_principal_ray_points_at_origin():
    for cam in S.make_cameras([(64, 64), (1280, 720), (1920, 1080)], seed=5):
        o, d = pixel_rays(cam, np.array([cam.cx - 0.5]), np.array([cam.cy - 0.5]))
        assert np.allclose(d[0], -o / np.linalg.norm(o), atol=1e-6)
        assert abs(np.linalg.norm(o) - 3.0) < 1e-5
        # pixel +x goes right: the ray's camera-frame x grows with the column
        _, d2 = pixel_rays(cam, np.array([cam.cx + 10]), np.array([cam.cy - 0.5]))
        assert (np.asarray(cam.R, float) @ d2[0])[0] > 0


def test_sphere_chord_length():
    """Equal scales r and identity rotation: chord length 2 sqrt(r^2 - b^2), b the
    distance between the sphere centre and the ray."""
    rng = np.random.default_rng(1)
    for _ in range(50):
        c = rng.uniform(-1, 1, 3)
        r = rng.uniform(0.05, 0.5)
        o = rng.standard_normal(3) * 3
        d = rng.standard_normal((8, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        disc, t0, t1 = intersect_ellipsoid(o, d, c, [r, r, r], np.eye(3))
        b = np.linalg.norm(np.cross(c - o, d), axis=1)
        hit = b < r
        assert np.array_equal(disc > 0, hit)
        assert np.allclose((t1 - t0)[hit], 2 * np.sqrt(r * r - b[hit] ** 2), atol=1e-12)


def test_endpoints_on_quadric_and_axis_swap_invariance():
    rng = np.random.default_rng(2)
    for _ in range(30):
        c = rng.uniform(-1, 1, 3)
        s = rng.uniform(0.02, 0.3, 3)
        q = rng.standard_normal(4)
        R = quat_to_rotmat(q)
        o = rng.standard_normal(3) * 3
        u = rng.standard_normal((16, 3)) * 0.4
        d = c + (R @ (s * u).T).T - o
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        disc, t0, t1 = intersect_ellipsoid(o, d, c, s, R)
        for t in (t0, t1):
            x = o + t[:, None] * d
            v = ((x - c) @ R) / s
            val = np.sum(v * v, axis=1)
            assert np.allclose(val[disc > 0], 1.0, atol=1e-10)
        # rotate the frame by 90 degrees about its own z axis and swap s_x, s_y
        c4 = np.cos(np.pi / 4)
        qz = np.array([c4, 0, 0, c4])
        w1, x1, y1, z1 = q
        w2, x2, y2, z2 = qz
        q2 = np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                       w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
        disc2, u0, u1 = intersect_ellipsoid(o, d, c, s[[1, 0, 2]], quat_to_rotmat(q2))
        assert np.array_equal(disc > 0, disc2 > 0)
        assert np.allclose(t0[disc > 0], u0[disc > 0], atol=1e-10)
        assert np.allclose(t1[disc > 0], u1[disc > 0], atol=1e-10)


def _surface_points(scene, p, n=20000, rng=None):
    rng = np.random.default_rng(0) if rng is None else rng
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    R = quat_to_rotmat(scene["quats"][p].astype(float))
    return scene["centers"][p].astype(float) + (R @ (scene["scales"][p].astype(float) * u).T).T


def test_outline_extent_is_tight_and_culling_is_exact():
    """The dual-quadric tangents bound the projections of sampled surface
    points and are attained by them within 1e-3 px; a primitive is culled iff
    some of its surface lies behind the near plane."""
    scene = S.custom_scene(200, 8, seed=3)
    cam = S.make_cameras([(320, 240)], seed=4)[0]
    pr = project_all(scene, cam, z_near=0.2)
    Rc, tc = np.asarray(cam.R, float), np.asarray(cam.t, float)
    rng = np.random.default_rng(1)
    for p in range(200):
        X = _surface_points(scene, p, 40000, rng) @ Rc.T + tc
        zmin = X[:, 2].min()
        if abs(zmin - 0.2) > 1e-3:
            assert pr["keep"][p] == (zmin > 0.2)
        if not pr["keep"][p]:
            continue
        px = float(cam.fx) * X[:, 0] / X[:, 2] + float(cam.cx)
        py = float(cam.fy) * X[:, 1] / X[:, 2] + float(cam.cy)
        lo_x, hi_x, lo_y, hi_y = pr["extent"][p]
        assert px.min() >= lo_x - 1e-9 and px.max() <= hi_x + 1e-9
        assert py.min() >= lo_y - 1e-9 and py.max() <= hi_y + 1e-9
        span = max(hi_x - lo_x, hi_y - lo_y)
        tol = 2e-3 * span + 1e-6
        assert px.min() - lo_x <= tol and hi_x - px.max() <= tol
        assert py.min() - lo_y <= tol and hi_y - py.max() <= tol


def test_near_plane_culling_of_close_primitives():
    cam = S.make_cameras([(64, 64)], seed=1)[0]
    o = camera_center(cam)
    fwd = -o / np.linalg.norm(o)
    scene = S.custom_scene(3, 8, seed=0)
    scene["centers"] = np.array([o + 0.25 * fwd, o + 0.5 * fwd, o - 0.5 * fwd], np.float32)
    scene["scales"] = np.full((3, 3), 0.1, np.float32)
    scene["quats"] = np.tile(np.array([1, 0, 0, 0], np.float32), (3, 1))
    pr = project_all(scene, cam, z_near=0.2)
    assert list(pr["keep"]) == [False, True, False]


@pytest.mark.parametrize("size,P", [((64, 64), 256), ((256, 256), 2000)])
def test_rect_contains_every_hit_pixel(size, P):
    """Brute force over every pixel of the image: each pixel whose ray meets
    a kept primitive's ellipsoid lies in that primitive's pixel rectangle, and
    the tangent rays at the outline extremes are (nearly) tangent."""
    scene = S.custom_scene(P, 8, seed=7)
    cam = S.make_cameras([size], seed=8)[0]
    pr = project_all(scene, cam)
    W, H = size
    rows, cols = np.mgrid[0:H, 0:W]
    o, d = pixel_rays(cam, cols.ravel(), rows.ravel())
    Rs = quat_to_rotmat(scene["quats"].astype(float))
    n_hit = 0
    for p in np.nonzero(pr["keep"])[0]:
        disc, _, _ = intersect_ellipsoid(o, d, scene["centers"][p], scene["scales"][p], Rs[p])
        hit = disc > 0
        n_hit += hit.sum()
        if not hit.any():
            continue
        assert pr["nonempty"][p]
        x0, x1, y0, y1 = pr["rect"][p]
        hc, hr = cols.ravel()[hit], rows.ravel()[hit]
        assert hc.min() >= x0 and hc.max() <= x1 and hr.min() >= y0 and hr.max() <= y1
    assert n_hit > 0


def test_tangent_rays_touch_the_ellipsoid():
    """Rays through points of the tangent line x = x_lo are tangent or miss;
    slightly inside that line some ray hits."""
    scene = S.custom_scene(40, 8, seed=21)
    cam = S.make_cameras([(512, 512)], seed=22)[0]
    pr = project_all(scene, cam)
    Rs = quat_to_rotmat(scene["quats"].astype(float))
    for p in np.nonzero(pr["keep"])[0][:20]:
        lo_x, hi_x, lo_y, hi_y = pr["extent"][p]
        ys = np.linspace(lo_y, hi_y, 4001)
        for xline, inward in ((lo_x, +1), (hi_x, -1)):
            o, d = pixel_rays(cam, np.full_like(ys, xline - 0.5), ys - 0.5)
            disc, _, _ = intersect_ellipsoid(o, d, scene["centers"][p], scene["scales"][p], Rs[p])
            dn = disc / np.max(np.abs(disc))
            assert dn.max() <= 1e-9
            o2, d2 = pixel_rays(cam, np.full_like(ys, xline + inward * 1e-2 - 0.5), ys - 0.5)
            disc2, _, _ = intersect_ellipsoid(o2, d2, scene["centers"][p], scene["scales"][p], Rs[p])
            assert disc2.max() > 0


def test_tile_lists_cover_hits_and_are_ordered():
    """Every (pixel, primitive) hit appears in the list of the pixel's tile; the
    lists are ordered by the float32 camera depth (computed here by a matrix
    product) and then by index; keys and ranges are consistent."""
    scene = S.custom_scene(300, 8, seed=31)
    cams = S.make_cameras([(96, 64), (64, 48)], seed=32)
    for tw, th in ((16, 16), (8, 8), (32, 16)):
        lists = tile_lists(scene, cams, tw, th)
        keys, vals = sorted_instances(lists)
        ranges = tile_ranges(lists)
        assert np.all(np.diff(keys.astype(np.uint64)) >= 0)
        gbase = 0
        for cam in cams:
            Rc, tc = np.asarray(cam.R, float), np.asarray(cam.t, float)
            zc = (scene["centers"].astype(float) @ Rc.T + tc)[:, 2].astype(np.float32)
            ntx = (cam.width + tw - 1) // tw
            nty = (cam.height + th - 1) // th
            for g in range(gbase, gbase + ntx * nty):
                lst = [p for _, p in lists[g]]
                z = zc[lst]
                assert all((z[i], lst[i]) < (z[i + 1], lst[i + 1]) for i in range(len(lst) - 1))
                s, e = ranges[g]
                assert list(vals[s:e]) == lst
                assert np.all((keys[s:e] >> np.uint64(31)) == g)
            rows, cols = np.mgrid[0:cam.height, 0:cam.width]
            o, d = pixel_rays(cam, cols.ravel(), rows.ravel())
            Rs = quat_to_rotmat(scene["quats"].astype(float))
            for p in range(0, 300, 7):
                disc, _, _ = intersect_ellipsoid(o, d, scene["centers"][p], scene["scales"][p], Rs[p])
                for pix in np.nonzero(disc > 0)[0][::13]:
                    g = gbase + (rows.ravel()[pix] // th) * ntx + cols.ravel()[pix] // tw
                    assert p in [q for _, q in lists[g]]
            gbase += ntx * nty


def test_depth_ties_break_by_index():
    scene = S.custom_scene(50, 8, seed=41)
    scene["centers"][10:20] = scene["centers"][5]
    cam = S.make_cameras([(64, 64)], seed=42)[0]
    lists = tile_lists(scene, [cam])
    for lst in lists:
        for (b0, p0), (b1, p1) in zip(lst[:-1], lst[1:]):
            assert b0 < b1 or (b0 == b1 and p0 < p1)
    assert any(sum(1 for _, p in lst if 5 <= p < 20) >= 2 for lst in lists)
