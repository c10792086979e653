"""Per-(primitive, view) culling, screen bounds, depth keys and tile lists (FP64).

Test infrastructure only (see the package docstring).

The paper renders with 3DGS-style tiling and depth sorting (Eq. 4: the
primitives N(r) along a ray are depth sorted; App. A names preprocessing and
primitive sorting/tiling as pipeline stages) but gives no formula for either.
The readings used here:

  * Near culling.  A primitive is kept for a view only if its whole ellipsoid
    lies in front of the plane z = z_near in camera space:
    mu_z - sqrt(Sigma_zz) > z_near, where mu and Sigma = R_c R diag(s^2) R^T R_c^T
    are the centre and shape matrix in camera coordinates.  Then every hit
    has t_in > 0 and the outline on the image is a bounded ellipse.
  * Screen bounds.  The exact bounding box of the projected ellipsoid, from
    its dual quadric: with M = Sigma - mu mu^T, the vertical lines x = u
    (normalised image coordinates) tangent to the outline solve
    M22 u^2 - 2 M02 u + M00 = 0 (rows: M11, M12).  Pixel column i can be hit
    only if its centre i + 0.5 lies strictly between the two tangents, so the
    pixel rectangle is [ceil(p_lo - 1/2 - eps), floor(p_hi - 1/2 + eps)],
    eps = 1/64 px, clipped to the image.
  * Depth.  The camera-space z of the centre, rounded to float32; its bit
    pattern (positive after culling, hence monotone) is the sort key.  Equal
    depths are ordered by primitive index.
  * Tiles.  Row-major tiles of tile_w x tile_h pixels; a primitive is listed
    in every tile its pixel rectangle touches.  The global tile id of view v
    is the number of tiles of views 0..v-1 plus the local id, and the sort key
    of an instance is (global tile id << 31) | depth bits (the depth is
    positive, so its sign bit is zero and is dropped).

The key path is evaluated in float64 with one fixed order of correctly
rounded operations (no fused multiply-add; each numpy elementwise operation
rounds once), so any other float64 implementation that follows the same
order produces the same integers bit for bit.  The order is written out
step by step below.
"""
from __future__ import annotations

import numpy as np

EPS_PX = 1.0 / 64.0


def project_all(scene, cam, tile_w=16, tile_h=16, z_near=0.2):
    """Key path for all primitives of `scene` in camera `cam`.

    Returns a dict of per-primitive arrays:
      keep (bool), rect (P,4) int64 [x0, x1, y0, y1] inclusive pixel bounds,
      nonempty (bool), trect (P,4) int64 [tx0, tx1, ty0, ty1],
      depth (float32), depth_bits (uint32), n_tiles (int64),
      extent (P,4) float64 [x_lo, x_hi, y_lo, y_hi]: pixel coordinates of the
      tangent lines of the projected outline (meaningful where keep).
    """
    f64 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    q = f64(scene["quats"])
    xb = f64(scene["centers"])
    s = f64(scene["scales"])
    C = f64(cam.R)
    t = f64(cam.t)
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    W, H = int(cam.width), int(cam.height)
    zn = float(np.float32(z_near))

    with np.errstate(all="ignore"):
        # 1. normalised quaternion
        qn = np.sqrt(((q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2]) + q[:, 3] * q[:, 3])
        w = q[:, 0] / qn
        x = q[:, 1] / qn
        y = q[:, 2] / qn
        z = q[:, 3] / qn
        # 2. rotation matrix
        xx = x * x; yy = y * y; zz = z * z
        xy = x * y; xz = x * z; yz = y * z
        wx = w * x; wy = w * y; wz = w * z
        Rp = np.empty((q.shape[0], 3, 3))
        Rp[:, 0, 0] = 1.0 - 2.0 * (yy + zz)
        Rp[:, 0, 1] = 2.0 * (xy - wz)
        Rp[:, 0, 2] = 2.0 * (xz + wy)
        Rp[:, 1, 0] = 2.0 * (xy + wz)
        Rp[:, 1, 1] = 1.0 - 2.0 * (xx + zz)
        Rp[:, 1, 2] = 2.0 * (yz - wx)
        Rp[:, 2, 0] = 2.0 * (xz - wy)
        Rp[:, 2, 1] = 2.0 * (yz + wx)
        Rp[:, 2, 2] = 1.0 - 2.0 * (xx + yy)
        # 3. camera-frame rotation  Rc = C Rp
        Rc = np.empty_like(Rp)
        for i in range(3):
            for j in range(3):
                Rc[:, i, j] = (C[i, 0] * Rp[:, 0, j] + C[i, 1] * Rp[:, 1, j]) + C[i, 2] * Rp[:, 2, j]
        # 4. camera-frame centre  mu = C x_B + t
        mu = np.empty_like(xb)
        for i in range(3):
            mu[:, i] = ((C[i, 0] * xb[:, 0] + C[i, 1] * xb[:, 1]) + C[i, 2] * xb[:, 2]) + t[i]
        # 5. camera-frame shape matrix  Sigma = Rc diag(s^2) Rc^T
        ss = s * s

        def sig(i, j):
            return (((Rc[:, i, 0] * ss[:, 0]) * Rc[:, j, 0] + (Rc[:, i, 1] * ss[:, 1]) * Rc[:, j, 1])
                    + (Rc[:, i, 2] * ss[:, 2]) * Rc[:, j, 2])

        S00, S02, S11, S12, S22 = sig(0, 0), sig(0, 2), sig(1, 1), sig(1, 2), sig(2, 2)
        # 6. near culling
        keep = (mu[:, 2] - np.sqrt(S22)) > zn
        # 7. dual-quadric outline  M = Sigma - mu mu^T
        M00 = S00 - mu[:, 0] * mu[:, 0]
        M02 = S02 - mu[:, 0] * mu[:, 2]
        M11 = S11 - mu[:, 1] * mu[:, 1]
        M12 = S12 - mu[:, 1] * mu[:, 2]
        M22 = S22 - mu[:, 2] * mu[:, 2]

        # 8. tangent lines -> pixel range
        def extent(Ma, Mb, f, cc, size):
            disc = Mb * Mb - Ma * M22
            disc = np.where(disc > 0.0, disc, 0.0)
            sq = np.sqrt(disc)
            u_lo = (Mb + sq) / M22
            u_hi = (Mb - sq) / M22
            p_lo = f * u_lo + cc
            p_hi = f * u_hi + cc
            lo = np.ceil((p_lo - 0.5) - EPS_PX)
            hi = np.floor((p_hi - 0.5) + EPS_PX)
            lo = np.where(lo > 0.0, lo, 0.0)
            hi = np.where(hi < size - 1.0, hi, size - 1.0)
            return lo, hi, p_lo, p_hi

        x0, x1, px_lo, px_hi = extent(M00, M02, fx, cx, float(W))
        y0, y1, py_lo, py_hi = extent(M11, M12, fy, cy, float(H))
        nonempty = keep & (x0 <= x1) & (y0 <= y1)
    rect = np.zeros((q.shape[0], 4), dtype=np.int64)
    rect[nonempty, 0] = x0[nonempty].astype(np.int64)
    rect[nonempty, 1] = x1[nonempty].astype(np.int64)
    rect[nonempty, 2] = y0[nonempty].astype(np.int64)
    rect[nonempty, 3] = y1[nonempty].astype(np.int64)
    trect = np.zeros_like(rect)
    trect[:, 0] = rect[:, 0] // tile_w
    trect[:, 1] = rect[:, 1] // tile_w
    trect[:, 2] = rect[:, 2] // tile_h
    trect[:, 3] = rect[:, 3] // tile_h
    n_tiles = np.where(nonempty, (trect[:, 1] - trect[:, 0] + 1) * (trect[:, 3] - trect[:, 2] + 1), 0)
    # 9. depth key: camera-space z rounded to the nearest float32
    depth = mu[:, 2].astype(np.float32)
    depth_bits = depth.view(np.uint32)
    return dict(keep=keep, rect=rect, nonempty=nonempty, trect=trect, depth=depth,
                depth_bits=depth_bits, n_tiles=n_tiles.astype(np.int64),
                extent=np.stack([px_lo, px_hi, py_lo, py_hi], axis=1))


def tiles_of(cam, tile_w, tile_h):
    """Number of tiles across and down the image."""
    return (cam.width + tile_w - 1) // tile_w, (cam.height + tile_h - 1) // tile_h


def tile_lists(scene, cams, tile_w=16, tile_h=16, z_near=0.2, projs=None):
    """Brute-force tile lists: for every global tile id, the primitives whose
    pixel rectangle touches it, ordered by (depth bits, primitive index) with
    Python's sorted().  Returns a list (one entry per global tile) of lists."""
    out = []
    for v, cam in enumerate(cams):
        pr = projs[v] if projs is not None else project_all(scene, cam, tile_w, tile_h, z_near)
        ntx, nty = tiles_of(cam, tile_w, tile_h)
        ids = np.nonzero(pr["nonempty"])[0]
        tr = pr["trect"][ids]
        bits = pr["depth_bits"][ids]
        for ty in range(nty):
            for tx in range(ntx):
                sel = (tr[:, 0] <= tx) & (tx <= tr[:, 1]) & (tr[:, 2] <= ty) & (ty <= tr[:, 3])
                out.append(sorted(zip(bits[sel].tolist(), ids[sel].tolist())))
    return out


def sorted_instances(lists):
    """Keys (uint64) and values (uint32) in sorted order, from tile lists."""
    keys, vals = [], []
    for gid, lst in enumerate(lists):
        for bits, p in lst:
            keys.append((gid << 31) | bits)
            vals.append(p)
    return np.array(keys, dtype=np.uint64), np.array(vals, dtype=np.uint32)


def tile_ranges(lists):
    """[start, end) of every global tile in the sorted instance arrays."""
    r = np.zeros((len(lists), 2), dtype=np.int64)
    pos = 0
    for gid, lst in enumerate(lists):
        r[gid] = (pos, pos + len(lst))
        pos += len(lst)
    return r
