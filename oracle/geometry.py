"""Primitive bounds, camera rays and the ray-ellipsoid intersection (FP64).

Test infrastructure only (see the package docstring).

Sec. 3.1 (Representation): every primitive is bounded by an ellipsoid with
centre x_B, a per-axis scaling vector s_B and a rotation quaternion q_B.
Readings used here, since the paper does not spell them out:
  * q_B = (w, x, y, z), normalised before use (Hamilton convention);
  * s_B holds the semi-axis lengths, so the ellipsoid is
    {x : || diag(1/s) R^T (x - x_B) || <= 1} with R = R(q_B);
  * view rays r(t) = o + t d with a unit direction d (Sec. 2.1: d lies on the
    sphere), t measured in world length.
"""
from __future__ import annotations

import numpy as np


def quat_to_rotmat(q) -> np.ndarray:
    """Rotation matrix R(q) for quaternions q (..., 4) stored (w, x, y, z);
    q is normalised first.  Columns of R are the ellipsoid's principal axes
    in world coordinates."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def camera_to_world(cam) -> np.ndarray:
    """Inverse of the camera's 3x3 matrix R (x_cam = R x_world + t).

    R is stored in float32, so it is orthogonal only to about 1e-7; rays are
    mapped back to the world with the exact inverse of the stored matrix so
    that they agree with the world-to-camera map used for culling, bounds and
    depth."""
    return np.linalg.inv(np.asarray(cam.R, dtype=np.float64))


def camera_center(cam) -> np.ndarray:
    """World position o of a camera with x_cam = R x_world + t."""
    t = np.asarray(cam.t, dtype=np.float64)
    return -camera_to_world(cam) @ t


def pixel_rays(cam, cols, rows):
    """Rays through pixel centres (cols + 0.5, rows + 0.5).

    Returns (o, d): o is the camera centre (3,), d (..., 3) unit world-space
    directions (Sec. 2.1, r(t) = o + t d with d on the unit sphere): the
    camera-space direction ((i+0.5-cx)/fx, (j+0.5-cy)/fy, 1) mapped by R^-1
    and normalised.
    """
    cols = np.asarray(cols, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.float64)
    xc = (cols + 0.5 - float(cam.cx)) / float(cam.fx)
    yc = (rows + 0.5 - float(cam.cy)) / float(cam.fy)
    dc = np.stack([xc, yc, np.ones_like(xc)], axis=-1)
    d = dc @ camera_to_world(cam).T
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return camera_center(cam), d


def intersect_ellipsoid(o, d, center, scale, R):
    """Analytic line-ellipsoid intersection (Sec. 3.2: entry and exit
    distances t_in, t_out).

    In the ellipsoid's normalised frame o' = diag(1/s) R^T (o - x_B) and
    d' = diag(1/s) R^T d the ellipsoid is the unit sphere, so t solves
    |o' + t d'|^2 = 1:  A t^2 + 2 B t + C = 0 with A = d'.d', B = o'.d',
    C = o'.o' - 1.  A ray hits when disc = B^2 - A C > 0.

    o: (3,), d: (..., 3).  Returns (disc, t_in, t_out); t_in/t_out are NaN
    where disc <= 0.
    """
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    center = np.asarray(center, dtype=np.float64)
    inv_s = 1.0 / np.asarray(scale, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    op = ((o - center) @ R) * inv_s          # diag(1/s) R^T (o - x_B)
    dp = (d @ R) * inv_s                     # diag(1/s) R^T d
    A = np.sum(dp * dp, axis=-1)
    B = dp @ op
    C = op @ op - 1.0
    disc = B * B - A * C
    with np.errstate(invalid="ignore"):
        sq = np.sqrt(np.where(disc > 0, disc, np.nan))
    t_in = (-B - sq) / A
    t_out = (-B + sq) / A
    return disc, t_in, t_out
