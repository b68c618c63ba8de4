"""Continuous per-Gaussian quantities in float64, as plain definitions
(test infrastructure).

For image (c, e) and every Gaussian g (standard 3DGS / EWA splatting, which the
paper renders; posing by the paper's Rigid-Link Gaussian Kinematics):

* posing: a body Gaussian's world mean is R(q_b) mu + t_b and its world
  covariance R(q_b) Sigma R(q_b)^T, where Sigma = R(q_g) S S^T R(q_g)^T; static
  Gaussians use the identity pose;
* camera space: t = W x + w_t for the viewmat [W | w_t];
* 2D covariance: J W Sigma_world W^T J^T + 0.3 I with the local affine
  Jacobian J of the pinhole projection at t (x/z and y/z clamped to 1.3 times
  the half field of view inside J only);
* conic = inverse of that 2x2 matrix; projected mean u = f_x t_x / t_z + c_x,
  v = f_y t_y / t_z + c_y; depth z = t_z;
* colour: the view direction from the camera centre to the Gaussian, expressed
  in the frame in which its SH coefficients are stored (its body frame), gives
  rgb = max(0, 0.5 + sum_k f_k Y_k(d)).

Nothing here is rounded to float32: inputs are float32 arrays converted to
float64 once.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from .sh import sh_colour


def quat_to_rot64(q: np.ndarray) -> np.ndarray:
    q = np.asarray(q, np.float64)
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


def viewmat64(batch, c: int, e: int):
    """World->camera (W, w) of image (c, e) in float64.  A camera slot attached
    to body k carries body->camera offsets (R_o, t_o): a world point p is
    first taken into the body frame, R_k^T (p - t_k), then into the camera,
    so W = R_o R_k^T and w = t_o - W t_k."""
    vm = np.asarray(batch.viewmats[c, e], np.float64)
    Ro, to = vm[:, :3], vm[:, 3]
    k = int(getattr(batch.cams[c], "attach_body", -1))
    if k < 0:
        return Ro, to
    pose = np.asarray(batch.poses[e, k], np.float64)
    Rk = quat_to_rot64(pose[None, 0:4])[0]
    W = Ro @ Rk.T
    return W, to - W @ pose[4:7]


def attrs64(scene, batch, c: int = 0, e: int = 0, attrs: Dict[str, np.ndarray] | None = None) -> Dict[str, np.ndarray]:
    """Float64 projection of every Gaussian into image (c, e).

    Returns u, v, conic (N, 3: inverse-covariance entries xx, xy, yy), opacity,
    rgb (N, 3), z, cov (N, 3: a=xx, b=xy, c=yy of the dilated covariance),
    det, t (N, 3) camera-space mean and a float64 visibility estimate
    ``visible64`` (finite, in front of the near plane, alpha reachable,
    positive determinant; no tile-rectangle test)."""
    at = attrs or {}
    cam = batch.cams[c]
    mu = np.asarray(at.get("means", scene.means), np.float64)
    s = np.asarray(at.get("scales", scene.scales), np.float64)
    qg = np.asarray(at.get("quats", scene.quats), np.float64)
    op = np.asarray(at.get("opacities", scene.opacities), np.float64)
    sh = np.asarray(at.get("sh", scene.sh), np.float64)
    N = mu.shape[0]

    body = scene.body_of()
    Rb = np.broadcast_to(np.eye(3), (N, 3, 3)).copy()
    tb = np.zeros((N, 3))
    if scene.n_bodies:
        pose = np.asarray(batch.poses[e], np.float64)
        Rbody = quat_to_rot64(pose[:, 0:4])
        m = body >= 0
        Rb[m] = Rbody[body[m]]
        tb[m] = pose[body[m], 4:7]

    Wc, wt = viewmat64(batch, c, e)

    mu_world = np.einsum("nij,nj->ni", Rb, mu) + tb
    t = mu_world @ Wc.T + wt
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]

    Rg = quat_to_rot64(qg)
    RS = Rg * s[:, None, :]
    Sigma_local = RS @ np.transpose(RS, (0, 2, 1))
    Sigma_world = Rb @ Sigma_local @ np.transpose(Rb, (0, 2, 1))
    Sigma_cam = Wc[None] @ Sigma_world @ Wc.T[None]

    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    with np.errstate(all="ignore"):
        lx = 1.3 * (0.5 * cam.width) / fx
        ly = 1.3 * (0.5 * cam.height) / fy
        xcl = np.clip(tx / tz, -lx, lx) * tz
        ycl = np.clip(ty / tz, -ly, ly) * tz
        J = np.zeros((N, 2, 3))
        J[:, 0, 0] = fx / tz
        J[:, 0, 2] = -fx * xcl / (tz * tz)
        J[:, 1, 1] = fy / tz
        J[:, 1, 2] = -fy * ycl / (tz * tz)
        S2 = J @ Sigma_cam @ np.transpose(J, (0, 2, 1)) + 0.3 * np.eye(2)[None]
        a, b, cc = S2[:, 0, 0], S2[:, 0, 1], S2[:, 1, 1]
        det = a * cc - b * b
        conic = np.stack([cc / det, -b / det, a / det], axis=1)
        u = fx * tx / tz + cx
        v = fy * ty / tz + cy

        # camera centre in world, then in each Gaussian's own (body) frame
        cam_centre = -Wc.T @ wt
        view_world = mu_world - cam_centre
        view_local = np.einsum("nji,nj->ni", Rb, view_world)   # R_b^T (mu_world - C)
        d = view_local / np.linalg.norm(view_local, axis=1, keepdims=True)
        rgb = sh_colour(sh, d, scene.sh_degree)

    visible64 = (np.isfinite(t).all(axis=1) & (tz > float(cam.near)) & (op >= 1.0 / 255.0)
                 & np.isfinite(det) & (det > 0))
    return dict(u=u, v=v, conic=conic, opacity=op, rgb=rgb, z=tz, cov=np.stack([a, b, cc], axis=1),
                det=det, t=t, visible64=visible64)
