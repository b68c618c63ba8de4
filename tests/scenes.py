"""Hand-built scenes and cameras for the closed-form tests."""
import math

import numpy as np

from paper_2604_25459_amd.synth import Batch, Camera, Scene

IDENTITY_VIEW = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float32)


def scene_from(means, scales, quats=None, opac=None, sh=None, degree=0, body_offsets=None):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    scales = np.broadcast_to(np.asarray(scales, np.float32), (n, 3)).copy() if np.ndim(scales) <= 1 \
        else np.asarray(scales, np.float32).reshape(n, 3)
    if quats is None:
        quats = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    quats = np.asarray(quats, np.float32).reshape(n, 4)
    opac = np.broadcast_to(np.asarray(0.9 if opac is None else opac, np.float32), (n,)).copy()
    K = (degree + 1) ** 2
    if sh is None:
        sh = np.zeros((n, K, 3), np.float32)
    sh = np.asarray(sh, np.float32).reshape(n, K, 3)
    if body_offsets is None:
        body_offsets = np.array([n], np.int64)
    return Scene(means=np.ascontiguousarray(means), scales=scales, quats=np.ascontiguousarray(quats),
                 opacities=opac, sh=np.ascontiguousarray(sh), sh_degree=degree,
                 body_offsets=np.asarray(body_offsets, np.int64))


def one_camera(W, H, f, cx=None, cy=None, near=0.01, viewmat=None, poses=None, bg=(0, 0, 0), n_bodies=0):
    cam = Camera(width=W, height=H, fx=float(np.float32(f)), fy=float(np.float32(f)),
                 cx=float(np.float32(W / 2 if cx is None else cx)), cy=float(np.float32(H / 2 if cy is None else cy)),
                 near=float(np.float32(near)))
    vm = IDENTITY_VIEW if viewmat is None else np.asarray(viewmat, np.float32)
    if poses is None:
        poses = np.zeros((1, n_bodies, 7), np.float32)
        poses[..., 0] = 1.0
    return Batch(cams=[cam], viewmats=vm.reshape(1, 1, 3, 4), poses=np.asarray(poses, np.float32).reshape(1, -1, 7),
                 bg=np.asarray(bg, np.float32))


def quat_axis_angle(axis, angle):
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    return np.concatenate([[math.cos(angle / 2)], math.sin(angle / 2) * axis]).astype(np.float32)


def pixel_centres(W, H):
    ys, xs = np.mgrid[0:H, 0:W]
    return xs + 0.5, ys + 0.5
