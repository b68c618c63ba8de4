"""Binning reference under an IEEE binary32 specification (test infrastructure).

The discrete outputs of the renderer -- which Gaussians are culled, the depth
bits in each 64-bit sort key, the tile rectangle of every splat and therefore
every tile list -- must be reproducible bit for bit on the GPU.  They are
defined here with numpy float32 arithmetic: every +, -, *, /, sqrt is rounded
separately to nearest-even, sums run left to right, no operation is fused,
division and square root are correctly rounded, denormals are kept, and every
constant is a float32 literal.

Steps follow standard 3DGS projection (Kerbl et al. 2023, cited by the paper as
its rendering representation; EWA splatting with a local affine Jacobian and a
0.3 px^2 low-pass dilation) and the paper's rigid-link posing (RLGK, Sec.
"Batch Renderer Optimization"): each Gaussian cluster moves with its rigid body.
Constants fixed by the target specification of this renderer: alpha threshold
1/255, 16x16 tiles by default, a 64-bit (image/tile, depth) key.

Readings where the paper is silent (also listed in the design notes):
* quaternions (w, x, y, z) are normalised before use;
* the Jacobian uses the camera-space mean with x/z and y/z clamped to 1.3 times
  the half field of view; the projected mean is not clamped;
* conservative radius r = ceil(3.33 * sqrt(lambda_max)); 3.33 >= sqrt(2 ln 255)
  so no pixel outside the square can reach alpha >= 1/255;
* the tile rectangle uses the tighter of that square and the axis-aligned box
  of the opacity-aware ellipse q <= 2 ln(255 o) (bounded per opacity bucket,
  QMAX below), which is still conservative;
* the determinant uses the Lagrange identity (no cancellation).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict

import numpy as np

F = np.float32
ONE, TWO, HALF = F(1.0), F(2.0), F(0.5)
DILATE = F(0.3)
DILATE_SQ = F(0.09)
EIG_FLOOR = F(0.1)
GUARD = F(1.3)
ALPHA_MIN = F(1.0) / F(255.0)

# Opacity-aware splat extent.  alpha >= 1/255 needs q <= 2 ln(255 o), q the
# Mahalanobis form of the dilated 2D covariance.  Opacities fall in buckets
# (2^-(k+1), 2^-k], k = 0..7 (k = 8 and beyond are culled by o >= 1/255), and
# QMAX[k] is 1.01 * 2 ln(255 * 2^-k) rounded up to binary32: a bound for the
# whole bucket with 1 % to spare for binary32 rounding of the extents below.
QMAX = np.array([float.fromhex(h) for h in (
    "0x1.662ff2p+3", "0x1.3961dcp+3", "0x1.0c93c4p+3", "0x1.bf8b5cp+2",
    "0x1.65ef2ep+2", "0x1.0c5300p+2", "0x1.656da6p+1", "0x1.646a94p+0")], F)


def quat_to_rot32(q: np.ndarray) -> np.ndarray:
    """Unit-quaternion rotation matrix from (w, x, y, z), float32 spec."""
    q = np.asarray(q, dtype=F)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    n = np.sqrt(((w * w + x * x) + y * y) + z * z)
    w, x, y, z = w / n, x / n, y / n, z / n
    xx, yy, zz = x * x, y * y, z * z
    xy, xz, yz = x * y, x * z, y * z
    wx, wy, wz = w * x, w * y, w * z
    R = np.empty(q.shape[:-1] + (3, 3), dtype=F)
    R[..., 0, 0] = ONE - TWO * (yy + zz)
    R[..., 0, 1] = TWO * (xy - wz)
    R[..., 0, 2] = TWO * (xz + wy)
    R[..., 1, 0] = TWO * (xy + wz)
    R[..., 1, 1] = ONE - TWO * (xx + zz)
    R[..., 1, 2] = TWO * (yz - wx)
    R[..., 2, 0] = TWO * (xz - wy)
    R[..., 2, 1] = TWO * (yz + wx)
    R[..., 2, 2] = ONE - TWO * (xx + yy)
    return R


def matmul32(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """(AB)_ij = (A_i0 B_0j + A_i1 B_1j) + A_i2 B_2j, rounded per operation."""
    A = np.asarray(A, F)
    B = np.asarray(B, F)
    shape = np.broadcast_shapes(A.shape, B.shape)
    out = np.empty(shape, F)
    for i in range(3):
        for j in range(3):
            out[..., i, j] = (A[..., i, 0] * B[..., 0, j] + A[..., i, 1] * B[..., 1, j]) + A[..., i, 2] * B[..., 2, j]
    return out


def affine32(A: np.ndarray, x: np.ndarray, a: np.ndarray) -> np.ndarray:
    """A x + a with ((A_i0 x0 + A_i1 x1) + A_i2 x2) + a_i per component."""
    A = np.asarray(A, F)
    x = np.asarray(x, F)
    a = np.asarray(a, F)
    comps = [((A[..., i, 0] * x[..., 0] + A[..., i, 1] * x[..., 1]) + A[..., i, 2] * x[..., 2]) + a[..., i]
             for i in range(3)]
    return np.stack(comps, axis=-1).astype(F)


def image_tiles(width: int, height: int, ts: int):
    return (width + ts - 1) // ts, (height + ts - 1) // ts


def tile_bases(batch, ts: int) -> np.ndarray:
    """First global tile id of every image, images in camera-slot-major order."""
    counts = []
    for c, cam in enumerate(batch.cams):
        tx, ty = image_tiles(cam.width, cam.height, ts)
        counts += [tx * ty] * batch.n_envs
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def viewmat32(batch, c: int, e: int):
    """World->camera (R_c, t_c) of image (c, e) in the float32 spec.  A camera
    slot attached to body k carries body->camera offsets [R_o | t_o] instead;
    then R_c = R_o R(q_k)^T (matmul32 with the transposed body rotation) and
    t_c = t_o - R_c t_k, the product summed left to right before the one
    subtraction (the camera rides rigidly on the body: its world pose is the
    body's pose followed by the offset)."""
    vm = np.asarray(batch.viewmats[c, e], F)
    Ro, to = vm[:, :3], vm[:, 3]
    k = int(getattr(batch.cams[c], "attach_body", -1))
    if k < 0:
        return Ro, to
    pose = np.asarray(batch.poses[e, k], F)
    Rk = quat_to_rot32(pose[0:4])
    Rc = matmul32(Ro, np.ascontiguousarray(Rk.T))
    tk = pose[4:7]
    Rt = np.array([(Rc[i, 0] * tk[0] + Rc[i, 1] * tk[1]) + Rc[i, 2] * tk[2] for i in range(3)], F)
    return Rc, (to - Rt).astype(F)


def compose32(batch, scene, c: int, e: int):
    """Per-body camera-from-body transforms (A, a) for image (c, e); slot 0 is
    the static background (A = R_c, a = t_c), slot b+1 is body b:
    A = R_c R(q_b), a = R_c t_b + t_c."""
    Rc, tc = viewmat32(batch, c, e)
    B = scene.n_bodies
    As = np.empty((B + 1, 3, 3), F)
    as_ = np.empty((B + 1, 3), F)
    As[0], as_[0] = Rc, tc
    if B:
        pose = np.asarray(batch.poses[e], F)
        Rb = quat_to_rot32(pose[:, 0:4])
        As[1:] = matmul32(Rc[None], Rb)
        as_[1:] = affine32(Rc[None], pose[:, 4:7], tc[None])
    return As, as_


@dataclass
class Bins:
    """Binning of one image.  Arrays over Gaussians have length N (scene
    storage order = Gaussian index g); pair arrays are sorted by (key, g)."""
    visible: np.ndarray   # (N,) bool
    zbits: np.ndarray     # (N,) uint32, bit pattern of camera-space z (float32)
    rect: np.ndarray      # (N, 4) int64: x0, x1, y0, y1 (tiles, half-open)
    count: np.ndarray     # (N,) int64, tiles touched (0 if culled)
    u: np.ndarray         # (N,) float32 projected mean x (pixels)
    v: np.ndarray
    conic: np.ndarray     # (N, 3) float32 (c/det, -b/det, a/det)
    radius: np.ndarray    # (N,) float32 integer-valued
    tz: np.ndarray        # (N,) float32
    keys: np.ndarray      # (P,) uint64 sorted ascending
    values: np.ndarray    # (P,) uint32 Gaussian index g
    ranges: np.ndarray    # (T, 2) int64 [start, end) into keys/values, per local tile
    tile_base: int
    tiles_x: int
    tiles_y: int
    cov: np.ndarray       # (N, 3) float32 (a, b, c) of the dilated 2D covariance
    det: np.ndarray       # (N,) float32


def project32(scene, batch, c: int, e: int, ts: int = 16, cutoff: float = 3.33,
              attrs: Dict[str, np.ndarray] | None = None):
    """Float32-spec projection of every Gaussian of ``scene`` into image (c, e).
    ``attrs`` optionally overrides the stored attributes (e.g. decoded
    half-precision ones); keys: means, scales, quats, opacities."""
    cam = batch.cams[c]
    at = attrs or {}
    means = np.asarray(at.get("means", scene.means), F)
    scales = np.asarray(at.get("scales", scene.scales), F)
    quats = np.asarray(at.get("quats", scene.quats), F)
    opac = np.asarray(at.get("opacities", scene.opacities), F)
    N = means.shape[0]
    As, as_ = compose32(batch, scene, c, e)
    slot = scene.body_of() + 1
    A = As[slot]
    a = as_[slot]
    with np.errstate(all="ignore"):
        t = affine32(A, means, a)
        tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
        Rg = quat_to_rot32(quats)
        M = matmul32(A, Rg)
        M = M * scales[:, None, :]          # M_ij <- M_ij * s_j (one rounding each)
        fx, fy, cx, cy = F(cam.fx), F(cam.fy), F(cam.cx), F(cam.cy)
        W, H = F(cam.width), F(cam.height)
        lx = GUARD * ((HALF * W) / fx)
        ly = GUARD * ((HALF * H) / fy)
        itz = ONE / tz                      # the one division by depth; products below
        itz2 = itz * itz
        xcl = np.minimum(lx, np.maximum(-lx, tx * itz)) * tz
        ycl = np.minimum(ly, np.maximum(-ly, ty * itz)) * tz
        j00 = fx * itz
        j02 = -((fx * xcl) * itz2)
        j11 = fy * itz
        j12 = -((fy * ycl) * itz2)
        v1 = np.stack([j00 * M[:, 0, k] + j02 * M[:, 2, k] for k in range(3)], axis=1)
        v2 = np.stack([j11 * M[:, 1, k] + j12 * M[:, 2, k] for k in range(3)], axis=1)
        n1 = (v1[:, 0] * v1[:, 0] + v1[:, 1] * v1[:, 1]) + v1[:, 2] * v1[:, 2]
        n2 = (v2[:, 0] * v2[:, 0] + v2[:, 1] * v2[:, 1]) + v2[:, 2] * v2[:, 2]
        ca = n1 + DILATE
        cc = n2 + DILATE
        cb = (v1[:, 0] * v2[:, 0] + v1[:, 1] * v2[:, 1]) + v1[:, 2] * v2[:, 2]
        w0 = v1[:, 1] * v2[:, 2] - v1[:, 2] * v2[:, 1]
        w1 = v1[:, 2] * v2[:, 0] - v1[:, 0] * v2[:, 2]
        w2 = v1[:, 0] * v2[:, 1] - v1[:, 1] * v2[:, 0]
        det = (((w0 * w0 + w1 * w1) + w2 * w2) + DILATE * (n1 + n2)) + DILATE_SQ
        m = HALF * (ca + cc)
        h = HALF * (ca - cc)
        lam = m + np.sqrt(np.maximum(EIG_FLOOR, h * h + cb * cb))
        r = np.ceil(F(cutoff) * np.sqrt(lam))
        u = (fx * tx) * itz + cx
        v = (fy * ty) * itz + cy
        # axis-aligned half-extents of the ellipse q <= QMAX[bucket of o]
        # (sqrt(Q Sigma_xx), sqrt(Q Sigma_yy)), never beyond the radius
        k = np.zeros(N, np.int64)
        for j in range(1, 8):
            k += (opac <= F(2.0 ** -j)).astype(np.int64)
        Q = QMAX[k]
        rx = np.minimum(r, np.sqrt(Q * ca))
        ry = np.minimum(r, np.sqrt(Q * cc))
        tsf = F(ts)
        TX, TY = image_tiles(cam.width, cam.height, ts)
        x0 = np.clip(np.floor((u - rx) / tsf), F(0), F(TX))
        x1 = np.clip(np.floor((u + rx) / tsf) + ONE, F(0), F(TX))
        y0 = np.clip(np.floor((v - ry) / tsf), F(0), F(TY))
        y1 = np.clip(np.floor((v + ry) / tsf) + ONE, F(0), F(TY))
        finite_t = np.isfinite(tx) & np.isfinite(ty) & np.isfinite(tz)
        vis = finite_t & (tz > F(cam.near)) & (opac >= ALPHA_MIN) & np.isfinite(det) & (det > F(0))
        vis &= np.isfinite(r) & np.isfinite(u) & np.isfinite(v)
        x0i = np.where(vis, x0, 0).astype(np.int64)
        x1i = np.where(vis, x1, 0).astype(np.int64)
        y0i = np.where(vis, y0, 0).astype(np.int64)
        y1i = np.where(vis, y1, 0).astype(np.int64)
        vis &= (x1i > x0i) & (y1i > y0i)
        conic = np.stack([cc / det, -cb / det, ca / det], axis=1).astype(F)
    count = np.where(vis, (x1i - x0i) * (y1i - y0i), 0)
    rect = np.stack([x0i, x1i, y0i, y1i], axis=1)
    rect[~vis] = 0
    return dict(visible=vis, zbits=tz.view(np.uint32).copy(), rect=rect, count=count,
                u=u.astype(F), v=v.astype(F), conic=conic, radius=r.astype(F), tz=tz.astype(F),
                cov=np.stack([ca, cb, cc], axis=1).astype(F), det=det.astype(F),
                tiles_x=TX, tiles_y=TY, n=N)


def bin_ref(scene, batch, c: int = 0, e: int = 0, ts: int = 16, cutoff: float = 3.33,
            attrs: Dict[str, np.ndarray] | None = None) -> Bins:
    """Keys, values and tile ranges of image (c, e) of ``batch``.

    Every visible Gaussian g emits one pair per touched tile, tiles in
    row-major order (ty outer); key = (global_tile << 32) | float32 bits of its
    camera-space depth; pairs are then sorted stably by key, so equal depth
    bits keep ascending g.  Global tile ids start at the image's tile base
    (images in camera-slot-major order, i = c * E + e)."""
    p = project32(scene, batch, c, e, ts, cutoff, attrs)
    TX, TY = p["tiles_x"], p["tiles_y"]
    base = int(tile_bases(batch, ts)[batch.image_index(c, e)])
    vis_idx = np.nonzero(p["visible"])[0]
    cnt = p["count"][vis_idx]
    g = np.repeat(vis_idx, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    s = np.arange(g.shape[0], dtype=np.int64) - start
    rect = p["rect"][g]
    nx = rect[:, 1] - rect[:, 0]
    tyy = rect[:, 2] + s // np.maximum(nx, 1)
    txx = rect[:, 0] + s % np.maximum(nx, 1)
    local = tyy * TX + txx
    keys = ((local + base).astype(np.uint64) << np.uint64(32)) | p["zbits"][g].astype(np.uint64)
    order = np.argsort(keys, kind="stable")
    keys = keys[order]
    values = g[order].astype(np.uint32)
    local_sorted = local[order]
    T = TX * TY
    cnt_t = np.bincount(local_sorted, minlength=T) if local_sorted.size else np.zeros(T, np.int64)
    ends = np.cumsum(cnt_t)
    ranges = np.stack([ends - cnt_t, ends], axis=1).astype(np.int64)
    return Bins(visible=p["visible"], zbits=p["zbits"], rect=p["rect"], count=p["count"],
                u=p["u"], v=p["v"], conic=p["conic"], radius=p["radius"], tz=p["tz"],
                keys=keys, values=values, ranges=ranges, tile_base=base, tiles_x=TX, tiles_y=TY,
                cov=p["cov"], det=p["det"])
