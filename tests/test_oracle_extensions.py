"""Pins of the oracle's extensions (CPU): body-attached cameras and the
observation epilogue.  Each check compares against something other than the
oracle's own formula: hand-derived closed forms, an independent camera built
with look-at, brute-force compositing, numpy's IEEE half conversion."""
import math

import numpy as np
import pytest

from oracle import attrs64, brute_ref, observe32, observe64, observe_codes, quantise_u8, render_ref
from oracle.attrs64 import viewmat64
from oracle.spec32 import viewmat32
from paper_2604_25459_amd import synth
from tests.scenes import quat_axis_angle, scene_from


def _attached_batch(pose, offset, W=96, H=72, f=70.0, attach=0, n_bodies=1):
    cam = synth.Camera(width=W, height=H, fx=f, fy=f, cx=W / 2, cy=H / 2, near=0.02, attach_body=attach)
    poses = np.asarray(pose, np.float32).reshape(1, n_bodies, 7)
    return synth.Batch(cams=[cam], viewmats=np.asarray(offset, np.float32).reshape(1, 1, 3, 4), poses=poses)


# ------------------------------------------------------------ attached cameras
def test_attached_viewmat_closed_form():
    """Body turned 90 degrees about +z and moved to (1, 2, 3); identity offset:
    the camera frame is the body frame, so world p -> Rz(-90)(p - t)."""
    q = quat_axis_angle([0, 0, 1], math.pi / 2)
    pose = np.array([[*q, 1.0, 2.0, 3.0]], np.float32)
    ident = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    b = _attached_batch(pose, ident)
    W, w = viewmat64(b, 0, 0)
    Rz_inv = np.array([[0, 1, 0], [-1, 0, 0], [0, 0, 1]], np.float64)     # rotation by -90 degrees about z
    np.testing.assert_allclose(W, Rz_inv, atol=1e-7)
    np.testing.assert_allclose(w, -Rz_inv @ np.array([1.0, 2.0, 3.0]), atol=1e-6)
    R32, t32 = viewmat32(b, 0, 0)
    np.testing.assert_allclose(R32, W, atol=2e-7)
    np.testing.assert_allclose(t32, w, atol=1e-6)


def test_attached_equals_world_camera_from_look_at():
    """A camera riding on a body at a fixed body-frame look-at offset sees the
    scene like a world camera placed with look-at at the transformed eye and
    target (independent construction of the same camera)."""
    rng = np.random.default_rng(3)
    n = 200
    means = rng.uniform(-1.5, 1.5, (n, 3))
    scene = scene_from(means, np.exp(rng.normal(math.log(0.05), 0.4, (n, 3))), rng.standard_normal((n, 4)),
                       1 / (1 + np.exp(-rng.standard_normal(n))),
                       np.concatenate([rng.uniform(0, 1, (n, 1, 3)), rng.normal(0, 0.1, (n, 3, 3))], axis=1),
                       degree=1, body_offsets=[n, n])                   # everything static, one (empty) body
    q = quat_axis_angle([0.2, 0.9, -0.4], 0.7)
    t = np.array([0.3, -0.4, 0.5])
    eye_b, target_b = np.array([0.0, -2.5, 1.0]), np.array([0.1, 0.2, -0.1])
    offset = synth.look_at(eye_b, target_b)                            # body -> camera
    b_att = _attached_batch(np.array([[*q, *t]]), offset)
    from oracle.attrs64 import quat_to_rot64
    R = quat_to_rot64(q.astype(np.float64))
    eye_w, target_w = R @ eye_b + t, R @ target_b + t
    V = synth.look_at(eye_w, target_w)        # world camera at the same eye and target (roll may differ)
    W, w = viewmat64(b_att, 0, 0)
    # both cameras sit at eye_w and look at target_w
    np.testing.assert_allclose(-W.T @ w, eye_w, atol=1e-5)
    np.testing.assert_allclose(W[2], V[2, :3], atol=1e-5)              # same viewing direction
    # and render the same as the world camera with the composed viewmat
    b_world = synth.Batch(cams=[synth.Camera(96, 72, 70.0, 70.0, 48.0, 36.0, 0.02)],
                          viewmats=np.concatenate([W, w[:, None]], axis=1).astype(np.float32).reshape(1, 1, 3, 4),
                          poses=b_att.poses)
    r1 = render_ref(scene, b_att, variants=False)
    r2 = render_ref(scene, b_world, variants=False)
    assert np.abs(r1.rgb - r2.rgb).max() < 5e-4


def test_attached_camera_co_moves_with_its_body():
    """A body-only scene seen by a camera attached to that body does not change
    when the body moves (rigid co-motion): poses far apart give one image."""
    rng = np.random.default_rng(11)
    n = 250
    means = rng.uniform(-0.25, 0.25, (n, 3))
    scene = scene_from(means, np.exp(rng.normal(math.log(0.02), 0.4, (n, 3))), rng.standard_normal((n, 4)),
                       1 / (1 + np.exp(-rng.standard_normal(n))),
                       np.concatenate([rng.uniform(0, 1, (n, 1, 3)), rng.normal(0, 0.2, (n, 8, 3))], axis=1),
                       degree=2, body_offsets=[0, n])
    offset = synth.look_at([0.0, -0.8, 0.3], [0.0, 0.0, 0.0])
    imgs = []
    for ax, ang, t in (([1, 0, 0], 0.0, [0, 0, 0]), ([0.3, -0.5, 0.8], 1.9, [2.0, -1.0, 0.5]),
                       ([0, 1, 0], -2.4, [-3.0, 0.5, 4.0])):
        b = _attached_batch(np.array([[*quat_axis_angle(ax, ang), *t]]), offset)
        imgs.append(render_ref(scene, b, variants=False).rgb)
    for im in imgs[1:]:
        assert np.abs(im - imgs[0]).max() < 5e-4


def test_attached_camera_tiled_equals_brute_force():
    rng = np.random.default_rng(21)
    n = 60
    means = rng.uniform(-1.0, 1.0, (n, 3))
    scene = scene_from(means, np.exp(rng.normal(math.log(0.05), 0.5, (n, 3))), rng.standard_normal((n, 4)),
                       1 / (1 + np.exp(-rng.standard_normal(n))),
                       np.concatenate([rng.uniform(0, 1, (n, 1, 3)), rng.normal(0, 0.1, (n, 3, 3))], axis=1),
                       degree=1, body_offsets=[30, 60])
    pose = np.array([[*quat_axis_angle([0.1, 0.4, 0.9], 0.8), 0.2, -0.1, 0.3]])
    b = _attached_batch(pose, synth.look_at([0.2, -2.2, 0.8], [0.0, 0.0, 0.0]), W=64, H=48, f=45.0)
    ref = render_ref(scene, b, variants=False)
    rgb, depth, alpha = brute_ref(scene, b)
    np.testing.assert_allclose(ref.rgb, rgb, atol=1e-12)
    np.testing.assert_allclose(ref.depth, depth, atol=1e-12)


# ------------------------------------------------------------ observation epilogue
def test_observe_identity_codes():
    k = np.arange(256)
    x = (k / 255.0).astype(np.float32)
    np.testing.assert_array_equal(quantise_u8(observe32(x)), k)
    lo, hi = observe_codes(k / 255.0)
    np.testing.assert_array_equal(lo, k)                 # exact code centres are never flagged
    np.testing.assert_array_equal(hi, k)


def test_observe_worked_example_and_clamp():
    # one stop of exposure, contrast 1.5 about mid-grey, brightness -0.1:
    # 0.3 -> 0.6 -> 0.65 -> 0.55 -> code floor(140.25 + 0.5) = 140
    assert observe64(0.3, 2.0, 1.5, -0.1) == pytest.approx(0.55, abs=1e-15)
    assert int(quantise_u8(observe32(0.3, 2.0, 1.5, -0.1))) == 140
    assert observe64(2.0) == 1.0 and observe64(0.2, 1.0, 1.0, -0.5) == 0.0
    np.testing.assert_array_equal(quantise_u8(observe32([2.0, -1.0, 0.5])), [255, 0, 128])
    # zero contrast: every colour becomes mid-grey plus brightness
    np.testing.assert_allclose(observe64(np.linspace(0, 1, 7), 1.3, 0.0, 0.1), 0.6, atol=1e-15)


def test_observe32_close_to_float64_and_half_rounding():
    rng = np.random.default_rng(5)
    rgb = rng.uniform(0, 1.2, (1000, 3))
    g, c, b = 1.4, 0.7, 0.05
    np.testing.assert_allclose(observe32(rgb, g, c, b), observe64(rgb, g, c, b), atol=3e-7)
    # halves: numpy's IEEE conversion (round to nearest, ties to even) of the binary32 value
    x32 = observe32(rgb, g, c, b)
    lo, hi = observe_codes(rgb, g, c, b, fmt="f16", tol=0.0)
    np.testing.assert_array_equal(lo, x32.astype(np.float16).astype(np.float64))
    np.testing.assert_array_equal(hi, lo)
    # ties to even at a half boundary: 1 + 2^-11 lies between 1 and 1 + 2^-10
    assert np.float32(1.0 + 2.0 ** -11).astype(np.float16) == np.float16(1.0)


def test_observe_codes_flags_only_near_boundaries():
    rng = np.random.default_rng(8)
    rgb = rng.uniform(0, 1, (20000, 3))
    lo, hi = observe_codes(rgb, 1.1, 1.2, -0.02, tol=1e-4)
    assert np.all(hi - lo <= 1)
    frac = np.mean(hi != lo)
    # a channel is flagged only within 1e-4 * gain * contrast * 255 codes of a boundary
    assert 0.0 < frac < 0.2


# ------------------------------------------------------------ opacity-aware extent
def test_qmax_table_is_the_rounded_up_bound():
    from oracle.spec32 import QMAX
    for k in range(8):
        x = 1.01 * 2.0 * math.log(255.0 * 2.0 ** -k)
        assert float(QMAX[k]) >= x                                        # a bound ...
        assert float(np.nextafter(QMAX[k], np.float32(0))) < x            # ... and the nearest one


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tight_extent_tiled_equals_brute_force(seed):
    """Needles and discs at every opacity bucket edge (o = 2^-k and just
    above), seen at an angle: the tighter tile rectangles still hold every
    pixel a Gaussian reaches with alpha >= 1/255, so tiled compositing equals
    the brute-force definition."""
    from tests.scenes import one_camera
    rng = np.random.default_rng(100 + seed)
    ops = []
    for k in range(8):
        ops += [2.0 ** -k, min(1.0, 2.0 ** -k * 1.0001)]
    n = len(ops) * 3
    op = np.array(ops * 3, np.float64)
    op = np.clip(op, 1.0 / 255.0, 0.999)
    means = rng.uniform([-1.2, -0.9, 1.5], [1.2, 0.9, 3.0], (n, 3))
    scales = np.exp(rng.normal(math.log(0.06), 0.9, (n, 3)))          # strongly anisotropic
    q = rng.standard_normal((n, 4))
    sh = rng.uniform(0, 1, (n, 1, 3))
    scene = scene_from(means, scales, q, op, sh, degree=0)
    batch = one_camera(80, 60, 50.0, bg=(0.2, 0.3, 0.4))
    ref = render_ref(scene, batch, ts=8, variants=False)
    rgb, depth, alpha = brute_ref(scene, batch)
    np.testing.assert_allclose(ref.rgb, rgb, atol=1e-12)
    np.testing.assert_allclose(ref.alpha, alpha, atol=1e-12)


def test_tight_extent_never_wider_than_radius_square():
    from oracle.spec32 import project32
    scene, batch = synth.make_config(1, n_envs=1)
    p = project32(scene, batch, 0, 0)
    vis = p["visible"]
    u, v, r = p["u"][vis], p["v"][vis], p["radius"][vis]
    ts = np.float32(16)
    TX, TY = p["tiles_x"], p["tiles_y"]
    sq = np.stack([np.clip(np.floor((u - r) / ts), 0, TX), np.clip(np.floor((u + r) / ts) + 1, 0, TX),
                   np.clip(np.floor((v - r) / ts), 0, TY), np.clip(np.floor((v + r) / ts) + 1, 0, TY)], axis=1)
    rect = p["rect"][vis]
    assert np.all(rect[:, 0] >= sq[:, 0]) and np.all(rect[:, 1] <= sq[:, 1])
    assert np.all(rect[:, 2] >= sq[:, 2]) and np.all(rect[:, 3] <= sq[:, 3])
    sq_count = ((sq[:, 1] - sq[:, 0]) * (sq[:, 3] - sq[:, 2])).sum()
    assert p["count"].sum() < 0.9 * sq_count
