"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact: cull set, depth-key bits, tile rectangles, sort keys, tile lists
and ranges (float32 binning specification).  Within tolerance: pixels
(max-abs 1e-3 RGB, 1e-3 relative depth beyond 1 m) against the float64
oracle, where a pixel may match any admissible result of a threshold decision
taken within rounding distance of its boundary."""
import math

import numpy as np
import pytest

from oracle import attrs64, bin_ref, render_ref
from oracle.spec32 import project32
from oracle.storage import decoded_attrs
from paper_2604_25459_amd import synth
from tests.parity import compare, psnr
from tests.scenes import one_camera, scene_from

pytestmark = pytest.mark.gpu

LOG2E = 1.4426950408889634


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def R():
    _torch()
    from paper_2604_25459_amd import gsr
    r = gsr.Renderer(0)
    yield r
    r.close()


def _upload(R, scene, storage="f32"):
    return R.add_synth_scene(scene, storage)


def _render(R, sid, batch, plain=False):
    from paper_2604_25459_amd import gsr
    cams, vm, poses = gsr.batch_tensors(batch)
    return R.render(sid, cams, vm, poses, bg=tuple(batch.bg), alpha=True, plain=plain)


def _img(got, c, e):
    """Image (c, e) of a render result as numpy (rgb, depth, alpha)."""
    r, d, a = got[c]
    return r[e].cpu().numpy(), d[e].cpu().numpy(), a[e].cpu().numpy()


def _same(x, y):
    import torch
    assert torch.equal(x, y)


def _check_bins(R, sid, scene, batch, c, e, attrs=None):
    """Keys, ids and ranges of image (c, e) as the render path builds them (its
    tuned parameters, chunks, graphs and streams) against the specification."""
    from paper_2604_25459_amd import gsr
    cams, vm, poses = gsr.batch_tensors(batch)
    image = batch.image_index(c, e)
    got = R.debug_bins(sid, cams, vm, poses, image)
    ref = bin_ref(scene, batch, c, e, got["tile_size"], attrs=attrs)
    assert got["n_visible"] == int(ref.visible.sum())
    assert got["tile_base"] == ref.tile_base
    np.testing.assert_array_equal(got["keys"], ref.keys)
    np.testing.assert_array_equal(got["values"], ref.values)
    np.testing.assert_array_equal(got["ranges"], ref.ranges)
    return ref


def _check_image(got, ref, label, rgb_tol=1e-3):
    """RGB, depth and alpha of every pixel against the oracle: the primary
    result, or for a pixel with flagged threshold decisions one of its
    admissible variants (all of them enumerated; rgb, depth and alpha from the
    same variant)."""
    rgb, depth, alpha = got
    res = compare(rgb, depth, ref, gpu_alpha=alpha, rgb_tol=rgb_tol)
    print(f"[{label}] {res}", flush=True)
    assert res["ok"], (label, res)
    return res


# ------------------------------------------------------------------ projection
def test_project_cfg0_matches_spec(R):
    scene, batch = synth.make_config(0)
    sid = _upload(R, scene)
    from paper_2604_25459_amd import gsr
    cams, vm, poses = gsr.batch_tensors(batch)
    got = R.debug_project(sid, cams, vm, poses, 0, scene.n)
    p = project32(scene, batch, 0, 0, R.tile_size)
    vis = p["visible"]
    np.testing.assert_array_equal(got["zkey"] != 0xFFFFFFFF, vis)
    np.testing.assert_array_equal(got["zkey"][vis], p["zbits"][vis])
    np.testing.assert_array_equal(got["rect"][vis], p["rect"][vis])
    rec = got["rec"][vis]
    # u, v and the radius follow the binary32 specification exactly
    np.testing.assert_array_equal(rec[:, 0], p["u"][vis])
    np.testing.assert_array_equal(rec[:, 1], p["v"][vis])
    np.testing.assert_array_equal(rec[:, 7], p["radius"][vis])
    np.testing.assert_array_equal(rec[:, 6].view(np.uint32), p["zbits"][vis])
    # whitened conic: 0.5 log2(e) q(dx, dy) = (a1 dx + b1 dy)^2 + (c1 dy)^2, from the
    # specification's dilated covariance (a, b, c) and determinant
    cov = p["cov"][vis].astype(np.float64)
    det = p["det"][vis].astype(np.float64)
    k = 0.5 * LOG2E
    a1 = np.sqrt(k * cov[:, 2] / det)
    np.testing.assert_allclose(rec[:, 2], a1, rtol=4e-6)
    np.testing.assert_allclose(rec[:, 3], -k * cov[:, 1] / (det * a1), rtol=4e-6, atol=1e-9)
    np.testing.assert_allclose(rec[:, 4], np.sqrt(k / cov[:, 2]), rtol=4e-6)
    # the factors reproduce the conic of the specification
    con = p["conic"][vis].astype(np.float64)
    r64 = rec.astype(np.float64)
    np.testing.assert_allclose(r64[:, 2] ** 2, k * con[:, 0], rtol=2e-5)
    np.testing.assert_allclose(2 * r64[:, 2] * r64[:, 3], 2 * k * con[:, 1], rtol=2e-5, atol=1e-9)
    np.testing.assert_allclose(r64[:, 3] ** 2 + r64[:, 4] ** 2, k * con[:, 2], rtol=2e-5)
    at = attrs64(scene, batch)
    np.testing.assert_allclose(rec[:, 8:11], at["rgb"][vis], atol=2e-6)
    np.testing.assert_allclose(rec[:, 5], np.log2(scene.opacities[vis].astype(np.float64)), atol=2e-6)
    R.remove_scene(sid)


# ------------------------------------------------------------------ config 0
def test_cfg0_bins_and_pixels(R):
    scene, batch = synth.make_config(0)
    sid = _upload(R, scene)
    _check_bins(R, sid, scene, batch, 0, 0)
    got = _render(R, sid, batch)
    ref = render_ref(scene, batch, 0, 0, R.tile_size)
    _check_image(_img(got, 0, 0), ref, "cfg0")
    # the plain per-image path gives the same bits
    plain = _render(R, sid, batch, plain=True)
    _same(plain[0][0], got[0][0])
    _same(plain[0][1], got[0][1])
    R.remove_scene(sid)


def test_work_counts_match_oracle(R):
    """Per-pixel list entries visited up to termination equal the oracle's count
    (pixels whose decisions are within rounding of a threshold excepted)."""
    import torch
    from paper_2604_25459_amd import gsr
    for cfg, e in ((0, 0), (1, 5)):
        scene, batch = synth.make_config(cfg, n_envs=e + 1)
        sid = _upload(R, scene)
        cams, vm, poses = gsr.batch_tensors(batch)
        rgb, depth, _ = R.alloc_outputs(cams, batch.n_envs)
        work = torch.zeros(rgb.numel() // 3 * 2, dtype=torch.int32, device=rgb.device)
        R.render_into(sid, cams, vm, poses, rgb, depth, work=work)
        cam = batch.cams[0]
        npx = cam.width * cam.height
        w = work.view(-1, 2)[e * npx:(e + 1) * npx].cpu().numpy().reshape(cam.height, cam.width, 2)
        ref = render_ref(scene, batch, 0, e, R.tile_size, variants=False)
        ok = ref.nflag == 0
        np.testing.assert_array_equal(w[..., 0][ok], ref.visited[ok])
        assert (w[..., 1] <= w[..., 0]).all()
        plain = R.render(sid, cams, vm, poses)          # counting changes no pixel
        assert torch.equal(plain[0][0].reshape(-1), rgb)
        R.remove_scene(sid)


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.2, 0.3, 0.4)])
def test_ragged_100x75_random_scene(R, bg):
    rng = np.random.default_rng(3)
    n = 3000
    means = rng.uniform([-1.2, -0.9, 1.0], [1.2, 0.9, 4.0], (n, 3))
    scales = np.exp(rng.normal(math.log(0.04), 0.6, (n, 3)))
    sh = np.concatenate([rng.uniform(0, 1, (n, 1, 3)), rng.normal(0, 0.1, (n, 15, 3))], axis=1)
    scene = scene_from(means, scales, rng.standard_normal((n, 4)), 1 / (1 + np.exp(-rng.standard_normal(n))), sh, 3)
    batch = one_camera(100, 75, 70.0, bg=bg)
    sid = _upload(R, scene)
    _check_bins(R, sid, scene, batch, 0, 0)
    got = _render(R, sid, batch)
    ref = render_ref(scene, batch, 0, 0, R.tile_size)
    _check_image(_img(got, 0, 0), ref, f"ragged bg={bg}")
    R.remove_scene(sid)


def test_full_survivor_batches_and_opaque_splats(R):
    """Every wave's batches of 64 candidates survive whole (wide, faint
    splats: survivor packs of 64, the last pair at the end of the slots), with
    near-opaque splats (opacity >= 0.99: the 0.99 clamp) in between that stop
    pixels; bins bit for bit, pixels against the oracle, at several LDS batch
    sizes."""
    rng = np.random.default_rng(17)
    n_faint, n_opaque = 300, 40
    means = np.concatenate([rng.uniform([-0.3, -0.2, 1.0], [0.3, 0.2, 3.0], (n_faint, 3)),
                            rng.uniform([-0.5, -0.35, 1.0], [0.5, 0.35, 3.0], (n_opaque, 3))])
    scales = np.concatenate([np.full((n_faint, 3), 0.6), np.exp(rng.normal(math.log(0.03), 0.3, (n_opaque, 3)))])
    opac = np.concatenate([rng.uniform(0.01, 0.03, n_faint), rng.choice([0.991, 0.995, 0.999, 1.0], n_opaque)])
    order = rng.permutation(n_faint + n_opaque)          # opaque splats interleaved in index order
    sh = rng.uniform(0, 1, (n_faint + n_opaque, 1, 3))
    scene = scene_from(means[order], scales[order], rng.standard_normal((n_faint + n_opaque, 4)), opac[order],
                       sh, 0)
    batch = one_camera(72, 56, 60.0, bg=(0.2, 0.3, 0.4))
    sid = _upload(R, scene)
    _check_bins(R, sid, scene, batch, 0, 0)
    ref = render_ref(scene, batch, 0, 0, R.tile_size)
    from paper_2604_25459_amd import gsr
    cams, vm, poses = gsr.batch_tensors(batch)
    for lds_batch in (64, 128, 256):
        R.set_tuning(sid, cams, vm, poses, lds_batch=lds_batch)
        got = _render(R, sid, batch)
        _check_image(_img(got, 0, 0), ref, f"full batches + opaque, lds_batch {lds_batch}")
    R.remove_scene(sid)


# ------------------------------------------------------------------ batched configs (sampled envs)
def test_cfg1_all_envs_batched(R):
    scene, batch = synth.make_config(1)
    sid = _upload(R, scene)
    got = _render(R, sid, batch)
    for e in (0, 17, 63):
        _check_bins(R, sid, scene, batch, 0, e)
        ref = render_ref(scene, batch, 0, e, R.tile_size)
        _check_image(_img(got, 0, e), ref, f"cfg1 env {e}")
    R.remove_scene(sid)


def test_cfg1_batch_independence_and_plain(R):
    scene, batch = synth.make_config(1, n_envs=8)
    sid = _upload(R, scene)
    full = _render(R, sid, batch)[0]
    plain = _render(R, sid, batch, plain=True)[0]
    _same(full[0], plain[0])
    _same(full[1], plain[1])
    alone = _render(R, sid, batch.subset([5]))[0]
    _same(alone[0][0], full[0][5])
    _same(alone[1][0], full[1][5])
    again = _render(R, sid, batch)[0]
    _same(again[0], full[0])      # deterministic
    _same(again[1], full[1])
    R.remove_scene(sid)


def test_cfg2_full_batch_sampled(R):
    """The benchmark's launch configuration: the autotuner's parameters (as the
    benchmark runs them), two 1024-image chunks from the 48 GiB working budget,
    the second chunk on the second stream, captured graphs; bins read from
    inside each sampled image's chunk, envs from both chunks."""
    scene, batch = synth.make_config(2)
    sid = _upload(R, scene)
    from paper_2604_25459_amd import gsr
    cams, vm, poses = gsr.batch_tensors(batch)
    rgb, depth, _ = R.alloc_outputs(cams, batch.n_envs)
    tuning = R.autotune(sid, cams, vm, poses, rgb, depth)
    print(f"[cfg2] autotuned {tuning}", flush=True)
    del rgb, depth
    got = _render(R, sid, batch)
    assert tuple(got[0][0].shape) == (2048, 480, 640, 3)
    for e in (0, 700, 1337, 2047):
        _check_bins(R, sid, scene, batch, 0, e)
        ref = render_ref(scene, batch, 0, e, R.tile_size)
        _check_image(_img(got, 0, e), ref, f"cfg2 env {e}")
    # the same render at 16 images per projection thread, the value the tuner picks on this workload
    R.set_tuning(sid, cams, vm, poses, images_per_thread=16)
    again = _render(R, sid, batch)
    _same(again[0][0], got[0][0])
    _same(again[0][1], got[0][1])
    _check_bins(R, sid, scene, batch, 0, 1337)
    R.remove_scene(sid)


def test_equal_depth_ties_follow_storage_order(R):
    """Two overlapping Gaussians at one depth (identical binary32 depth bits):
    composited in index order; swapping their storage slots swaps which one is
    in front, in the keys, the lists and the pixels."""
    W, H, f = 64, 48, 40.0
    sh = np.zeros((2, 1, 3), np.float32)
    sh[0, 0] = [1.0, -1.0, 0.0]
    sh[1, 0] = [-1.0, 1.0, 0.5]
    means = [[0.01, 0.0, 2.0], [-0.01, 0.0, 2.0]]
    s1 = scene_from(means, [0.1] * 3, opac=[0.6, 0.6], sh=sh, degree=0)
    s2 = scene_from(means[::-1], [0.1] * 3, opac=[0.6, 0.6], sh=sh[::-1].copy(), degree=0)
    batch = one_camera(W, H, f, bg=(0.2, 0.3, 0.4))
    imgs = []
    for sc in (s1, s2):
        b = bin_ref(sc, batch)
        assert b.zbits[0] == b.zbits[1]
        sid = _upload(R, sc)
        _check_bins(R, sid, sc, batch, 0, 0)
        got = _img(_render(R, sid, batch), 0, 0)
        _check_image(got, render_ref(sc, batch, 0, 0, R.tile_size), "equal depth")
        imgs.append(got[0])
        R.remove_scene(sid)
    # slot 0 is in front in both: the swap changes the pixels where the splats overlap
    assert np.abs(imgs[0] - imgs[1]).max() > 0.05


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_half_storage_cfg1(R, storage):
    scene, batch = synth.make_config(1, n_envs=4)
    sid = _upload(R, scene, storage)
    at = decoded_attrs(scene, storage)
    got = _render(R, sid, batch)
    for e in (0, 3):
        _check_bins(R, sid, scene, batch, 0, e, attrs=at)
        ref = render_ref(scene, batch, 0, e, R.tile_size, attrs=at)
        img = _img(got, 0, e)
        _check_image(img, ref, f"cfg1 {storage} env {e} (decoded attributes)")
        full = render_ref(scene, batch, 0, e, R.tile_size, variants=False)
        print(f"[cfg1 {storage} env {e} vs float32 attributes] max-abs {np.abs(img[0] - full.rgb).max():.4g} "
              f"mean-abs {np.abs(img[0] - full.rgb).mean():.4g} PSNR {psnr(img[0], full.rgb):.2f} dB", flush=True)
    R.remove_scene(sid)


def test_scene_replaced_in_one_context(R):
    """A scene destroyed and replaced by one of the same size but another
    storage format: the replacement's renders (captured as graphs by the
    first) must read the new scene, not replay the old one's launches."""
    scene, batch = synth.make_config(1, n_envs=4)
    first = _upload(R, scene, "f16")
    for _ in range(2):                       # the second render replays the captured graphs
        _render(R, first, batch)
    _torch().cuda.synchronize()              # destroying a scene with renders in flight is refused
    R.remove_scene(first)
    sid = _upload(R, scene, "bf16")
    at = decoded_attrs(scene, "bf16")
    for _ in range(2):
        got = _render(R, sid, batch)
    for e in (0, 3):
        _check_bins(R, sid, scene, batch, 0, e, attrs=at)
        ref = render_ref(scene, batch, 0, e, R.tile_size, attrs=at)
        _check_image(_img(got, 0, e), ref, f"cfg1 bf16 after f16 env {e}")
    R.remove_scene(sid)


def test_cfg3_uneven_two_slots(R):
    scene, batch = synth.make_config(3, n_envs=16)
    sid = _upload(R, scene, "bf16")
    at = decoded_attrs(scene, "bf16")
    got = _render(R, sid, batch)
    assert tuple(got[0][0].shape) == (16, 128, 128, 3) and tuple(got[1][0].shape) == (16, 480, 640, 3)
    for c, e in ((0, 3), (1, 3), (1, 15)):
        _check_bins(R, sid, scene, batch, c, e, attrs=at)
        ref = render_ref(scene, batch, c, e, R.tile_size, attrs=at)
        _check_image(_img(got, c, e), ref, f"cfg3 slot {c} env {e}")
    R.remove_scene(sid)


# ------------------------------------------------------------------ invariances and edge cases
def test_tile_size_invariance():
    _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(0)
    outs = {}
    for ts in (8, 16, 32):
        r = gsr.Renderer(0, tile_size=ts)
        sid = r.add_synth_scene(scene)
        if ts != 16:
            cams, vm, poses = gsr.batch_tensors(batch)
            got = r.debug_bins(sid, cams, vm, poses, 0)
            ref = bin_ref(scene, batch, 0, 0, ts)
            np.testing.assert_array_equal(got["keys"], ref.keys)
            np.testing.assert_array_equal(got["values"], ref.values)
        outs[ts] = _img(_render(r, sid, batch), 0, 0)
        r.close()
    for ts in (8, 32):
        np.testing.assert_array_equal(outs[ts][0], outs[16][0])
        np.testing.assert_array_equal(outs[ts][1], outs[16][1])


def test_empty_and_degenerate_scenes(R):
    bg = (0.1, 0.6, 0.3)
    batch = one_camera(40, 30, 30.0, bg=bg)
    for label, scene in (("empty", scene_from(np.zeros((0, 3)), np.zeros((0, 3)), degree=0)),
                         ("behind", scene_from([[0, 0, -1.0], [0.1, 0, -0.5], [0, 0, 0.005]], [0.3] * 3, degree=0)),
                         ("transparent", scene_from([[0, 0, 2.0]], [0.3] * 3, opac=[0.5 / 255], degree=0))):
        sid = _upload(R, scene)
        rgb, depth, alpha = _img(_render(R, sid, batch), 0, 0)
        np.testing.assert_array_equal(rgb, np.broadcast_to(np.float32(bg), (30, 40, 3)), err_msg=label)
        assert (depth == 0).all() and (alpha == 0).all(), label
        R.remove_scene(sid)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_sh_degrees(R, degree):
    scene, batch = synth.make_config(1, n_envs=1)
    K = (degree + 1) ** 2
    sub = np.arange(0, scene.n, 7)
    keep = [int(np.searchsorted(sub, o)) for o in scene.body_offsets]
    s = scene_from(scene.means[sub], scene.scales[sub], scene.quats[sub], scene.opacities[sub],
                   scene.sh[sub][:, :K], degree=degree, body_offsets=keep)
    sid = _upload(R, s)
    got = _render(R, sid, batch)
    ref = render_ref(s, batch, 0, 0, R.tile_size)
    _check_image(_img(got, 0, 0), ref, f"degree {degree}")
    R.remove_scene(sid)


def test_invalid_render_arguments(R):
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(0)
    sid = _upload(R, scene)
    cams, vm, poses = gsr.batch_tensors(batch)
    with pytest.raises(gsr.GsrError) as ei:
        R.render(sid + 1000, cams, vm, poses)
    assert ei.value.code == gsr.GSR_E_NOT_FOUND
    bad = [gsr.Camera(0, 96, 100.0, 100.0, 64.0, 48.0)]
    with pytest.raises(gsr.GsrError) as ei:
        R.render(sid, bad, vm, poses)
    assert ei.value.code == gsr.GSR_E_INVALID
    R.remove_scene(sid)


def test_large_image_near_the_tile_limit(R):
    """1920 x 1080 (8160 tiles of 16, a ragged last tile row) with a dense
    scene: tile ids, pair offsets and the raster grid at their largest test
    sizes; tile lists bit-exact, pixels within tolerance."""
    scene = synth.make_scene(61, 60_000, 2, 5_000, sh_degree=1, half_box=4.0)
    rng = np.random.default_rng(12)
    cam = synth.pinhole(1920, 1080, 70.0)
    batch = synth.Batch(cams=[cam], viewmats=synth.orbit_viewmats(rng, 2, 3.0, 5.0)[None],
                        poses=synth.random_poses(rng, 2, scene.n_bodies), bg=np.array([0.2, 0.3, 0.4], np.float32))
    sid = _upload(R, scene)
    got = _render(R, sid, batch)
    ref = _check_bins(R, sid, scene, batch, 0, 1)
    assert ref.ranges.shape[0] == 120 * 68
    _check_image(_img(got, 0, 1), render_ref(scene, batch, 0, 1, R.tile_size), "1920x1080")
    R.remove_scene(sid)


def test_many_tiny_images_one_launch(R):
    """4096 environments of 24 x 16 (two ragged tiles each): many images per
    chunk and per raster segment; sampled images against the oracle."""
    scene = synth.make_scene(62, 3_000, 2, 500, sh_degree=0, half_box=2.0)
    rng = np.random.default_rng(13)
    E = 4096
    cam = synth.pinhole(24, 16, 60.0)
    batch = synth.Batch(cams=[cam], viewmats=synth.orbit_viewmats(rng, E, 2.5, 4.0)[None],
                        poses=synth.random_poses(rng, E, scene.n_bodies))
    sid = _upload(R, scene)
    got = _render(R, sid, batch)
    for e in (0, 1, 2049, E - 1):
        _check_image(_img(got, 0, e), render_ref(scene, batch, 0, e, R.tile_size), f"tiny env {e}")
    _check_bins(R, sid, scene, batch, 0, E - 1)
    R.remove_scene(sid)


def test_rectangles_beyond_255_tiles_per_axis(R):
    """A 4160 x 64 panorama: 260 tile columns, more than the packed 4-byte
    rectangle holds, so the chunk keeps the 2 x 16-bit rectangle format;
    projection rectangles, tile lists and pixels still match the oracle."""
    scene = synth.make_scene(64, 20_000, 1, 2_000, sh_degree=1, half_box=5.0)
    rng = np.random.default_rng(14)
    cam = synth.pinhole(4160, 64, 120.0)
    batch = synth.Batch(cams=[cam], viewmats=synth.orbit_viewmats(rng, 1, 1.0, 1.5)[None],
                        poses=synth.random_poses(rng, 1, scene.n_bodies))
    sid = _upload(R, scene)
    from paper_2604_25459_amd import gsr
    cams, vm, poses = gsr.batch_tensors(batch)
    proj = R.debug_project(sid, cams, vm, poses, 0, scene.n)
    p = project32(scene, batch, 0, 0, R.tile_size)
    vis = p["visible"]
    assert p["rect"][vis][:, 1].max() > 255
    np.testing.assert_array_equal(proj["rect"][vis], p["rect"][vis])
    ref = _check_bins(R, sid, scene, batch, 0, 0)
    assert ref.tiles_x == 260
    got = _render(R, sid, batch)
    _check_image(_img(got, 0, 0), render_ref(scene, batch, 0, 0, R.tile_size), "4160x64")
    R.remove_scene(sid)


def test_depth_sort_with_wide_and_narrow_key_spans(R):
    """One chunk with an image whose visible depths span 0.02 m .. 4 km (keys
    2^27 or more apart: the depth sort takes its fourth pass) and an image whose
    depths lie within 4 .. 6 m (three passes): keys, ids and ranges of both
    equal the oracle's bit for bit, and so do the pixels within tolerance."""
    rng = np.random.default_rng(23)
    n1, n2 = 3000, 2000
    z = np.exp(rng.uniform(np.log(0.02), np.log(4000.0), n1))
    far = np.stack([rng.uniform(-0.4, 0.4, n1) * z, rng.uniform(-0.3, 0.3, n1) * z, z], 1)
    near = np.stack([rng.uniform(-2.0, 2.0, n2), rng.uniform(-1.5, 1.5, n2), rng.uniform(-6.0, -4.0, n2)], 1)
    means = np.concatenate([far, near])
    scales = np.concatenate([np.repeat((0.01 * z)[:, None], 3, 1), np.full((n2, 3), 0.05)])
    scene = scene_from(means, scales * np.exp(rng.normal(0, 0.2, (n1 + n2, 3))), rng.standard_normal((n1 + n2, 4)),
                       rng.uniform(0.1, 0.9, n1 + n2), rng.uniform(0, 1, (n1 + n2, 1, 3)), degree=0)
    cam = one_camera(320, 240, 200.0).cams[0]
    back = np.array([[-1, 0, 0, 0], [0, 1, 0, 0], [0, 0, -1, 0]], np.float32)   # looks along -z
    vms = np.stack([np.eye(3, 4, dtype=np.float32), back])[None]
    batch = synth.Batch(cams=[cam], viewmats=vms, poses=np.zeros((2, 0, 7), np.float32),
                        bg=np.zeros(3, np.float32))
    spans = []
    for e in range(2):
        p = project32(scene, batch, 0, e)
        zb = p["zbits"][p["visible"]].astype(np.int64)
        spans.append(int(zb.max() - zb.min()))
    assert spans[0] >= 1 << 27 and spans[1] < 1 << 27
    sid = _upload(R, scene)
    for e in range(2):
        _check_bins(R, sid, scene, batch, 0, e)
    got = _render(R, sid, batch)
    for e in range(2):
        _check_image(_img(got, 0, e), render_ref(scene, batch, 0, e, R.tile_size), f"span env {e}")
    R.remove_scene(sid)


def test_stage_totals_match_oracle_bins():
    """The profiled renderer's totals of visible Gaussians and (tile,
    Gaussian) pairs equal the sums of the oracle's binning over the images."""
    _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(1, n_envs=6)
    r = gsr.Renderer(0, profile=True)
    sid = r.add_synth_scene(scene)
    cams, vm, poses = gsr.batch_tensors(batch)
    r.stage_times(reset=True)
    r.render(sid, cams, vm, poses)
    st = r.stage_times(reset=True)
    vis = pairs = 0
    for e in range(batch.n_envs):
        b = bin_ref(scene, batch, 0, e, r.tile_size)
        vis += int(b.visible.sum())
        pairs += len(b.keys)
    assert st["renders"] == 1
    assert st["visible"] == vis and st["pairs"] == pairs
    r.close()
